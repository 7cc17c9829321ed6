"""Checkpointed, compressed adjoint acoustic gradients on MI355X (gfx950).

The compute path is the HIP library ``libwv.so`` (C ABI in ``include/wv.h``);
this package only marshals arguments to it:

* ``_binding``: ctypes declarations and thin wrappers of every C entry point;
* ``shot.DeviceShot``: device buffers of one shot;
* ``autograd.WaveMisfit``: torch.autograd.Function velocity -> misfit;
* ``serving``: continuous-batching shot-gradient engine;
* ``build``: compiles the HIP sources in-tree for gfx950.
"""
from ._binding import (OP_FORWARD, OP_GRADIENT, Problem, WvError, adjoint_src, batch_misfit_gradient,  # noqa
                       batch_workspace_bytes, cfl_dt, forward, gradient,
                       choose, costs_from_stats, lib, misfit_gradient, misfit_gradient_auto, pad_velocity, plan, predict, schedule,
                       schedule_forward_steps, stream_ceiling, velocity_gradient, zfpk_decode, zfpk_encode, zfpk_encode_noalloc,
                       zfpk_max_bytes, zfpk_workspace_bytes)

__all__ = ["OP_FORWARD", "OP_GRADIENT", "Problem", "WvError", "adjoint_src", "batch_misfit_gradient",
           "batch_workspace_bytes", "cfl_dt", "choose", "costs_from_stats",
           "forward",
           "gradient", "lib", "misfit_gradient", "misfit_gradient_auto", "pad_velocity", "plan", "predict", "schedule", "schedule_forward_steps", "stream_ceiling",
           "velocity_gradient",
           "zfpk_decode", "zfpk_encode", "zfpk_encode_noalloc", "zfpk_max_bytes", "zfpk_workspace_bytes"]
