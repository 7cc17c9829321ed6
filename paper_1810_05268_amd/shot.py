"""Device buffers for one shot, on top of the C ABI (marshalling only).

A ``DeviceShot`` owns the torch tensors the C calls read and write (padded
velocity, wavelet samples, data, gradient, workspace) and forwards each call to
libwv.  No solver arithmetic happens here.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding as B


class DeviceShot:
    def __init__(self, ndim, n, h, nbl, space_order, nt, dt, vmax, vel_padded, wavelet, src, rec,
                 device="cuda", time_order=2):
        self.device = torch.device(device)
        self.vel = torch.as_tensor(np.ascontiguousarray(vel_padded, dtype=np.float32), device=self.device)
        self.wavelet = torch.as_tensor(np.ascontiguousarray(wavelet, dtype=np.float32), device=self.device)
        self.pb = B.Problem(ndim, n, h, nbl, space_order, nt, dt, vmax, self.vel, src, self.wavelet, rec,
                            time_order=time_order)
        self.shape = tuple(reversed(self.pb.padded))
        self.nt, self.nrec, self.P = self.pb.nt, self.pb.nrec, self.pb.P
        # bytes of one uncompressed checkpoint slot (two pitched field arrays)
        self.slot_bytes = 8 * self.pb.field_elements()
        self._ws = None

    def set_velocity(self, vel_padded) -> None:
        v = vel_padded if isinstance(vel_padded, torch.Tensor) else torch.as_tensor(
            np.ascontiguousarray(vel_padded, dtype=np.float32), device=self.device)
        self.vel = v.contiguous()
        self.pb.set_vel(self.vel)

    def workspace(self, op: int, mem_budget: int = 0) -> torch.Tensor:
        nb = self.pb.workspace_bytes(op, mem_budget)
        if self._ws is None or self._ws.numel() < nb:
            self._ws = None
            torch.cuda.synchronize(self.device)
            self._ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        # 256-byte aligned view
        off = (-self._ws.data_ptr()) % 256
        return self._ws[off: off + nb]

    def new_data(self) -> torch.Tensor:
        return torch.empty((self.nt + 1, self.nrec), dtype=torch.float32, device=self.device)

    def forward(self, want_state: bool = False):
        data = self.new_data()
        state = torch.empty((2,) + self.shape, dtype=torch.float32, device=self.device) if want_state else None
        B.forward(self.pb, data, self.workspace(B.OP_FORWARD), state_out=state)
        return (data, state) if want_state else data

    def gradient(self, residual, mem_budget: int, tol: float = 0.0, ratio_hint: float = 0.0,
                 timing: bool = False, out=None):
        g = out if out is not None else torch.empty(self.shape, dtype=torch.float64, device=self.device)
        st = B.gradient(self.pb, residual, mem_budget, tol, g, self.workspace(B.OP_GRADIENT, mem_budget),
                        ratio_hint=ratio_hint, timing=timing)
        return g, st

    def misfit_gradient(self, d_obs, mem_budget: int, tol: float = 0.0, ratio_hint: float = 0.0,
                        want_dsim: bool = False, timing: bool = False, out=None):
        g = out if out is not None else torch.empty(self.shape, dtype=torch.float64, device=self.device)
        dsim = self.new_data() if want_dsim else None
        phi, st = B.misfit_gradient(self.pb, d_obs, mem_budget, tol, g, self.workspace(B.OP_GRADIENT, mem_budget),
                                    ratio_hint=ratio_hint, d_sim=dsim, timing=timing)
        return (phi, g, st, dsim) if want_dsim else (phi, g, st)

    def adjoint_src(self, residual):
        out = torch.empty(self.nt, dtype=torch.float32, device=self.device)
        B.adjoint_src(self.pb, residual, out, self.workspace(B.OP_GRADIENT, 0))
        return out

    def compressibility(self, tol: float, stride: int) -> list:
        """Stream bytes of u^n every `stride` steps of a forward run (wv_compressibility)."""
        return B.compressibility(self.pb, tol, stride, self.workspace(B.OP_COMPRESSIBILITY))

    def checkpoint_bytes(self) -> int:
        """Bytes of one uncompressed checkpoint (two binary32 fields)."""
        return 8 * self.P
