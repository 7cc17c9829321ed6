"""Shared test helpers: build the oracle and the GPU path from one seeded workload.

Each side computes its own dt from its own CFL formula (they agree to the last
bit, see test_lib_host.py); the Ricker samples come from the input generator."""
from __future__ import annotations

import numpy as np

import oracle
import workloads as W


def has_gpu() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:        # noqa: BLE001
        return False


def oracle_side(shot: W.Shot, which: str = "vel", nthreads=None, time_order: int = 2):
    dt = shot.cfl_frac * oracle.cfl_dt(shot.ndim, shot.h, shot.order, shot.vmax, time_order=time_order)
    spec = oracle.ModelSpec(shot.ndim, shot.n, shot.h, shot.nbl, shot.order, shot.nt, dt, shot.vmax,
                            time_order=time_order)
    q = W.ricker(shot.f0, dt, shot.nt)
    vel = shot.padded(which).astype(np.float64)
    return oracle.Solver(spec, vel, shot.src, q, shot.rec, nthreads=nthreads), dt


def gpu_side(shot: W.Shot, which: str = "vel", time_order: int = 2):
    import paper_1810_05268_amd as P
    from paper_1810_05268_amd.shot import DeviceShot
    dt = shot.cfl_frac * P.cfl_dt(shot.ndim, shot.h, shot.order, shot.vmax, time_order=time_order)
    q = W.ricker(shot.f0, dt, shot.nt).astype(np.float32)
    return DeviceShot(shot.ndim, shot.n, shot.h, shot.nbl, shot.order, shot.nt, dt, shot.vmax,
                      shot.padded(which), q, shot.src, shot.rec, time_order=time_order), dt


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def small_3d(n=(44, 38, 41), nbl=8, order=8, nt=120, f0=25.0, seed=2) -> W.Shot:
    """Ragged 3-D case: extents not multiples of the 32-wide tiles, several z chunks."""
    return W.layered_noise_3d(n=n, h=(10.0, 10.0, 10.0), nbl=nbl, nt=nt, order=order, seed=seed, f0=f0)
