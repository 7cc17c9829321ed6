"""Writes fault_body_3000.npz: the FP64 oracle's forward run of the large 3-D shot
(320^3 interior + 40 absorbing cells per side = 400^3 points, 12.5 m, space order 16,
all 3000 steps, Ricker 8 Hz, 320 x 320 surface receivers), sampled so that a GPU test
can measure the long-run drift of the binary32 stencils against it.

Calls only the oracle and the seeded input generator (no GPU code).  Stored:
  u_sub, up_sub  u^3000 and u^2999 on the subgrid of every 10th point per axis
                 (binary64 values rounded to binary32, 40^3 each);
  u_norm, up_norm, data_norm  2-norms of the full fields and of all receiver data;
  rec_idx, data_sub  the traces (all 3001 rows) of 36 receivers (x, y = 20, 70, ..., 270).
Run:  python tests/golden/make_fault_body_3000.py   (about 45 minutes on 8 cores)."""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

SUB = 10
REC_XY = list(range(20, 320, 50))


def main(out=os.path.join(os.path.dirname(os.path.abspath(__file__)), "fault_body_3000.npz")):
    shot = W.fault_body_3d()
    dt = shot.cfl_frac * oracle.cfl_dt(shot.ndim, shot.h, shot.order, shot.vmax)
    spec = oracle.ModelSpec(shot.ndim, shot.n, shot.h, shot.nbl, shot.order, shot.nt, dt, shot.vmax)
    q = W.ricker(shot.f0, dt, shot.nt)
    S = oracle.Solver(spec, shot.padded("vel").astype(np.float64), shot.src, q, shot.rec)
    t0 = time.time()
    fw = S.forward(want_last=True)
    print(f"oracle forward: {time.time() - t0:.0f} s", flush=True)
    u, up = fw["last"]
    data = fw["data"]
    rec_idx = np.array([iy * shot.n[0] + ix for iy in REC_XY for ix in REC_XY], dtype=np.int64)
    with open(os.path.join(ROOT, "oracle", "wv_oracle.c"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    np.savez_compressed(out, u_sub=u[::SUB, ::SUB, ::SUB].astype(np.float32),
                        up_sub=up[::SUB, ::SUB, ::SUB].astype(np.float32),
                        u_norm=np.linalg.norm(u), up_norm=np.linalg.norm(up), data_norm=np.linalg.norm(data),
                        rec_idx=rec_idx, data_sub=data[:, rec_idx].astype(np.float32), dt=dt, sub=SUB,
                        oracle_sha256=sha)
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main()
