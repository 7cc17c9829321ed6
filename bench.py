#!/usr/bin/env python3
"""Shot-gradient benchmark on one MI355X: compressed vs plain Revolve checkpointing.

One step = one checkpointed misfit + gradient evaluation of one shot (the whole
hot path: forward stencil with source injection and receiver gather, misfit,
Revolve schedule, checkpoint stores/restores through the codec, adjoint stencil
with the binary64 gradient accumulation), through the C ABI of libwv.

Default workload (the large 3-D shot): 320^3 interior + 40 absorbing cells per
side (400^3 = 64.0 M points), 12.5 m, space order 16, 3000 steps, Ricker 8 Hz,
320x320 surface receivers, 16e9 bytes of checkpoint memory.  Inputs are seeded
and synthetic (layered model with a dipping fault and a fast ellipsoid), resident
in HBM before timing starts.

Prints one JSON line.  ``value`` = effective Gpt/s of the compressed shot
gradient (P * 2N stencil updates of the forward + adjoint problem / wall time).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FWD_BYTES_PER_POINT = 20.0     # read u^n, d^n, w; write u^{n+1}, d^{n+1}
ADJ_BYTES_PER_POINT = 40.0     # read lam^k, mu, w, u^k, G(8); write lam^{k-1}, mu, G(8)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_shot(args):
    import workloads as W
    if args.quick:
        return W.fault_body_3d(n=(96, 96, 96), nbl=16, nt=400, order=16, f0=15.0)
    if args.workload == "fault_body_3d":
        return W.fault_body_3d()
    if args.workload == "layered_noise_3d":
        return W.layered_noise_3d()
    raise SystemExit(f"unknown workload {args.workload}")


def cpu_baseline(shot, counts, tol):
    """The FP64 oracle on the host cores, on a bounded sample of the same shot:
    two forward steps, two adjoint steps and the codec on a slab of one field,
    extrapolated with the schedule's exact counts."""
    import numpy as np

    import oracle
    import workloads as W
    dt = shot.cfl_frac * oracle.cfl_dt(shot.ndim, shot.h, shot.order, shot.vmax)
    q = W.ricker(shot.f0, dt, shot.nt)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    spec = oracle.ModelSpec(shot.ndim, shot.n, shot.h, shot.nbl, shot.order, shot.nt, dt, shot.vmax)
    S = oracle.Solver(spec, shot.padded("vel").astype(np.float64), shot.src, q, shot.rec, nthreads=threads)
    shape = spec.array_shape()
    rng = np.random.default_rng(0)
    cur = rng.standard_normal(shape) * 1e-3
    prev = rng.standard_normal(shape) * 1e-3
    t0 = time.perf_counter()
    for n in range(2):
        nxt = S.forward_step(n, cur, prev)
        prev, cur = cur, nxt
    t_fwd = (time.perf_counter() - t0) / 2
    res_row = rng.standard_normal(len(shot.rec))
    t0 = time.perf_counter()
    lam, lamp = cur, prev
    for _ in range(2):
        lm = S.adjoint_step(res_row, lam, lamp)
        lamp, lam = lam, lm
    t_adj = (time.perf_counter() - t0) / 2
    # codec on a slab of a smooth field (a quarter of the depth), scaled to a field
    nz = max(4, shape[0] // 4)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(shape[1]), np.arange(shape[2]), indexing="ij")
    slab = (np.sin(0.05 * x) * np.cos(0.07 * y) * np.sin(0.03 * z + 0.5)).astype(np.float32)
    t0 = time.perf_counter()
    s = oracle.encode(slab, tol)
    t_enc = (time.perf_counter() - t0) * shape[0] / nz
    t0 = time.perf_counter()
    oracle.decode(s)
    t_dec = (time.perf_counter() - t0) * shape[0] / nz
    total = (t_fwd * counts["advances"] + t_adj * counts["reverses"] + 2 * t_enc * counts["stores"]
             + 2 * t_dec * counts["restores"])
    P = int(np.prod(shape))
    return {"value": P * 2 * shot.nt / total / 1e9, "unit": "Gpt/s", "cores": threads, "kind": "oracle",
            "sample": (f"2 forward + 2 adjoint FP64 steps of the full {shape} grid and the codec on a "
                       f"{nz}-plane slab, extrapolated with the compressed run's counts "
                       f"(advances {counts['advances']}, reverses {counts['reverses']}, "
                       f"stores {counts['stores']}, restores {counts['restores']})"),
            "seconds_extrapolated": total, "s_per_forward_step": t_fwd, "s_per_adjoint_step": t_adj,
            "s_per_field_encode": t_enc, "s_per_field_decode": t_dec}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fault_body_3d")
    ap.add_argument("--tol", type=float, default=1e-4, help="codec tolerance of the headline run")
    ap.add_argument("--sweep", default="1e-3,1e-6", help="extra tolerances timed once each ('' = none)")
    ap.add_argument("--budget", type=float, default=16e9, help="checkpoint memory, bytes")
    ap.add_argument("--quick", action="store_true", help="small grid for a fast functional run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not part of it"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1810_05268_amd as P
    import workloads as W
    from paper_1810_05268_amd.shot import DeviceShot

    torch.cuda.set_device(0)
    shot = make_shot(args)
    dt = shot.cfl_frac * P.cfl_dt(shot.ndim, shot.h, shot.order, shot.vmax)
    q = W.ricker(shot.f0, dt, shot.nt)
    log(f"workload {shot.name} interior {shot.n} nbl {shot.nbl} order {shot.order} nt {shot.nt} dt {dt:.3e}")
    G = DeviceShot(shot.ndim, shot.n, shot.h, shot.nbl, shot.order, shot.nt, dt, shot.vmax, shot.padded("vel"),
                   q.astype(np.float32), shot.src, shot.rec)
    budget = int(args.budget)
    Pn = G.P
    # observed data from the model with the anomaly (untimed set-up)
    G.set_velocity(shot.padded("true"))
    d_obs = G.forward()
    G.set_velocity(shot.padded("vel"))
    torch.cuda.synchronize()
    g_plain = torch.empty(G.shape, dtype=torch.float64, device="cuda")
    g_comp = torch.empty(G.shape, dtype=torch.float64, device="cuda")

    def timed(tol, hint, out, n):
        walls, stats = [], []
        for _ in range(n):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            phi, _, st = G.misfit_gradient(d_obs, budget, tol, hint, timing=True, out=out)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            stats.append(st)
        return walls, stats, phi

    # plain Revolve (no compression)
    log("plain revolve ...")
    timed(0.0, 0.0, g_plain, args.warmup)
    w_plain, st_plain, phi_plain = timed(0.0, 0.0, g_plain, args.steps)
    log(f"plain: {statistics.mean(w_plain):.3f} s  M={st_plain[0]['slots']} advances={st_plain[0]['advances']}")

    # compressed: the first (warm-up) call measures the ratio on the final state; later
    # calls reuse it as the hint, as an optimisation loop would from one iteration to the next
    log("compressed ...")
    _, st0, _ = timed(args.tol, 0.0, g_comp, max(1, args.warmup))
    hint = 0.95 * st0[-1]["ratio_planned"]
    w_comp, st_comp, phi_comp = timed(args.tol, hint, g_comp, args.steps)
    err = float(torch.linalg.vector_norm(g_comp - g_plain) / torch.linalg.vector_norm(g_plain))
    log(f"compressed tol {args.tol}: {statistics.mean(w_comp):.3f} s  M={st_comp[0]['slots']} "
        f"ratio={st_comp[0]['ratio']:.1f} advances={st_comp[0]['advances']} grad err vs plain {err:.3e}")

    sweep = []
    for tol in [float(t) for t in args.sweep.split(",") if t.strip()]:
        _, sp0, _ = timed(tol, 0.0, g_comp, 1)
        ws_, ss_, _ = timed(tol, 0.95 * sp0[-1]["ratio_planned"], g_comp, 1)
        e = float(torch.linalg.vector_norm(g_comp - g_plain) / torch.linalg.vector_norm(g_plain))
        sweep.append({"tol": tol, "shot_s": ws_[0], "slots": ss_[0]["slots"], "ratio": ss_[0]["ratio"],
                      "advances": ss_[0]["advances"], "grad_rel_err_vs_plain": e,
                      "speedup_vs_plain": statistics.mean(w_plain) / ws_[0]})
        log(f"sweep tol {tol}: {ws_[0]:.3f} s ratio {ss_[0]['ratio']:.1f} err {e:.3e}")

    # per-phase device times over the timed compressed steps (HIP events on the call's stream)
    adv = sum(s["advances"] for s in st_comp)
    rev = sum(s["reverses"] for s in st_comp)
    ms_f = sum(s["ms_forward"] for s in st_comp)
    ms_a = sum(s["ms_adjoint"] for s in st_comp)
    fwd_ms = ms_f / adv
    adj_ms = ms_a / rev
    fwd_gbs = FWD_BYTES_PER_POINT * Pn / (fwd_ms * 1e-3) / 1e9
    adj_gbs = ADJ_BYTES_PER_POINT * Pn / (adj_ms * 1e-3) / 1e9
    dom = "adjoint" if ms_a >= ms_f else "forward"
    ach = adj_gbs if dom == "adjoint" else fwd_gbs
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "stencil3d adjoint+gradient step" if dom == "adjoint" else "stencil3d forward step",
            "bytes_per_launch": (ADJ_BYTES_PER_POINT if dom == "adjoint" else FWD_BYTES_PER_POINT) * Pn,
            "avg_launch_ms": adj_ms if dom == "adjoint" else fwd_ms,
            "forward_step": {"avg_ms": fwd_ms, "GBs": round(fwd_gbs, 1), "frac": round(fwd_gbs / HBM_PEAK_GBS, 4)},
            "adjoint_step": {"avg_ms": adj_ms, "GBs": round(adj_gbs, 1), "frac": round(adj_gbs / HBM_PEAK_GBS, 4)}}
    st = st_comp[0]
    enc_gbs = 8.0 * Pn * st["stores"] / (st["ms_store"] * 1e-3) / 1e9 if st["ms_store"] > 0 else None
    dec_gbs = 8.0 * Pn * st["decodes"] / (st["ms_restore"] * 1e-3) / 1e9 if st["ms_restore"] > 0 else None

    ms_step = 1e3 * statistics.mean(w_comp)
    value = Pn * 2 * shot.nt / (ms_step * 1e-3) / 1e9
    lat = sorted(1e3 * w for w in w_comp)
    out = {
        "metric": "shot-gradient s & Gpt/s vs plain at fixed grad err; HBM GB/s; p50/p99 lat",
        "value": round(value, 3), "unit": "Gpt/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"{shot.name} {shot.n[0]}x{shot.n[1]}x{shot.n[2]} + {shot.nbl} layer, "
                                f"order {shot.order}, {shot.nt} steps, budget {budget:.3g} B, tol {args.tol:g}"),
                   "points": Pn, "nt": shot.nt, "mem_budget": budget, "tol": args.tol},
        "shot_gradient_s": {"compressed": round(ms_step / 1e3, 4), "plain": round(statistics.mean(w_plain), 4)},
        "speedup_vs_plain": round(statistics.mean(w_plain) * 1e3 / ms_step, 4),
        "grad_rel_err_vs_plain": err,
        "plain_gpts": round(Pn * 2 * shot.nt / statistics.mean(w_plain) / 1e9, 3),
        "latency_ms": {"p50": lat[len(lat) // 2], "p99": lat[min(len(lat) - 1, math.ceil(0.99 * len(lat)) - 1)]},
        "schedule": {"compressed": {k: st[k] for k in ("slots", "advances", "stores", "restores", "decodes",
                                                         "ratio")},
                     "plain": {k: st_plain[0][k] for k in ("slots", "advances", "stores", "restores")}},
        "phase_ms": {"compressed": {k: st[k] for k in ("ms_forward", "ms_adjoint", "ms_store", "ms_restore")},
                     "plain": {k: st_plain[0][k] for k in ("ms_forward", "ms_adjoint", "ms_store", "ms_restore")}},
        "codec_GBs_uncompressed": {"encode": enc_gbs, "decode": dec_gbs},
        "misfit": {"compressed": phi_comp, "plain": phi_plain},
        "sweep": sweep,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample) ...")
        out["cpu_baseline"] = cpu_baseline(shot, {"advances": st["advances"], "reverses": st["reverses"],
                                                  "stores": st["stores"], "restores": st["decodes"]}, args.tol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
