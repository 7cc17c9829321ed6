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

Beside it: the plain (recompute-only) Revolve time at the same memory budget and
the gradient error between the two; a tolerance sweep; per-kernel device times
of the stencil launches (HIP events on the call's stream) priced at the
algorithmic bytes per point (forward 16 B, adjoint + gradient 36 B); the serving
stream (200 Poisson requests at 2/s of mixed 2-D / 3-D shots through the
continuous-batching engine: p50/p99 latency from arrival, throughput); and the
FP64 oracle timed on a bounded sample on the host cores.

``--kernels`` runs only a short kernel workload for hardware-counter passes
(a 1 GiB copy for calibration, then 12 forward and 12 adjoint steps of the
large grid).
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
# algorithmic bytes per point and step (what the method must move):
FWD_BYTES_PER_POINT = 16.0     # read u^n, u^{n-1}, w; write u^{n+1}
ADJ_BYTES_PER_POINT = 36.0     # read lam^k, lam^{k+1}, w, u^k; write lam^{k-1}; read + write the FP64 gradient
COUNTERS = os.path.join(ROOT, "profiles", "stencil3d_fault_body_3d_counters.txt")
STENCIL_SRC = [os.path.join(ROOT, "paper_1810_05268_amd", "csrc", f) for f in ("wv_stencil.hip", "wv_stencil_dev.h")]


def stencil_source_sha256() -> str:
    """sha256 of the stencil kernels' sources (the kernel file, then its device header)."""
    import hashlib
    h = hashlib.sha256()
    for f in STENCIL_SRC:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


# wv_stats.timing bits: 1 = HIP events around every schedule action (per-phase device
# times, for the run-time model), 2 = events recorded by every stencil dispatch (the
# roofline).  The timed steps use launch events only; per-action events add dependent
# packets between kernels and cost about 4 % of the wall time.
TIMING_ACTIONS = 1
TIMING_LAUNCHES = 2


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


def ot4_block(shot, budget, tol, steps, codec_costs):
    """The same shot with the OT4 kernel (fourth order in time: two stencil passes per
    forward step, three per adjoint step), at 0.4 of its own stability limit: plain
    against compressed Revolve at the same memory budget, with the model's predictions.
    As the paper validates its model on OT4 with compression, the compressed OT4 run is
    predicted from other runs' costs: the OT4 plain run's stencil costs and the OT2
    compressed run's codec costs (the codec does not depend on the time order), at the
    planning ratio of the OT4 run's own profile."""
    import numpy as np
    import torch

    import paper_1810_05268_amd as P
    import workloads as W
    from paper_1810_05268_amd.shot import DeviceShot
    dt = shot.cfl_frac * P.cfl_dt(shot.ndim, shot.h, shot.order, shot.vmax, time_order=4)
    q = W.ricker(shot.f0, dt, shot.nt).astype(np.float32)
    G = DeviceShot(shot.ndim, shot.n, shot.h, shot.nbl, shot.order, shot.nt, dt, shot.vmax, shot.padded("true"),
                   q, shot.src, shot.rec, time_order=4)
    d_obs = G.forward()
    G.set_velocity(shot.padded("vel"))
    gp = torch.empty(G.shape, dtype=torch.float64, device="cuda")
    gc = torch.empty(G.shape, dtype=torch.float64, device="cuda")

    def run(tol_, hint, out, n, timing):
        walls, st = [], None
        for _ in range(n):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, st = G.misfit_gradient(d_obs, budget, tol_, hint, timing=timing, out=out)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
        return walls, st
    log("OT4 plain ...")
    wp, sp = run(0.0, 0.0, gp, steps, TIMING_LAUNCHES)
    _, sp_ph = run(0.0, 0.0, gp, 1, TIMING_ACTIONS)
    log("OT4 compressed ...")
    _, s0 = run(tol, 0.0, gc, 1, 0)
    h = plan_hint(s0, G.P, shot.nt, budget)
    wc, sc = run(tol, h, gc, steps, TIMING_LAUNCHES)
    _, sc_ph = run(tol, h, gc, 1, TIMING_ACTIONS)
    err = float(torch.linalg.vector_norm(gc - gp) / torch.linalg.vector_norm(gp))
    cp, cc = P.costs_from_stats(sp_ph), P.costs_from_stats(sc_ph)
    pp = P.predict(shot.nt, G.P, budget, False, cp["c_f"], cp["c_r"], t_copy=cp["t_store"], slot_bytes=G.slot_bytes)
    px = P.predict(shot.nt, G.P, budget, True, cp["c_f"], cp["c_r"], t_c=codec_costs["t_store"],
                   t_d=codec_costs["t_d"], ratio=h)
    meas_c = sum(sc_ph[k] for k in ("ms_forward", "ms_adjoint", "ms_store", "ms_restore"))
    out = {"dt": dt, "shot_gradient_s": {"plain": statistics.mean(wp), "compressed": statistics.mean(wc)},
           "speedup_vs_plain": statistics.mean(wp) / statistics.mean(wc), "grad_rel_err_vs_plain": err,
           "schedule": {"plain": {k: sp[k] for k in ("slots", "advances", "stores")},
                        "compressed": {k: sc[k] for k in ("slots", "advances", "stores", "decodes", "ratio")}},
           "step_ms": {"forward": sp["ms_fwd_kernel"] / sp["advances"], "adjoint": sp["ms_adj_kernel"] / sp["reverses"]},
           "model": {"plain": {"predicted_ms": pp["ms_total"], "measured_ms": sum(sp_ph[k] for k in (
                         "ms_forward", "ms_adjoint", "ms_store", "ms_restore"))},
                     "compressed": {"predicted_ms": px["ms_total"], "measured_ms": meas_c,
                                    "rel_err": (px["ms_total"] - meas_c) / meas_c, "slots": px["slots"],
                                    "advances": px["advances"],
                                    "costs_from": "OT4 plain run (stencils) and OT2 compressed run (codec)"},
                     "full_storage_ms": pp["ms_full_storage"]}}
    log(f"OT4: plain {out['shot_gradient_s']['plain']:.3f} s, compressed {out['shot_gradient_s']['compressed']:.3f} s "
        f"({out['speedup_vs_plain']:.2f}x), grad err {err:.2e}")
    return out


def plan_hint(st, points, nt, budget):
    """Planning ratio for the next call of the same shot and tolerance, as an
    optimisation loop would carry it from one iteration to the next: the slot count
    wv_plan finds for the compressibility profile the previous call measured (stream
    sizes of its stored states over time), as the ratio that makes the call plan it."""
    import paper_1810_05268_amd as P
    prof = st["profile"]
    if all(x > 0 for x in prof):
        _, h = P.plan(nt, points, budget, prof)
        if h > 0:
            return h
    return 0.95 * st["ratio_planned"]


def full_trajectory_bytes(st, nt):
    """Compressed bytes of all states u^1..u^nt from a call's profile (linear between
    the samples), each stream rounded up to 256 bytes."""
    import numpy as np
    ks = [0] + [-(-(j * nt) // 16) for j in range(1, 17)]
    sizes = np.interp(np.arange(1, nt + 1), ks, st["profile"])
    return float(np.sum(np.ceil(sizes / 256.0) * 256.0))


def stream_ceilings(stream_bytes=256 * 1000 * 1000, reps=10):
    """Measured HBM ceilings in this process (wv_stream_ceiling): streams of 3 reads + 1
    write (the forward stencil's mix) and 4 reads + 1 write, 256 MB each (the large grid's
    field size), the first read through the caches and the others and the write
    nontemporal, as the stencils access their arrays; GB/s of bytes read plus written,
    the best of reps."""
    import torch
    import paper_1810_05268_amd as P
    ws = torch.empty(5 * stream_bytes + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    out = {f"{r}r1w_gbs": round(P.stream_ceiling(r, stream_bytes, ws[off:], reps), 1) for r in (3, 4)}
    del ws
    torch.cuda.empty_cache()
    return out


def raw_gpts(stats, points):
    """Stencil point updates per second of stencil kernel time over calls timed with
    per-launch events (Gpt/s)."""
    upd = sum(s["advances"] + s["reverses"] for s in stats)
    ms = sum(s["ms_fwd_kernel"] + s["ms_adj_kernel"] for s in stats)
    return round(points * upd / (ms * 1e-3) / 1e9, 3) if ms > 0 else None


def performance_model(nt, points, slot_bytes, budget, st_plain, st_comp, hint, sweep_stats):
    """The run-time model (wv_predict) fed with the per-unit costs of the timed plain
    and compressed calls: predicted against measured device time of each run, as the
    paper validates its model.  Sweep runs are predicted with the headline costs and
    their own planning ratio."""
    import paper_1810_05268_amd as P

    def phases(st):
        return st["ms_forward"] + st["ms_adjoint"] + st["ms_store"] + st["ms_restore"]
    cp, cc = P.costs_from_stats(st_plain), P.costs_from_stats(st_comp)
    rows = []
    pr = P.predict(nt, points, budget, False, cp["c_f"], cp["c_r"], t_copy=cp["t_store"], slot_bytes=slot_bytes)
    rows.append({"run": "plain", "predicted_ms": pr["ms_total"], "measured_ms": phases(st_plain),
                 "slots": pr["slots"], "advances": pr["advances"]})
    pr = P.predict(nt, points, budget, True, cc["c_f"], cc["c_r"], t_c=cc["t_store"], t_d=cc["t_d"], ratio=hint)
    rows.append({"run": "compressed", "predicted_ms": pr["ms_total"], "measured_ms": phases(st_comp),
                 "slots": pr["slots"], "advances": pr["advances"]})
    for tol, h, st in sweep_stats:
        pr = P.predict(nt, points, budget, True, cc["c_f"], cc["c_r"], t_c=cc["t_store"], t_d=cc["t_d"], ratio=h)
        rows.append({"run": f"compressed tol {tol:g}", "predicted_ms": pr["ms_total"], "measured_ms": phases(st),
                     "slots": pr["slots"], "advances": pr["advances"]})
    for r in rows:
        r["rel_err"] = (r["predicted_ms"] - r["measured_ms"]) / r["measured_ms"]
    full = P.predict(nt, points, budget, False, cp["c_f"], cp["c_r"], t_copy=cp["t_store"],
                     slot_bytes=slot_bytes)["ms_full_storage"]
    # the decision the model exists for: compress at this budget or not (from the timed
    # compressed call's compressibility profile), against which run measured faster
    ch = P.choose(nt, points, budget, cp, cc, profile=st_comp["profile"], slot_bytes=slot_bytes)
    ch["measured_faster"] = "compressed" if phases(st_comp) < phases(st_plain) else "plain"
    # the paper's predicted speed-up against memory (its Fig. 5): the same costs and
    # profile over budgets from 0.5 GB to 4 TB; compressed storage of the whole trajectory
    # and plain full storage mark the two regime boundaries
    curve = []
    for gb in (0.5, 1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 1536, 2048, 4096):
        b = int(gb * 1e9)
        c = P.choose(nt, points, b, cp, cc, profile=st_comp["profile"], slot_bytes=slot_bytes)
        pp = P.predict(nt, points, b, False, cp["c_f"], cp["c_r"], t_copy=cp["t_store"], slot_bytes=slot_bytes)
        mc, _ = P.plan(nt, points, b, st_comp["profile"])
        curve.append({"budget_gb": gb, "ms_plain": c["ms_plain"], "ms_compressed": c["ms_compressed"],
                      "speedup": c["ms_plain"] / c["ms_compressed"], "slots_plain": pp["slots"],
                      "slots_compressed": mc})
    regimes = {"compressed_trajectory_gb": full_trajectory_bytes(st_comp, nt) / 1e9,
               "plain_full_storage_gb": (nt + 1) * slot_bytes / 1e9}
    # and against the number of steps and the cost of a step (its Fig. 6), at this budget:
    # the profile read as a function of relative time; the stencil costs scaled, the codec
    # costs kept (a costlier physics per step with the same fields)
    steps_curve = []
    for n in (500, 1000, 2000, 3000, 6000, 12000):
        c = P.choose(n, points, budget, cp, cc, profile=st_comp["profile"], slot_bytes=slot_bytes)
        steps_curve.append({"nt": n, "ms_plain": c["ms_plain"], "ms_compressed": c["ms_compressed"],
                            "speedup": c["ms_plain"] / c["ms_compressed"]})
    cost_curve = []
    for f in (0.25, 0.5, 1.0, 2.0, 4.0, 8.0):
        cpf = dict(cp, c_f=cp["c_f"] * f, c_r=cp["c_r"] * f)
        ccf = dict(cc, c_f=cc["c_f"] * f, c_r=cc["c_r"] * f)
        c = P.choose(nt, points, budget, cpf, ccf, profile=st_comp["profile"], slot_bytes=slot_bytes)
        cost_curve.append({"step_cost_factor": f, "ms_plain": c["ms_plain"], "ms_compressed": c["ms_compressed"],
                           "speedup": c["ms_plain"] / c["ms_compressed"]})
    return {"costs_plain": cp, "costs_compressed": cc, "full_storage_ms": full, "runs": rows, "choice": ch,
            "speedup_vs_memory": curve, "regimes": regimes, "speedup_vs_steps": steps_curve,
            "speedup_vs_step_cost": cost_curve}


def traffic_per_launch():
    """HBM bytes per launch of the forward and adjoint stencils from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each
    scaled by what the counter reads for a plain copy of known size), or None when
    the stencil source has changed since the counters were taken."""
    if not os.path.exists(COUNTERS):
        return None
    kv = {}
    for line in open(COUNTERS):
        if ":" in line and not line.lstrip().startswith(("#", "|", "`")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("stencil_source_sha256") != stencil_source_sha256():
        return None
    ff, wf = float(kv["fetch_scale"]), float(kv["write_scale"])
    out = {}
    for k in ("forward", "adjoint"):
        out[k] = 1024.0 * (ff * float(kv[f"{k}_fetch_kib"]) + wf * float(kv[f"{k}_write_kib"]))
    return out


def kernels_mode():
    """Short workload for counter passes: 1 GiB copy (calibration), 12 forward steps,
    12 adjoint steps of the large grid."""
    import numpy as np
    import torch

    import paper_1810_05268_amd as P
    import workloads as W
    from paper_1810_05268_amd.shot import DeviceShot
    n = 256 * 1024 * 1024
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    del a, b
    nt = 12
    shot = W.fault_body_3d(nt=nt)
    dt = shot.cfl_frac * P.cfl_dt(shot.ndim, shot.h, shot.order, shot.vmax)
    q = W.ricker(shot.f0, dt, nt).astype(np.float32)
    G = DeviceShot(3, shot.n, shot.h, shot.nbl, shot.order, nt, dt, shot.vmax, shot.padded("vel"), q,
                   shot.src, shot.rec)
    G.forward()
    res = torch.randn(nt + 1, len(shot.rec), device="cuda") * 1e-3
    g, st = G.gradient(res, 8 * G.P * (nt + 2), timing=3)
    torch.cuda.synchronize()
    print(json.dumps({"kernels": "copy 1 GiB x3, forward x12 (+12 in the gradient call), adjoint x12",
                      "fwd_ms": st["ms_fwd_kernel"] / st["advances"], "adj_ms": st["ms_adj_kernel"] / st["reverses"],
                      "points": G.P}), flush=True)


def codec_kernels_mode(nt=1500, tol=1e-4, reps=5):
    """Short workload for the codec's counter and trace passes: the large shot's forward
    run to step nt (1500: a mid-run state, compressed about 70x at 1e-4; 2900: a late
    one, about 20x), then `reps` encodes
    and decodes of u^nt alone and `reps` encodes of u^nt - u^(nt-1) (the second-level
    form the compressed reversal stores)."""
    import numpy as np
    import torch

    import paper_1810_05268_amd as P
    import workloads as W
    from paper_1810_05268_amd.shot import DeviceShot
    shot = W.fault_body_3d(nt=nt)
    dt = shot.cfl_frac * P.cfl_dt(shot.ndim, shot.h, shot.order, shot.vmax)
    q = W.ricker(shot.f0, dt, nt).astype(np.float32)
    G = DeviceShot(3, shot.n, shot.h, shot.nbl, shot.order, nt, dt, shot.vmax, shot.padded("vel"), q,
                   shot.src, shot.rec)
    data, state = G.forward(want_state=True)
    u, up = state[0].contiguous(), state[1].contiguous()
    del data, state, G
    dims = list(reversed(u.shape))
    cap = P.zfpk_max_bytes(3, dims)
    out = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    wsb = P.zfpk_workspace_bytes(3, dims)
    ws = torch.zeros(wsb + 256, dtype=torch.uint8, device="cuda")
    wso = (-ws.data_ptr()) % 256
    dec = torch.empty_like(u)
    nb = 0
    for _ in range(reps):
        nb = P.zfpk_encode(u, tol, out, ws[wso: wso + wsb])
    for _ in range(reps):
        P.zfpk_decode(out, dec, nbytes=nb)
    d = u - up                       # the same binary32 difference the reversal's encoder forms
    nbd = 0
    for _ in range(reps):
        nbd = P.zfpk_encode(d, tol, out, ws[wso: wso + wsb])
    torch.cuda.synchronize()
    print(json.dumps({"codec_kernels": f"forward {nt} steps, then encode x{reps}, decode x{reps}, encode of the "
                      f"difference x{reps}", "tol": tol, "field_bytes": 4 * u.numel(), "stream_bytes": nb,
                      "diff_stream_bytes": nbd, "ratio": 4 * u.numel() / nb}), flush=True)


PROFILED_PER_CLASS = 3


SERVING_VMAX = 3700.0   # m/s: bound of every serving model (layers up to 3.5 km/s plus the 0.2 km/s anomaly)


def serving_leg(nreq, rate, pool_bytes, max_active, tol, cap, max_batch, saturation):
    """The serving stream: seeded Poisson arrivals of mixed shots through the engine, 2-D
    shots batched (one persistent launch per batch).  Untimed calls measure the
    compressibility profiles of each class's first requests; every request of the class
    then gets a checkpoint budget of 1.5 x the compressed full trajectory of their
    elementwise maximum (capped) and the plan for it as the hint.  All shots take their
    time step from one velocity bound, so a class shares dt and can share a batch.
    Then the saturation runs: the first half of the stream replayed at multiples of the
    rate, until the engine's throughput stops growing (queueing dominates)."""
    import numpy as np
    import torch

    import paper_1810_05268_amd as P
    import workloads as W
    from paper_1810_05268_amd.serving import Engine, replay
    from paper_1810_05268_amd.shot import DeviceShot
    reqs = W.serving_stream(nreq=nreq, rate=rate, seed=5)
    items, hints, budgets, profs, cls = [], {}, {}, {}, []
    for i, r in enumerate(reqs):
        s = r.shot
        dt = s.cfl_frac * P.cfl_dt(s.ndim, s.h, s.order, SERVING_VMAX)
        q = W.ricker(s.f0, dt, s.nt).astype(np.float32)
        G = DeviceShot(s.ndim, s.n, s.h, s.nbl, s.order, s.nt, dt, SERVING_VMAX, s.padded("true"), q, s.src,
                       s.rec)
        d_obs = G.forward()
        G.set_velocity(s.padded("vel"))
        c = s.extra["class"]
        if len(profs.setdefault(c, [])) < PROFILED_PER_CLASS:
            # untimed calls measure the compressibility profiles of the class's first requests
            _, _, st = G.misfit_gradient(d_obs, min(4 * G.P * (s.nt + 1), cap), tol)
            profs[c].append((s.nt, G.P, st["profile"]))
            G._ws = None
            torch.cuda.empty_cache()
        items.append([r.arrival, G, d_obs, 0, tol, 0.0])
        cls.append(c)
        if (i + 1) % 50 == 0:
            log(f"serving set-up: {i + 1}/{nreq} requests prepared")
    # shots of a class differ (peak frequency, layering), so their compressibility does:
    # plan from the largest stream sizes seen and leave 1.5 x the trajectory they give
    for c, lst in profs.items():
        nt, pts = lst[0][0], lst[0][1]
        pmax = [max(p[2][j] for p in lst) for j in range(17)]
        budgets[c] = int(min(cap, 1.5 * full_trajectory_bytes({"profile": pmax}, nt)))
        _, hints[c] = P.plan(nt, pts, budgets[c], pmax)
        profs[c] = pmax
    # Per class, the run-time model (wv_choose, fed with the per-unit costs of one plain and
    # one compressed call of the class's first request at its budget) decides whether
    # compression pays at that budget; plain checkpoints are exact, so they meet the
    # tolerance too.  The same calls, run again without events, check the choice.
    choice, tols = {}, {}
    for c in sorted(profs):
        i0 = cls.index(c)
        _, G, d_obs, _, _, _ = items[i0]
        _, _, stp = G.misfit_gradient(d_obs, budgets[c], 0.0, timing=TIMING_ACTIONS)
        _, _, stc = G.misfit_gradient(d_obs, budgets[c], tol, hints[c], timing=TIMING_ACTIONS)
        ch = P.choose(G.nt, G.P, budgets[c], P.costs_from_stats(stp), P.costs_from_stats(stc), profile=profs[c],
                      slot_bytes=G.slot_bytes)
        walls = {}
        for name, t_, h_ in (("plain", 0.0, 0.0), ("compressed", tol, hints[c])):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            G.misfit_gradient(d_obs, budgets[c], t_, h_)
            torch.cuda.synchronize()
            walls[name] = (time.perf_counter() - t0) * 1e3
        G._ws = None
        torch.cuda.empty_cache()
        tols[c] = tol if ch["compressed"] else 0.0
        choice[str(c)] = {"choice": "compressed" if ch["compressed"] else "plain",
                          "model_ms": {"plain": ch["ms_plain"], "compressed": ch["ms_compressed"]},
                          "measured_ms": walls}
        log(f"serving class {c}: model {ch['ms_plain']:.1f} ms plain, {ch['ms_compressed']:.1f} ms compressed -> "
            f"{choice[str(c)]['choice']}; measured {walls['plain']:.1f} / {walls['compressed']:.1f} ms")
    for it, c in zip(items, cls):
        it[3], it[4], it[5] = budgets[c], tols[c], (hints[c] if tols[c] > 0 else 0.0)
    items = [tuple(it) for it in items]
    torch.cuda.synchronize()
    eng = Engine(pool_bytes=pool_bytes, max_active=max_active, max_batch=max_batch)
    log(f"serving: replaying {nreq} requests at {rate}/s ...")
    res, wall = replay(eng, items, time_scale=1.0, timeout_s=150.0)
    eng.close()
    del eng
    torch.cuda.empty_cache()
    bad = [r["status"] for r in res if r["status"] != 0]
    for r, (arr, G, _, b, _, h) in zip(res, items):
        if r["status"] != 0 or r["stats"]["retries"]:
            log(f"serving: request at {arr:.2f} s (shape {G.shape}, budget {b:.3g}, hint {h:.1f}) status "
                f"{r['status']} retries {r['stats']['retries']}")
    lat = sorted(r["latency_ms"] for r in res)
    pts = sum(G.P * 2 * G.nt for _, G, _, _, _, _ in items)

    def pct(v, p):
        return v[min(len(v) - 1, max(0, math.ceil(p * len(v)) - 1))]
    per_class = {}
    for c in sorted(set(cls)):
        lc = sorted(r["latency_ms"] for r, k in zip(res, cls) if k == c)
        per_class[str(c)] = {"n": len(lc), "p50_ms": pct(lc, 0.5), "p99_ms": pct(lc, 0.99)}
    two_d = [r for r, k in zip(res, cls) if k == 0]
    batches = len({(r["t_start_ms"], r["t_end_ms"]) for r in two_d})
    # saturation: the first half of the stream at higher arrival rates
    sat = []
    half = items[: max(1, nreq // 2)]
    for mult in saturation:
        log(f"saturation x{mult}: replaying {len(half)} requests at {rate * mult:g}/s ...")
        eng = Engine(pool_bytes=pool_bytes, max_active=max_active, max_batch=max_batch)
        rs, w = replay(eng, half, time_scale=1.0 / mult, timeout_s=150.0)
        eng.close()
        del eng
        torch.cuda.empty_cache()
        ls = sorted(r["latency_ms"] for r in rs)
        sat.append({"offered_per_s": rate * mult, "req_per_s": len(half) / w, "p50_ms": pct(ls, 0.5),
                    "p99_ms": pct(ls, 0.99), "failed": sum(1 for r in rs if r["status"] != 0),
                    "queue_p50_ms": pct(sorted(r["queue_ms"] for r in rs), 0.5),
                    "retried": sum(1 for r in rs if r["stats"]["retries"])})
        log(f"saturation x{mult}: offered {rate * mult:.0f}/s -> {len(half) / w:.2f} req/s, p50 "
            f"{sat[-1]['p50_ms']:.0f} ms, p99 {sat[-1]['p99_ms']:.0f} ms, failed {sat[-1]['failed']}, "
            f"retried {sat[-1]['retried']}")
        if len(sat) >= 2 and sat[-1]["req_per_s"] < 1.1 * sat[-2]["req_per_s"]:
            break   # throughput no longer grows with the load: the engine is saturated
    return {"requests": nreq, "rate_per_s": rate, "failed": len(bad), "wall_s": wall,
            "max_batch": max_batch, "two_d_requests": len(two_d), "two_d_batches": batches,
            "saturation": sat, "capacity_req_per_s": max([x["req_per_s"] for x in sat] + [nreq / wall]),
            "capacity_note": "the largest throughput over the saturation runs (the stream's first half replayed "
                             "at multiples of the rate), where queueing dominates the latency",
            "retried": sum(1 for r in res if r["stats"]["retries"]),
            "p50_ms": pct(lat, 0.5), "p99_ms": pct(lat, 0.99), "req_per_s": nreq / wall,
            "gpts": pts / wall / 1e9, "per_class": per_class, "pool_bytes": pool_bytes, "max_active": max_active,
            "tol": tol, "ratio_hints": hints, "budgets": budgets, "class_choice": choice,
            "classes": "0: 2-D 512^2 order 8 1500 steps; 1: 3-D 160^3 order 8 1200 steps; "
                       "2: 3-D 256^3 order 12 2000 steps (interior; 20-cell layer; h = 10 m)"}


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


def oracle_errors(dt, threads):
    """Error of the GPU path against the FP64 oracle on the large shot's full 400^3 grid,
    on samples the oracle finishes in seconds (it cannot run the shot itself in minutes):
    a 20-step forward run (data and the final wavefield), an 8-step checkpointed gradient
    with 3 slots for a seeded residual (recomputation on), and the whole 3000-step
    forward run against the oracle's stored run of it (tests/golden/fault_body_3000.npz,
    written by tests/golden/make_fault_body_3000.py) when that file is present."""
    import numpy as np
    import torch

    import oracle
    import workloads as W
    from oracle import schedule as SC
    from paper_1810_05268_amd.shot import DeviceShot

    def rel(a, b):
        a = np.asarray(a, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

    out = {}
    for nt in (20, 8):
        sh = W.fault_body_3d(nt=nt)
        dto = sh.cfl_frac * oracle.cfl_dt(3, sh.h, sh.order, sh.vmax)
        spec = oracle.ModelSpec(3, sh.n, sh.h, sh.nbl, sh.order, nt, dto, sh.vmax)
        q = W.ricker(sh.f0, dto, nt)
        S = oracle.Solver(spec, sh.padded("vel").astype(np.float64), sh.src, q, sh.rec, nthreads=threads)
        G = DeviceShot(3, sh.n, sh.h, sh.nbl, sh.order, nt, dt, sh.vmax, sh.padded("vel"), q.astype(np.float32),
                       sh.src, sh.rec)
        if nt == 20:
            ref = S.forward(want_last=True)
            data, state = G.forward(want_state=True)
            out["forward_20_steps"] = {"data": rel(data.cpu().numpy(), ref["data"]),
                                       "u_N": rel(state[0].cpu().numpy(), ref["last"][0]),
                                       "u_N_1": rel(state[1].cpu().numpy(), ref["last"][1])}
            del ref, data, state
        else:
            M = 3
            res = np.random.default_rng(11).standard_normal((nt + 1, len(sh.rec))) * 1e-3
            res[0] = 0.0
            acts = SC.schedule(nt, M, write_min=True)
            g_or, st_or = S.gradient_actions(res, acts, M)
            g, st = G.gradient(torch.as_tensor(res.astype(np.float32), device="cuda"), G.slot_bytes * (M - 1))
            out["gradient_8_steps_3_slots"] = {"gradient": rel(g.cpu().numpy(), g_or),
                                               "advances": [st["advances"], st_or["advances"]]}
            del g
        del S, G
        torch.cuda.empty_cache()
    gold = os.path.join(ROOT, "tests", "golden", "fault_body_3000.npz")
    if os.path.exists(gold):
        ref = np.load(gold)
        sh = W.fault_body_3d()
        q = W.ricker(sh.f0, dt, sh.nt).astype(np.float32)
        G = DeviceShot(3, sh.n, sh.h, sh.nbl, sh.order, sh.nt, dt, sh.vmax, sh.padded("vel"), q, sh.src, sh.rec)
        data, state = G.forward(want_state=True)
        k = int(ref["sub"])
        out["forward_3000_steps"] = {
            "u_N_subgrid": rel(state[0][::k, ::k, ::k].cpu().numpy(), ref["u_sub"]),
            "u_N_1_subgrid": rel(state[1][::k, ::k, ::k].cpu().numpy(), ref["up_sub"]),
            "u_N_norm": abs(float(state[0].double().norm()) / float(ref["u_norm"]) - 1.0),
            "data_norm": abs(float(data.double().norm()) / float(ref["data_norm"]) - 1.0),
            "traces": rel(data[:, torch.as_tensor(ref["rec_idx"], device=data.device)].cpu().numpy(),
                          ref["data_sub"])}
        del G, data, state
        torch.cuda.empty_cache()
    out["note"] = ("relative L2 errors of the binary32 GPU path against the binary64 oracle on the full grid; "
                   "the compressed gradient's codec share is compared with the oracle's in the parity tests")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fault_body_3d")
    ap.add_argument("--tol", type=float, default=1e-4, help="codec tolerance of the headline run")
    ap.add_argument("--sweep", default="1e-3,1e-6", help="extra tolerances timed once each ('' = none)")
    ap.add_argument("--budget", type=float, default=16e9, help="checkpoint memory, bytes")
    ap.add_argument("--budget-sweep", default="2e9,4e9,64e9", help="other checkpoint budgets (bytes, comma "
                                                                   "separated) timed plain and compressed once "
                                                                   "each ('' = none)")
    ap.add_argument("--quick", action="store_true", help="small grid for a fast functional run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=200, help="0 = skip the serving stream")
    ap.add_argument("--serving-rate", type=float, default=2.0)
    ap.add_argument("--serving-pool", type=float, default=200e9)
    ap.add_argument("--serving-active", type=int, default=8)
    ap.add_argument("--serving-batch", type=int, default=16, help="2-D requests per batched launch (0 = no batching)")
    ap.add_argument("--serving-saturation", default="2,4,8,16", help="rate multiples of the saturation runs "
                                                                      "('' = none)")
    ap.add_argument("--kernels", action="store_true", help="short kernel workload for counter passes only")
    ap.add_argument("--codec-kernels", action="store_true", help="short codec workload for counter passes only")
    ap.add_argument("--codec-nt", type=int, default=1500, help="state the codec workload encodes (its step)")
    ap.add_argument("--no-ot4", action="store_true", help="skip the OT4 comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not part of it"}))
        sys.exit(2)
    if args.codec_kernels:
        codec_kernels_mode(nt=args.codec_nt)
        return
    if args.kernels:
        kernels_mode()
        return

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

    def timed(tol, hint, out, n, timing=TIMING_LAUNCHES):
        walls, stats, phi = [], [], None
        for _ in range(n):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            phi, _, st = G.misfit_gradient(d_obs, budget, tol, hint, timing=timing, out=out)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            stats.append(st)
        return walls, stats, phi

    # plain Revolve (no compression)
    log("plain revolve ...")
    timed(0.0, 0.0, g_plain, args.warmup)
    w_plain, st_plain, phi_plain = timed(0.0, 0.0, g_plain, args.steps)
    _, st_plain_ph, _ = timed(0.0, 0.0, g_plain, 1, TIMING_ACTIONS)   # per-phase times (untimed call)
    log(f"plain: {statistics.mean(w_plain):.3f} s  M={st_plain[0]['slots']} advances={st_plain[0]['advances']}")

    # compressed: the first (warm-up) call has no hint; later calls plan with the profile
    # it measured, as an optimisation loop would carry it from one iteration to the next
    log("compressed ...")
    w_cold, st0, _ = timed(args.tol, 0.0, g_comp, max(1, args.warmup))
    hint = plan_hint(st0[-1], Pn, shot.nt, budget)
    w_comp, st_comp, phi_comp = timed(args.tol, hint, g_comp, args.steps)
    _, st_comp_ph, _ = timed(args.tol, hint, g_comp, 1, TIMING_ACTIONS)
    err = float(torch.linalg.vector_norm(g_comp - g_plain) / torch.linalg.vector_norm(g_plain))
    log(f"compressed tol {args.tol}: {statistics.mean(w_comp):.3f} s  M={st_comp[0]['slots']} "
        f"ratio={st_comp[0]['ratio']:.1f} advances={st_comp[0]['advances']} grad err vs plain {err:.3e}")

    sweep, sweep_stats = [], []
    for tol in [float(t) for t in args.sweep.split(",") if t.strip()]:
        _, sp0, _ = timed(tol, 0.0, g_comp, 1, 0)
        h = plan_hint(sp0[-1], Pn, shot.nt, budget)
        ws_, ss_, _ = timed(tol, h, g_comp, 1)
        _, sph_, _ = timed(tol, h, g_comp, 1, TIMING_ACTIONS)
        e = float(torch.linalg.vector_norm(g_comp - g_plain) / torch.linalg.vector_norm(g_plain))
        sweep.append({"tol": tol, "shot_s": ws_[0], "slots": ss_[0]["slots"], "ratio": ss_[0]["ratio"],
                      "advances": ss_[0]["advances"], "grad_rel_err_vs_plain": e,
                      "speedup_vs_plain": statistics.mean(w_plain) / ws_[0]})
        sweep_stats.append((tol, h, sph_[0]))
        log(f"sweep tol {tol}: {ws_[0]:.3f} s ratio {ss_[0]['ratio']:.1f} err {e:.3e}")

    # per-phase device times over the timed compressed steps (HIP events on the call's stream)
    adv = sum(s["advances"] for s in st_comp)
    rev = sum(s["reverses"] for s in st_comp)
    ms_f = sum(s["ms_fwd_kernel"] for s in st_comp)
    ms_a = sum(s["ms_adj_kernel"] for s in st_comp)
    fwd_ms = ms_f / adv
    adj_ms = ms_a / rev
    fwd_gbs = FWD_BYTES_PER_POINT * Pn / (fwd_ms * 1e-3) / 1e9
    adj_gbs = ADJ_BYTES_PER_POINT * Pn / (adj_ms * 1e-3) / 1e9
    dom = "adjoint" if ms_a >= ms_f else "forward"
    ach = adj_gbs if dom == "adjoint" else fwd_gbs
    tr = traffic_per_launch()
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": (tr[dom] if tr else None),
            "traffic_note": ("HBM bytes per launch from FETCH_SIZE/WRITE_SIZE, copy-calibrated"
                             if tr else "counters absent or taken on a different stencil source"),
            "kernel": "stencil3d adjoint+gradient step" if dom == "adjoint" else "stencil3d forward step",
            "bytes_per_launch": (ADJ_BYTES_PER_POINT if dom == "adjoint" else FWD_BYTES_PER_POINT) * Pn,
            "avg_launch_ms": adj_ms if dom == "adjoint" else fwd_ms,
            "forward_step": {"avg_ms": fwd_ms, "GBs": round(fwd_gbs, 1), "frac": round(fwd_gbs / HBM_PEAK_GBS, 4),
                             "traffic": tr["forward"] if tr else None,
                             "hbm_gbs": round(tr["forward"] / (fwd_ms * 1e-3) / 1e9, 1) if tr else None},
            "adjoint_step": {"avg_ms": adj_ms, "GBs": round(adj_gbs, 1), "frac": round(adj_gbs / HBM_PEAK_GBS, 4),
                             "traffic": tr["adjoint"] if tr else None,
                             "hbm_gbs": round(tr["adjoint"] / (adj_ms * 1e-3) / 1e9, 1) if tr else None}}
    # counted HBM bytes (traffic) over the same launch time: the real rate, against the
    # algorithmic rate of "achieved"
    roof["hbm_gbs"] = roof["adjoint_step" if dom == "adjoint" else "forward_step"]["hbm_gbs"]
    roof["ceiling"] = stream_ceilings()
    roof["ceiling_note"] = ("hand-written streams (wv_stream_ceiling), 256 MB per array, one read through the "
                            "caches and the others and the write nontemporal, bytes read plus written per second: "
                            "the measured ceiling for the stencils' access mix")
    st = st_comp_ph[0]
    ms_per_store = st["ms_store"] / st["stores"] if st["stores"] else None
    ms_per_decode = st["ms_restore"] / st["decodes"] if st["decodes"] else None

    model = performance_model(shot.nt, Pn, G.slot_bytes, budget, st_plain_ph[0], st_comp_ph[0], hint, sweep_stats)
    # compressibility over time at the headline tolerance (untimed)
    stride = max(1, shot.nt // 10)
    cb = G.compressibility(args.tol, stride)
    compressibility = {"tol": args.tol, "steps": [(i + 1) * stride for i in range(len(cb))],
                       "ratio": [4.0 * Pn / b for b in cb]}
    log("compressibility (ratio of u^n): " + ", ".join(f"{n}:{r:.0f}" for n, r in
                                                         zip(compressibility["steps"], compressibility["ratio"])))

    # optional: plain against compressed at other checkpoint budgets (each run once; the
    # compressed call plans from the profile a first (cold, unhinted) compressed call measured)
    budget_sweep = []
    for bb in [int(float(x)) for x in args.budget_sweep.split(",") if x.strip()]:
        def once(tol, hint, out):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, st_ = G.misfit_gradient(d_obs, bb, tol, hint, out=out)
            torch.cuda.synchronize()
            return time.perf_counter() - t0, st_
        wp_, sp_ = once(0.0, 0.0, g_plain)
        wcold_, s0_ = once(args.tol, 0.0, g_comp)
        h_ = plan_hint(s0_, Pn, shot.nt, bb)
        wc_, sc_ = once(args.tol, h_, g_comp)
        ch_ = P.choose(shot.nt, Pn, bb, P.costs_from_stats(st_plain_ph[0]), P.costs_from_stats(st_comp_ph[0]),
                       profile=s0_["profile"], slot_bytes=G.slot_bytes)
        e_ = float(torch.linalg.vector_norm(g_comp - g_plain) / torch.linalg.vector_norm(g_plain))
        budget_sweep.append({"budget": bb, "plain_s": wp_, "plain_slots": sp_["slots"],
                             "plain_advances": sp_["advances"], "compressed_s": wc_,
                             "compressed_slots": sc_["slots"], "compressed_advances": sc_["advances"],
                             "compressed_cold_s": wcold_,
                             "retries": sc_["retries"], "speedup_vs_plain": wp_ / wc_,
                             "grad_rel_err_vs_plain": e_,
                             "model_choice": "compressed" if ch_["compressed"] else "plain",
                             "model_ms": {"plain": ch_["ms_plain"], "compressed": ch_["ms_compressed"]}})
        log(f"budget {bb:.3g} B: plain {wp_:.3f} s (M={sp_['slots']}, {sp_['advances']} advances), compressed "
            f"{wc_:.3f} s (M={sc_['slots']}, {sc_['advances']} advances; cold {wcold_:.3f} s), {wp_ / wc_:.2f}x, "
            f"err {e_:.2e}")

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
        "shot_gradient_s": {"compressed": round(ms_step / 1e3, 4), "plain": round(statistics.mean(w_plain), 4),
                            "compressed_cold": round(w_cold[0], 4),
                            "cold_note": "first compressed call, no ratio hint: it stores every state when "
                                         "they all fit the budget (as here), else it first measures their stream "
                                         "sizes in a forward run that stops before the reversal; the timed calls "
                                         "plan from the profile it measured"},
        "speedup_vs_plain": round(statistics.mean(w_plain) * 1e3 / ms_step, 4),
        "grad_rel_err_vs_plain": err,
        "plain_gpts": round(Pn * 2 * shot.nt / statistics.mean(w_plain) / 1e9, 3),
        # raw rate: stencil point updates executed (forward advances and adjoint steps, with
        # recomputation) over the stencil kernels' own time, from the timed steps
        "raw_gpts": {"compressed": raw_gpts(st_comp, Pn), "plain": raw_gpts(st_plain, Pn)},
        "latency_ms": {"p50": lat[len(lat) // 2], "p99": lat[min(len(lat) - 1, math.ceil(0.99 * len(lat)) - 1)]},
        "schedule": {"compressed": {k: st[k] for k in ("slots", "advances", "stores", "restores", "decodes",
                                                         "ratio", "ratio_planned", "peak_bytes", "retries")},
                     "plain": {k: st_plain[0][k] for k in ("slots", "advances", "stores", "restores")}},
        "phase_ms": {"compressed": {k: st[k] for k in ("ms_forward", "ms_adjoint", "ms_store", "ms_restore")},
                     "plain": {k: st_plain_ph[0][k] for k in ("ms_forward", "ms_adjoint", "ms_store", "ms_restore")},
                     "note": "one extra call each with per-action events (they cost about 4 % of wall time, "
                             "so the timed steps record only the stencil launches)"},
        "codec": {"ms_per_store": ms_per_store, "ms_per_field_decode": ms_per_decode,
                  "fields_per_store": (st["bytes_stored"] * st["ratio"]) / (4.0 * Pn * st["stores"])
                  if st["stores"] else None},
        "misfit": {"compressed": phi_comp, "plain": phi_plain},
        "sweep": sweep,
        "model": model,
        "compressibility": compressibility,
        "roofline": roof,
    }
    if budget_sweep:
        out["budget_sweep"] = budget_sweep
    if not args.no_ot4:
        del g_plain, g_comp
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out["ot4"] = ot4_block(shot, budget, args.tol, 1, model["costs_compressed"])
        torch.cuda.empty_cache()
        g_plain = g_comp = None
    if args.serving_requests > 0 and not args.quick:
        del G, g_plain, g_comp, d_obs
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out["serving"] = serving_leg(args.serving_requests, args.serving_rate, int(args.serving_pool),
                                     args.serving_active, 1e-4, int(16e9), args.serving_batch,
                                     [float(x) for x in args.serving_saturation.split(",") if x.strip()])
        out["latency_ms"] = {"p50": out["serving"]["p50_ms"], "p99": out["serving"]["p99_ms"],
                             "of": "serving stream, from arrival to completion"}
        log(f"serving: p50 {out['serving']['p50_ms']:.1f} ms p99 {out['serving']['p99_ms']:.1f} ms "
            f"{out['serving']['req_per_s']:.2f} req/s failed {out['serving']['failed']}")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample) ...")
        out["cpu_baseline"] = cpu_baseline(shot, {"advances": st["advances"], "reverses": st["reverses"],
                                                  "stores": st["stores"], "restores": st["decodes"]}, args.tol)
        if not args.quick:
            log("errors against the FP64 oracle (bounded samples of the large shot) ...")
            out["err_vs_fp64_oracle"] = oracle_errors(dt, out["cpu_baseline"]["cores"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
