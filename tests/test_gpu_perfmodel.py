"""The performance model against measured gradient times (the paper validates its
model the same way: predicted against measured run time).  Costs are measured in one
call at one memory budget; the model must predict the device time of calls at other
budgets, where the schedule (recomputation, stores, decodes) differs."""
import numpy as np
import pytest

import workloads as W
from tests.helpers import gpu_side, has_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not has_gpu(), reason="needs a GPU")]


@pytest.mark.parametrize("tol", [0.0, 1e-4])
def test_model_predicts_other_budgets(tol):
    import torch
    import paper_1810_05268_amd as P
    shot = W.layered_noise_3d(n=(120, 112, 104), nt=400, order=8)
    G, _ = gpu_side(shot)
    rng = np.random.default_rng(3)
    res = torch.as_tensor((rng.standard_normal((shot.nt + 1, len(shot.rec))) * 1e-3).astype(np.float32),
                          device="cuda")
    S = 8 * G.P
    G.gradient(res, 20 * S, tol=tol, ratio_hint=8.0 if tol else 0.0)        # warm-up
    _, st = G.gradient(res, 20 * S, tol=tol, ratio_hint=8.0 if tol else 0.0, timing=1)
    c = P.costs_from_stats(st)
    for slots in (6, 60):
        _, sm = G.gradient(res, slots * S, tol=tol, ratio_hint=8.0 if tol else 0.0, timing=1)
        if tol:
            pr = P.predict(shot.nt, G.P, slots * S, True, c["c_f"], c["c_r"], t_c=c["t_store"], t_d=c["t_d"],
                           ratio=8.0)
        else:
            pr = P.predict(shot.nt, G.P, slots * S, False, c["c_f"], c["c_r"], t_copy=c["t_store"],
                           slot_bytes=G.slot_bytes)
        phases = sm["ms_forward"] + sm["ms_adjoint"] + sm["ms_store"] + sm["ms_restore"]
        print(f"tol {tol:g} budget {slots} S: predicted {pr['ms_total']:.2f} ms, measured {phases:.2f} ms "
              f"(call {sm['ms_total']:.2f} ms), advances {pr['advances']} / {sm['advances']}")
        assert pr["slots"] == sm["slots"]
        assert pr["advances"] == sm["advances"] and pr["stores"] == sm["stores"]
        assert pr["fields"] == sm["fields"] and pr["decodes"] == sm["decodes"]
        assert abs(pr["ms_total"] - phases) <= 0.15 * phases
        assert abs(pr["ms_total"] - sm["ms_total"]) <= 0.25 * sm["ms_total"]


def test_model_chooses_the_faster_strategy():
    """wv_choose against measurement, with costs from one plain and one compressed call. At a
    budget of 2 slots plain Revolve recomputes quadratically and compression must win; at a
    budget that holds every state uncompressed, plain Revolve (copies, no codec) must win; at
    6 slots the two are within a few percent (this 400-step shot recomputes cheaply), and
    whichever is chosen must measure within 5 % of the faster."""
    import torch
    import paper_1810_05268_amd as P
    shot = W.layered_noise_3d(n=(120, 112, 104), nt=400, order=8)
    G, _ = gpu_side(shot)
    rng = np.random.default_rng(3)
    res = torch.as_tensor((rng.standard_normal((shot.nt + 1, len(shot.rec))) * 1e-3).astype(np.float32),
                          device="cuda")
    tol = 1e-4

    def phases(st):
        return st["ms_forward"] + st["ms_adjoint"] + st["ms_store"] + st["ms_restore"]
    G.gradient(res, 20 * G.slot_bytes, timing=1)                                  # warm-up
    _, sp = G.gradient(res, 20 * G.slot_bytes, timing=1)
    _, sc = G.gradient(res, 20 * G.slot_bytes, tol=tol, ratio_hint=8.0, timing=1)
    cp, cc = P.costs_from_stats(sp), P.costs_from_stats(sc)
    for slots, expect in ((2, 1), (6, None), (shot.nt, 0)):
        budget = slots * G.slot_bytes
        ch = P.choose(shot.nt, G.P, budget, cp, cc, profile=sc["profile"], slot_bytes=G.slot_bytes)
        _, mp = G.gradient(res, budget, timing=1)
        _, mc = G.gradient(res, budget, tol=tol, ratio_hint=ch["ratio_hint"] if ch["compressed"] else 0.0,
                           timing=1)
        t = {0: phases(mp), 1: phases(mc)}
        print(f"{slots} slots: chose {'compressed' if ch['compressed'] else 'plain'} (predicted plain "
              f"{ch['ms_plain']:.1f} ms, compressed {ch['ms_compressed']:.1f} ms); measured plain {t[0]:.1f} ms, "
              f"compressed {t[1]:.1f} ms")
        if expect is not None:
            assert ch["compressed"] == expect
        assert t[ch["compressed"]] <= 1.05 * min(t.values())


def test_misfit_gradient_auto_takes_the_models_choice():
    """wv_misfit_gradient_auto makes wv_choose's decision per call, from the costs and the
    profile of earlier calls: at 2 slots it compresses (plain Revolve would recompute
    quadratically), with every state in memory it runs plain Revolve, and each result is
    bit-identical to the explicit call it chose."""
    import torch
    import paper_1810_05268_amd as P
    from paper_1810_05268_amd.shot import DeviceShot
    shot = W.layered_noise_3d(n=(120, 112, 104), nt=400, order=8)
    G, dt = gpu_side(shot)
    q = W.ricker(shot.f0, dt, shot.nt).astype(np.float32)
    Gt = DeviceShot(3, shot.n, shot.h, shot.nbl, shot.order, shot.nt, dt, shot.vmax, shot.padded("true"), q,
                    shot.src, shot.rec)
    d_obs = Gt.forward()
    del Gt
    tol = 1e-4
    G.misfit_gradient(d_obs, 20 * G.slot_bytes, timing=1)                          # warm-up
    _, _, sp = G.misfit_gradient(d_obs, 20 * G.slot_bytes, timing=1)
    _, _, sc = G.misfit_gradient(d_obs, 20 * G.slot_bytes, tol, ratio_hint=8.0, timing=1)
    cp, cc = P.costs_from_stats(sp), P.costs_from_stats(sc)
    for slots, expect in ((2, 1), (shot.nt, 0)):
        budget = slots * G.slot_bytes
        g = torch.empty(G.shape, dtype=torch.float64, device="cuda")
        phi, st, ch = P.misfit_gradient_auto(G.pb, d_obs, budget, tol, cp, cc, g, G.workspace(1, budget),
                                             profile=sc["profile"], slot_bytes=G.slot_bytes)
        print(f"{slots} slots: {'compressed' if ch['compressed'] else 'plain'}, M {st['slots']}, "
              f"predicted plain {ch['ms_plain']:.1f} ms, compressed {ch['ms_compressed']:.1f} ms")
        assert ch["compressed"] == expect and st["slots"] == ch["slots"]
        phi2, g2, st2 = G.misfit_gradient(d_obs, budget, tol if expect else 0.0,
                                          ratio_hint=ch["ratio_hint"] if expect else 0.0)
        assert phi2 == phi and torch.equal(g2, g) and st2["slots"] == st["slots"]
