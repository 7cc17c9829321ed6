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
