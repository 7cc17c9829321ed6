"""Compressed checkpoints on the GPU against the oracle's compressed gradient.

Both sides run the same Revolve schedule (same N and M) with every stored state
(u^k, d^k = u^k - u^{k-1}) passed through the codec at the same absolute tolerance.
Their quantisation decisions are taken on slightly different inputs (binary32
vs binary64 wavefields), so the two compressed gradients are not bitwise equal;
the bound is the oracle's own compression error at that tolerance (the measured
constant C of ||g_tol - g_0|| <= C tol), doubled, plus the uncompressed binary32
tolerance."""
import numpy as np
import pytest

import workloads as W
from oracle import schedule as SC
from tests.helpers import gpu_side, has_gpu, oracle_side, rel_l2, small_3d

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not has_gpu(), reason="needs a GPU")]

GRAD_TOL = 1e-4


def _problem(shot):
    S, _ = oracle_side(shot)
    St, _ = oracle_side(shot, "true")
    fw = S.forward(want_traj=True)
    res = fw["data"] - St.forward()["data"]
    g0 = S.gradient_full(fw["traj"], res)
    return S, res, g0


@pytest.mark.parametrize("case", ["2d", "3d"])
@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_compressed_gradient_within_codec_bound(case, tol):
    import torch
    shot = W.near_anomaly_2d() if case == "2d" else small_3d(nt=100)
    M = 8
    S, res, g0 = _problem(shot)
    acts = SC.schedule(shot.nt, M)
    g_or, st_or = S.gradient_actions(res, acts, M, tol=tol, increment=True)
    e_or = rel_l2(g_or, g0)
    G, _ = gpu_side(shot)
    rt = torch.as_tensor(res.astype(np.float32), device="cuda")
    # ratio hint 1 and a budget of M-1 raw states plus 5 % (room for the per-stream
    # prefix the planner adds to a compressed slot): the schedule has exactly M slots
    budget = int(8 * G.P * (M - 1) * 1.05)
    g, st = G.gradient(rt, budget, tol=tol, ratio_hint=1.0)
    e_gpu = rel_l2(g.cpu().numpy(), g0)
    g_plain, _ = G.gradient(rt, G.slot_bytes * (M - 1))
    e_plain = rel_l2(g_plain.cpu().numpy(), g0)
    print(f"{case} tol {tol:g}: oracle compressed {e_or:.3e}  GPU compressed {e_gpu:.3e}  GPU plain {e_plain:.3e}"
          f"  ratio {st['ratio']:.1f}")
    assert st["slots"] == M
    assert st["advances"] == st_or["advances"] == SC.p_closed(shot.nt + 1, M)
    assert st["stores"] == st_or["stores"]
    assert st["reverses"] == shot.nt
    assert st["ratio"] > 1.0
    assert e_plain <= GRAD_TOL
    assert e_gpu <= 2.0 * e_or + GRAD_TOL
    # against the GPU's own uncompressed gradient on the same schedule
    assert rel_l2(g.cpu().numpy(), g_plain.cpu().numpy()) <= 2.0 * e_or + GRAD_TOL


def test_compressed_gradient_error_falls_with_tolerance():
    import torch
    shot = small_3d(nt=100)
    M = 6
    S, res, g0 = _problem(shot)
    G, _ = gpu_side(shot)
    rt = torch.as_tensor(res.astype(np.float32), device="cuda")
    errs, sizes = [], []
    for tol in (1e-3, 1e-4, 1e-5):
        g, st = G.gradient(rt, int(8 * G.P * (M - 1) * 1.05), tol=tol, ratio_hint=1.0)
        assert st["slots"] == M
        errs.append(rel_l2(g.cpu().numpy(), g0))
        sizes.append(st["bytes_stored"])
    print("errors", errs, "bytes", sizes)
    assert errs[0] > errs[1] > errs[2]
    assert sizes[0] < sizes[1] < sizes[2]


@pytest.mark.parametrize("tol", [1e-3, 1e-5])
def test_compression_only_gradient_within_pointwise_bound(tol):
    """Every state stored compressed (M = N, no recomputation).  The adjoint states are the
    same as in the plain run, and each decoded state is within tol of the stored one, so
    at every point |g_tol - g_plain| <= tol (1/dt^2) sum_k |(1+a) lam^{k-1} - 2 lam^k +
    (1-a) lam^{k+1}|; the sum comes from the FP64 oracle, with 5 % for the binary32
    adjoint."""
    import torch
    shot = small_3d(nt=100)
    S, res, _ = _problem(shot)
    B = S.gradient_bound(res)
    G, _ = gpu_side(shot)
    rt = torch.as_tensor(res.astype(np.float32), device="cuda")
    g_plain, _ = G.gradient(rt, G.slot_bytes * 9)
    g, st = G.gradient(rt, G.slot_bytes * shot.nt, tol=tol, ratio_hint=1.0)
    assert st["slots"] == shot.nt and st["advances"] == shot.nt
    d = (g - g_plain).abs().cpu().numpy()
    top = float(np.abs(g_plain.cpu().numpy()).max())
    print(f"tol {tol:g}: worst share of the bound {float(np.max(d / np.maximum(tol * B, 1e-300))):.3f}")
    assert np.all(d <= 1.05 * tol * B + 1e-9 * top)
    assert d.max() > 0.0
