"""Compressed checkpoints on the GPU against the oracle's compressed gradient.

Both sides run the same Revolve schedule (same N and M) with every stored state
(u^k, d^k = u^k - u^{k-1}) passed through the codec at the same absolute tolerance.
Their quantisation decisions are taken on slightly different inputs (binary32
vs binary64 wavefields), so the two compressed gradients are not bitwise equal;
what is compared is the codec's share of each: the change compression makes to the
gradient on the GPU against the change it makes in the FP64 oracle on the same
schedule, with an allowance of twice the binary32 floor of the plain run."""
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


def check_codec_parity(tag, g_tol, g_plain, g_or_tol, g0):
    """The codec's share of a compressed GPU gradient against the oracle's.

    e_or    = ||g_or,tol - g0|| / ||g0||: what compression changes in the FP64 oracle
              on the same schedule (the quantity under test);
    d_gpu   = ||g_gpu,tol - g_gpu,plain|| / ||g0||: what it changes on the GPU;
    e_plain = ||g_gpu,plain - g0|| / ||g0||: the binary32 floor of the plain run.
    The GPU's change must be the oracle's within a factor of 3 either way, with an
    additive allowance of twice the binary32 floor (the two sides quantise binary32 and
    binary64 wavefields, so a few coefficients round differently); and the GPU's
    compressed gradient must sit closer to the oracle's compressed gradient than the
    codec's own change plus that floor, i.e. both sides dropped the same bits."""
    e_or = rel_l2(g_or_tol, g0)
    d_gpu = rel_l2(g_tol, g_plain) * float(np.linalg.norm(g_plain) / np.linalg.norm(g0))
    e_plain = rel_l2(g_plain, g0)
    e_pair = rel_l2(g_tol, g_or_tol)
    print(f"{tag}: oracle codec change {e_or:.3e}  GPU codec change {d_gpu:.3e}  (ratio {d_gpu / e_or:.3f})"
          f"  GPU plain floor {e_plain:.3e}  GPU vs oracle compressed {e_pair:.3e}")
    assert e_plain <= GRAD_TOL
    assert d_gpu <= 3.0 * e_or + 2.0 * e_plain
    assert d_gpu >= e_or / 3.0 - 2.0 * e_plain
    assert e_pair <= 0.5 * e_or + 2.0 * e_plain
    return e_or, d_gpu, e_plain, e_pair


@pytest.mark.parametrize("case", ["2d", "3d"])
@pytest.mark.parametrize("tol", [1e-3, 1e-4, 1e-6])
def test_compressed_gradient_within_codec_bound(case, tol):
    """Compressed checkpoints with recomputation (M = 8 slots): the codec's effect on the
    gradient matches the oracle's compressed reversal on the same schedule."""
    import torch
    shot = W.near_anomaly_2d() if case == "2d" else small_3d(nt=100)
    M = 8
    S, res, g0 = _problem(shot)
    acts = SC.schedule(shot.nt, M)
    g_or, st_or = S.gradient_actions(res, acts, M, tol=tol, increment=True)
    G, _ = gpu_side(shot)
    rt = torch.as_tensor(res.astype(np.float32), device="cuda")
    # ratio hint 1 and a budget of M-1 raw states plus 5 % (room for the per-stream
    # prefix the planner adds to a compressed slot): the schedule has exactly M slots
    budget = int(8 * G.P * (M - 1) * 1.05)
    g, st = G.gradient(rt, budget, tol=tol, ratio_hint=1.0)
    g_plain, _ = G.gradient(rt, G.slot_bytes * (M - 1))
    assert st["slots"] == M
    assert st["advances"] == st_or["advances"] == SC.p_closed(shot.nt + 1, M)
    assert st["stores"] == st_or["stores"]
    assert st["reverses"] == shot.nt
    assert st["ratio"] > 1.0
    check_codec_parity(f"{case} tol {tol:g} ratio {st['ratio']:.1f}", g.cpu().numpy(), g_plain.cpu().numpy(),
                       g_or, g0)


def test_arena_overflow_replans_and_equals_a_direct_plan():
    """A ratio hint far too optimistic makes every slot count the planner tries overflow
    the arena: the call re-plans with half the ratio (the last time at the uncompressed
    size) and reports the repeats; its gradient equals, bit for bit, a call planned at the
    final ratio from the start."""
    import torch
    shot = small_3d(nt=100)
    S, res, g0 = _problem(shot)
    G, _ = gpu_side(shot)
    rt = torch.as_tensor(res.astype(np.float32), device="cuda")
    # a third of one raw state: a hint of 1e6 plans every state (M = N), whose streams
    # (about 0.9 MB here) cannot fit; half of that hint plans the same; the last re-plan
    # takes the uncompressed size, M = 1 (recomputation from x_0 alone)
    budget = int(8 * G.P * 0.3)
    g1, st1 = G.gradient(rt, budget, tol=1e-4, ratio_hint=1e6)
    print("forced overflow:", {k: st1[k] for k in ("retries", "slots", "ratio_planned", "peak_bytes")})
    assert st1["retries"] >= 1
    assert st1["peak_bytes"] <= budget
    g2, st2 = G.gradient(rt, budget, tol=1e-4, ratio_hint=st1["ratio_planned"])
    assert st2["retries"] == 0 and st2["slots"] == st1["slots"]
    assert st2["advances"] == st1["advances"] and st2["stores"] == st1["stores"]
    assert torch.equal(g1, g2)
    assert rel_l2(g1.cpu().numpy(), g0) <= 1e-3


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
