"""GPU OT4 kernel (two stencil passes per forward step, three per adjoint step)
against the oracle's OT4: wavefields and data, adjoint, gradient (with the term from
the m inside the fourth-order operator), checkpointed reversal and compression."""
import numpy as np
import pytest

import workloads as W
from oracle import schedule as SC
from tests.test_gpu_compressed import check_codec_parity
from tests.helpers import gpu_side, has_gpu, oracle_side, rel_l2, small_3d

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not has_gpu(), reason="needs a GPU")]

WAVEFIELD_TOL = 1e-5
GRAD_TOL = 1e-4


@pytest.mark.parametrize("order", [2, 8, 16])
@pytest.mark.parametrize("nxi", [44, 45])
def test_forward_3d(order, nxi):
    shot = small_3d(n=(nxi, 38, 41), order=order, nt=80)
    S, _ = oracle_side(shot, time_order=4)
    G, _ = gpu_side(shot, time_order=4)
    ref = S.forward(want_last=True)
    data, state = G.forward(want_state=True)
    e_d = rel_l2(data.cpu().numpy(), ref["data"])
    e_u = rel_l2(state[0].cpu().numpy(), ref["last"][0])
    e_p = rel_l2(state[1].cpu().numpy(), ref["last"][1])
    print(f"OT4 order {order} nx {nxi}: data {e_d:.2e} u^N {e_u:.2e} u^(N-1) {e_p:.2e}")
    assert e_d <= WAVEFIELD_TOL and e_u <= WAVEFIELD_TOL and e_p <= WAVEFIELD_TOL


def test_forward_2d_full_size():
    shot = W.two_layer_2d()
    S, _ = oracle_side(shot, time_order=4)
    G, _ = gpu_side(shot, time_order=4)
    ref = S.forward(want_last=True)
    data, state = G.forward(want_state=True)
    assert rel_l2(data.cpu().numpy(), ref["data"]) <= WAVEFIELD_TOL
    assert rel_l2(state[0].cpu().numpy(), ref["last"][0]) <= WAVEFIELD_TOL


@pytest.mark.parametrize("ndim", [2, 3])
def test_adjoint_source(ndim):
    import torch
    shot = W.two_layer_2d(n=(61, 53), nt=150) if ndim == 2 else small_3d(nt=60)
    r = np.random.default_rng(5).standard_normal((shot.nt + 1, len(shot.rec))).astype(np.float32)
    S, _ = oracle_side(shot, time_order=4)
    G, _ = gpu_side(shot, time_order=4)
    ref = S.adjoint_src(r.astype(np.float64))
    got = G.adjoint_src(torch.as_tensor(r, device="cuda")).cpu().numpy()
    assert rel_l2(got, ref) <= GRAD_TOL


def _residual(shot):
    S, _ = oracle_side(shot, time_order=4)
    St, _ = oracle_side(shot, "true", time_order=4)
    fw = S.forward(want_traj=True)
    res = fw["data"] - St.forward()["data"]
    return S, res, S.gradient_full(fw["traj"], res)


@pytest.mark.parametrize("ndim", [2, 3])
def test_gradient_uncompressed(ndim):
    import torch
    shot = W.near_anomaly_2d() if ndim == 2 else small_3d(nt=100)
    S, res, gref = _residual(shot)
    G, _ = gpu_side(shot, time_order=4)
    g, st = G.gradient(torch.as_tensor(res.astype(np.float32), device="cuda"), G.slot_bytes * shot.nt)
    e = rel_l2(g.cpu().numpy(), gref)
    print("OT4 gradient rel-L2", e)
    assert e <= GRAD_TOL


def test_revolve_bit_identical_and_compressed():
    import torch
    shot = small_3d(nt=90)
    S, res, gref = _residual(shot)
    G, _ = gpu_side(shot, time_order=4)
    rt = torch.as_tensor(res.astype(np.float32), device="cuda")
    full, _ = G.gradient(rt, G.slot_bytes * shot.nt)
    for M in (3, 12):
        g, st = G.gradient(rt, G.slot_bytes * (M - 1))
        assert st["advances"] == SC.p_closed(shot.nt + 1, M)
        assert torch.equal(g, full), M
    M = 8
    g_plain, _ = G.gradient(rt, G.slot_bytes * (M - 1))
    for tol in (1e-3, 1e-5):
        acts = SC.schedule(shot.nt, M)
        g_or, _ = S.gradient_actions(res, acts, M, tol=tol, increment=True)
        g, st = G.gradient(rt, int(8 * G.P * (M - 1) * 1.05), tol=tol, ratio_hint=1.0)
        assert st["slots"] == M
        check_codec_parity(f"OT4 tol {tol:g}", g.cpu().numpy(), g_plain.cpu().numpy(), g_or, gref)
