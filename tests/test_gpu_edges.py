"""Degenerate and boundary cases of the GPU path against the oracle: one time step, one
checkpoint slot (quadratic recomputation), no absorbing layer, second-order stencil,
a compressed 2-D gradient and a grid that is a single z plane of tiles."""
import numpy as np
import pytest

import workloads as W
from oracle import schedule as SC
from tests.helpers import gpu_side, has_gpu, oracle_side, rel_l2, small_3d

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not has_gpu(), reason="needs a GPU")]


def _gradient_case(shot, slots, tol=0.0):
    import torch
    S, _ = oracle_side(shot)
    St, _ = oracle_side(shot, "true")
    fw = S.forward(want_traj=True)
    res = fw["data"] - St.forward()["data"]
    gref = S.gradient_full(fw["traj"], res)
    G, _ = gpu_side(shot)
    rt = torch.as_tensor(res.astype(np.float32), device="cuda")
    g, st = G.gradient(rt, 8 * G.P * (slots - 1), tol=tol, ratio_hint=1.0 if tol else 0.0)
    return rel_l2(g.cpu().numpy(), gref), st, res


def test_single_time_step():
    shot = small_3d(nt=1)
    S, _ = oracle_side(shot)
    G, _ = gpu_side(shot)
    ref = S.forward(want_last=True)
    data, state = G.forward(want_state=True)
    assert np.all(data.cpu().numpy()[0] == 0.0)
    assert rel_l2(state[0].cpu().numpy(), ref["last"][0]) <= 1e-5
    e, st, res = _gradient_case(shot, 2)
    assert st["advances"] == 1 and st["reverses"] == 1
    if np.any(res):
        assert e <= 1e-4


def test_one_slot_quadratic_recomputation():
    shot = W.near_anomaly_2d(n=(41, 37), nt=60)
    e, st, _ = _gradient_case(shot, 1)
    assert st["slots"] == 1
    assert st["advances"] == SC.p_closed(shot.nt + 1, 1) == shot.nt * (shot.nt + 1) // 2
    assert e <= 1e-4


def test_no_absorbing_layer_and_second_order():
    shot = W.replace(small_3d(n=(30, 28, 26), nt=60, order=2), nbl=0)
    S, _ = oracle_side(shot)
    G, _ = gpu_side(shot)
    ref = S.forward(want_last=True)
    data, state = G.forward(want_state=True)
    assert rel_l2(data.cpu().numpy(), ref["data"]) <= 1e-5
    assert rel_l2(state[0].cpu().numpy(), ref["last"][0]) <= 1e-5
    e, st, _ = _gradient_case(shot, 6)
    assert e <= 1e-4


def test_compressed_2d_gradient_and_thin_grid():
    e, st, _ = _gradient_case(W.near_anomaly_2d(), 8, tol=1e-6)
    assert st["ratio"] > 1.0 and e <= 1e-3
    # a grid only a few planes deep: one z chunk shorter than the stencil reach
    shot = W.replace(small_3d(n=(36, 34, 3), nt=40, order=8), nbl=2)
    S, _ = oracle_side(shot)
    G, _ = gpu_side(shot)
    ref = S.forward(want_last=True)
    data, state = G.forward(want_state=True)
    assert rel_l2(state[0].cpu().numpy(), ref["last"][0]) <= 1e-5
