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
    # uncompressed slots are two pitched field arrays; compressed ones are sized from the
    # dense field bytes and the hint
    budget = 8 * G.P * (slots - 1) if tol else G.slot_bytes * (slots - 1)
    g, st = G.gradient(rt, budget, tol=tol, ratio_hint=1.0 if tol else 0.0)
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


@pytest.mark.parametrize("order,tol", [(8, 0.0), (12, 1e-4)])
def test_workspace_contents_do_not_matter(order, tol):
    """Field rows are pitched (pad columns beyond nx): a workspace full of NaN bytes must
    give bit-identical data, final state and gradient to a zeroed one (76 x 72 x 70
    padded points, rows pitched to 96)."""
    import torch
    shot = W.random_layers((36, 32, 30), (10.0,) * 3, 20, order, 120, np.random.default_rng(4), 15.0)
    G, _ = gpu_side(shot)
    rng = np.random.default_rng(1)
    res = torch.as_tensor((rng.standard_normal((shot.nt + 1, len(shot.rec))) * 1e-3).astype(np.float32),
                          device="cuda")
    budget = G.slot_bytes * 10
    out = []
    for fill in (0, 0xFF):          # 0xFF bytes are NaN in binary32 and binary64
        ws = G.workspace(1, budget)
        G._ws.fill_(fill)
        data, state = G.forward(want_state=True)
        G._ws.fill_(fill)
        g, st = G.gradient(res, budget, tol=tol, ratio_hint=4.0 if tol else 0.0)
        assert torch.isfinite(g).all()
        out.append((data.clone(), state.clone(), g.clone(), st["slots"]))
        del ws
    for a, b in zip(out[0][:3], out[1][:3]):
        assert torch.equal(a, b)
    assert out[0][3] == out[1][3]


@pytest.mark.parametrize("n,order,nbl", [((300, 4), 16, 2), ((70, 203), 4, 20), ((520, 61), 8, 20)])
def test_2d_strip_and_chunk_edges(n, order, nbl):
    """2-D grids against the oracle where the z chunking is at its edges: a strip shallower
    than the stencil reach (a single chunk), many chunks of a few planes with a ragged
    last one, and more than one 256-wide x strip with a ragged last strip."""
    shot = W.near_anomaly_2d(n=n, nt=60, order=order, nbl=nbl)
    S, _ = oracle_side(shot)
    G, _ = gpu_side(shot)
    ref = S.forward(want_last=True)
    data, state = G.forward(want_state=True)
    assert np.any(ref["data"])
    assert rel_l2(data.cpu().numpy(), ref["data"]) <= 1e-5
    assert rel_l2(state[0].cpu().numpy(), ref["last"][0]) <= 1e-5
    e, st, _ = _gradient_case(shot, 6)
    assert st["advances"] == SC.p_closed(shot.nt + 1, 6)
    assert e <= 1e-4
