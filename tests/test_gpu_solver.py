"""GPU solver parity against the FP64 oracle (wavefield, data, adjoint, gradient)."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import schedule as SC
from tests.helpers import gpu_side, has_gpu, oracle_side, rel_l2, small_3d

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not has_gpu(), reason="needs a GPU")]

WAVEFIELD_TOL = 1e-5     # rel-L2 of wavefields and data vs the FP64 oracle
GRAD_TOL = 1e-4          # rel-L2 of the uncompressed gradient


def test_forward_2d_two_layer_full_size():
    """2-D two-layer model at its full size (101^2 + 20-cell layer, 500 steps, order 4)."""
    shot = W.two_layer_2d()
    S, _ = oracle_side(shot)
    G, _ = gpu_side(shot)
    ref = S.forward(want_last=True)
    data, state = G.forward(want_state=True)
    print("data rel-L2", rel_l2(data.cpu().numpy(), ref["data"]))
    assert rel_l2(data.cpu().numpy(), ref["data"]) <= WAVEFIELD_TOL
    assert rel_l2(state[0].cpu().numpy(), ref["last"][0]) <= WAVEFIELD_TOL
    assert rel_l2(state[1].cpu().numpy(), ref["last"][1]) <= WAVEFIELD_TOL


@pytest.mark.parametrize("order", [2, 4, 8, 12, 16])
@pytest.mark.parametrize("nxi", [44, 45, 48])
def test_forward_3d_orders_ragged(order, nxi):
    """nxi = 44: padded x extent 60, a multiple of 4 (vector path), rows pitched to 64;
    45: 61, scalar path; 48: 64, rows already a multiple of 32 (no pad columns)."""
    shot = small_3d(n=(nxi, 38, 41), order=order, nt=80)
    S, _ = oracle_side(shot)
    G, _ = gpu_side(shot)
    ref = S.forward(want_last=True)
    data, state = G.forward(want_state=True)
    e_d = rel_l2(data.cpu().numpy(), ref["data"])
    e_u = rel_l2(state[0].cpu().numpy(), ref["last"][0])
    print(f"order {order}: data {e_d:.2e} field {e_u:.2e}")
    assert e_d <= WAVEFIELD_TOL and e_u <= WAVEFIELD_TOL


@pytest.mark.parametrize("ndim", [2, 3])
def test_receivers_on_nodes_lines_and_between(ndim):
    """Sources and receivers with every mix of zero interpolation weights: on grid nodes
    (one nonzero corner), on grid lines (two or four) and between them (all corners).  The
    sparse tables keep only the nonzero corners, padded per point; data, final state and
    the uncompressed gradient against the oracle."""
    import dataclasses
    import torch
    base = W.near_anomaly_2d(n=(61, 57), nt=200) if ndim == 2 else small_3d(nt=80)
    h = np.array(base.h)
    rng = np.random.default_rng(11)
    ext = (np.array(base.n) - 1) * h
    pts = []
    for kind in range(4):
        for _ in range(6):
            x = rng.uniform(0.1, 0.9, ndim) * ext
            if kind == 0:
                x = np.round(x / h) * h                      # a node
            elif kind == 1:
                x[0] = np.round(x[0] / h[0]) * h[0]          # on a line through x
            elif kind == 2:
                x[1:] = np.round(x[1:] / h[1:]) * h[1:]      # on lines through the other axes
            pts.append(x)
    rec = np.array(pts, dtype=np.float64)
    src = np.array([np.round(ext * 0.5 / h) * h], dtype=np.float64)   # a node
    shot = dataclasses.replace(base, src=src, rec=rec)
    S, _ = oracle_side(shot)
    G, _ = gpu_side(shot)
    ref = S.forward(want_last=True, want_traj=True)
    data, state = G.forward(want_state=True)
    assert rel_l2(data.cpu().numpy(), ref["data"]) <= WAVEFIELD_TOL
    assert rel_l2(state[0].cpu().numpy(), ref["last"][0]) <= WAVEFIELD_TOL
    res = np.random.default_rng(12).standard_normal(ref["data"].shape) * 1e-3
    gref = S.gradient_full(ref["traj"], res)
    g, _ = G.gradient(torch.as_tensor(res.astype(np.float32), device="cuda"), G.slot_bytes * shot.nt)
    assert rel_l2(g.cpu().numpy(), gref) <= GRAD_TOL


def test_forward_3d_longer_run():
    shot = small_3d(n=(60, 52, 70), nbl=10, order=8, nt=400, f0=15.0)
    S, _ = oracle_side(shot)
    G, _ = gpu_side(shot)
    ref = S.forward(want_last=True)
    data, state = G.forward(want_state=True)
    assert rel_l2(data.cpu().numpy(), ref["data"]) <= WAVEFIELD_TOL
    assert rel_l2(state[0].cpu().numpy(), ref["last"][0]) <= WAVEFIELD_TOL


@pytest.mark.parametrize("ndim", [2, 3])
def test_adjoint_source_and_dot_product(ndim):
    import torch
    shot = W.two_layer_2d(n=(61, 53), nt=150) if ndim == 2 else small_3d(nt=60)
    rng = np.random.default_rng(5)
    r = rng.standard_normal((shot.nt + 1, len(shot.rec))).astype(np.float32)
    S, _ = oracle_side(shot)
    G, _ = gpu_side(shot)
    ref = S.adjoint_src(r.astype(np.float64))
    got = G.adjoint_src(torch.as_tensor(r, device="cuda")).cpu().numpy()
    assert rel_l2(got, ref) <= GRAD_TOL
    # dot test on the GPU path itself: <F q, r> = <q, F^T r>
    d = G.forward().cpu().numpy().astype(np.float64)
    q = G.wavelet.cpu().numpy().astype(np.float64)
    lhs, rhs = float(np.dot(d.ravel(), r.ravel())), float(np.dot(q, got.astype(np.float64)))
    assert abs(lhs - rhs) <= 1e-4 * abs(rhs)


def _residual(shot):
    S, _ = oracle_side(shot)
    St, _ = oracle_side(shot, "true")
    fw = S.forward(want_traj=True)
    dobs = St.forward()["data"]
    res = fw["data"] - dobs
    g = S.gradient_full(fw["traj"], res)
    return S, res, dobs, g


def test_two_layer_full_size_full_storage_and_revolve_10():
    """The 2-D two-layer model at its full size (101^2 + 20-cell layer, 500 steps, order 4):
    gradient with full storage and with uncompressed Revolve on 10 checkpoints (M = 11 with
    the initial zero state), against the oracle's full-storage gradient.  The two GPU
    gradients are bit-identical (recomputation is deterministic and the reverse sweep sums
    in the same order), and the recomputation count is the binomial closed form."""
    import torch
    shot = W.two_layer_2d()
    S, res, _, gref = _residual(shot)
    G, _ = gpu_side(shot)
    rt = torch.as_tensor(res.astype(np.float32), device="cuda")
    full, st_full = G.gradient(rt, G.slot_bytes * shot.nt)
    M = 11
    g, st = G.gradient(rt, G.slot_bytes * (M - 1))
    e = rel_l2(full.cpu().numpy(), gref)
    print(f"two-layer full size: gradient rel-L2 {e:.2e}, Revolve advances {st['advances']}")
    assert st_full["advances"] == shot.nt
    assert st["slots"] == M and st["advances"] == SC.p_closed(shot.nt + 1, M)
    assert torch.equal(g, full)
    assert e <= GRAD_TOL


@pytest.mark.parametrize("ndim", [2, 3])
def test_gradient_uncompressed(ndim):
    import torch
    shot = W.near_anomaly_2d() if ndim == 2 else small_3d(nt=100)
    S, res, dobs, gref = _residual(shot)
    G, _ = gpu_side(shot)
    rt = torch.as_tensor(res.astype(np.float32), device="cuda")
    budget = G.slot_bytes * shot.nt      # every state stored
    g, st = G.gradient(rt, budget)
    e = rel_l2(g.cpu().numpy(), gref)
    print("gradient rel-L2", e, st)
    assert e <= GRAD_TOL
    assert st["advances"] == shot.nt and st["reverses"] == shot.nt


def test_revolve_bit_identical_to_full_storage():
    import torch
    shot = small_3d(nt=90)
    S, res, dobs, gref = _residual(shot)
    G, _ = gpu_side(shot)
    rt = torch.as_tensor(res.astype(np.float32), device="cuda")
    full, st_full = G.gradient(rt, G.slot_bytes * shot.nt)
    for M in (2, 5, 12):
        g, st = G.gradient(rt, G.slot_bytes * (M - 1))
        assert st["slots"] == M
        assert st["advances"] == SC.p_closed(shot.nt + 1, M)
        assert torch.equal(g, full), M


def test_gradient_3d_odd_step_count():
    """3-D adjoint steps update the binary64 gradient once per pair: the step k = 2j
    leaves its term, rounded to binary32, for the step k = 2j - 1 to add with its own.
    With an odd step count the first reverse step (k = nt) adds its own term alone.  The
    gradient stays within the oracle tolerance, and Revolve (whose reverse sweep visits the
    same k in the same order) stays bit-identical to full storage."""
    import torch
    shot = small_3d(nt=91)
    S, res, dobs, gref = _residual(shot)
    G, _ = gpu_side(shot)
    rt = torch.as_tensor(res.astype(np.float32), device="cuda")
    full, st_full = G.gradient(rt, G.slot_bytes * shot.nt)
    e = rel_l2(full.cpu().numpy(), gref)
    print(f"odd nt: gradient rel-L2 {e:.2e}")
    assert st_full["reverses"] == shot.nt
    assert e <= GRAD_TOL
    for M in (3, 8):
        g, st = G.gradient(rt, G.slot_bytes * (M - 1))
        assert st["slots"] == M
        assert torch.equal(g, full), M


def test_misfit_gradient_one_sweep():
    import torch
    shot = W.near_anomaly_2d()
    S, res, dobs, gref = _residual(shot)
    phi_ref = 0.5 * float(np.sum(res ** 2))
    G, _ = gpu_side(shot)
    d_obs = torch.as_tensor(dobs.astype(np.float32), device="cuda")
    phi, g, st, dsim = G.misfit_gradient(d_obs, 8 * G.P * 20, want_dsim=True)
    assert abs(phi - phi_ref) <= 1e-4 * phi_ref
    assert rel_l2(g.cpu().numpy(), gref) <= GRAD_TOL
    assert st["slots"] == 21
