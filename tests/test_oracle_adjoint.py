"""Pins of the oracle's adjoint-state gradient (Sec. "Problem and test case", eqs. (7)-(8)):
dot-product test, Lagrangian form vs reversed-sum form, finite differences, Taylor
remainder, and bit-identity of the checkpointed (Revolve) reversal with full storage."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import schedule as SC


def tiny_problem(ndim=2, nt=80, order=4, nbl=5, n=None, f0=30.0):
    n = n or ((21, 21) if ndim == 2 else (12, 11, 10))
    h = (10.0,) * ndim
    shape = tuple(reversed(n))
    grids = np.meshgrid(*(np.arange(m) * 10.0 for m in shape), indexing="ij")
    z = grids[0]
    coords = list(reversed(grids))
    vel_i = np.where(z < (n[-1] // 2) * 10.0, 1500.0, 2500.0)
    centre = [(n[d] - 1) * 5.0 for d in range(ndim)]
    r2 = sum((coords[d] - centre[d]) ** 2 for d in range(ndim))
    velt_i = vel_i + 200.0 * np.exp(-r2 / (2 * 40.0 ** 2))
    vmax = float(max(vel_i.max(), velt_i.max()))
    dt = 0.4 * oracle.cfl_dt(ndim, h, order, vmax)
    spec = oracle.ModelSpec(ndim, tuple(n), h, nbl, order, nt, dt, vmax)
    src, rec = W.surface_geometry(n, h)
    q = W.ricker(f0, dt, nt)
    vel = np.pad(vel_i, nbl, mode="edge")
    velt = np.pad(velt_i, nbl, mode="edge")
    return spec, vel, velt, src, rec, q


@pytest.fixture(scope="module")
def prob2d():
    spec, vel, velt, src, rec, q = tiny_problem()
    S = oracle.Solver(spec, vel, src, q, rec)
    St = oracle.Solver(spec, velt, src, q, rec)
    fw = S.forward(want_traj=True)
    dobs = St.forward()["data"]
    res = fw["data"] - dobs
    g, lam = S.gradient_full(fw["traj"], res, want_lam=True)
    return dict(spec=spec, vel=vel, src=src, rec=rec, q=q, S=S, fw=fw, dobs=dobs, res=res, g=g, lam=lam)


@pytest.mark.parametrize("ndim", [2, 3])
def test_dot_product(ndim):
    """<R U(q), r> = <q, S^T lam(r)>: forward and adjoint are exact transposes."""
    spec, vel, _, src, rec, _ = tiny_problem(ndim=ndim, nt=40 if ndim == 3 else 80)
    rng = np.random.default_rng(7)
    q = rng.standard_normal(spec.nt)
    S = oracle.Solver(spec, vel, src, q, rec)
    d = S.forward()["data"]
    r = rng.standard_normal(d.shape)
    lhs = float(np.dot(d.ravel(), r.ravel()))
    rhs = float(np.dot(q, S.adjoint_src(r)))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_summation_by_parts(prob2d):
    """The per-step Lagrangian derivative sum equals the reversed k-sum the solver uses."""
    p = prob2d
    gn = p["S"].gradient_nform(p["fw"]["traj"], p["lam"])
    assert np.linalg.norm(gn - p["g"]) <= 1e-12 * np.linalg.norm(p["g"])


def _phi(p, vel):
    s = oracle.Solver(p["spec"], vel, p["src"], p["q"], p["rec"])
    return oracle.misfit(s.forward()["data"], p["dobs"])


def test_central_finite_differences(prob2d):
    p = prob2d
    gc = -2.0 * p["g"] / p["vel"] ** 3              # chain rule m = c^-2
    rng = np.random.default_rng(11)
    for _ in range(3):
        dv = rng.standard_normal(p["vel"].shape)
        errs = []
        for rel in (1e-3, 1e-4):
            eps = rel * np.linalg.norm(p["vel"]) / np.linalg.norm(dv)
            fd = (_phi(p, p["vel"] + eps * dv) - _phi(p, p["vel"] - eps * dv)) / (2 * eps)
            errs.append(abs(fd - np.sum(gc * dv)) / abs(fd))
        assert errs[1] < 1e-4
        assert errs[1] < errs[0] / 30          # O(eps^2) convergence


def test_taylor_remainder_second_order(prob2d):
    p = prob2d
    m = 1.0 / p["vel"] ** 2
    rng = np.random.default_rng(12)
    dm = rng.standard_normal(m.shape) * m.mean() * 1e-2
    phi0 = _phi(p, p["vel"])
    rs = []
    for eps in (0.1, 0.05, 0.025):
        rs.append(_phi(p, 1.0 / np.sqrt(m + eps * dm)) - phi0 - eps * np.sum(p["g"] * dm))
    assert rs[0] / rs[1] == pytest.approx(4.0, rel=0.05)
    assert rs[1] / rs[2] == pytest.approx(4.0, rel=0.05)


def test_misfit_definition():
    a = np.array([[1.0, 2.0], [3.0, 4.0]])
    b = np.array([[0.0, 2.5], [3.0, 2.0]])
    assert oracle.misfit(a, b) == 0.5 * (1.0 + 0.25 + 0.0 + 4.0)


@pytest.mark.parametrize("write_min", [False, True])
@pytest.mark.parametrize("M", [1, 2, 3, 5, 12, 80, 200])
def test_revolve_bit_identical_to_full_storage(prob2d, M, write_min):
    p = prob2d
    acts = SC.schedule(p["spec"].nt, M, write_min=write_min)
    g, st = p["S"].gradient_actions(p["res"], acts, M)
    assert np.array_equal(g, p["g"])
    c = SC.counts(acts)
    assert st["advances"] == c["advances"] == SC.p_closed(p["spec"].nt + 1, M)
    assert st["reverses"] == p["spec"].nt


def test_compressed_gradient_error_trend(prob2d):
    """Checkpoints through the codec: error falls with the tolerance, roughly linearly
    (the paper's tolerance-vs-gradient-error table shows the same monotone trend)."""
    p = prob2d
    acts = SC.schedule(p["spec"].nt, 6)
    gref = np.linalg.norm(p["g"])
    errs = []
    for tol in (1e-3, 1e-4, 1e-5, 1e-6):
        g, _ = p["S"].gradient_actions(p["res"], acts, 6, tol=tol, increment=True)
        errs.append(np.linalg.norm(g - p["g"]) / gref)
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))
    for i in range(len(errs) - 1):
        assert errs[i] / errs[i + 1] < 30.0          # no faster than ~linear in tol
    # levels and increment representations agree to within the same order
    g_lv, _ = p["S"].gradient_actions(p["res"], acts, 6, tol=1e-5, increment=False)
    assert np.linalg.norm(g_lv - p["g"]) / gref < 10 * errs[2] + 1e-9


@pytest.mark.parametrize("tol", [1e-3, 1e-5])
def test_compression_only_gradient_within_pointwise_bound(prob2d, tol):
    """Every state stored compressed (M = N, no recomputation): the adjoint states do not
    depend on u, so by the gradient's definition
        |g_tol - g_0| <= e (1/dt^2) sum_k |(1+a) lam^{k-1} - 2 lam^k + (1-a) lam^{k+1}|
    at every point, with e the largest change of a stored state: the codec's tol plus the
    rounding of the state to binary32 before encoding.  A reversal that reads the state of
    the neighbouring step (a planted mistake) breaks the bound."""
    p = prob2d
    N = p["spec"].nt
    g, st = p["S"].gradient_actions(p["res"], SC.schedule(N, N), N, tol=tol, increment=True)
    assert st["advances"] == N
    B = p["S"].gradient_bound(p["res"])
    e = tol + 2.0 ** -24 * np.abs(p["fw"]["traj"]).max()
    d = np.abs(g - p["g"])
    assert np.all(d <= e * B * (1.0 + 1e-9))
    assert d.max() > 0.0
    # planted mistake: every reverse step reads u^{k-1} instead of u^k
    traj = p["fw"]["traj"]
    shifted = np.concatenate([np.zeros_like(traj[:1]), traj[:-1]])
    wrong = p["S"].gradient_full(shifted, p["res"])
    assert np.any(np.abs(wrong - p["g"]) > e * B)
