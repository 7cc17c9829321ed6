"""Pins of the oracle's OT4 kernel: the fourth-order-in-time (modified-equation) scheme
the paper runs beside OT2 (Sec. "Problem and test case"), with spatial operator
B(m) u = lap u + (dt^2/12) lap((1/m) lap u).  Checked against a closed-form single-mode
solution, its fourth-order convergence in time, its stability limit, the dot-product
test, finite differences of the misfit and the checkpointed reversal."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import schedule as SC
from tests.test_oracle_adjoint import tiny_problem


def _homog(n, h, order, nt, dt, vel, time_order):
    nd = len(n)
    spec = oracle.ModelSpec(nd, tuple(n), tuple(h), 0, order, nt, dt, vel, time_order=time_order)
    src = np.array([[(n[d] - 1) * h[d] / 2 for d in range(nd)]])
    return oracle.Solver(spec, np.full(spec.array_shape(), vel), src, np.zeros(max(nt, 1)), src.copy()), spec


def _mode(n, h, px=3, pz=2):
    z, x = np.meshgrid(np.arange(n[1]), np.arange(n[0]), indexing="ij")
    phi = np.sin(math.pi * px * (x + 1) / (n[0] + 1)) * np.sin(math.pi * pz * (z + 1) / (n[1] + 1))
    lam = -4 / h[0] ** 2 * (math.sin(math.pi * px / (2 * (n[0] + 1))) ** 2 +
                            math.sin(math.pi * pz / (2 * (n[1] + 1))) ** 2)
    return phi, lam


def test_single_mode_closed_form():
    """Order 2, no damping: a discrete sine mode phi is an exact eigenvector of lap (zero
    halo), so B phi = (lam + w lam^2 / 12) phi and u^n = cos(n Om) phi with
    cos Om = 1 + (w lam + (w lam)^2 / 12) / 2."""
    n, h, vel = (15, 11), (10.0, 10.0), 1800.0
    dt = 0.5 * oracle.cfl_dt(2, h, 2, vel, time_order=4)
    S, _ = _homog(n, h, 2, 1, dt, vel, 4)
    phi, lam = _mode(n, h)
    wl = dt * dt * vel * vel * lam
    Om = math.acos(1 + (wl + wl * wl / 12) / 2)
    prev, cur = math.cos(-Om) * phi, phi.copy()
    for step in range(1, 200):
        prev, cur = cur, S.forward_step(0, cur, prev)
        assert np.allclose(cur, math.cos(step * Om) * phi, atol=1e-9)


@pytest.mark.parametrize("time_order,ratio", [(2, 4.0), (4, 16.0)])
def test_convergence_order_in_time(time_order, ratio):
    """Against the exact solution cos(omega t) phi of the semi-discrete equation
    u'' = c^2 lap u, halving dt at a fixed final time divides the error by 2^order."""
    n, h, vel = (15, 11), (10.0, 10.0), 1800.0
    phi, lam = _mode(n, h, 5, 4)
    om = vel * math.sqrt(-lam)
    T = 4.3 * 2 * math.pi / om     # not a whole number of periods: sin(omega T) != 0
    errs = []
    for k in range(3):
        dt = 0.1 * oracle.cfl_dt(2, h, 2, vel) / 2 ** k
        steps = int(round(T / dt))
        dt = T / steps
        S, _ = _homog(n, h, 2, 1, dt, vel, time_order)
        prev, cur = math.cos(-om * dt) * phi, phi.copy()
        for _ in range(steps):
            prev, cur = cur, S.forward_step(0, cur, prev)
        errs.append(float(np.abs(cur - math.cos(om * T) * phi).max()))
    print(time_order, errs)
    assert errs[0] / errs[1] == pytest.approx(ratio, rel=0.15)
    assert errs[1] / errs[2] == pytest.approx(ratio, rel=0.15)


def test_stability_limit():
    """The OT4 limit is sqrt(3) times the OT2 one; at 0.98 of it the undamped scheme
    stays bounded, at 1.05 it blows up."""
    n, h, order, vel = (16, 16), (10.0, 10.0), 8, 2000.0
    lim = oracle.cfl_dt(2, h, order, vel, time_order=4)
    assert lim == pytest.approx(math.sqrt(3.0) * oracle.cfl_dt(2, h, order, vel), rel=1e-14)
    rng = np.random.default_rng(0)
    for frac, bounded in [(0.98, True), (1.05, False)]:
        S, spec = _homog(n, h, order, 1, frac * lim, vel, 4)
        prev = np.zeros(spec.array_shape())
        cur = rng.standard_normal(spec.array_shape())
        for _ in range(600):
            prev, cur = cur, S.forward_step(0, cur, prev)
        assert (np.abs(cur).max() < 1e3) == bounded


def ot4_problem(ndim=2, nt=80, order=4, nbl=5, n=None, f0=30.0):
    spec, vel, velt, src, rec, _ = tiny_problem(ndim=ndim, nt=nt, order=order, nbl=nbl, n=n, f0=f0)
    dt = 0.4 * oracle.cfl_dt(ndim, spec.h, order, spec.vmax, time_order=4)
    spec = dataclasses.replace(spec, dt=dt, time_order=4)
    return spec, vel, velt, src, rec, W.ricker(f0, dt, nt)


@pytest.fixture(scope="module")
def prob_ot4():
    spec, vel, velt, src, rec, q = ot4_problem()
    S = oracle.Solver(spec, vel, src, q, rec)
    St = oracle.Solver(spec, velt, src, q, rec)
    fw = S.forward(want_traj=True)
    dobs = St.forward()["data"]
    res = fw["data"] - dobs
    g, lam = S.gradient_full(fw["traj"], res, want_lam=True)
    return dict(spec=spec, vel=vel, src=src, rec=rec, q=q, S=S, fw=fw, dobs=dobs, res=res, g=g, lam=lam)


@pytest.mark.parametrize("ndim", [2, 3])
def test_dot_product(ndim):
    spec, vel, _, src, rec, _ = ot4_problem(ndim=ndim, nt=40 if ndim == 3 else 80)
    rng = np.random.default_rng(7)
    q = rng.standard_normal(spec.nt)
    S = oracle.Solver(spec, vel, src, q, rec)
    d = S.forward()["data"]
    r = rng.standard_normal(d.shape)
    lhs = float(np.dot(d.ravel(), r.ravel()))
    rhs = float(np.dot(q, S.adjoint_src(r)))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_differs_from_ot2(prob_ot4):
    """The OT4 data are not the OT2 data of the same dt (the correction term acts)."""
    p = prob_ot4
    S2 = oracle.Solver(dataclasses.replace(p["spec"], time_order=2), p["vel"], p["src"], p["q"], p["rec"])
    d2 = S2.forward()["data"]
    rel = np.linalg.norm(d2 - p["fw"]["data"]) / np.linalg.norm(p["fw"]["data"])
    assert rel > 1e-4


def test_summation_by_parts(prob_ot4):
    p = prob_ot4
    gn = p["S"].gradient_nform(p["fw"]["traj"], p["lam"])
    assert np.linalg.norm(gn - p["g"]) <= 1e-12 * np.linalg.norm(p["g"])


def _phi(p, vel):
    s = oracle.Solver(p["spec"], vel, p["src"], p["q"], p["rec"])
    return oracle.misfit(s.forward()["data"], p["dobs"])


def test_central_finite_differences(prob_ot4):
    """Pins the gradient including the term from the m inside B(m): the central
    difference converges to it as eps^2 (a missing or wrong term would leave a
    plateau instead)."""
    p = prob_ot4
    gc = -2.0 * p["g"] / p["vel"] ** 3
    rng = np.random.default_rng(11)
    for _ in range(3):
        dv = rng.standard_normal(p["vel"].shape)
        errs = []
        for rel in (1e-3, 1e-4, 1e-5):
            eps = rel * np.linalg.norm(p["vel"]) / np.linalg.norm(dv)
            fd = (_phi(p, p["vel"] + eps * dv) - _phi(p, p["vel"] - eps * dv)) / (2 * eps)
            errs.append(abs(fd - np.sum(gc * dv)) / abs(fd))
        print("fd errors", errs)
        assert errs[2] < 1e-5
        assert errs[1] < errs[0] / 30 and errs[2] < errs[1] / 30


@pytest.mark.parametrize("write_min", [False, True])
@pytest.mark.parametrize("M", [1, 3, 12, 80])
def test_revolve_bit_identical_to_full_storage(prob_ot4, M, write_min):
    p = prob_ot4
    acts = SC.schedule(p["spec"].nt, M, write_min=write_min)
    g, st = p["S"].gradient_actions(p["res"], acts, M)
    assert np.array_equal(g, p["g"])
    assert st["advances"] == SC.p_closed(p["spec"].nt + 1, M)
