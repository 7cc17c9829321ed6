"""Pins of the oracle's discretisation of eq. (7) against closed forms and exact identities."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W


def exact_coeffs(K):
    """Taylor conditions solved exactly in rationals: sum_k a_k k^(2j) = [j == 1] for
    j = 1..K (a_k symmetric), a_0 = -2 sum a_k.  Independent of the closed form."""
    A = [[Fraction(k) ** (2 * j) for k in range(1, K + 1)] for j in range(1, K + 1)]
    b = [Fraction(1 if j == 1 else 0) for j in range(1, K + 1)]
    n = K
    for i in range(n):                       # Gauss-Jordan in exact arithmetic
        piv = next(r for r in range(i, n) if A[r][i] != 0)
        A[i], A[piv] = A[piv], A[i]
        b[i], b[piv] = b[piv], b[i]
        for r in range(n):
            if r != i and A[r][i] != 0:
                f = A[r][i] / A[i][i]
                A[r] = [x - f * y for x, y in zip(A[r], A[i])]
                b[r] -= f * b[i]
    ak = [b[i] / A[i][i] for i in range(n)]
    return [-2 * sum(ak)] + ak


@pytest.mark.parametrize("K", range(1, 9))
def test_fd_coeffs_match_taylor_conditions(K):
    a = oracle.fd_coeffs(K)
    ex = exact_coeffs(K)
    for k in range(K + 1):
        assert a[k] == pytest.approx(float(ex[k]), rel=1e-13, abs=1e-15)


def test_fd_coeffs_printed_values():
    # order 4 and order 8 second-derivative weights (standard tables)
    assert np.allclose(oracle.fd_coeffs(2), [-5 / 2, 4 / 3, -1 / 12], rtol=1e-15)
    assert np.allclose(oracle.fd_coeffs(4), [-205 / 72, 8 / 5, -1 / 5, 8 / 315, -1 / 560], rtol=1e-14)


@pytest.mark.parametrize("order,S", [(2, 4.0), (4, 5.3333), (8, 6.5016), (12, 7.0729), (16, 7.4269)])
def test_cfl_constant(order, S):
    # dt_cfl = 2 h / (c sqrt(d S)); brute-force the symbol max over wavenumbers
    a = oracle.fd_coeffs(order // 2)
    th = np.linspace(0, math.pi, 20001)
    symbol = a[0] + 2 * sum(a[k] * np.cos(k * th) for k in range(1, order // 2 + 1))
    assert np.max(np.abs(symbol)) == pytest.approx(S, abs=1e-4)
    h, c = 10.0, 2000.0
    assert oracle.cfl_dt(3, (h, h, h), order, c) == pytest.approx(2 * h / (c * math.sqrt(3 * np.max(np.abs(symbol)))),
                                                                  rel=1e-9)


def _homog(n, h, nbl, order, nt, dt, vel=2000.0, src=None, rec=None, wavelet=None):
    nd = len(n)
    spec = oracle.ModelSpec(nd, tuple(n), tuple(h), nbl, order, nt, dt, vel)
    shape = spec.array_shape()
    v = np.full(shape, vel)
    src = src if src is not None else np.array([[(n[d] - 1) * h[d] / 2 for d in range(nd)]])
    rec = rec if rec is not None else src.copy()
    wavelet = wavelet if wavelet is not None else np.zeros(max(nt, 1))
    return oracle.Solver(spec, v, src, wavelet, rec), spec


@pytest.mark.parametrize("order", [2, 4, 8, 16])
def test_laplacian_exact_on_polynomials(order):
    """A 2K-th order centred second difference is exact on polynomials of degree <= 2K+1."""
    K = order // 2
    n, h = (30, 28, 26), (10.0, 12.5, 7.5)
    S, spec = _homog(n, h, 0, order, 1, 1e-4)
    z, y, x = np.meshgrid(*(np.arange(m) * hh for m, hh in zip(reversed(n), reversed(h))), indexing="ij")
    deg = min(2 * K + 1, 5)
    u = (x / 100) ** deg + 0.5 * (y / 100) ** 2 * (z / 100) - (z / 100) ** 3 + 2.0
    lap_ex = deg * (deg - 1) * (x / 100) ** (deg - 2) / 100 ** 2 + (z / 100) / 100 ** 2 - 6 * (z / 100) / 100 ** 2
    lap = S.laplacian(u)
    sl = (slice(K, -K),) * 3
    assert np.allclose(lap[sl], lap_ex[sl], rtol=1e-9, atol=1e-12)


def test_laplacian_zero_halo():
    """Outside the padded grid the field is zero: the stencil at the edge sees zeros."""
    S, spec = _homog((12, 12), (10.0, 10.0), 0, 4, 1, 1e-4)
    u = np.ones(spec.array_shape())
    lap = S.laplacian(u)
    a = oracle.fd_coeffs(2)
    # corner point: each axis misses both +-1, +-2 neighbours on one side
    corner = 2 * (a[0] + a[1] + a[2]) / 100.0
    assert lap[0, 0] == pytest.approx(corner, rel=1e-14)
    assert lap[6, 6] == pytest.approx(0.0, abs=1e-15)


def test_leapfrog_single_mode_closed_form():
    """Order 2, no damping: discrete sine modes are exact eigenvectors of the Laplacian
    with the zero halo, so u^n = cos(n Omega) phi with cos Omega = 1 - w lambda / 2."""
    n, h = (15, 11), (10.0, 10.0)
    vel = 1800.0
    dt = 0.5 * oracle.cfl_dt(2, h, 2, vel)
    S, spec = _homog(n, h, 0, 2, 1, dt, vel=vel)
    z, x = np.meshgrid(np.arange(n[1]), np.arange(n[0]), indexing="ij")
    px, pz = 3, 2
    phi = np.sin(math.pi * px * (x + 1) / (n[0] + 1)) * np.sin(math.pi * pz * (z + 1) / (n[1] + 1))
    lam = -4 / h[0] ** 2 * (math.sin(math.pi * px / (2 * (n[0] + 1))) ** 2 +
                            math.sin(math.pi * pz / (2 * (n[1] + 1))) ** 2)
    w = dt * dt * vel * vel
    Om = math.acos(1 + w * lam / 2)
    prev, cur = math.cos(-Om) * phi, phi.copy()
    for step in range(1, 200):
        nxt = S.forward_step(0, cur, prev)
        prev, cur = cur, nxt
        assert np.allclose(cur, math.cos(step * Om) * phi, atol=1e-9)


def test_damped_update_single_step():
    """Where the Laplacian of a field vanishes, one step gives u^1 = (2u^0 - (1-a)u^-1)/(1+a)."""
    S, spec = _homog((30, 30), (10.0, 10.0), 20, 4, 1, 1e-3, vel=2500.0)
    a = S.damp()
    u0 = np.full(spec.array_shape(), 1.0)
    um = np.full(spec.array_shape(), 0.25)
    u1 = S.forward_step(0, u0, um)
    inner = (slice(4, -4),) * 2       # at least K cells from the zero halo
    expect = (2 - (1 - a) * 0.25) / (1 + a)
    assert np.allclose(u1[inner], expect[inner], rtol=1e-14)


def test_damping_profile():
    nbl, vmax, h, dt = 10, 3000.0, (10.0, 20.0), 1e-3
    S, spec = _homog((20, 16), h, nbl, 4, 1, dt, vel=vmax)
    a = S.damp()
    assert (a >= 0).all()
    assert (a[nbl:-nbl, nbl:-nbl] == 0).all()
    # outermost corner: delta = nbl on both axes
    smax = [3 * vmax * math.log(1000) / (2 * nbl * hh) for hh in h]
    assert a[0, 0] == pytest.approx(0.5 * dt * (smax[0] + smax[1]), rel=1e-14)
    # first layer cell along x only: delta = 1
    assert a[nbl + 3, nbl - 1] == pytest.approx(0.5 * dt * smax[0] / nbl ** 2, rel=1e-14)
    # monotone towards the edge
    assert np.all(np.diff(a[nbl + 3, :nbl]) < 0)


def test_interpolation_reproduces_affine_functions():
    rng = np.random.default_rng(1)
    n, h, nbl = (12, 10, 9), (10.0, 12.5, 7.5), 3
    pts = rng.uniform(0, 1, size=(50, 3)) * np.array([(n[d] - 1) * h[d] for d in range(3)])
    S, spec = _homog(n, h, nbl, 4, 1, 1e-4, src=pts[:1], rec=pts)
    idx, wt = S.interp(1)
    assert np.allclose(wt.sum(1), 1.0, rtol=1e-14)
    assert (wt >= 0).all()
    N = spec.padded()
    lin = np.unravel_index(idx, tuple(reversed(N)))          # (z, y, x)
    coords = [(lin[2 - d] - nbl) * h[d] for d in range(3)]
    f = lambda c: 1.5 * c[0] - 0.25 * c[1] + 3.0 * c[2] + 7.0
    approx = (wt * f(coords)).sum(1)
    assert np.allclose(approx, f(pts.T), rtol=1e-12)


def test_ricker_input_generator():
    f0, dt = 10.0, 1e-3
    q = W.ricker(f0, dt, 400)
    assert q[100] == pytest.approx(1.0)                      # peak at t0 = 1/f0
    tz = 1 / f0 + 1 / (math.pi * f0 * math.sqrt(2))          # zero crossing
    assert W.ricker(f0, tz, 2)[1] == pytest.approx(0.0, abs=1e-12)


def test_cfl_stability_boundary():
    """At 0.98 of the limit the undamped scheme stays bounded; at 1.05 it blows up."""
    n, h, order, vel = (16, 16), (10.0, 10.0), 8, 2000.0
    lim = oracle.cfl_dt(2, h, order, vel)
    rng = np.random.default_rng(0)
    for frac, bounded in [(0.98, True), (1.05, False)]:
        S, spec = _homog(n, h, 0, order, 1, frac * lim, vel=vel)
        prev = np.zeros(spec.array_shape())
        cur = rng.standard_normal(spec.array_shape())
        for _ in range(600):
            prev, cur = cur, S.forward_step(0, cur, prev)
        mx = np.abs(cur).max()
        assert (mx < 1e3) == bounded
