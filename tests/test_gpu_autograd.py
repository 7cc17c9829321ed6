"""Autograd path: interior velocity -> misfit through the C ABI (pad, one checkpointed
sweep, chain rule and pad adjoint), checked against the oracle and finite differences."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.helpers import has_gpu, oracle_side, rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not has_gpu(), reason="needs a GPU")]


def make_problem(shot, tol, budget_states, headroom=1.0):
    """headroom > 1 raises the velocity bound (damping and stability limit) so that
    perturbed velocities stay admissible."""
    import torch
    import paper_1810_05268_amd as P
    from paper_1810_05268_amd.autograd import WaveProblem
    vmax = headroom * shot.vmax
    dt = shot.cfl_frac * P.cfl_dt(shot.ndim, shot.h, shot.order, vmax)
    q = W.ricker(shot.f0, dt, shot.nt).astype(np.float32)
    St, _ = oracle_side(shot, "true") if headroom == 1.0 else (None, None)
    if St is not None:
        d_obs = St.forward()["data"].astype(np.float32)
    else:   # observed data from the GPU forward on the true model (same dt, same damping)
        from paper_1810_05268_amd.shot import DeviceShot
        Gt = DeviceShot(shot.ndim, shot.n, shot.h, shot.nbl, shot.order, shot.nt, dt, vmax, shot.padded("true"),
                        q, shot.src, shot.rec)
        d_obs = Gt.forward().cpu().numpy()
    S = 8 * int(np.prod(shot.padded_shape()))
    pb = WaveProblem(shot.ndim, shot.n, shot.h, shot.nbl, shot.order, shot.nt, dt, vmax, q, shot.src,
                     shot.rec, d_obs, budget_states * S, tol=tol)
    vel = torch.tensor(shot.vel, dtype=torch.float32, device="cuda", requires_grad=True)
    return pb, vel, d_obs


def pad_adjoint(g, nbl):
    """Sum layer cells into the interior cell they copy (numpy, test side)."""
    out = g.copy()
    for ax in range(g.ndim):
        out = np.moveaxis(out, ax, 0)
        lo = out[:nbl + 1].sum(0)
        hi = out[-nbl - 1:].sum(0)
        out = out[nbl:-nbl].copy() if nbl else out.copy()
        out[0] = lo
        out[-1] = hi
        out = np.moveaxis(out, 0, ax)
    return out


def test_velocity_gradient_matches_oracle():
    import paper_1810_05268_amd.autograd as A
    shot = W.near_anomaly_2d(n=(61, 57), nt=300)
    pb, vel, d_obs = make_problem(shot, 0.0, 40)
    phi = A.wave_misfit(vel, pb)
    phi.backward()
    S, _ = oracle_side(shot)
    fw = S.forward(want_traj=True)
    res = fw["data"] - d_obs.astype(np.float64)
    gm = S.gradient_full(fw["traj"], res)
    vp = shot.padded("vel").astype(np.float64)
    gref = pad_adjoint(-2.0 * gm / vp ** 3, shot.nbl)
    assert abs(float(phi.detach()) - 0.5 * float(np.sum(res ** 2))) <= 1e-4 * float(phi.detach())
    assert rel_l2(vel.grad.double().cpu().numpy(), gref) <= 1e-4


def _c3_oracle(shot, vmax):
    """The FP64 oracle on the smooth random 2-D medium (400^2 interior at 5 m, 2000 steps,
    order 8) at the raised velocity bound vmax: observed data from the true model
    (rounded to binary32, the GPU's input too), and the misfit, residual and full-storage
    gradient with respect to m and to the interior velocity."""
    dt = shot.cfl_frac * oracle.cfl_dt(shot.ndim, shot.h, shot.order, vmax)
    spec = oracle.ModelSpec(shot.ndim, shot.n, shot.h, shot.nbl, shot.order, shot.nt, dt, vmax)
    q = W.ricker(shot.f0, dt, shot.nt)
    St = oracle.Solver(spec, shot.padded("true").astype(np.float64), shot.src, q, shot.rec)
    d_obs = St.forward()["data"].astype(np.float32)
    del St
    S = oracle.Solver(spec, shot.padded("vel").astype(np.float64), shot.src, q, shot.rec)
    fw = S.forward(want_traj=True)
    res = fw["data"] - d_obs.astype(np.float64)
    phi = 0.5 * float(np.sum(res ** 2))
    gm = S.gradient_full(fw["traj"], res)
    del fw
    vp = shot.padded("vel").astype(np.float64)
    return S, d_obs, res, phi, gm, pad_adjoint(-2.0 * gm / vp ** 3, shot.nbl)


def test_smooth_random_full_size_against_oracle_and_finite_differences():
    """The autograd configuration at its own size: the 2-D smooth random medium (400^2
    interior at 5 m, 20-cell layer, 2000 steps, order 8), checkpoints compressed at 1e-5.

    Against the FP64 oracle at full size:
      * forward data: rel-L2 <= 1e-5.  The residual d_sim - d_obs is a small difference of
        large data, so its relative error e_r = ||d_gpu - d_or|| / ||d_or - d_obs|| is the
        data error times ||d|| / ||r||; it is measured and carried below;
      * the adjoint gradient for the oracle's own residual (wv_gradient, 20 checkpoints):
        rel-L2 <= 1e-4, the stencil and gradient accuracy alone;
      * the autograd path (misfit and gradient from the GPU's own residual): the misfit
        within its exact bound 2 e_r + e_r^2 (phi = ||r||^2 / 2); the velocity gradient is
        the chain rule and the pad adjoint of the GPU's m-gradient for that residual
        (checked against the same map in numpy), and its distance to the oracle's is
        reported: the adjoint maps the residual error e_r into the gradient with a gain
        the test does not bound, so the adjoint's own accuracy is the check above;
      * compressed at 1e-5 with the configuration's budget (20 raw states): the slot count
        the call planned, replayed by the oracle's compressed reversal on the same schedule
        for the same residual; the codec's share of the gradient matches
        (check_codec_parity).
    Finite differences, per direction (the normalised gradient and 20 seeded smooth unit
    directions, white noise filtered by a Gaussian of 10 cells): the GPU misfit at
    v + s eps dv for s = 0, +-1/8, ..., +-1 (eps = 1e-3 ||v||) and a least-squares
    polynomial of degree 7 in s through the 17 values; its linear coefficient / eps is the
    derivative (truncation O(eps^8): along these directions a 1e-3 ||v|| step shifts the
    waveforms by a sizeable fraction of a period, and a Richardson central difference,
    printed beside it, keeps an O(eps^4) term of the size of the small derivatives).  The
    fit's residuals along the random directions measure the misfit's binary32 rounding
    noise sigma (pooled, 180 degrees of freedom); the fitted derivative then has std
    2.77 sigma / eps, and the floor is three of those.  In every direction whose exact
    derivative (the oracle's <g, dv>) exceeds 10 times the floor, the fitted derivative
    must agree with it to 1e-3 relative plus the floor; along the gradient it must also
    agree so with the GPU adjoint's <g, dv>.  (In the random directions the GPU
    gradient's own error, the residual's rounding e_r mapped by the adjoint, is of the
    size of these small derivatives' floor; it is reported per direction, and the adjoint
    itself is checked above on the oracle's residual.)"""
    import torch
    import paper_1810_05268_amd.autograd as A
    from paper_1810_05268_amd.autograd import WaveProblem
    from paper_1810_05268_amd.shot import DeviceShot
    from scipy.ndimage import gaussian_filter
    from oracle import schedule as SC
    from tests.test_gpu_compressed import check_codec_parity
    import paper_1810_05268_amd as P
    shot = W.smooth_random_2d()
    vmax = 1.02 * shot.vmax              # headroom: perturbed velocities stay admissible
    S, d_obs, res, phi_or, gm_or, gv_or = _c3_oracle(shot, vmax)
    dt = shot.cfl_frac * P.cfl_dt(shot.ndim, shot.h, shot.order, vmax)
    q = W.ricker(shot.f0, dt, shot.nt).astype(np.float32)
    Sb = 8 * int(np.prod(shot.padded_shape()))
    vp = shot.padded("vel").astype(np.float64)

    # forward data and the residual's conditioning
    G = DeviceShot(shot.ndim, shot.n, shot.h, shot.nbl, shot.order, shot.nt, dt, vmax, shot.padded("vel"), q,
                   shot.src, shot.rec)
    d_gpu = G.forward().double().cpu().numpy()
    d_or = res + d_obs.astype(np.float64)
    e_d = rel_l2(d_gpu, d_or)
    e_r = float(np.linalg.norm(d_gpu - d_or) / np.linalg.norm(res))
    print(f"C3 data rel-L2 {e_d:.2e}, residual rel error e_r {e_r:.2e}")
    assert e_d <= 1e-5

    # the adjoint gradient for the oracle's residual
    rt = torch.as_tensor(res.astype(np.float32), device="cuda")
    gm, stg = G.gradient(rt, 20 * Sb)
    e_gm = rel_l2(gm.cpu().numpy(), gm_or)
    print(f"C3 gradient for the oracle residual: slots {stg['slots']} rel-L2 {e_gm:.2e}")
    assert stg["slots"] == 21 and e_gm <= 1e-4

    # compressed at 1e-5 for the same residual; the oracle replays the planned schedule
    gc_m, stc_m = G.gradient(rt, 20 * Sb, tol=1e-5)
    M = int(stc_m["slots"])
    assert M > 21 and stc_m["retries"] == 0          # compression bought more slots
    acts = SC.schedule(shot.nt, M)
    g_or_tol, st_or = S.gradient_actions(res, acts, M, tol=1e-5, increment=True)
    assert st_or["advances"] == stc_m["advances"] and st_or["stores"] == stc_m["stores"]
    gp_m, stp = G.gradient(rt, (M - 1) * Sb)          # plain on the same slot count
    assert stp["slots"] == M and stp["advances"] == stc_m["advances"]
    check_codec_parity(f"C3 tol 1e-5 M {M}", gc_m.cpu().numpy(), gp_m.cpu().numpy(), g_or_tol, gm_or)
    del G, gm, gc_m, gp_m

    def problem(budget, tol):
        return WaveProblem(shot.ndim, shot.n, shot.h, shot.nbl, shot.order, shot.nt, dt, vmax, q, shot.src,
                           shot.rec, d_obs, budget, tol=tol)

    def run(pb):
        vel = torch.tensor(shot.vel, dtype=torch.float32, device="cuda", requires_grad=True)
        phi = A.wave_misfit(vel, pb)
        phi.backward()
        return float(phi.detach()), vel.grad.double().cpu().numpy(), pb.last_stats

    # the autograd path, uncompressed and compressed
    phi0, g0, st0 = run(problem(20 * Sb, 0.0))
    e_phi = abs(phi0 - phi_or) / phi_or
    e_g0 = rel_l2(g0, gv_or)
    print(f"C3 autograd plain: slots {st0['slots']} misfit rel err {e_phi:.2e} (bound {2 * e_r + e_r ** 2:.2e}) "
          f"gradient rel-L2 to the oracle's {e_g0:.2e}")
    assert st0["slots"] == 21
    assert e_phi <= 2.0 * e_r + e_r ** 2
    # the velocity gradient is the chain rule and pad adjoint of the m-gradient
    Gm = DeviceShot(shot.ndim, shot.n, shot.h, shot.nbl, shot.order, shot.nt, dt, vmax, shot.padded("vel"), q,
                    shot.src, shot.rec)
    phim, gmm, _ = Gm.misfit_gradient(torch.as_tensor(d_obs, device="cuda"), 20 * Sb)
    assert phim == phi0
    del Gm
    # vel.grad is stored in vel's dtype (float32): each element is rounded once, so the
    # relative L2 difference is at most the unit roundoff 2^-24 (plus the FP64 rounding)
    assert rel_l2(g0, pad_adjoint(-2.0 * gmm.cpu().numpy() / vp ** 3, shot.nbl)) <= 2.0 ** -24 + 1e-12
    pbc = problem(20 * Sb, 1e-5)
    phic, gc, stc = run(pbc)
    e_gc = rel_l2(gc, g0)
    print(f"C3 autograd compressed: slots {stc['slots']} rel-L2 to plain {e_gc:.2e}")
    assert phic == phi0 and stc["slots"] == M and e_gc <= 1e-4

    # finite differences of the GPU misfit, per direction
    v0 = torch.tensor(shot.vel, dtype=torch.float64, device="cuda")
    vnorm = float(torch.linalg.vector_norm(v0))
    gcd = torch.as_tensor(gc, device="cuda")

    def misfit_at(v):
        with torch.no_grad():
            return float(A.wave_misfit(v.float(), pbc))

    dphi = abs(phic - phi_or)
    eps = 1e-3 * vnorm
    sg = np.arange(-8, 9) / 8.0                   # t = s eps, s = 0, +-1/8, ..., +-1
    X = np.stack([sg ** k for k in range(8)], 1)
    XtXi = np.linalg.inv(X.T @ X)
    gvo = torch.as_tensor(gv_or, device="cuda")
    dirs = [gvo / torch.linalg.vector_norm(gvo)]
    for seed in range(30, 50):
        noise = np.random.default_rng(seed).standard_normal(tuple(shot.vel.shape))
        dv = torch.as_tensor(gaussian_filter(noise, sigma=10.0, mode="reflect"), device="cuda")
        dirs.append(dv / torch.linalg.vector_norm(dv))
    rows, rss = [], 0.0
    for j, dv in enumerate(dirs):
        ph = np.array([phic if s_ == 0.0 else misfit_at(v0 + (s_ * eps) * dv) for s_ in sg])
        coef = XtXi @ (X.T @ ph)                  # least-squares degree-7 polynomial in s
        fd = coef[1] / eps
        rich = (4.0 * (ph[12] - ph[4]) / eps - (ph[16] - ph[0]) / (2 * eps)) / 3.0
        if j > 0:
            rss += float(np.sum((ph - X @ coef) ** 2))
        rows.append((j, fd, rich, float(torch.sum(gcd * dv)), float(torch.sum(gvo * dv))))
    dof = (len(sg) - 8) * (len(dirs) - 1)
    sigma = (rss / dof) ** 0.5
    se = np.sqrt(XtXi[1, 1]) * sigma / eps       # std of the fitted derivative: 2.77 sigma / eps
    floor = 3.0 * se
    print(f"misfit rounding noise: sigma {sigma:.3e} ({dof} dof; |phi - oracle| at v0: {dphi:.3e}); "
          f"FD std {se:.3e}, floor {floor:.3e}")
    checked = 0
    for j, fd, rich, ad, ad_or in rows:
        big = abs(ad_or) >= 10.0 * floor
        print(f"direction {j}: fd {fd:+.6e} (Richardson {rich:+.6e}) adjoint {ad:+.6e} oracle {ad_or:+.6e}  "
              f"|fd-or|/|or| {abs(fd - ad_or) / abs(ad_or):.2e}  |fd-ad|/|ad| {abs(fd - ad) / abs(ad):.2e}  "
              f"|ad-or|/|or| {abs(ad - ad_or) / abs(ad_or):.2e}  floor/|or| {floor / abs(ad_or):.2e}"
              f"{'' if big else '  (below 10x the floor: reported only)'}")
        if big:
            checked += 1
            assert abs(fd - ad_or) <= 1e-3 * abs(ad_or) + floor
        if j == 0:
            assert abs(fd - ad) <= 1e-3 * abs(ad) + floor
    assert checked >= 8
    # along the gradient a plain central difference converges quadratically
    gn = float(torch.sum(gcd * dirs[0]))

    def central(frac):
        e = frac * vnorm
        return (misfit_at(v0 + e * dirs[0]) - misfit_at(v0 - e * dirs[0])) / (2 * e)
    e_big = abs(central(1e-3) - gn)
    e_small = abs(central(1e-4) - gn)
    print(f"along g: error {e_big:.3e} at 1e-3, {e_small:.3e} at 1e-4")
    assert 30.0 < e_big / e_small < 300.0
