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
    Finite differences, per direction (the normalised gradient and 10 seeded smooth unit
    directions, white noise filtered by a Gaussian of 10 cells): a Richardson-extrapolated
    central difference of the GPU misfit, R = (4 D(eps/2) - D(eps)) / 3 with
    D(e) = (phi(v + e dv) - phi(v - e dv)) / (2 e) and eps = 1e-3 ||v|| (truncation
    O(eps^4)), against the GPU adjoint's directional derivative <g, dv> (the same misfit
    function); the oracle's is reported beside it.  The binary32 floor of R is
    3 dphi / eps, dphi = |phi_gpu - phi_oracle| (each of the four misfits is within dphi of
    exact and R weighs them by 4/(3 eps) and 1/(6 eps)); every direction whose derivative
    exceeds 10 times that floor must agree to 1e-3 relative plus the floor, and the others
    are reported."""
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
    assert rel_l2(g0, pad_adjoint(-2.0 * gmm.cpu().numpy() / vp ** 3, shot.nbl)) <= 1e-12
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

    def richardson(dv, eps):
        def D(e):
            return (misfit_at(v0 + e * dv) - misfit_at(v0 - e * dv)) / (2 * e)
        return (4.0 * D(eps / 2) - D(eps)) / 3.0

    dphi = abs(phic - phi_or)
    eps = 1e-3 * vnorm
    floor = 3.0 * dphi / eps
    gvo = torch.as_tensor(gv_or, device="cuda")
    dirs = [gvo / torch.linalg.vector_norm(gvo)]
    for seed in range(30, 40):
        noise = np.random.default_rng(seed).standard_normal(tuple(shot.vel.shape))
        dv = torch.as_tensor(gaussian_filter(noise, sigma=10.0, mode="reflect"), device="cuda")
        dirs.append(dv / torch.linalg.vector_norm(dv))
    checked = 0
    for j, dv in enumerate(dirs):
        ad_or = float(torch.sum(gvo * dv))
        ad = float(torch.sum(gcd * dv))
        fd = richardson(dv, eps)
        big = abs(ad) >= 10.0 * floor
        print(f"direction {j}: fd {fd:+.6e} adjoint {ad:+.6e} oracle {ad_or:+.6e}  |fd-ad|/|ad| "
              f"{abs(fd - ad) / abs(ad):.2e}  |ad-or|/|or| {abs(ad - ad_or) / abs(ad_or):.2e}  floor/|ad| "
              f"{floor / abs(ad):.2e}{'' if big else '  (below 10x the floor: reported only)'}")
        if big:
            checked += 1
            assert abs(fd - ad) <= 1e-3 * abs(ad) + floor
    assert checked >= 6
    # along the gradient a plain central difference converges quadratically
    gn = float(torch.sum(gcd * dirs[0]))

    def central(frac):
        e = frac * vnorm
        return (misfit_at(v0 + e * dirs[0]) - misfit_at(v0 - e * dirs[0])) / (2 * e)
    e_big = abs(central(1e-3) - gn)
    e_small = abs(central(1e-4) - gn)
    print(f"along g: error {e_big:.3e} at 1e-3, {e_small:.3e} at 1e-4")
    assert 30.0 < e_big / e_small < 300.0
