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


def test_central_finite_differences_smooth_random():
    """The 2-D smooth random medium (400^2 at 5 m, 2000 steps, order 8) with checkpoints
    compressed at 1e-5, checked against central differences of the misfit itself.
    Directions: the normalised gradient and 10 seeded smooth unit directions (white
    noise filtered by a Gaussian of 10 cells).  The truncation error of a central
    difference is O(eps^2) (it is what separates the two at eps = 1e-3 ||v||), so
    eps = 3e-5 ||v||, where binary32 rounding of the misfit is the floor (about
    1e-5 of phi, i.e. 1.5e-4 of ||g|| in the quotient); errors are measured against
    ||g||, the largest directional derivative, since a random direction may be
    nearly orthogonal to g.  Along g the error must also fall quadratically from
    eps = 1e-3 ||v|| to 1e-4 ||v||."""
    from scipy.ndimage import gaussian_filter
    import torch
    import paper_1810_05268_amd.autograd as A
    shot = W.smooth_random_2d()
    pb, vel, _ = make_problem(shot, 1e-5, 20, headroom=1.02)
    phi = A.wave_misfit(vel, pb)
    phi.backward()
    g = vel.grad.double()
    assert pb.last_stats["slots"] > 20          # compression bought more slots than 20 plain ones
    gnorm = float(torch.linalg.vector_norm(g))
    vnorm = float(torch.linalg.vector_norm(vel.detach().double()))

    def central(dv, frac):
        eps = frac * vnorm
        with torch.no_grad():
            fp = float(A.wave_misfit((vel.detach().double() + eps * dv).float(), pb))
            fm = float(A.wave_misfit((vel.detach().double() - eps * dv).float(), pb))
        return (fp - fm) / (2 * eps)

    dirs = [g / gnorm]
    for seed in range(30, 40):
        noise = np.random.default_rng(seed).standard_normal(tuple(vel.shape))
        dv = torch.as_tensor(gaussian_filter(noise, sigma=10.0, mode="reflect"), device="cuda")
        dirs.append(dv / torch.linalg.vector_norm(dv))
    errs = []
    for j, dv in enumerate(dirs):
        ad = float(torch.sum(g * dv))
        fd = central(dv, 3e-5)
        errs.append(abs(fd - ad) / gnorm)
        print(f"direction {j}: fd {fd:.6e} adjoint {ad:.6e} |fd-ad|/|g| {errs[-1]:.2e}")
    assert errs[0] < 5e-4
    assert max(errs) < 1e-3
    e_big = abs(central(dirs[0], 1e-3) - gnorm)
    e_small = abs(central(dirs[0], 1e-4) - gnorm)
    print(f"along g: error {e_big:.3e} at 1e-3, {e_small:.3e} at 1e-4")
    assert 30.0 < e_big / e_small < 300.0
