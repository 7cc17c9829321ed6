"""Checkpoint planning from a measured compressibility profile (wv_plan).

Compressibility falls as the wavefield spreads, so a single ratio taken from the
final state plans too few slots, and one taken from an early state overflows.
Planning from the profile of stream sizes over time (the sizes a previous call of
the same shot measured) fits the budget without a retry and holds at least as many
slots as the final-state plan."""
import numpy as np
import pytest

from tests.helpers import gpu_side, has_gpu, rel_l2, small_3d

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not has_gpu(), reason="needs a GPU")]


def _trajectory_bytes(prof, nt):
    ks = [0] + [-(-(j * nt) // 16) for j in range(1, 17)]
    sizes = np.interp(np.arange(1, nt + 1), ks, prof)
    return float(np.sum(np.ceil(sizes / 256.0) * 256.0))


@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_profile_plan_fits_without_retry(tol):
    import paper_1810_05268_amd as P
    shot = small_3d(nt=240)
    Gt, _ = gpu_side(shot, "true")
    d_obs = Gt.forward()
    G, _ = gpu_side(shot)
    raw_full = 8 * G.P * (shot.nt + 1)
    _, g_ref, st0 = G.misfit_gradient(d_obs, raw_full, tol)       # every state stored: the whole profile
    prof = st0["profile"]
    assert all(x > 0 for x in prof)
    # the wavefield spreads, so its stream grows from the first stored state to the last
    assert prof[16] > prof[1]
    for frac in (0.1, 0.25, 0.5):
        budget = int(frac * _trajectory_bytes(prof, shot.nt))
        M, h = P.plan(shot.nt, G.P, budget, prof)
        assert 1 < M < shot.nt
        _, g, st = G.misfit_gradient(d_obs, budget, tol, ratio_hint=h)
        print(f"tol {tol:g} budget {frac:.2f} x trajectory: slots {st['slots']} peak {st['peak_bytes']:.0f} "
              f"of {budget} retries {st['retries']}")
        assert st["retries"] == 0
        assert st["slots"] == M
        assert st["peak_bytes"] <= budget
        # same codec tolerance, another schedule: the gradient differs only by codec error
        assert rel_l2(g.cpu().numpy(), g_ref.cpu().numpy()) < 1e-2
        # the plan from the final state's ratio holds no more slots
        final_ratio = 4.0 * G.P / prof[16]
        m_final = P.predict(shot.nt, G.P, budget, True, 1.0, 1.0, ratio=final_ratio)["slots"]
        assert M >= m_final


def test_cold_call_stores_every_state_when_it_fits():
    """Without a hint, a budget that holds every compressed state is used on the first
    attempt: every state is stored, with no plan and no repeat, and the gradient is the
    one a hinted call with the same slots computes."""
    import paper_1810_05268_amd as P
    shot = small_3d(nt=240)
    Gt, _ = gpu_side(shot, "true")
    d_obs = Gt.forward()
    G, _ = gpu_side(shot)
    budget = 8 * G.P * (shot.nt + 1)
    phi, g, st = G.misfit_gradient(d_obs, budget, 1e-4)
    assert st["retries"] == 0 and st["slots"] == shot.nt
    assert st["stores"] == shot.nt - 1 and st["advances"] == shot.nt
    assert st["peak_bytes"] <= budget
    M, h = P.plan(shot.nt, G.P, budget, st["profile"])
    assert M == shot.nt
    phi2, g2, st2 = G.misfit_gradient(d_obs, budget, 1e-4, ratio_hint=h)
    assert st2["slots"] == shot.nt and st2["retries"] == 0
    assert phi2 == phi
    assert np.array_equal(g.cpu().numpy(), g2.cpu().numpy())


def test_no_hint_plans_from_a_probe():
    """Without a hint, a budget too small for every state: the first attempt stops before
    the reversal with the states' stream sizes measured, and the call plans from them the
    slots wv_plan gives for the same profile, with no repeat of the planned run."""
    import paper_1810_05268_amd as P
    shot = small_3d(nt=240)
    Gt, _ = gpu_side(shot, "true")
    d_obs = Gt.forward()
    G, _ = gpu_side(shot)
    _, _, st0 = G.misfit_gradient(d_obs, 8 * G.P * (shot.nt + 1), 1e-4)
    budget = int(0.25 * _trajectory_bytes(st0["profile"], shot.nt))
    phi, g, st = G.misfit_gradient(d_obs, budget, 1e-4)
    assert st["retries"] == 0
    assert st["peak_bytes"] <= budget
    M, h = P.plan(shot.nt, G.P, budget, st0["profile"])
    assert 1 < st["slots"] == M < shot.nt
    # the hinted call with that plan computes the same gradient
    phi2, g2, st2 = G.misfit_gradient(d_obs, budget, 1e-4, ratio_hint=h)
    assert st2["slots"] == M
    assert phi2 == phi
    assert np.array_equal(g.cpu().numpy(), g2.cpu().numpy())
