"""Batched 2-D shots (wv_batch_misfit_gradient): one persistent launch runs the whole
checkpointed reversal of several shots.  Each shot's misfit, data and gradient must be
bit-identical to a solo wv_misfit_gradient of that shot with the same slot count, and to
the same shot in a batch of one; an uncompressed gradient is also checked against the
FP64 oracle."""
import numpy as np
import pytest

import workloads as W
from tests.helpers import has_gpu, oracle_side, rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not has_gpu(), reason="needs a GPU")]


def _shots(n, nt, order, count, seed):
    """count 2-D shots sharing grid, order, nt, dt and vmax (3.5 km/s, as the serving
    stream's classes) with their own layered velocity, peak frequency and source position."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        sh = W.random_layers(n, (10.0, 10.0), 20, order, nt, rng, float(rng.uniform(10.0, 20.0)))
        sh.src = sh.src.copy()
        sh.src[0, 0] += 10.0 * i                  # the source moves along the surface
        out.append(sh)
    return out


def _device(shots, vmax=3700.0):
    import torch
    import paper_1810_05268_amd as P
    from paper_1810_05268_amd.shot import DeviceShot
    s0 = shots[0]
    dt = s0.cfl_frac * P.cfl_dt(2, s0.h, s0.order, vmax)
    devs, dobs = [], []
    for sh in shots:
        q = W.ricker(sh.f0, dt, sh.nt).astype(np.float32)
        Gt = DeviceShot(2, sh.n, sh.h, sh.nbl, sh.order, sh.nt, dt, vmax, sh.padded("true"), q, sh.src, sh.rec)
        dobs.append(Gt.forward())
        del Gt
        devs.append(DeviceShot(2, sh.n, sh.h, sh.nbl, sh.order, sh.nt, dt, vmax, sh.padded("vel"), q, sh.src,
                               sh.rec))
    torch.cuda.synchronize()
    return devs, dobs, dt


def _batch(devs, dobs, budget, tol, hint):
    import torch
    import paper_1810_05268_amd as P
    pbs = [d.pb for d in devs]
    nb = P.batch_workspace_bytes(pbs, budget)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    grads = [torch.empty(d.shape, dtype=torch.float64, device="cuda") for d in devs]
    dsims = [d.new_data() for d in devs]
    phis, sts = P.batch_misfit_gradient(pbs, dobs, budget, tol, grads, ws[off: off + nb], ratio_hint=hint,
                                        d_sims=dsims)
    return phis, grads, dsims, sts


@pytest.mark.parametrize("n,nt,order", [((97, 90), 160, 8), ((300, 120), 120, 4)], ids=["ragged", "two_tiles"])
@pytest.mark.parametrize("mode", ["plain", "compressed_recompute", "compressed_all"])
def test_batch_bit_identical_to_solo_and_alone(n, nt, order, mode):
    import torch
    shots = _shots(n, nt, order, 4, seed=70 + len(mode))
    devs, dobs, _ = _device(shots)
    S = devs[0].slot_bytes
    if mode == "plain":
        budget, tol, hint = 7 * S, 0.0, 0.0
    elif mode == "compressed_recompute":
        # a ratio hint that plans 9 slots: recomputation and second-level decodes happen
        budget, tol, hint = int(8 * 1.05 * S), 1e-4, 1.0
    else:
        budget, tol, hint = nt * S, 1e-5, 1.0             # every state stored compressed
    phis, grads, dsims, sts = _batch(devs, dobs, budget, tol, hint)
    for i, d in enumerate(devs):
        phi, g, st, ds = d.misfit_gradient(dobs[i], budget, tol, ratio_hint=hint, want_dsim=True)
        print(f"{mode} shot {i}: phi {phi:.6e} slots {st['slots']} advances {st['advances']} "
              f"decodes {st['decodes']} ratio {st['ratio']:.1f}")
        assert sts[i]["slots"] == st["slots"] and sts[i]["advances"] == st["advances"]
        assert sts[i]["stores"] == st["stores"] and sts[i]["decodes"] == st["decodes"]
        assert sts[i]["bytes_stored"] == st["bytes_stored"] and sts[i]["peak_bytes"] == st["peak_bytes"]
        assert phis[i] == phi
        assert torch.equal(dsims[i], ds)
        assert torch.equal(grads[i], g)
    if mode == "compressed_recompute":
        assert sts[0]["slots"] == 9 and sts[0]["advances"] > nt and sts[0]["decodes"] > 0
    # the same shot alone, as a batch of one, and in another order
    phis1, grads1, _, _ = _batch([devs[2]], [dobs[2]], budget, tol, hint)
    assert phis1[0] == phis[2] and torch.equal(grads1[0], grads[2])
    order_ = [3, 0, 2, 1]
    phis2, grads2, _, _ = _batch([devs[i] for i in order_], [dobs[i] for i in order_], budget, tol, hint)
    for k, i in enumerate(order_):
        assert phis2[k] == phis[i] and torch.equal(grads2[k], grads[i])


def test_batch_gradient_against_oracle():
    """An uncompressed batched gradient against the FP64 oracle's (residual from each
    side's own forward run, small enough a grid that the residual is well conditioned)."""
    import torch
    import oracle
    shots = _shots((61, 57), 500, 4, 2, seed=80)
    for sh in shots:                               # an anomaly the wave reaches in 500 steps
        sh.vel_true = (sh.vel + W.gaussian_anomaly(sh.n, sh.h, 200.0, 80.0, [300.0, 150.0])).astype(np.float32)
    vmax = 3700.0
    devs, _, dt = _device(shots, vmax)
    refs, dobs = [], []
    for sh in shots:
        dto = sh.cfl_frac * oracle.cfl_dt(2, sh.h, sh.order, vmax)
        assert dto == dt
        spec = oracle.ModelSpec(2, sh.n, sh.h, sh.nbl, sh.order, sh.nt, dto, vmax)
        q = W.ricker(sh.f0, dto, sh.nt)
        St = oracle.Solver(spec, sh.padded("true").astype(np.float64), sh.src, q, sh.rec)
        d_obs = St.forward()["data"].astype(np.float32)
        S = oracle.Solver(spec, sh.padded("vel").astype(np.float64), sh.src, q, sh.rec)
        fw = S.forward(want_traj=True)
        res = fw["data"] - d_obs.astype(np.float64)
        refs.append((0.5 * float(np.sum(res ** 2)), S.gradient_full(fw["traj"], res)))
        dobs.append(torch.as_tensor(d_obs, device="cuda"))
    phis, grads, _, sts = _batch(devs, dobs, 10 * devs[0].slot_bytes, 0.0, 0.0)
    for i, (phi_or, g_or) in enumerate(refs):
        e = rel_l2(grads[i].cpu().numpy(), g_or)
        print(f"shot {i}: misfit rel err {abs(phis[i] - phi_or) / phi_or:.2e} gradient rel-L2 {e:.2e}")
        assert abs(phis[i] - phi_or) <= 1e-4 * phi_or and e <= 1e-4


def test_batch_launch_that_ends_early_falls_back_to_solo(monkeypatch):
    """A barrier that cannot complete ends the launch and every shot runs alone.  The
    condition is forced from the host: a poll bound of 0 makes the first workgroup that
    has to wait at the first barrier give up (a wide batch is first relaunched with half
    the workgroups).  Results stay bit-identical to solo calls, and each shot's stats
    count the aborted launches."""
    import torch
    shots = _shots((97, 90), 160, 8, 3, seed=91)
    devs, dobs, _ = _device(shots)
    S = devs[0].slot_bytes
    budget, tol, hint = int(8 * 1.05 * S), 1e-4, 1.0
    monkeypatch.setenv("WV_BATCH_SPIN_LIMIT", "0")
    phis, grads, dsims, sts = _batch(devs, dobs, budget, tol, hint)
    monkeypatch.delenv("WV_BATCH_SPIN_LIMIT")
    for i, d in enumerate(devs):
        phi, g, st, ds = d.misfit_gradient(dobs[i], budget, tol, ratio_hint=hint, want_dsim=True)
        assert sts[i]["retries"] >= st["retries"] + 1
        assert phis[i] == phi
        assert torch.equal(grads[i], g) and torch.equal(dsims[i], ds)
    # and the next batch, with the default bound, runs in one launch again
    phis2, grads2, _, sts2 = _batch(devs, dobs, budget, tol, hint)
    assert all(st["retries"] == 0 for st in sts2)
    assert phis2 == phis and all(torch.equal(a, b) for a, b in zip(grads2, grads))
