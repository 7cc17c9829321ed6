"""Serving engine: continuous batching; every result equals the same request alone."""
import numpy as np
import pytest

import workloads as W
from tests.helpers import has_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not has_gpu(), reason="needs a GPU")]


def device_requests(nreq=8, seed=5):
    import torch
    import paper_1810_05268_amd as P
    from paper_1810_05268_amd.shot import DeviceShot
    classes = [(0.5, 2, (120, 100), 8, 300), (0.3, 3, (36, 32, 30), 8, 160), (0.2, 3, (40, 36, 44), 12, 200)]
    reqs = W.serving_stream(nreq=nreq, rate=50.0, seed=seed, classes=classes)
    out = []
    for r in reqs:
        s = r.shot
        dt = s.cfl_frac * P.cfl_dt(s.ndim, s.h, s.order, s.vmax)
        q = W.ricker(s.f0, dt, s.nt).astype(np.float32)
        G = DeviceShot(s.ndim, s.n, s.h, s.nbl, s.order, s.nt, dt, s.vmax, s.padded("true"), q, s.src, s.rec)
        d_obs = G.forward()
        G.set_velocity(s.padded("vel"))
        budget = 8 * G.P * max(4, s.nt // 10)
        tol = 1e-4 if r.rid % 2 else 0.0
        out.append((r.arrival, G, d_obs, budget, tol, 0.0))
    torch.cuda.synchronize()
    return out


def test_alone_equals_mix():
    import torch
    from paper_1810_05268_amd.serving import Engine, replay
    items = device_requests()
    alone = []
    for arrival, G, d_obs, budget, tol, hint in items:
        phi, g, st = G.misfit_gradient(d_obs, budget, tol, hint)
        alone.append((phi, g.clone()))
    eng = Engine(pool_bytes=sum(G.pb.workspace_bytes(1, b) + 4096 for _, G, _, b, _, _ in items), max_active=4)
    res, wall = replay(eng, items, time_scale=1.0)
    eng.close()
    for (phi, g), r in zip(alone, res):
        assert r["status"] == 0
        assert r["misfit"] == phi
        assert torch.equal(r["grad"], g)
        assert r["t_start_ms"] >= r["t_submit_ms"] and r["t_end_ms"] > r["t_start_ms"]


def test_admission_under_a_tight_pool():
    """A pool that holds one workspace at a time still serves every request.  Admission is
    first fit in arrival order: a request that started before an earlier one needed less
    pool memory than it (it fitted where the earlier one did not)."""
    from paper_1810_05268_amd.serving import Engine
    items = device_requests(nreq=6, seed=7)
    ws = [G.pb.workspace_bytes(1, b) for _, G, _, b, _, _ in items]
    eng = Engine(pool_bytes=max(ws) + 4096, max_active=4)
    ids = [eng.submit(G, d, b, t, h) for _, G, d, b, t, h in items]
    res = [eng.wait(i) for i in ids]
    eng.close()
    assert all(r["status"] == 0 for r in res)
    for i in range(len(res)):
        for j in range(i + 1, len(res)):
            if res[j]["t_start_ms"] < res[i]["t_start_ms"]:
                assert ws[j] < ws[i]


def test_batch_lane_alone_equals_mix():
    """Batching on: the 2-D requests of a mixed stream run in batches on the batch lane
    (requests of one batch share their start and end times), the 3-D ones on the solo
    workers, and every result is bit-identical to the same request alone."""
    import torch
    from paper_1810_05268_amd.serving import Engine, replay
    from paper_1810_05268_amd.shot import DeviceShot
    import paper_1810_05268_amd as P
    classes = [(0.7, 2, (120, 100), 8, 300), (0.3, 3, (36, 32, 30), 8, 160)]
    reqs = W.serving_stream(nreq=12, rate=200.0, seed=11, classes=classes)
    vmax = 3700.0
    items = []
    for r in reqs:
        s = r.shot
        dt = s.cfl_frac * P.cfl_dt(s.ndim, s.h, s.order, vmax)     # one time step per class
        q = W.ricker(s.f0, dt, s.nt).astype(np.float32)
        G = DeviceShot(s.ndim, s.n, s.h, s.nbl, s.order, s.nt, dt, vmax, s.padded("true"), q, s.src, s.rec)
        d_obs = G.forward()
        G.set_velocity(s.padded("vel"))
        # one budget and hint per class, so that a class's requests can share a batch
        budget = int(8 * 1.05 * 12 * (s.n[0] + 40) * (s.n[1] + 40) * (s.n[2] + 40 if s.ndim == 3 else 1))
        items.append((r.arrival, G, d_obs, budget, 1e-4, 1.0))
    torch.cuda.synchronize()
    alone = []
    for _, G, d_obs, b, tol, h in items:
        phi, g, _ = G.misfit_gradient(d_obs, b, tol, h)
        alone.append((phi, g.clone()))
        G._ws = None
    torch.cuda.empty_cache()
    pool = 2 * sum(G.pb.workspace_bytes(1, b) + 65536 for _, G, _, b, _, _ in items)
    eng = Engine(pool_bytes=pool, max_active=4, max_batch=8)
    res, wall = replay(eng, items, time_scale=1.0)
    eng.close()
    for (phi, g), r in zip(alone, res):
        assert r["status"] == 0
        assert r["misfit"] == phi
        assert torch.equal(r["grad"], g)
    two_d = [r for r, (_, G, _, _, _, _) in zip(res, items) if len(G.shape) == 2]
    spans = {(r["t_start_ms"], r["t_end_ms"]) for r in two_d}
    print(f"{len(two_d)} 2-D requests in {len(spans)} batches; wall {wall:.2f} s")
    assert len(spans) < len(two_d)                      # some 2-D requests shared a batch


def test_request_larger_than_pool_is_rejected():
    import paper_1810_05268_amd as P
    from paper_1810_05268_amd.serving import Engine
    items = device_requests(nreq=1, seed=9)
    _, G, d, b, t, h = items[0]
    eng = Engine(pool_bytes=1 << 20, max_active=1)
    with pytest.raises(P.WvError):
        eng.submit(G, d, b, t, h)
    eng.close()


def test_many_concurrent_compressed_requests():
    """Twelve compressed requests submitted at once to eight workers: the encoders of
    different shots run concurrently on their own streams; every request completes and
    equals the same request run alone."""
    import torch
    import paper_1810_05268_amd as P
    from paper_1810_05268_amd.serving import Engine, replay
    from paper_1810_05268_amd.shot import DeviceShot
    classes = [(0.5, 3, (72, 64, 60), 8, 150), (0.5, 3, (96, 80, 70), 8, 120)]
    reqs = W.serving_stream(nreq=12, rate=1e6, seed=9, classes=classes)
    items = []
    for r in reqs:
        s = r.shot
        dt = s.cfl_frac * P.cfl_dt(s.ndim, s.h, s.order, s.vmax)
        q = W.ricker(s.f0, dt, s.nt).astype(np.float32)
        G = DeviceShot(s.ndim, s.n, s.h, s.nbl, s.order, s.nt, dt, s.vmax, s.padded("true"), q, s.src, s.rec)
        d_obs = G.forward()
        G.set_velocity(s.padded("vel"))
        items.append((r.arrival, G, d_obs, 8 * G.P * 12, 1e-4, 4.0))
    torch.cuda.synchronize()
    alone = [G.misfit_gradient(d_obs, b, tol, h)[1].clone() for _, G, d_obs, b, tol, h in items]
    for _, G, _, _, _, _ in items:
        G._ws = None
    eng = Engine(pool_bytes=sum(G.pb.workspace_bytes(1, b) + 4096 for _, G, _, b, _, _ in items), max_active=8)
    res, wall = replay(eng, items, time_scale=0.0)
    eng.close()
    for g, r in zip(alone, res):
        assert r["status"] == 0
        assert torch.equal(r["grad"], g)
