"""Failure paths on the GPU, each forced from the host with an input the library must
refuse or detect, none of which can fault the device: a velocity outside (0, vmax] or
not finite (checked by the set-up kernel: WV_EINVAL), a non-finite value given to the
encoder (WV_EINVAL), and a wavefield that overflows binary32 (a source of amplitude
3e38: WV_EUNSTABLE, from the forward call, the gradient call and a batch)."""
import numpy as np
import pytest

import workloads as W
from tests.helpers import has_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not has_gpu(), reason="needs a GPU")]


def _shot(vel_edit=None, amp=1.0, nt=120):
    import paper_1810_05268_amd as P
    from paper_1810_05268_amd.shot import DeviceShot
    sh = W.random_layers((61, 57), (10.0, 10.0), 20, 4, nt, np.random.default_rng(4), 15.0)
    vmax = 3700.0
    dt = sh.cfl_frac * P.cfl_dt(2, sh.h, sh.order, vmax)
    q = (amp * W.ricker(sh.f0, dt, sh.nt)).astype(np.float32)
    vel = sh.padded("vel").copy()
    if vel_edit is not None:
        vel_edit(vel)
    return DeviceShot(2, sh.n, sh.h, sh.nbl, sh.order, sh.nt, dt, vmax, vel, q, sh.src, sh.rec)


@pytest.mark.parametrize("bad", [np.nan, np.inf, -1500.0, 0.0, 3800.0], ids=["nan", "inf", "negative", "zero",
                                                                             "above_vmax"])
def test_velocity_outside_its_range_is_refused(bad):
    import paper_1810_05268_amd as P
    import paper_1810_05268_amd._binding as B

    def edit(v):
        v[40, 30] = bad
    G = _shot(edit)
    with pytest.raises(P.WvError) as ex:
        G.forward()
    assert ex.value.code == B.WV_EINVAL
    d_obs = G.new_data()
    with pytest.raises(P.WvError) as ex:
        G.misfit_gradient(d_obs, 8 * G.slot_bytes)
    assert ex.value.code == B.WV_EINVAL


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf], ids=["nan", "inf", "-inf"])
def test_encoder_refuses_non_finite_values(bad):
    import torch
    import paper_1810_05268_amd as P
    import paper_1810_05268_amd._binding as B
    f = torch.zeros((37, 41, 29), dtype=torch.float32, device="cuda")
    f[20, 7, 3] = float(bad)
    dims = list(reversed(f.shape))
    out = torch.zeros(P.zfpk_max_bytes(3, dims), dtype=torch.uint8, device="cuda")
    wsb = P.zfpk_workspace_bytes(3, dims)
    ws = torch.zeros(wsb + 256, dtype=torch.uint8, device="cuda")
    wso = (-ws.data_ptr()) % 256
    with pytest.raises(P.WvError) as ex:
        P.zfpk_encode(f, 1e-3, out, ws[wso: wso + wsb])
    assert ex.value.code == B.WV_EINVAL
    with pytest.raises(P.WvError) as ex:
        P.zfpk_encode_noalloc(f, 1e-3, out)
    assert ex.value.code == B.WV_EINVAL
    f[20, 7, 3] = 0.0                     # the same call on the clean field succeeds
    assert P.zfpk_encode(f, 1e-3, out, ws[wso: wso + wsb]) > 0


def test_binary32_overflow_is_reported_unstable():
    import torch
    import paper_1810_05268_amd as P
    import paper_1810_05268_amd._binding as B
    G = _shot(amp=3e38)                   # the first injections already overflow binary32
    with pytest.raises(P.WvError) as ex:
        G.forward()
    assert ex.value.code == B.WV_EUNSTABLE
    d_obs = torch.zeros((G.nt + 1, G.nrec), dtype=torch.float32, device="cuda")
    for tol in (0.0, 1e-4):
        with pytest.raises(P.WvError) as ex:
            G.misfit_gradient(d_obs, 8 * G.slot_bytes, tol, ratio_hint=1.0 if tol else 0.0)
        assert ex.value.code == B.WV_EUNSTABLE
    # in a batch, beside a well-behaved shot
    H = _shot()
    ws_b = P.batch_workspace_bytes([G.pb, H.pb], 8 * G.slot_bytes)
    ws = torch.empty(ws_b + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    grads = [torch.empty(s.shape, dtype=torch.float64, device="cuda") for s in (G, H)]
    with pytest.raises(P.WvError) as ex:
        P.batch_misfit_gradient([G.pb, H.pb], [d_obs, d_obs], 8 * G.slot_bytes, 0.0, grads,
                                ws[off: off + ws_b])
    assert ex.value.code == B.WV_EUNSTABLE
