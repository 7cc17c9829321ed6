"""wv_zfpk_encode_noalloc: the allocation-free encode (fixed device scratch, no
workspace) gives the same stream as wv_zfpk_encode, call after call."""
import ctypes as C

import numpy as np
import pytest

import oracle
from tests.helpers import has_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not has_gpu(), reason="needs a GPU")]


def _field(shape, seed):
    rng = np.random.default_rng(seed)
    g = np.meshgrid(*(np.linspace(0, 5, s) for s in shape), indexing="ij")
    f = np.sin(sum(g)) * np.exp(-0.05 * sum(x * x for x in g)) + 1e-3 * rng.standard_normal(shape)
    return f.astype(np.float32)


def _encode_both(field, tol):
    import torch
    import paper_1810_05268_amd as P
    f = torch.as_tensor(field, device="cuda")
    dims = list(reversed(field.shape))
    cap = P.zfpk_max_bytes(field.ndim, dims)
    ws = torch.zeros(P.zfpk_workspace_bytes(field.ndim, dims) + 256, dtype=torch.uint8, device="cuda")
    wso = (-ws.data_ptr()) % 256
    ref = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    nref = P.zfpk_encode(f, tol, ref, ws[wso:])
    # the output buffer starts dirty: the stream must not depend on it
    out = torch.full((cap,), 0xA5, dtype=torch.uint8, device="cuda")
    n = P.zfpk_encode_noalloc(f, tol, out)
    torch.cuda.synchronize()
    return ref[:nref].cpu().numpy().tobytes(), out[:n].cpu().numpy().tobytes(), out


def test_noalloc_encode_equals_workspace_encode_twice():
    import torch
    import paper_1810_05268_amd as P
    big = _field((72, 66, 90), 1)        # 2 x 17 x 23 ... blocks: several chunks
    small = _field((9, 13, 7), 2)        # one chunk, ragged blocks
    for field, tol in ((big, 1e-4), (small, 1e-3)):
        ref, got, out = _encode_both(field, tol)
        assert got == ref
        assert got == oracle.encode(field, tol)
        dec = torch.empty(field.shape, dtype=torch.float32, device="cuda")
        P.zfpk_decode(out, dec, nbytes=len(got))
        assert float(np.max(np.abs(dec.cpu().numpy() - field))) <= tol
    # 2-D after 3-D, on the same scratch
    f2 = _field((130, 70), 3)
    ref, got, _ = _encode_both(f2, 1e-5)
    assert got == ref


def test_noalloc_encode_rejects_fields_beyond_its_scratch():
    import torch
    import paper_1810_05268_amd as P
    from paper_1810_05268_amd._binding import WV_ENOMEM
    L = P.lib()
    f = torch.zeros(64, dtype=torch.float32, device="cuda")
    out = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    nb = C.c_size_t(0)
    dims = (C.c_int * 3)(1024, 1024, 1024)     # 16.8 M blocks: rejected before any launch
    rc = L.wv_zfpk_encode_noalloc(f.data_ptr(), 3, dims, C.c_double(1e-3), out.data_ptr(), out.numel(),
                                  C.byref(nb), None)
    assert rc == WV_ENOMEM
    assert b"scratch" in L.wv_last_error()
    assert b"at most 4172288 blocks" in L.wv_last_error()   # the limit wv.h states (640^3 = 4096000 blocks fit)
