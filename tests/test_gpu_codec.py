"""GPU codec: byte-identical streams and bit-identical decodes against the oracle codec."""
import numpy as np
import pytest

import oracle
from tests.helpers import has_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not has_gpu(), reason="needs a GPU")]


def gpu_roundtrip(field: np.ndarray, tol: float):
    import torch
    import paper_1810_05268_amd as P
    f = torch.as_tensor(np.ascontiguousarray(field, dtype=np.float32), device="cuda")
    dims = list(reversed(field.shape))
    cap = P.zfpk_max_bytes(field.ndim, dims)
    out = torch.zeros(cap + 64, dtype=torch.uint8, device="cuda")
    ws = torch.zeros(P.zfpk_workspace_bytes(field.ndim, dims) + 256, dtype=torch.uint8, device="cuda")
    wso = (-ws.data_ptr()) % 256
    nb = P.zfpk_encode(f, tol, out, ws[wso:])
    dec = torch.empty_like(f)
    P.zfpk_decode(out, dec)
    torch.cuda.synchronize()
    return out[:nb].cpu().numpy().tobytes(), dec.cpu().numpy()


def fields():
    rng = np.random.default_rng(0)
    out = []
    for shape in [(16, 16), (9, 13), (130, 70), (555, 17), (8, 8, 8), (7, 6, 5), (13, 3, 22), (40, 41, 42),
                  (33, 97, 65)]:
        g = np.meshgrid(*(np.linspace(0, 4, s) for s in shape), indexing="ij")
        smooth = np.sin(sum(g)) * np.exp(-0.1 * sum(x * x for x in g))
        out.append((f"smooth{shape}", (smooth + 1e-3 * rng.standard_normal(shape)).astype(np.float32)))
    out.append(("noise3d", rng.standard_normal((24, 20, 36)).astype(np.float32)))
    out.append(("mixed3d", (rng.standard_normal((12, 12, 12)) * 2.0 ** rng.integers(-60, 60, (12, 12, 12)))
                .astype(np.float32)))
    sub = (rng.integers(-2 ** 23, 2 ** 23, (8, 12, 16)) * 2.0 ** -149).astype(np.float32)
    out.append(("subnormal3d", sub))
    z = np.zeros((20, 24, 28), np.float32)
    z[5:9, 4:8, 8:12] = 1.0
    out.append(("mostly_zero3d", z))
    return out


@pytest.mark.parametrize("name,field", fields(), ids=[n for n, _ in fields()])
@pytest.mark.parametrize("tol", [1e-1, 1e-3, 1e-5, 1e-7])
def test_stream_byte_identical(name, field, tol):
    ref = oracle.encode(field, tol)
    got, dec = gpu_roundtrip(field, tol)
    assert len(got) == len(ref)
    assert got == ref
    refdec = oracle.decode(ref)
    assert np.array_equal(dec.view(np.uint32), refdec.view(np.uint32))
    floor = float(np.max(np.abs(field))) * 2.0 ** -23
    assert float(np.max(np.abs(dec.astype(np.float64) - field))) <= max(tol, floor)


def test_many_chunks_wavefield_like():
    """Several hundred chunks: every chunk placed at the offset the scan of the chunk word counts gives."""
    rng = np.random.default_rng(3)
    z, y, x = np.meshgrid(np.arange(90), np.arange(100), np.arange(110), indexing="ij")
    r = np.sqrt((x - 55) ** 2 + (y - 50) ** 2 + (z - 10) ** 2)
    f = (np.sin(0.4 * r) * np.exp(-0.02 * r) + 1e-4 * rng.standard_normal(r.shape)).astype(np.float32)
    for tol in (1e-3, 1e-5):
        ref = oracle.encode(f, tol)
        got, dec = gpu_roundtrip(f, tol)
        assert got == ref
        assert np.max(np.abs(dec - f)) <= tol


def test_decode_rejects_mismatched_or_truncated_streams():
    """The decoder checks the stream header against the caller's dims and readable
    bytes on the host and launches nothing on a mismatch; a valid stream decodes
    exactly when nbytes covers it."""
    import torch
    import paper_1810_05268_amd as P
    from paper_1810_05268_amd._binding import WV_EINVAL, WvError
    rng = np.random.default_rng(7)
    field = rng.standard_normal((20, 24, 28)).astype(np.float32)
    ref = oracle.encode(field, 1e-3)
    buf = torch.as_tensor(np.frombuffer(ref, dtype=np.uint8).copy(), device="cuda")
    dec = torch.full(field.shape, 7.0, dtype=torch.float32, device="cuda")
    P.zfpk_decode(buf, dec, nbytes=len(ref))
    assert np.array_equal(dec.cpu().numpy().view(np.uint32), oracle.decode(ref).view(np.uint32))
    cases = []
    # other dims, other ndim, a stream cut one word short, a stream cut inside its prefix
    cases.append((torch.empty((20, 24, 29), dtype=torch.float32, device="cuda"), len(ref)))
    cases.append((torch.empty((20, 24 * 28), dtype=torch.float32, device="cuda"), len(ref)))
    cases.append((torch.empty(field.shape, dtype=torch.float32, device="cuda"), len(ref) - 8))
    cases.append((torch.empty(field.shape, dtype=torch.float32, device="cuda"), 100))
    for out, nb in cases:
        out.fill_(3.0)
        with pytest.raises(WvError) as ei:
            P.zfpk_decode(buf, out, nbytes=nb)
        assert ei.value.code == WV_EINVAL
        torch.cuda.synchronize()
        assert bool(torch.all(out == 3.0))     # nothing was launched
    # a corrupt magic word
    bad = buf.clone()
    bad[0] ^= 1
    out = torch.full(field.shape, 3.0, dtype=torch.float32, device="cuda")
    with pytest.raises(WvError):
        P.zfpk_decode(bad, out, nbytes=len(ref))
    assert bool(torch.all(out == 3.0))
