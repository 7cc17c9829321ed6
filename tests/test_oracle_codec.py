"""Pins of the oracle's ZFP-kind fixed-accuracy codec (Sec. "Lossy Compression": ZFP in
fixed-tolerance mode, i.e. an absolute error bound; block scheme after Lindstrom 2014)."""
import json
import math
import os

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")

A = np.array([[4, 4, 4, 4], [5, 1, -1, -5], [-4, 4, 4, -4], [-2, 6, -6, 2]]) / 16.0
AINV = np.array([[4, 6, -4, -1], [4, 2, 4, 5], [4, -2, 4, -5], [4, -6, -4, 1]]) / 4.0


def bits_of(words, nbits):
    w = np.asarray(words, dtype=np.uint64)
    return [int((int(w[i // 64]) >> (i % 64)) & 1) for i in range(nbits)]


def test_golden_constant_block():
    g = json.load(open(os.path.join(GOLD, "codec_block_2d_const.json")))
    words, nb = oracle.encode_block(np.array(g["values"], np.float32), g["ndim"], g["tol"])
    assert nb == len(g["bits"])
    assert bits_of(words, nb) == g["bits"]
    out = oracle.decode_block(words, 0, g["ndim"], g["tol"])
    assert out.tolist() == g["decoded"]


def test_transform_matrices_are_inverse():
    assert np.allclose(A @ AINV, np.eye(4), atol=1e-15)


def test_lifting_is_the_matrix_when_exact():
    """On inputs that are multiples of 16 every shift is exact, so the integer lifting
    equals A x and its inverse returns x exactly."""
    rng = np.random.default_rng(0)
    for _ in range(2000):
        x = rng.integers(-2 ** 25, 2 ** 25, size=4) * 16
        y = oracle.fwd_lift4(x)
        assert np.array_equal(y, (A @ x).astype(np.int64))
        assert np.array_equal(oracle.inv_lift4(y), x)


def test_negabinary_definition():
    rng = np.random.default_rng(1)
    vals = [0, 1, -1, 2, -2, 3, -3, 2 ** 29, -2 ** 29 + 5] + rng.integers(-2 ** 30, 2 ** 30, 500).tolist()
    for x in vals:
        u = oracle.negabinary(x)
        assert sum(((u >> i) & 1) * (-2) ** i for i in range(32)) == x
    assert [oracle.negabinary(v) for v in (0, 1, -1, 2, -2, -3)] == [0, 1, 3, 6, 2, 13]


@pytest.mark.parametrize("ndim", [2, 3])
def test_sequency_order(ndim):
    perm = oracle.sequency_perm(ndim)
    S = 64 if ndim == 3 else 16
    assert sorted(perm.tolist()) == list(range(S))
    key = [((v & 3) + ((v >> 2) & 3) + ((v >> 4) & 3)) for v in perm]
    assert key == sorted(key) and perm[0] == 0


def test_sequency_order_all_three_keys_2d():
    """The whole 2-D order, worked out by hand (v = i + 4 j): total degree i + j first,
    then i^2 + j^2 ((1,1) before (2,0) and (0,2)), then the slower index j, then i."""
    expect = [0, 1, 4, 5, 2, 8, 6, 9, 3, 12, 10, 7, 13, 11, 14, 15]
    assert oracle.sequency_perm(2).tolist() == expect


def test_sequency_order_all_three_keys_3d():
    """The 3-D order at its head and tail, worked out by hand (v = i + 4 j + 16 k).
    Degree 1: (1,0,0), (0,1,0), (0,0,1).  Degree 2: squares 2 before 4, and within each
    the slowest index k, then j: (1,1,0), (1,0,1), (0,1,1), (2,0,0), (0,2,0), (0,0,2).
    Degree 3: (1,1,1) (square 3) first; then the six of square 5 by (k, j):
    (2,1,0), (1,2,0), (2,0,1), (0,2,1), (1,0,2), (0,1,2); then (3,0,0), (0,3,0), (0,0,3).
    Degree 8 (all of square 22): (3,3,2), (3,2,3), (2,3,3); then (3,3,3)."""
    perm = oracle.sequency_perm(3).tolist()
    assert perm[:20] == [0, 1, 4, 16, 5, 17, 20, 2, 8, 32, 21, 6, 9, 18, 24, 33, 36, 3, 12, 48]
    assert perm[-4:] == [47, 59, 62, 63]


# ---------------------------------------------------------------- error bound on blocks

def family_block(kind, rng, S):
    if kind == "uniform":
        return rng.uniform(-1, 1, S)
    if kind == "gauss":
        return rng.standard_normal(S) * 10.0 ** rng.integers(-6, 4)
    if kind == "smooth":
        i, j, k = np.arange(S) & 3, (np.arange(S) >> 2) & 3, (np.arange(S) >> 4) & 3
        c = rng.standard_normal(6)
        return c[0] + c[1] * i + c[2] * j + c[3] * k + c[4] * i * j + c[5] * k * k
    if kind == "spike":
        v = np.zeros(S)
        v[rng.integers(S)] = rng.choice([-1, 1]) * 10.0 ** rng.uniform(-5, 5)
        return v
    if kind == "mixed":
        return rng.standard_normal(S) * 2.0 ** rng.integers(-100, 100, S)
    if kind == "subnormal":
        return rng.integers(-2 ** 23, 2 ** 23, S) * 2.0 ** -149
    if kind == "equal":
        return np.full(S, rng.standard_normal() * 10.0 ** rng.integers(-3, 3))
    if kind == "zeros":
        return np.zeros(S)
    if kind == "alternate":
        return (-1.0) ** np.arange(S) * rng.uniform(0.5, 1, S) * 10.0 ** rng.integers(-3, 3)
    raise ValueError(kind)


FAMILIES = ["uniform", "gauss", "smooth", "spike", "mixed", "subnormal", "equal", "zeros", "alternate"]


@settings(max_examples=400, deadline=None, derandomize=True, suppress_health_check=list(HealthCheck))
@given(kind=st.sampled_from(FAMILIES), ndim=st.sampled_from([2, 3]), seed=st.integers(0, 2 ** 31),
       logtol=st.floats(-9, 2))
def test_block_error_bound(kind, ndim, seed, logtol):
    rng = np.random.default_rng(seed)
    S = 64 if ndim == 3 else 16
    v = family_block(kind, rng, S).astype(np.float32)
    tol = 10.0 ** logtol
    words, nb = oracle.encode_block(v, ndim, tol)
    out = oracle.decode_block(words, 0, ndim, tol)
    err = np.max(np.abs(out.astype(np.float64) - v.astype(np.float64)))
    # the bound holds unless tol is below what binary32 can resolve at this magnitude
    floor = np.max(np.abs(v.astype(np.float64))) * 2.0 ** -23
    assert err <= max(tol, floor)


def test_wavefield_like_blocks_error_bound():
    rng = np.random.default_rng(3)
    x = np.linspace(0, 1, 4)
    for _ in range(300):
        f, ph = rng.uniform(1, 30, 3), rng.uniform(0, 6.3, 3)
        amp = 10.0 ** rng.uniform(-4, 1)
        z, y, xx = np.meshgrid(x, x, x, indexing="ij")
        v = (amp * np.sin(f[0] * xx + ph[0]) * np.cos(f[1] * y + ph[1]) * np.sin(f[2] * z + ph[2])).astype(np.float32)
        for tol in (1e-3, 1e-4, 1e-6):
            words, nb = oracle.encode_block(v.ravel(), 3, tol)
            out = oracle.decode_block(words, 0, 3, tol)
            assert np.max(np.abs(out - v.ravel())) <= tol


def test_huge_tolerance_costs_one_bit():
    rng = np.random.default_rng(4)
    for ndim in (2, 3):
        S = 64 if ndim == 3 else 16
        v = rng.standard_normal(S).astype(np.float32)
        tol = 1024.0 * float(np.max(np.abs(v)))
        words, nb = oracle.encode_block(v, ndim, tol)
        assert nb == 1
        assert np.all(oracle.decode_block(words, 0, ndim, tol) == 0)


def test_tiny_tolerance_is_near_lossless():
    """With all 32 planes coded only the transform's dropped low bits and the final
    rounding to binary32 remain: |x - x~| <= 2^(emax-26) + ulp/2."""
    rng = np.random.default_rng(5)
    for _ in range(500):
        v = (rng.standard_normal(64) * 10.0 ** rng.integers(-8, 8)).astype(np.float32)
        words, nb = oracle.encode_block(v, 3, 1e-38)
        out = oracle.decode_block(words, 0, 3, 1e-38)
        emax = max(math.frexp(float(abs(t)))[1] for t in v)
        bound = 2.0 ** (emax - 26) + 2.0 ** (emax - 25)
        assert np.max(np.abs(out.astype(np.float64) - v.astype(np.float64))) <= bound


def test_embedded_prefix_property():
    """Fixed-accuracy coding is embedded: a looser tolerance codes a prefix of the bits of a
    tighter one (same header), so sizes are monotone in the tolerance."""
    rng = np.random.default_rng(6)
    for _ in range(200):
        v = (rng.standard_normal(64) * 10.0 ** rng.integers(-3, 3)).astype(np.float32)
        prev = None
        for tol in (1e-7, 1e-5, 1e-3, 1e-1, 10.0):
            words, nb = oracle.encode_block(v, 3, tol)
            b = bits_of(words, nb)
            if prev is not None and nb > 1:
                assert nb <= len(prev)
                assert b == prev[:nb]
            prev = b


# ---------------------------------------------------------------- whole fields

@pytest.mark.parametrize("shape", [(9, 13), (16, 16), (1, 5), (7, 6, 5), (8, 12, 16), (13, 3, 22)])
def test_field_roundtrip_ragged(shape):
    rng = np.random.default_rng(sum(shape))
    grids = np.meshgrid(*(np.linspace(0, 3, s) for s in shape), indexing="ij")
    f = (np.sin(sum(grids)) + 0.01 * rng.standard_normal(shape)).astype(np.float32)
    sizes = []
    for tol in (1e-6, 1e-4, 1e-2):
        s = oracle.encode(f, tol)
        out = oracle.decode(s)
        assert out.shape == f.shape
        assert np.max(np.abs(out - f)) <= tol
        sizes.append(len(s))
    assert sizes[0] >= sizes[1] >= sizes[2]


def test_field_stream_layout():
    f = np.random.default_rng(9).standard_normal((6, 10, 11)).astype(np.float32)
    s = oracle.encode(f, 1e-3)
    hdr = np.frombuffer(s[:64], dtype=np.uint32)
    assert hdr[0] == 0x4B50465A and hdr[1] == 1 and hdr[2] == 3
    assert hdr[3:6].tolist() == [11, 10, 6]
    nblocks = 3 * 3 * 2
    assert hdr[8] == nblocks and hdr[9] == 1 and hdr[10] == 256
    total = int(np.frombuffer(s[56:64], dtype=np.uint64)[0])
    assert total == len(s)
    # per-block lengths sum to the data bits, padded to a 64-bit word per chunk
    lens = np.frombuffer(s[64 + 8: 64 + 8 + 2 * nblocks], dtype=np.uint16)
    dw = int(np.frombuffer(s[48:56], dtype=np.uint64)[0])
    assert dw == (int(lens.sum()) + 63) // 64


def test_non_finite_rejected():
    f = np.ones((8, 8), np.float32)
    f[3, 3] = np.nan
    with pytest.raises(ValueError):
        oracle.encode(f, 1e-3)


def test_early_wavefields_compress_better():
    """Sec. "Results": compressibility falls as the wave fills the domain."""
    from tests.test_oracle_adjoint import tiny_problem
    spec, vel, _, src, rec, q = tiny_problem(n=(61, 61), nt=240, nbl=10)
    S = oracle.Solver(spec, vel, src, q, rec)
    fw = S.forward(want_traj=True)
    sizes = [len(oracle.encode(fw["traj"][k].astype(np.float32), 1e-6)) for k in (40, 120, 240)]
    assert sizes[0] < sizes[1] < sizes[2]
