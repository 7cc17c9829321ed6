"""Oracle: plain FP64 CPU reference of the checkpointed adjoint solver and codec.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no
code with the GPU library (``paper_1810_05268_amd``) and never imports it.

The numerical core is ``wv_oracle.c`` (binary64, OpenMP over the slowest
axis); ``schedule.py`` holds the Revolve schedule oracle.  This module
compiles the C file with gcc on first use and wraps it with ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from . import schedule  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (always when force=True)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Model(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double * 3), ("nbl", C.c_int),
                ("order", C.c_int), ("nt", C.c_int), ("dt", C.c_double), ("vmax", C.c_double),
                ("time_order", C.c_int)]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        vp, dp, ip, lp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_long)
        L.or_fd_coeffs.argtypes = [C.c_int, dp]
        L.or_cfl_dt.argtypes = [C.c_int, dp, C.c_int, C.c_double]
        L.or_cfl_dt.restype = C.c_double
        L.or_cfl_dt_to.argtypes = [C.c_int, dp, C.c_int, C.c_double, C.c_int]
        L.or_cfl_dt_to.restype = C.c_double
        L.or_create.argtypes = [C.POINTER(_Model), dp, C.c_int, dp, dp, C.c_int, dp, C.c_int, ip]
        L.or_create.restype = vp
        L.or_destroy.argtypes = [vp]
        L.or_npoints.argtypes = [vp]
        L.or_npoints.restype = C.c_long
        L.or_get_w.argtypes = [vp, dp]
        L.or_get_damp.argtypes = [vp, dp]
        L.or_get_interp.argtypes = [vp, C.c_int, lp, dp]
        L.or_laplacian.argtypes = [vp, dp, dp]
        L.or_forward_step.argtypes = [vp, C.c_int, dp, dp, dp, dp]
        L.or_forward.argtypes = [vp, dp, dp, dp]
        L.or_forward.restype = C.c_int
        L.or_misfit.argtypes = [C.c_long, dp, dp]
        L.or_misfit.restype = C.c_double
        L.or_adjoint_step.argtypes = [vp, dp, dp, dp, dp, dp]
        L.or_gradient_full.argtypes = [vp, dp, dp, dp, dp]
        L.or_gradient_full.restype = C.c_int
        L.or_gradient_nform.argtypes = [vp, dp, dp, dp]
        L.or_gradient_bound.argtypes = [vp, dp, dp]
        L.or_gradient_bound.restype = C.c_int
        L.or_adjoint_src.argtypes = [vp, dp, dp]
        L.or_adjoint_src.restype = C.c_int
        L.or_gradient_actions.argtypes = [vp, dp, C.POINTER(C.c_int32), C.c_long, C.c_int, C.c_double, C.c_int,
                                          dp, lp]
        L.or_gradient_actions.restype = C.c_int
        L.or_zk_encode_block_buf.argtypes = [C.POINTER(C.c_float), C.c_int, C.c_double, C.POINTER(C.c_uint64),
                                             C.c_long]
        L.or_zk_encode_block_buf.restype = C.c_long
        L.or_zk_decode_block_buf.argtypes = [C.POINTER(C.c_uint64), C.c_long, C.c_long, C.c_int, C.c_double,
                                             C.POINTER(C.c_float)]
        L.or_zk_decode_block_buf.restype = C.c_int
        L.or_zk_prefix_bytes.argtypes = [C.c_int, ip]
        L.or_zk_prefix_bytes.restype = C.c_long
        L.or_zk_encode.argtypes = [C.POINTER(C.c_float), C.c_int, ip, C.c_double, C.POINTER(C.c_uint8), C.c_long,
                                   lp]
        L.or_zk_encode.restype = C.c_int
        L.or_zk_decode.argtypes = [C.POINTER(C.c_uint8), C.c_long, C.POINTER(C.c_float)]
        L.or_zk_decode.restype = C.c_int
        L.or_zk_fwd_lift4.argtypes = [C.POINTER(C.c_int32)]
        L.or_zk_inv_lift4.argtypes = [C.POINTER(C.c_int32)]
        L.or_zk_perm.argtypes = [C.c_int, C.POINTER(C.c_int)]
        L.or_zk_negabinary.argtypes = [C.c_int32]
        L.or_zk_negabinary.restype = C.c_uint32
        _lib = L
    return _lib


def default_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


# ---------------------------------------------------------------- discretisation

def fd_coeffs(K: int) -> np.ndarray:
    a = np.zeros(K + 1)
    lib().or_fd_coeffs(K, _dp(a))
    return a


def cfl_dt(ndim: int, h, order: int, vmax: float, time_order: int = 2) -> float:
    """Stability limit of the leapfrog (OT2) or modified-equation (OT4) scheme."""
    hh = np.zeros(3)
    hh[:ndim] = h[:ndim]
    if time_order == 2:
        return lib().or_cfl_dt(ndim, _dp(hh), order, vmax)
    return lib().or_cfl_dt_to(ndim, _dp(hh), order, vmax, time_order)


@dataclass
class ModelSpec:
    ndim: int
    n: tuple            # interior points, axis 0 fastest (x), last axis = depth
    h: tuple
    nbl: int
    order: int
    nt: int
    dt: float
    vmax: float
    time_order: int = 2     # 2: OT2 leapfrog; 4: OT4 modified-equation scheme

    def padded(self) -> tuple:
        return tuple(self.n[d] + 2 * self.nbl for d in range(self.ndim))

    def array_shape(self) -> tuple:
        """C-order array shape (depth slowest): [z][y][x] or [z][x]."""
        return tuple(reversed(self.padded()))


class Solver:
    """FP64 forward / adjoint / gradient on one shot."""

    def __init__(self, spec: ModelSpec, vel: np.ndarray, src: np.ndarray, wavelet: np.ndarray,
                 rec: np.ndarray, nthreads: int | None = None):
        self.spec = spec
        m = _Model()
        m.ndim = spec.ndim
        for d in range(3):
            m.n[d] = spec.n[d] if d < spec.ndim else 1
            m.h[d] = spec.h[d] if d < spec.ndim else 1.0
        m.nbl, m.order, m.nt, m.dt, m.vmax = spec.nbl, spec.order, spec.nt, spec.dt, spec.vmax
        m.time_order = spec.time_order
        self._m = m
        self.vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1)
        self.src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, spec.ndim)
        self.rec = np.ascontiguousarray(rec, dtype=np.float64).reshape(-1, spec.ndim)
        self.wavelet = np.ascontiguousarray(wavelet, dtype=np.float64)
        assert self.wavelet.size >= spec.nt
        st = C.c_int(0)
        self._h = lib().or_create(C.byref(m), _dp(self.vel), len(self.src), _dp(self.src), _dp(self.wavelet),
                                  len(self.rec), _dp(self.rec), nthreads or default_threads(), C.byref(st))
        if not self._h:
            raise ValueError(f"oracle rejected the model (status {st.value})")
        self.P = lib().or_npoints(self._h)
        self.shape = spec.array_shape()
        self.nrec = len(self.rec)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_destroy(h)
            self._h = None

    def w(self):
        out = np.zeros(self.P)
        lib().or_get_w(self._h, _dp(out))
        return out.reshape(self.shape)

    def damp(self):
        out = np.zeros(self.P)
        lib().or_get_damp(self._h, _dp(out))
        return out.reshape(self.shape)

    def interp(self, which: int):
        nc = 8 if self.spec.ndim == 3 else 4
        n = self.nrec if which else len(self.src)
        idx = np.zeros(n * nc, dtype=np.int64)
        wt = np.zeros(n * nc)
        lib().or_get_interp(self._h, which, idx.ctypes.data_as(C.POINTER(C.c_long)), _dp(wt))
        return idx.reshape(n, nc), wt.reshape(n, nc)

    def laplacian(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros(self.P)
        lib().or_laplacian(self._h, _dp(u), _dp(out))
        return out.reshape(self.shape)

    def forward_step(self, n, cur, prev):
        cur = np.ascontiguousarray(cur, dtype=np.float64)
        prev = np.ascontiguousarray(prev, dtype=np.float64)
        nxt = np.zeros(self.P)
        lap = np.zeros(self.P)
        lib().or_forward_step(self._h, n, _dp(cur), _dp(prev), _dp(nxt), _dp(lap))
        return nxt.reshape(self.shape)

    def adjoint_step(self, res_k, lam_k, lam_kp1):
        res_k = np.ascontiguousarray(res_k, dtype=np.float64)
        lam_k = np.ascontiguousarray(lam_k, dtype=np.float64)
        lam_kp1 = np.ascontiguousarray(lam_kp1, dtype=np.float64)
        out = np.zeros(self.P)
        lap = np.zeros(self.P)
        lib().or_adjoint_step(self._h, _dp(res_k), _dp(lam_k), _dp(lam_kp1), _dp(out), _dp(lap))
        return out.reshape(self.shape)

    def forward(self, want_traj: bool = False, want_last: bool = False):
        nt = self.spec.nt
        data = np.zeros((nt + 1, self.nrec))
        traj = np.zeros((nt + 1,) + self.shape) if want_traj else None
        last = np.zeros((2,) + self.shape) if want_last else None
        rc = lib().or_forward(self._h, _dp(data), _dp(traj) if traj is not None else None,
                              _dp(last) if last is not None else None)
        if rc:
            raise RuntimeError(f"or_forward failed: {rc}")
        out = {"data": data}
        if want_traj:
            out["traj"] = traj
        if want_last:
            out["last"] = last
        return out

    def gradient_full(self, traj, residual, want_lam: bool = False):
        residual = np.ascontiguousarray(residual, dtype=np.float64)
        traj = np.ascontiguousarray(traj, dtype=np.float64)
        g = np.zeros(self.P)
        lam = np.zeros((self.spec.nt,) + self.shape) if want_lam else None
        rc = lib().or_gradient_full(self._h, _dp(traj), _dp(residual), _dp(g),
                                    _dp(lam) if lam is not None else None)
        if rc:
            raise RuntimeError(f"or_gradient_full failed: {rc}")
        return (g.reshape(self.shape), lam) if want_lam else g.reshape(self.shape)

    def gradient_nform(self, traj, lam):
        g = np.zeros(self.P)
        lib().or_gradient_nform(self._h, _dp(np.ascontiguousarray(traj)), _dp(np.ascontiguousarray(lam)), _dp(g))
        return g.reshape(self.shape)

    def gradient_bound(self, residual):
        """B with |g(u~) - g(u)| <= e B at every point when every forward state the
        reverse steps read is within e of the exact one (OT2; or_gradient_bound)."""
        residual = np.ascontiguousarray(residual, dtype=np.float64)
        b = np.zeros(self.P)
        rc = lib().or_gradient_bound(self._h, _dp(residual), _dp(b))
        if rc:
            raise RuntimeError(f"or_gradient_bound failed: {rc}")
        return b.reshape(self.shape)

    def adjoint_src(self, residual):
        residual = np.ascontiguousarray(residual, dtype=np.float64)
        out = np.zeros(self.spec.nt)
        rc = lib().or_adjoint_src(self._h, _dp(residual), _dp(out))
        if rc:
            raise RuntimeError(f"or_adjoint_src failed: {rc}")
        return out

    def gradient_actions(self, residual, actions, nslots: int, tol: float = 0.0, increment: bool = False):
        residual = np.ascontiguousarray(residual, dtype=np.float64)
        acts = np.ascontiguousarray(actions, dtype=np.int32)
        g = np.zeros(self.P)
        st = np.zeros(6, dtype=np.int64)
        rc = lib().or_gradient_actions(self._h, _dp(residual), acts.ctypes.data_as(C.POINTER(C.c_int32)),
                                       len(acts), nslots, tol, 1 if increment else 0, _dp(g),
                                       st.ctypes.data_as(C.POINTER(C.c_long)))
        if rc:
            raise RuntimeError(f"or_gradient_actions failed: {rc}")
        keys = ["advances", "stores", "restores", "reverses", "bytes_stored", "peak_bytes"]
        return g.reshape(self.shape), dict(zip(keys, st.tolist()))


def misfit(dsim, dobs) -> float:
    a = np.ascontiguousarray(dsim, dtype=np.float64).reshape(-1)
    b = np.ascontiguousarray(dobs, dtype=np.float64).reshape(-1)
    return lib().or_misfit(a.size, _dp(a), _dp(b))


# ---------------------------------------------------------------- codec

def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def encode_block(vals, ndim: int, tol: float) -> tuple[np.ndarray, int]:
    v = np.ascontiguousarray(vals, dtype=np.float32).reshape(-1)
    assert v.size == (64 if ndim == 3 else 16)
    words = np.zeros(80, dtype=np.uint64)
    nb = lib().or_zk_encode_block_buf(_fp(v), ndim, tol, words.ctypes.data_as(C.POINTER(C.c_uint64)), len(words))
    if nb < 0:
        raise RuntimeError("block overflow")
    return words, int(nb)


def decode_block(words, nbits_start: int, ndim: int, tol: float) -> np.ndarray:
    w = np.ascontiguousarray(words, dtype=np.uint64)
    out = np.zeros(64 if ndim == 3 else 16, dtype=np.float32)
    rc = lib().or_zk_decode_block_buf(w.ctypes.data_as(C.POINTER(C.c_uint64)), len(w), nbits_start, ndim, tol,
                                      _fp(out))
    if rc:
        raise RuntimeError("block decode overrun")
    return out


def fwd_lift4(v) -> np.ndarray:
    a = np.ascontiguousarray(v, dtype=np.int32).copy()
    lib().or_zk_fwd_lift4(a.ctypes.data_as(C.POINTER(C.c_int32)))
    return a


def inv_lift4(v) -> np.ndarray:
    a = np.ascontiguousarray(v, dtype=np.int32).copy()
    lib().or_zk_inv_lift4(a.ctypes.data_as(C.POINTER(C.c_int32)))
    return a


def sequency_perm(ndim: int) -> np.ndarray:
    out = (C.c_int * 64)()
    lib().or_zk_perm(ndim, out)
    return np.array(out[: (64 if ndim == 3 else 16)])


def negabinary(x: int) -> int:
    return int(lib().or_zk_negabinary(int(x)))


def stream_prefix_bytes(ndim: int, dims) -> int:
    d = (C.c_int * 3)(*(list(dims) + [1] * (3 - len(dims))))
    return lib().or_zk_prefix_bytes(ndim, d)


def encode(field: np.ndarray, tol: float) -> bytes:
    """Encode a 2-D ([z][x]) or 3-D ([z][y][x]) binary32 field."""
    f = np.ascontiguousarray(field, dtype=np.float32)
    ndim = f.ndim
    dims = list(reversed(f.shape)) + [1] * (3 - ndim)
    d = (C.c_int * 3)(*dims)
    cap = stream_prefix_bytes(ndim, dims) + 9 * f.size + 4096
    out = np.zeros(cap, dtype=np.uint8)
    nb = C.c_long(0)
    rc = lib().or_zk_encode(_fp(f), ndim, d, tol, out.ctypes.data_as(C.POINTER(C.c_uint8)), cap, C.byref(nb))
    if rc:
        raise ValueError(f"encode failed: {rc}")
    return out[: nb.value].tobytes()


def decode(stream: bytes) -> np.ndarray:
    buf = np.frombuffer(stream, dtype=np.uint8).copy()
    hdr = buf[:64].view(np.uint32)
    ndim = int(hdr[2])
    dims = [int(hdr[3]), int(hdr[4]), int(hdr[5])]
    shape = tuple(reversed(dims[:ndim]))
    out = np.zeros(shape, dtype=np.float32)
    rc = lib().or_zk_decode(buf.ctypes.data_as(C.POINTER(C.c_uint8)), len(buf), _fp(out))
    if rc:
        raise ValueError(f"decode failed: {rc}")
    return out
