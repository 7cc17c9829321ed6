"""ctypes binding of libwv.so (the C ABI declared in include/wv.h).

Argument marshalling only: every step of the solver, schedule and codec runs in
the library.  Device buffers are torch tensors on a ROCm device; their raw
pointers and the current HIP stream are handed to the C functions.  The library
must have been built (``paper_1810_05268_amd.build``); if it is missing this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwv.so")

WV_OK, WV_EINVAL, WV_ECFL, WV_EBUDGET, WV_EARENA, WV_ENOMEM, WV_EHIP, WV_EUNSTABLE, WV_ENOTIMPL, WV_ECAP = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9)
WV_ETIMEOUT = -10
OP_FORWARD, OP_GRADIENT, OP_COMPRESSIBILITY = 0, 1, 2
ADVANCE, STORE, RESTORE, FREE, REVERSE = 1, 2, 3, 4, 5


class WvError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        detail = ""
        if code == WV_EHIP:
            try:
                detail = " [" + lib().wv_last_error().decode() + "]"
            except Exception:    # noqa: BLE001 - formatting only
                pass
        super().__init__(f"{where}: {strerror(code)} ({code}){detail}")


class WvModel(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double * 3), ("nbl", C.c_int),
                ("space_order", C.c_int), ("nt", C.c_int), ("dt", C.c_double), ("vmax", C.c_double),
                ("vel", C.c_void_p), ("time_order", C.c_int)]


class WvGeom(C.Structure):
    _fields_ = [("nsrc", C.c_int), ("src_xyz", C.POINTER(C.c_double)), ("wavelet", C.c_void_p),
                ("nrec", C.c_int), ("rec_xyz", C.POINTER(C.c_double))]


class WvStats(C.Structure):
    _fields_ = [("timing", C.c_int), ("advances", C.c_long), ("stores", C.c_long), ("restores", C.c_long),
                ("fields", C.c_long), ("decodes", C.c_long), ("reverses", C.c_long), ("slots", C.c_long), ("bytes_stored", C.c_double),
                ("peak_bytes", C.c_double), ("ratio", C.c_double), ("ratio_planned", C.c_double),
                ("misfit", C.c_double), ("ms_total", C.c_double), ("ms_forward", C.c_double),
                ("ms_adjoint", C.c_double), ("ms_store", C.c_double), ("ms_restore", C.c_double),
                ("ms_fwd_kernel", C.c_double), ("ms_adj_kernel", C.c_double), ("retries", C.c_long),
                ("profile", C.c_double * 17)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "profile"}
        d["profile"] = list(self.profile)
        return d


class WvCosts(C.Structure):
    _fields_ = [("c_f", C.c_double), ("c_r", C.c_double), ("t_copy", C.c_double), ("t_c", C.c_double),
                ("t_d", C.c_double), ("ratio", C.c_double), ("slot_bytes", C.c_double)]


class WvChoice(C.Structure):
    _fields_ = [("compressed", C.c_int), ("slots", C.c_int), ("ratio_hint", C.c_double), ("ms_plain", C.c_double),
                ("ms_compressed", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class WvPrediction(C.Structure):
    _fields_ = [("slots", C.c_int), ("advances", C.c_long), ("stores", C.c_long), ("fields", C.c_long),
                ("decodes", C.c_long), ("ms_forward", C.c_double), ("ms_adjoint", C.c_double),
                ("ms_store", C.c_double), ("ms_restore", C.c_double), ("ms_total", C.c_double),
                ("ms_full_storage", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class WvResult(C.Structure):
    _fields_ = [("status", C.c_int), ("misfit", C.c_double), ("t_submit_ms", C.c_double),
                ("t_start_ms", C.c_double), ("t_end_ms", C.c_double), ("stats", WvStats)]


# every symbol include/wv.h declares
SYMBOLS = ["wv_cfl_dt", "wv_cfl_dt_to", "wv_workspace_bytes", "wv_field_elements", "wv_forward", "wv_gradient", "wv_misfit_gradient", "wv_adjoint_src",
           "wv_pad_velocity", "wv_velocity_gradient", "wv_zfpk_workspace_bytes", "wv_zfpk_max_bytes",
           "wv_zfpk_encode", "wv_zfpk_encode_noalloc", "wv_zfpk_decode", "wv_schedule", "wv_schedule_forward_steps", "wv_predict", "wv_choose", "wv_plan", "wv_compressibility", "wv_stream_ceiling", "wv_misfit_gradient_auto", "wv_strerror",
           "wv_last_error", "wv_version", "wv_batch_workspace_bytes", "wv_batch_misfit_gradient", "wv_engine_create", "wv_engine_set_batching", "wv_engine_submit", "wv_engine_wait",
           "wv_engine_pending", "wv_engine_destroy"]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -m paper_1810_05268_amd.build)")
        # torch ships its own HIP runtime under the same soname; load it first so that
        # the library and torch share one runtime (and one device context) in the process
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, dp, ip, sz = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_size_t
        mp, gp, stp = C.POINTER(WvModel), C.POINTER(WvGeom), C.POINTER(WvStats)
        L.wv_cfl_dt.argtypes = [C.c_int, dp, C.c_int, C.c_double]
        L.wv_cfl_dt.restype = C.c_double
        L.wv_cfl_dt_to.argtypes = [C.c_int, dp, C.c_int, C.c_double, C.c_int]
        L.wv_cfl_dt_to.restype = C.c_double
        L.wv_workspace_bytes.argtypes = [mp, gp, C.c_int, sz]
        L.wv_workspace_bytes.restype = sz
        L.wv_field_elements.argtypes = [mp]
        L.wv_field_elements.restype = C.c_longlong
        L.wv_forward.argtypes = [mp, gp, vp, vp, vp, sz, vp]
        L.wv_gradient.argtypes = [mp, gp, vp, sz, C.c_double, C.c_double, vp, stp, vp, sz, vp]
        L.wv_misfit_gradient.argtypes = [mp, gp, vp, sz, C.c_double, C.c_double, dp, vp, vp, stp, vp, sz, vp]
        L.wv_adjoint_src.argtypes = [mp, gp, vp, vp, vp, sz, vp]
        L.wv_pad_velocity.argtypes = [C.c_int, ip, C.c_int, vp, vp, vp]
        L.wv_velocity_gradient.argtypes = [C.c_int, ip, C.c_int, vp, vp, vp, vp]
        L.wv_zfpk_workspace_bytes.argtypes = [C.c_int, ip]
        L.wv_zfpk_workspace_bytes.restype = sz
        L.wv_zfpk_max_bytes.argtypes = [C.c_int, ip]
        L.wv_zfpk_max_bytes.restype = sz
        L.wv_zfpk_encode.argtypes = [vp, C.c_int, ip, C.c_double, vp, sz, C.POINTER(C.c_size_t), vp, sz, vp]
        L.wv_zfpk_encode_noalloc.argtypes = [vp, C.c_int, ip, C.c_double, vp, sz, C.POINTER(C.c_size_t), vp]
        L.wv_zfpk_decode.argtypes = [vp, sz, C.c_int, ip, vp, vp]
        L.wv_schedule.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int32), sz, C.POINTER(C.c_size_t)]
        L.wv_schedule_forward_steps.argtypes = [C.c_int, C.c_int]
        L.wv_schedule_forward_steps.restype = C.c_long
        L.wv_predict.argtypes = [C.c_int, C.c_longlong, sz, C.c_int, C.POINTER(WvCosts), C.POINTER(WvPrediction)]
        L.wv_choose.argtypes = [C.c_int, C.c_longlong, sz, C.POINTER(WvCosts), C.POINTER(WvCosts),
                                C.POINTER(C.c_double), C.c_int, C.POINTER(WvChoice)]
        L.wv_plan.argtypes = [C.c_int, C.c_longlong, sz, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_int),
                              C.POINTER(C.c_double)]
        L.wv_compressibility.argtypes = [mp, gp, C.c_double, C.c_int, C.POINTER(C.c_size_t), C.c_int,
                                         C.POINTER(C.c_int), vp, sz, vp]
        L.wv_batch_workspace_bytes.argtypes = [C.c_int, mp, gp, sz]
        L.wv_batch_workspace_bytes.restype = sz
        L.wv_batch_misfit_gradient.argtypes = [C.c_int, mp, gp, C.POINTER(C.c_void_p), sz, C.c_double, C.c_double,
                                               C.POINTER(C.c_double), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                               stp, vp, sz, vp]
        L.wv_misfit_gradient_auto.argtypes = [mp, gp, vp, sz, C.c_double, C.POINTER(WvCosts), C.POINTER(WvCosts),
                                              C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double), vp, vp, stp,
                                              C.POINTER(WvChoice), vp, sz, vp]
        L.wv_stream_ceiling.argtypes = [C.c_int, sz, vp, sz, C.c_int, C.POINTER(C.c_double), vp]
        L.wv_strerror.argtypes = [C.c_int]
        L.wv_strerror.restype = C.c_char_p
        L.wv_version.restype = C.c_char_p
        L.wv_last_error.restype = C.c_char_p
        L.wv_engine_create.argtypes = [vp, sz, C.c_int, C.POINTER(C.c_void_p)]
        L.wv_engine_set_batching.argtypes = [vp, C.c_int]
        L.wv_engine_submit.argtypes = [vp, mp, gp, vp, sz, C.c_double, C.c_double, vp, vp]
        L.wv_engine_wait.argtypes = [vp, C.c_int, C.c_double, C.POINTER(WvResult)]
        L.wv_engine_pending.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.wv_engine_destroy.argtypes = [vp]
        for name in SYMBOLS:
            getattr(L, name)
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().wv_strerror(code).decode()
    except Exception:        # noqa: BLE001 - used while formatting another error
        return "error"


def _check(rc: int, where: str) -> None:
    if rc != WV_OK:
        raise WvError(rc, where)


def _ptr(t) -> int | None:
    """Raw device pointer of a torch tensor (or an int, or None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream=None) -> int | None:
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _dims(ndim, dims):
    d = (C.c_int * 3)(*(list(dims) + [1] * (3 - len(dims))))
    return d


# ------------------------------------------------------------------ host-only calls

def cfl_dt(ndim: int, h, space_order: int, vmax: float, time_order: int = 2) -> float:
    hh = (C.c_double * 3)(*(list(h)[:ndim] + [1.0] * (3 - ndim)))
    if time_order == 2:
        return float(lib().wv_cfl_dt(ndim, hh, space_order, vmax))
    return float(lib().wv_cfl_dt_to(ndim, hh, space_order, vmax, time_order))


def schedule(nt: int, M: int, write_min: bool = True) -> np.ndarray:
    """wv_schedule: write_min=True is what uncompressed gradient calls run, False what
    compressed ones run."""
    n = C.c_size_t(0)
    wm = 1 if write_min else 0
    lib().wv_schedule(nt, M, wm, None, 0, C.byref(n))
    out = np.zeros((max(n.value, 1), 3), dtype=np.int32)
    _check(lib().wv_schedule(nt, M, wm, out.ctypes.data_as(C.POINTER(C.c_int32)), n.value, C.byref(n)),
           "wv_schedule")
    return out[: n.value]


def schedule_forward_steps(nt: int, M: int) -> int:
    return int(lib().wv_schedule_forward_steps(nt, M))


def compressibility(pb: Problem, tol: float, stride: int, ws, stream=None) -> list:
    """Stream bytes of u^n for n = stride, 2 stride, ... (see wv_compressibility)."""
    cap = pb.nt // stride
    out = (C.c_size_t * max(1, cap))()
    n = C.c_int(0)
    _check(lib().wv_compressibility(C.byref(pb.model), C.byref(pb.geom), float(tol), int(stride), out, cap,
                                    C.byref(n), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)),
           "wv_compressibility")
    return [int(out[i]) for i in range(n.value)]


def plan(nt: int, points: int, mem_budget: int, profile) -> tuple[int, float]:
    """(slots, ratio_hint) for a compressibility profile (see wv_plan)."""
    prof = (C.c_double * 17)(*[float(x) for x in profile])
    m, h = C.c_int(0), C.c_double(0.0)
    _check(lib().wv_plan(int(nt), int(points), int(mem_budget), prof, 17, C.byref(m), C.byref(h)), "wv_plan")
    return int(m.value), float(h.value)


def predict(nt: int, points: int, mem_budget: int, compressed: bool, c_f: float, c_r: float, t_copy: float = 0.0,
            t_c: float = 0.0, t_d: float = 0.0, ratio: float = 1.0, slot_bytes: float = 0.0) -> dict:
    """Predicted gradient time (ms) and counts for the given per-unit costs (host only).
    slot_bytes: bytes of one uncompressed slot (8 x wv_field_elements; 0 = 8 x points)."""
    costs = WvCosts(float(c_f), float(c_r), float(t_copy), float(t_c), float(t_d), float(ratio), float(slot_bytes))
    out = WvPrediction()
    _check(lib().wv_predict(int(nt), int(points), int(mem_budget), 1 if compressed else 0, C.byref(costs),
                            C.byref(out)), "wv_predict")
    return out.as_dict()


def choose(nt: int, points: int, mem_budget: int, plain: dict, compressed: dict, profile=None,
           slot_bytes: float = 0.0) -> dict:
    """Plain or compressed checkpoints for this budget, whichever the run-time model predicts
    faster (see wv_choose).  plain / compressed: per-unit costs as costs_from_stats returns
    them; compressed["ratio"] is used when no profile is given."""
    cp = WvCosts(plain["c_f"], plain["c_r"], plain.get("t_store", 0.0), 0.0, 0.0, 1.0, float(slot_bytes))
    cc = WvCosts(compressed["c_f"], compressed["c_r"], 0.0, compressed.get("t_store", 0.0), compressed.get("t_d", 0.0),
                 float(compressed.get("ratio", 0.0)), 0.0)
    prof = (C.c_double * 17)(*[float(x) for x in profile]) if profile is not None else None
    out = WvChoice()
    _check(lib().wv_choose(int(nt), int(points), int(mem_budget), C.byref(cp), C.byref(cc), prof,
                           17 if profile is not None else 0, C.byref(out)), "wv_choose")
    return out.as_dict()


def costs_from_stats(st: dict) -> dict:
    """Per-unit costs measured by a gradient call with timing (see wv_costs)."""
    return {"c_f": st["ms_forward"] / max(1, st["advances"]), "c_r": st["ms_adjoint"] / max(1, st["reverses"]),
            "t_store": st["ms_store"] / max(1, st["fields"]),
            "t_d": st["ms_restore"] / st["decodes"] if st["decodes"] else 0.0, "ratio": st["ratio"]}


def zfpk_max_bytes(ndim: int, dims) -> int:
    return int(lib().wv_zfpk_max_bytes(ndim, _dims(ndim, dims)))


def zfpk_workspace_bytes(ndim: int, dims) -> int:
    return int(lib().wv_zfpk_workspace_bytes(ndim, _dims(ndim, dims)))


# ------------------------------------------------------------------ model / geometry structs

class Problem:
    """C structs for one shot.  vel and wavelet are device tensors (float32);
    src/rec are host float64 arrays (metres, axis order x[, y], z)."""

    def __init__(self, ndim, n, h, nbl, space_order, nt, dt, vmax, vel, src, wavelet, rec, time_order=2):
        self.model = WvModel()
        self.model.ndim = ndim
        self.model.time_order = int(time_order)
        for a in range(3):
            self.model.n[a] = int(n[a]) if a < ndim else 1
            self.model.h[a] = float(h[a]) if a < ndim else 1.0
        self.model.nbl, self.model.space_order, self.model.nt = int(nbl), int(space_order), int(nt)
        self.model.dt, self.model.vmax = float(dt), float(vmax)
        self.vel = vel
        self.model.vel = _ptr(vel)
        self.src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, ndim)
        self.rec = np.ascontiguousarray(rec, dtype=np.float64).reshape(-1, ndim)
        self.wavelet = wavelet
        self.geom = WvGeom()
        self.geom.nsrc = len(self.src)
        self.geom.src_xyz = self.src.ctypes.data_as(C.POINTER(C.c_double))
        self.geom.wavelet = _ptr(wavelet)
        self.geom.nrec = len(self.rec)
        self.geom.rec_xyz = self.rec.ctypes.data_as(C.POINTER(C.c_double))
        self.ndim, self.nt, self.nrec = ndim, int(nt), len(self.rec)
        self.padded = tuple(int(n[a]) + 2 * int(nbl) for a in range(ndim))
        self.P = int(np.prod(self.padded))

    def set_vel(self, vel) -> None:
        self.vel = vel
        self.model.vel = _ptr(vel)

    def field_elements(self) -> int:
        """Elements of one solver field array (rows pitched; 8 x this = one uncompressed slot)."""
        n = int(lib().wv_field_elements(C.byref(self.model)))
        if n <= 0:
            raise WvError(WV_EINVAL, "wv_field_elements")
        return n

    def workspace_bytes(self, op: int, mem_budget: int = 0) -> int:
        b = int(lib().wv_workspace_bytes(C.byref(self.model), C.byref(self.geom), op, int(mem_budget)))
        if b == 0:
            raise WvError(WV_EINVAL, "wv_workspace_bytes")
        return b


# ------------------------------------------------------------------ device calls

def forward(pb: Problem, data, ws, state_out=None, stream=None) -> None:
    _check(lib().wv_forward(C.byref(pb.model), C.byref(pb.geom), _ptr(data), _ptr(state_out), _ptr(ws),
                            ws.numel() * ws.element_size(), _stream(stream)), "wv_forward")


def gradient(pb: Problem, residual, mem_budget: int, tol: float, grad, ws, ratio_hint: float = 0.0,
             stream=None, timing: bool = False) -> dict:
    st = WvStats()
    st.timing = int(timing)
    _check(lib().wv_gradient(C.byref(pb.model), C.byref(pb.geom), _ptr(residual), int(mem_budget), float(tol),
                             float(ratio_hint), _ptr(grad), C.byref(st), _ptr(ws), ws.numel() * ws.element_size(),
                             _stream(stream)), "wv_gradient")
    return st.as_dict()


def misfit_gradient(pb: Problem, d_obs, mem_budget: int, tol: float, grad, ws, ratio_hint: float = 0.0,
                    d_sim=None, stream=None, timing: bool = False) -> tuple[float, dict]:
    st = WvStats()
    st.timing = int(timing)
    phi = C.c_double(0.0)
    _check(lib().wv_misfit_gradient(C.byref(pb.model), C.byref(pb.geom), _ptr(d_obs), int(mem_budget), float(tol),
                                    float(ratio_hint), C.byref(phi), _ptr(grad), _ptr(d_sim), C.byref(st), _ptr(ws),
                                    ws.numel() * ws.element_size(), _stream(stream)), "wv_misfit_gradient")
    return float(phi.value), st.as_dict()


def stream_ceiling(reads: int, stream_bytes: int, ws, reps: int = 10, stream=None) -> float:
    """GB/s of a nontemporal stream of `reads` input arrays and one output (wv_stream_ceiling)."""
    out = C.c_double(0.0)
    _check(lib().wv_stream_ceiling(int(reads), int(stream_bytes), _ptr(ws), ws.numel() * ws.element_size(), int(reps),
                                   C.byref(out), _stream(stream)), "wv_stream_ceiling")
    return float(out.value)


def _batch_structs(pbs):
    models = (WvModel * len(pbs))(*[pb.model for pb in pbs])
    geoms = (WvGeom * len(pbs))(*[pb.geom for pb in pbs])
    return models, geoms


def batch_workspace_bytes(pbs, mem_budget: int) -> int:
    models, geoms = _batch_structs(pbs)
    b = int(lib().wv_batch_workspace_bytes(len(pbs), models, geoms, int(mem_budget)))
    if b == 0:
        raise WvError(WV_EINVAL, "wv_batch_workspace_bytes")
    return b


def batch_misfit_gradient(pbs, d_obs, mem_budget: int, tol: float, grads, ws, ratio_hint: float = 0.0,
                          d_sims=None, stream=None) -> tuple[list, list]:
    """wv_batch_misfit_gradient over the shots pbs (Problem each); d_obs, grads, d_sims:
    lists of device tensors, one per shot.  Returns (misfits, stats dicts)."""
    n = len(pbs)
    models, geoms = _batch_structs(pbs)
    vp_arr = C.c_void_p * n
    dobs = vp_arr(*[_ptr(t) for t in d_obs])
    gs = vp_arr(*[_ptr(t) for t in grads])
    ds = vp_arr(*[_ptr(t) for t in d_sims]) if d_sims is not None else None
    phis = (C.c_double * n)()
    sts = (WvStats * n)()
    _check(lib().wv_batch_misfit_gradient(n, models, geoms, dobs, int(mem_budget), float(tol), float(ratio_hint),
                                          phis, gs, ds, sts, _ptr(ws), ws.numel() * ws.element_size(),
                                          _stream(stream)), "wv_batch_misfit_gradient")
    return [float(phis[i]) for i in range(n)], [sts[i].as_dict() for i in range(n)]


def misfit_gradient_auto(pb: Problem, d_obs, mem_budget: int, tol: float, plain: dict, compressed: dict, grad, ws,
                         profile=None, slot_bytes: float = 0.0, d_sim=None, stream=None) -> tuple[float, dict, dict]:
    """wv_misfit_gradient_auto: the model's choice of plain or compressed checkpoints made
    per call from earlier calls' costs (as costs_from_stats returns them).  Returns
    (misfit, stats, choice)."""
    cp = WvCosts(plain["c_f"], plain["c_r"], plain.get("t_store", 0.0), 0.0, 0.0, 1.0, float(slot_bytes))
    cc = WvCosts(compressed["c_f"], compressed["c_r"], 0.0, compressed.get("t_store", 0.0), compressed.get("t_d", 0.0),
                 float(compressed.get("ratio", 0.0)), 0.0)
    prof = (C.c_double * 17)(*[float(x) for x in profile]) if profile is not None else None
    st, ch, phi = WvStats(), WvChoice(), C.c_double(0.0)
    _check(lib().wv_misfit_gradient_auto(C.byref(pb.model), C.byref(pb.geom), _ptr(d_obs), int(mem_budget),
                                         float(tol), C.byref(cp), C.byref(cc), prof, 17 if profile is not None else 0,
                                         C.byref(phi), _ptr(grad), _ptr(d_sim), C.byref(st), C.byref(ch), _ptr(ws),
                                         ws.numel() * ws.element_size(), _stream(stream)), "wv_misfit_gradient_auto")
    return float(phi.value), st.as_dict(), ch.as_dict()


def adjoint_src(pb: Problem, residual, src_adj, ws, stream=None) -> None:
    _check(lib().wv_adjoint_src(C.byref(pb.model), C.byref(pb.geom), _ptr(residual), _ptr(src_adj), _ptr(ws),
                                ws.numel() * ws.element_size(), _stream(stream)), "wv_adjoint_src")


def pad_velocity(ndim: int, n, nbl: int, vel_interior, vel_padded, stream=None) -> None:
    _check(lib().wv_pad_velocity(ndim, _dims(ndim, n), nbl, _ptr(vel_interior), _ptr(vel_padded),
                                 _stream(stream)), "wv_pad_velocity")


def velocity_gradient(ndim: int, n, nbl: int, vel_padded, grad_m, grad_vel, stream=None) -> None:
    _check(lib().wv_velocity_gradient(ndim, _dims(ndim, n), nbl, _ptr(vel_padded), _ptr(grad_m), _ptr(grad_vel),
                                      _stream(stream)), "wv_velocity_gradient")


def zfpk_encode(field, tol: float, out, ws, stream=None) -> int:
    """Encode a device float32 field ([z][x] or [z][y][x]); returns the stream bytes."""
    ndim = field.dim()
    dims = list(reversed(field.shape))
    nb = C.c_size_t(0)
    _check(lib().wv_zfpk_encode(_ptr(field), ndim, _dims(ndim, dims), float(tol), _ptr(out),
                                out.numel() * out.element_size(), C.byref(nb), _ptr(ws),
                                ws.numel() * ws.element_size(), _stream(stream)), "wv_zfpk_encode")
    return int(nb.value)


def zfpk_encode_noalloc(field, tol: float, out, stream=None) -> int:
    """As zfpk_encode, with the library's fixed device scratch instead of a workspace."""
    ndim = field.dim()
    dims = list(reversed(field.shape))
    nb = C.c_size_t(0)
    _check(lib().wv_zfpk_encode_noalloc(_ptr(field), ndim, _dims(ndim, dims), float(tol), _ptr(out),
                                        out.numel() * out.element_size(), C.byref(nb), _stream(stream)),
           "wv_zfpk_encode_noalloc")
    return int(nb.value)


def zfpk_decode(stream_buf, field, nbytes=None, stream=None) -> None:
    """Decode the stream in the device buffer stream_buf (nbytes readable bytes, default
    the whole buffer) into the device float32 field."""
    ndim = field.dim()
    dims = list(reversed(field.shape))
    if nbytes is None:
        nbytes = stream_buf.numel() * stream_buf.element_size()
    _check(lib().wv_zfpk_decode(_ptr(stream_buf), int(nbytes), ndim, _dims(ndim, dims), _ptr(field),
                                _stream(stream)), "wv_zfpk_decode")
