"""CPU-side checks of the C ABI: the library loads, exports every declared symbol,
and its host logic (schedule, CFL limit, validation) agrees with the oracle."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from oracle import schedule as SC

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wv.h")


def lib():
    import paper_1810_05268_amd as P
    return P.lib()


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wv_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported():
    import paper_1810_05268_amd._binding as B
    lib()
    names = declared_functions()
    assert set(names) == set(B.SYMBOLS)
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (wv_[a-z0-9_]+)", out))
    assert set(names) <= exported, set(names) - exported


@pytest.mark.parametrize("N,M", [(1, 1), (2, 1), (7, 2), (30, 3), (100, 7), (500, 10), (1000, 20), (3000, 31),
                                 (3000, 312), (3000, 1250), (40, 40), (40, 100)])
def test_schedule_identical_to_oracle(N, M):
    import paper_1810_05268_amd as P
    a = P.schedule(N, M)
    b = SC.schedule(N, M)
    assert np.array_equal(a, b)
    assert P.schedule_forward_steps(N, M) == SC.p_closed(N + 1, M)


def test_schedule_forward_steps_grid():
    import paper_1810_05268_amd as P
    for N in range(1, 80):
        for M in range(1, 12):
            assert P.schedule_forward_steps(N, M) == SC.p_closed(N + 1, M)


@pytest.mark.parametrize("ndim,order", [(2, 2), (2, 4), (2, 8), (3, 8), (3, 12), (3, 16)])
def test_cfl_matches_oracle(ndim, order):
    import paper_1810_05268_amd as P
    h = (10.0, 12.5, 7.5)[:ndim]
    assert P.cfl_dt(ndim, h, order, 3000.0) == oracle.cfl_dt(ndim, h, order, 3000.0)


def test_invalid_arguments():
    import paper_1810_05268_amd as P
    assert P.cfl_dt(4, (1.0, 1.0, 1.0), 8, 1.0) <= 0
    assert P.cfl_dt(3, (1.0, 1.0, 1.0), 7, 1.0) <= 0
    assert P.cfl_dt(3, (1.0, 1.0, 1.0), 18, 1.0) <= 0
    assert lib().wv_strerror(-2).decode() == "time step above the stability limit"


def host_problem(dt_factor=0.4, **kw):
    import paper_1810_05268_amd._binding as B
    import workloads as W
    shot = W.two_layer_2d(n=(31, 29), nt=20)
    dt = dt_factor * B.cfl_dt(2, shot.h, shot.order, shot.vmax)
    args = dict(ndim=2, n=shot.n, h=shot.h, nbl=shot.nbl, space_order=shot.order, nt=shot.nt, dt=dt,
                vmax=shot.vmax, vel=0x1000, src=shot.src, wavelet=0x2000, rec=shot.rec)
    args.update(kw)
    return B.Problem(**args)


def test_workspace_query_and_validation():
    import paper_1810_05268_amd._binding as B
    pb = host_problem()
    f = pb.workspace_bytes(B.OP_FORWARD)
    g0 = pb.workspace_bytes(B.OP_GRADIENT, 0)
    g1 = pb.workspace_bytes(B.OP_GRADIENT, 10 ** 8)
    assert 0 < f < g0 < g1 and g1 - g0 >= 10 ** 8
    with pytest.raises(B.WvError):
        host_problem(dt_factor=1.01).workspace_bytes(B.OP_FORWARD)
    with pytest.raises(B.WvError):
        host_problem(space_order=5).workspace_bytes(B.OP_FORWARD)
    with pytest.raises(B.WvError):   # receiver outside the padded grid
        host_problem(rec=np.array([[1e6, 20.0]])).workspace_bytes(B.OP_FORWARD)


def test_cfl_violation_reported_before_device_work():
    """An unstable dt is rejected in host validation (no kernel is launched)."""
    import paper_1810_05268_amd._binding as B
    pb = host_problem(dt_factor=1.05)
    rc = lib().wv_forward(C.byref(pb.model), C.byref(pb.geom), None, None, None, 0, None)
    assert rc == B.WV_ECFL
