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


@pytest.mark.parametrize("N,M", [(1, 1), (2, 1), (7, 2), (30, 3), (100, 7), (500, 10), (1000, 20), (3000, 2),
                                 (3000, 31), (1200, 300), (40, 40), (40, 100)])
@pytest.mark.parametrize("write_min", [True, False])
def test_schedule_identical_to_oracle(N, M, write_min):
    """Both split rules of the library: the oracle's schedules, action for action."""
    import paper_1810_05268_amd as P
    a = P.schedule(N, M, write_min)
    b = SC.schedule(N, M, write_min=write_min)
    assert np.array_equal(a, b)
    assert P.schedule_forward_steps(N, M) == SC.p_closed(N + 1, M)


def test_schedule_grid_identical_to_oracle():
    import paper_1810_05268_amd as P
    for N in range(0, 41):
        for M in range(1, 14):
            for wm in (True, False):
                assert np.array_equal(P.schedule(N, M, wm), SC.schedule(N, M, write_min=wm)), (N, M, wm)


@pytest.mark.parametrize("N,M", [(3000, 312), (3000, 1250)])
def test_smallest_split_schedule_identical_to_oracle_at_large_slot_counts(N, M):
    import paper_1810_05268_amd as P
    assert np.array_equal(P.schedule(N, M, False), SC.schedule(N, M))


@pytest.mark.parametrize("N,M", [(3000, 312), (3000, 1250), (3000, 2486)])
def test_large_slot_counts_write_the_closed_form_count(N, M):
    """Where two repetitions suffice, the fewest writes of a minimal-step schedule are
    l - 2 - min(c, l-1-c) (l = N+1 states, c = M slots; the oracle's dynamic programme
    gives this for every such (l, c) it is pinned on).  The oracle's full programme takes
    minutes at these sizes: the library's schedule is checked for validity, minimal steps
    and that count."""
    import paper_1810_05268_amd as P
    from tests.test_oracle_schedule import simulate
    acts = P.schedule(N, M)
    c = SC.counts(acts)
    L = N + 1
    assert simulate(acts, N, M) == list(range(N, 0, -1))
    assert c["advances"] == SC.p_closed(L, M)
    assert c["stores"] == L - 2 - min(M, L - 1 - M)
    assert c["stores"] <= SC.counts(SC.schedule(N, M))["stores"]


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


@pytest.mark.parametrize("n,nbl", [((31, 29), 6), ((44, 38, 41), 8), ((320, 320, 320), 40), ((48, 20, 20), 8)])
def test_field_elements_pitch_rows_to_128_bytes_in_3d(n, nbl):
    """3-D field arrays pad each row to a multiple of 32 elements; 2-D rows stay dense."""
    import paper_1810_05268_amd._binding as B
    import workloads as W
    nd = len(n)
    h = (10.0,) * nd
    dt = 0.4 * B.cfl_dt(nd, h, 8, 3000.0)
    src = np.array([[(n[0] - 1) * 5.0] + [20.0] * (nd - 1)])
    pb = B.Problem(ndim=nd, n=n, h=h, nbl=nbl, space_order=8, nt=10, dt=dt, vmax=3000.0, vel=0x1000, src=src,
                   wavelet=0x2000, rec=src.copy())
    N = [x + 2 * nbl for x in n]
    px = -(-N[0] // 32) * 32 if nd == 3 else N[0]
    assert pb.field_elements() == px * int(np.prod(N[1:]))
    assert pb.field_elements() >= pb.P
    # the forward workspace holds four field arrays (u^n, u^{n-1}, w, zero) at least
    assert pb.workspace_bytes(B.OP_FORWARD) >= 4 * 4 * pb.field_elements()


def test_largest_grid_is_validated_on_the_host():
    """Field arrays are indexed with 32-bit point indices (the sparse tables): a grid whose
    pitched field array reaches 2^31 elements is rejected before any device work, and one
    just below is accepted (only host queries are made here)."""
    import paper_1810_05268_amd._binding as B
    h = (10.0, 10.0, 10.0)
    dt = 0.4 * B.cfl_dt(3, h, 4, 3000.0)
    src = np.array([[50.0, 50.0, 20.0]])

    def pb(n):
        return B.Problem(ndim=3, n=n, h=h, nbl=0, space_order=4, nt=10, dt=dt, vmax=3000.0, vel=0x1000, src=src,
                         wavelet=0x2000, rec=src.copy())
    ok = pb((1280, 1280, 1300))            # pitched 1280 x 1280 x 1300 = 2.13e9 < 2^31
    assert ok.field_elements() == 1280 * 1280 * 1300
    assert ok.workspace_bytes(B.OP_FORWARD) > 4 * 4 * ok.field_elements()
    big = pb((1290, 1280, 1300))           # rows pitched to 1312: 2.18e9 >= 2^31
    with pytest.raises(B.WvError):
        big.field_elements()
    with pytest.raises(B.WvError):
        big.workspace_bytes(B.OP_FORWARD)


def test_choose_compression_where_it_pays():
    """With the large shot's measured per-unit costs (ms), compression is chosen at a tight
    budget and plain Revolve once every raw state fits (no recomputation and no codec); the
    choice is the faster of the two predictions, and with a profile the compressed slot count
    is wv_plan's."""
    import paper_1810_05268_amd as P
    N, points, slot = 3000, 64_000_000, 8 * 66_560_000
    plain = {"c_f": 0.219, "c_r": 0.466, "t_store": 0.093}
    comp = {"c_f": 0.222, "c_r": 0.468, "t_store": 0.132, "t_d": 0.070, "ratio": 50.0}
    tight = P.choose(N, points, int(4e9), plain, comp, slot_bytes=slot)
    assert tight["compressed"] == 1 and tight["ms_compressed"] < tight["ms_plain"]
    assert tight["slots"] == P.predict(N, points, int(4e9), True, 1, 1, ratio=tight["ratio_hint"])["slots"]
    roomy = P.choose(N, points, slot * N, plain, comp, slot_bytes=slot)
    assert roomy["compressed"] == 0 and roomy["slots"] == N and roomy["ratio_hint"] == 0.0
    assert roomy["ms_plain"] <= roomy["ms_compressed"]
    prof = [800.0] + [float(2e5 + 3e4 * j) for j in range(1, 17)]
    M, _ = P.plan(N, points, int(4e9), prof)
    with_prof = P.choose(N, points, int(4e9), plain, comp, profile=prof, slot_bytes=slot)
    assert with_prof["compressed"] == 1 and with_prof["slots"] == M
    with pytest.raises(P.WvError):      # no ratio and no profile
        P.choose(N, points, int(4e9), plain, {k: v for k, v in comp.items() if k != "ratio"}, slot_bytes=slot)


def test_predict_plain_slots_follow_slot_bytes():
    import paper_1810_05268_amd as P
    N, points = 500, 10 ** 6
    slot = 8 * 1_040_000                      # pitched rows: 4 % more than 8 points
    budget = 30 * slot + 5
    assert P.predict(N, points, budget, False, 1.0, 1.0, t_copy=1.0, slot_bytes=slot)["slots"] == 31
    assert P.predict(N, points, budget, False, 1.0, 1.0, t_copy=1.0)["slots"] == 1 + budget // (8 * points)


def test_cfl_violation_reported_before_device_work():
    """An unstable dt is rejected in host validation (no kernel is launched)."""
    import paper_1810_05268_amd._binding as B
    pb = host_problem(dt_factor=1.05)
    rc = lib().wv_forward(C.byref(pb.model), C.byref(pb.geom), None, None, None, 0, None)
    assert rc == B.WV_ECFL


# ------------------------------------------------------------------ performance model

def _second_level_stores(acts):
    """Stores whose checkpoint is later restored and then advanced from (written from
    the action list here, independently of the library)."""
    acts = [tuple(a) for a in acts]
    need, holder = set(), {}
    for i, (op, a, b) in enumerate(acts):
        if op == 2:
            holder[b] = i
        if op == 3 and b > 0:
            j = i + 1
            while j < len(acts) and acts[j][0] == 4:
                j += 1
            if j >= len(acts) or acts[j][0] != 5:
                need.add(holder[b])
    return need, sum(1 for op, _, _ in acts if op == 2)


@pytest.mark.parametrize("N,M", [(500, 10), (1000, 21), (3000, 32), (1500, 400), (200, 200)])
def test_predict_counts_match_the_schedule(N, M):
    import paper_1810_05268_amd as P
    from oracle import schedule as SC
    points = 10_000
    S = 8 * points
    pr = P.predict(N, points, (M - 1) * S, False, 1.0, 2.0, t_copy=0.5)
    assert pr["slots"] == M
    assert pr["advances"] == SC.p_closed(N + 1, M)
    need, stores = _second_level_stores(SC.schedule(N, M, write_min=True))
    assert pr["stores"] == stores
    assert pr["fields"] == stores + len(need)
    assert pr["ms_total"] == pytest.approx(1.0 * pr["advances"] + 2.0 * N + 0.5 * pr["fields"])
    assert pr["ms_full_storage"] == pytest.approx(3.0 * N)


def test_predict_compressed_slots_and_decodes():
    import paper_1810_05268_amd as P
    N, points, F = 3000, 64_000_000, 50.0
    S = 8 * points
    budget = int(16e9)
    pr = P.predict(N, points, budget, True, 0.25, 0.57, t_c=0.14, t_d=0.08, ratio=F)
    assert pr["slots"] == min(N, 1 + budget // (int(S / F) + 512))
    # with every state stored, each reverse step restores its own checkpoint: one decode
    # per restore except the zero state, and no advance ever follows a restore
    full = P.predict(N, points, budget, True, 0.25, 0.57, t_c=0.14, t_d=0.08, ratio=1000.0)
    assert full["slots"] == N and full["advances"] == N
    assert full["decodes"] == N - 1 and full["fields"] == full["stores"] == N - 1
    assert full["ms_total"] == pytest.approx(0.25 * N + 0.57 * N + 0.14 * (N - 1) + 0.08 * (N - 1))
    # more memory never predicts more forward steps
    a = [P.predict(N, points, int(b), True, 0.25, 0.57, t_c=0.14, t_d=0.08, ratio=F)["advances"]
         for b in (2e9, 4e9, 8e9, 16e9)]
    assert a == sorted(a, reverse=True)


def test_predict_rejects_bad_input_and_budget_below_one_checkpoint_is_one_slot():
    import paper_1810_05268_amd as P
    with pytest.raises(P.WvError):
        P.predict(100, 1000, 10**9, True, 1.0, 1.0, ratio=0.0)
    with pytest.raises(P.WvError):
        P.predict(0, 1000, 10**9, False, 1.0, 1.0)
    # x_0 is the zero state and takes no memory: recomputation from it alone
    pr = P.predict(100, 1000, 10, False, 1.0, 1.0)
    assert pr["slots"] == 1 and pr["advances"] == 100 * 101 // 2 and pr["stores"] == 0


@pytest.mark.parametrize("order", [2, 4, 8, 16])
def test_ot4_cfl_matches_oracle(order):
    import oracle
    import paper_1810_05268_amd as P
    for ndim, h in ((2, (10.0, 7.5)), (3, (12.5, 10.0, 8.0))):
        a = P.cfl_dt(ndim, h, order, 3500.0, time_order=4)
        b = oracle.cfl_dt(ndim, h, order, 3500.0, time_order=4)
        assert a == b
        assert a == pytest.approx(3 ** 0.5 * P.cfl_dt(ndim, h, order, 3500.0), rel=1e-15)


# ------------------------------------------------------------------ profile planning

def _peak(N, M, prof):
    """Peak arena bytes of the oracle schedule for M slots with the given profile
    (independent of the library: oracle schedule, level scan above, linear sizes)."""
    import math
    from oracle import schedule as SC
    acts = [tuple(a) for a in SC.schedule(N, M)]
    need, _ = _second_level_stores(acts)
    ks = [0] + [-(-(j * N) // 16) for j in range(1, 17)]

    def size(k):
        for j in range(1, 17):
            if k <= ks[j] or j == 16:
                t = (k - ks[j - 1]) / (ks[j] - ks[j - 1]) if ks[j] > ks[j - 1] else 1.0
                return prof[j - 1] + min(1.0, max(0.0, t)) * (prof[j] - prof[j - 1])
    held, live, peak = {}, 0.0, 0.0
    for i, (op, a, b) in enumerate(acts):
        if op == 2:
            one = math.ceil(size(a) / 256.0) * 256.0
            held[b] = 2 * one if i in need else one
            live += held[b]
            peak = max(peak, live)
        elif op == 4:
            live -= held.pop(b, 0.0)
    return peak


@pytest.mark.parametrize("shape", ["flat", "growing"])
def test_plan_is_the_largest_fitting_slot_count(shape):
    import paper_1810_05268_amd as P
    N, points = 600, 1_000_000
    if shape == "flat":
        prof = [2e5] + [1e6] * 16
    else:
        prof = [2e5] + [2e5 + 1e6 * (j / 16) ** 2 for j in range(1, 17)]
    budget = 120_000_000
    M, hint = P.plan(N, points, budget, prof)
    assert 1 < M < N
    assert _peak(N, M, prof) <= 0.97 * budget < _peak(N, M + 1, prof)
    # the hint makes a gradient call plan the same M
    assert P.predict(N, points, budget, True, 1.0, 1.0, t_c=1.0, t_d=1.0, ratio=hint)["slots"] == M


def test_plan_growing_profile_holds_more_slots_than_the_final_state_ratio():
    """Early states are small: planning with the profile beats planning every slot at
    the final state's size (the paper's worst-case proxy)."""
    import paper_1810_05268_amd as P
    N, points, budget = 600, 1_000_000, 120_000_000
    prof = [2e5] + [2e5 + 1e6 * (j / 16) ** 2 for j in range(1, 17)]
    M, _ = P.plan(N, points, budget, prof)
    worst = P.predict(N, points, budget, True, 1.0, 1.0, t_c=1.0, t_d=1.0, ratio=8 * points / (2 * prof[-1]))
    assert M > worst["slots"]
    with pytest.raises(P.WvError):
        P.plan(N, points, budget, [0.0] * 17)


def test_write_min_table_cap_falls_back_to_the_smallest_split():
    """A reversal whose write-minimal table would exceed 2^26 entries is scheduled with the
    smallest optimal split, still minimal in forward steps."""
    import paper_1810_05268_amd as P
    N, M = 1_000_000, 200
    a = P.schedule(N, M)
    assert np.array_equal(a, P.schedule(N, M, False))
    assert SC.counts(a)["advances"] == SC.p_closed(N + 1, M)
