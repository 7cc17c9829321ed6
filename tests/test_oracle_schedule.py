"""Pins of the Revolve schedule oracle (Sec. "Checkpointing performance model", eqs. (2)-(3))."""
import numpy as np
import pytest

from oracle import schedule as SC


def test_recurrence_equals_closed_form():
    L, Cmax = 120, 14
    p, _ = SC.p_recurrence_table(L, Cmax)
    for c in range(1, Cmax + 1):
        for l in range(1, L + 1):
            assert p[c, l] == SC.p_closed(l, c), (l, c)


@pytest.mark.parametrize("l,c", [(l, c) for l in range(2, 11) for c in range(1, 5)])
def test_recurrence_is_optimal_by_exhaustive_search(l, c):
    assert SC.brute_force_min(l - 1, c) == SC.p_closed(l, c)


def test_recompute_zero_iff_enough_slots():
    """p(N+1, M) - N is the recomputation count: zero iff M >= N (remark after eq. (3))."""
    for N in range(1, 60):
        for M in range(1, 70):
            rec = SC.p_closed(N + 1, M) - N
            assert (rec == 0) == (M >= N)
            assert rec >= 0


def test_single_slot_is_quadratic():
    for N in range(1, 40):
        assert SC.p_closed(N + 1, 1) == N * (N + 1) // 2


PINNED = [  # N, M, forward steps t(N+1, M), stores W
    (500, 10, 1640, 346),
    (1000, 20, 2750, 847),
    (3000, 31, 8442, 2674),
    (3000, 312, 5688, 2927),
    (3000, 1250, 4750, 2941),
    (3000, 3000, 3000, 2999),
]


@pytest.mark.parametrize("N,M,t,Wn", PINNED)
def test_pinned_counts(N, M, t, Wn):
    acts = SC.schedule(N, M)
    c = SC.counts(acts)
    assert c["advances"] == t == SC.p_closed(N + 1, M)
    assert c["stores"] == Wn
    assert c["reverses"] == N
    assert c["max_slot"] <= M - 1


def simulate(acts, N, M):
    """Execute an action list symbolically; return the reverse order and check every rule."""
    wm, stack, held, order = 0, [], {0: 0}, []
    for op, a, b in acts.tolist():
        if op == SC.ADVANCE:
            assert wm == a and b > a
            wm = b
        elif op == SC.STORE:
            assert wm == a and b == len(stack) + 1 and b <= M - 1
            stack.append(a)
            held[b] = a
        elif op == SC.RESTORE:
            assert held.get(b) == a and wm != a
            wm = a
        elif op == SC.FREE:
            assert stack and stack[-1] == a and b == len(stack)
            stack.pop()
            del held[b]
        elif op == SC.REVERSE:
            assert wm == a
            order.append(a)
        else:
            raise AssertionError(op)
    assert not stack
    return order


@pytest.mark.parametrize("N,M", [(1, 1), (2, 1), (7, 2), (30, 3), (64, 5), (100, 7), (250, 16), (40, 40), (40, 100)])
def test_schedule_is_valid(N, M):
    acts = SC.schedule(N, M)
    assert simulate(acts, N, M) == list(range(N, 0, -1))
    assert SC.counts(acts)["advances"] == SC.p_closed(N + 1, M)


def test_first_advance_is_smallest_optimal():
    p, kmin = SC.p_recurrence_table(60, 8)
    for c in range(2, 9):
        for l in range(2, 61):
            assert SC._first_advance(l, c) == kmin[c, l]


# ------------------------------------------------------------------ write-minimal tie-break

@pytest.mark.parametrize("N", range(1, 12))
def test_write_min_is_optimal_by_exhaustive_search(N):
    """Among all schedules with the fewest forward steps, none writes fewer checkpoints
    than the write-minimal recursion (lexicographic shortest path over every schedule)."""
    for M in range(1, 6):
        c = SC.counts(SC.schedule(N, M, write_min=True))
        assert SC.brute_force_min_writes(N, M) == (SC.p_closed(N + 1, M), c["stores"]), M


def test_write_min_closed_form_where_two_repetitions_suffice():
    """W(l, c) = l - 2 where every state fits (c >= l-1), and l - 2 - min(c, l-1-c)
    wherever two repetitions suffice (beta(c, 2) >= l)."""
    L = C = 240
    W, _ = SC.write_min_table(L, C)
    n = 0
    for c in range(2, C + 1):
        for l in range(2, L + 1):
            if c >= l - 1:
                assert W[l, c] == l - 2, (l, c)
            elif SC.beta(c, 2) >= l:
                assert W[l, c] == l - 2 - min(c, l - 1 - c), (l, c)
                n += 1
    assert n > 10_000


@pytest.mark.parametrize("N,M", [(1, 1), (2, 1), (7, 2), (30, 3), (64, 5), (100, 7), (250, 16), (40, 40), (40, 100)])
def test_write_min_schedule_is_valid(N, M):
    acts = SC.schedule(N, M, write_min=True)
    assert simulate(acts, N, M) == list(range(N, 0, -1))
    assert SC.counts(acts)["advances"] == SC.p_closed(N + 1, M)


def test_write_min_never_writes_more_and_keeps_the_step_count():
    for N in range(1, 61):
        for M in range(1, 11):
            a, b = SC.counts(SC.schedule(N, M)), SC.counts(SC.schedule(N, M, write_min=True))
            assert b["advances"] == a["advances"]
            assert b["stores"] <= a["stores"]
            assert b["max_slot"] <= M - 1


PINNED_WRITE_MIN = [  # N, M, forward steps t(N+1, M), stores W (write-minimal)
    (500, 10, 1640, 219),
    (1000, 20, 2750, 769),
    (3000, 2, 152000, 75),
    (3000, 31, 8442, 2472),
]


@pytest.mark.parametrize("N,M,t,Wn", PINNED_WRITE_MIN)
def test_write_min_pinned_counts(N, M, t, Wn):
    c = SC.counts(SC.schedule(N, M, write_min=True))
    assert c["advances"] == t == SC.p_closed(N + 1, M)
    assert c["stores"] == Wn
    assert c["reverses"] == N


def test_smallest_split_minimises_the_peak_of_growing_streams():
    """Compressed checkpoints grow over a run (the wavefield spreads), and the schedule
    compressed gradient calls run takes the smallest optimal first advance at every split.
    For any nondecreasing stream sizes that schedule's peak arena equals the smallest peak
    over every step-optimal schedule, found by exhaustive dynamic programming over the
    split choices: no other choice of optimal splits lets more slots fit a budget."""
    rng = np.random.default_rng(21)
    for N, M in [(30, 3), (40, 5), (60, 4), (80, 8), (120, 6), (90, 12)]:
        for _ in range(3):
            size = np.cumsum(rng.uniform(0.0, 1.0, N + 1)) + rng.uniform(0.1, 2.0)
            acts = SC.schedule(N, M)
            assert SC.counts(acts)["advances"] == SC.p_closed(N + 1, M)
            assert SC.peak_bytes(acts, size) == pytest.approx(SC.min_peak(N, M, size), rel=1e-12)


def test_split_choice_matters_for_shrinking_streams():
    """The rule is not vacuous: with stream sizes that fall over the run, some other
    choice of optimal splits holds a smaller peak than the smallest splits do."""
    N, M = 60, 4
    size = np.linspace(10.0, 1.0, N + 1)
    acts = SC.schedule(N, M)
    assert SC.min_peak(N, M, size) < SC.peak_bytes(acts, size) - 1e-9
