"""Revolve schedule oracle (test infrastructure only: never imported by the product path).

The checkpointed reversal of Sec. "Checkpointing performance model" of the paper:
classic Revolve (Griewank) with one memory level and a fixed number of steps.

Mapping used here.  The forward states are x_0..x_N with x_k = (u^k, u^{k-1});
reverse step k (k = N..1) needs x_k.  This is Griewank's chain with l = N + 1
steps and c = M checkpoint slots, x_0 held in one of them; Griewank's last
reverse step (it needs x_0) is dropped, because u^0 = 0 contributes nothing to
the gradient.

Three independent routes to the forward-step count are provided so that each
pins the others:
  * ``p_recurrence``: recurrence (3) of the paper, read as
        p(l, 1) = l(l-1)/2,  p(1, c) = 0,
        p(l, c) = min_{1 <= k <= l-1} { k + p(k, c) + p(l-k, c-1) }
    (the printed range 1 <= k <= l would make p(l, c) refer to itself);
  * ``p_closed``: Griewank's binomial closed form
        t(l, c) = r l - beta(c+1, r-1),  beta(c, r) = C(c+r, c),
        r = min{ r : beta(c, r) >= l };
  * ``brute_force_min``: exhaustive shortest-path search over every schedule
    for tiny l.
The recomputation count of eq. (2) is p(N+1, M) - N: zero iff M >= N, as the
paper remarks after eq. (3).

``schedule(N, M)`` emits the action list of the recursion with the smallest
optimal first advance k (ties broken towards the left).  ``schedule(N, M,
write_min=True)`` breaks the tie instead towards the fewest checkpoint writes:
among the optimal first advances it takes the k that minimises the stores of the
whole recursion (``write_min_table``, a dynamic programme over segments; smallest
k among equal counts): every write is charged in the storage overhead W S / B of the
checkpointing performance model, and any k of the interval is optimal in steps.
A right part of a single state is then not stored: it is the state just reached,
reversed at once from the working state.  Actions are int32
triples (op, a, b):
  1 ADVANCE x_a -> x_b, 2 STORE x_a in slot b, 3 RESTORE x_a from slot b,
  4 FREE slot b (holding x_a), 5 REVERSE step a.
Slot 0 holds x_0 (the state at rest) for the whole run; slots are used as a
stack (slot b is the b-th nested checkpoint).  A RESTORE is emitted only when
the working state is not already the one needed.
"""
from __future__ import annotations

import heapq
import sys
from math import comb

import numpy as np

ADVANCE, STORE, RESTORE, FREE, REVERSE = 1, 2, 3, 4, 5


def beta(c: int, r: int) -> int:
    if r < 0 or c < 0:
        return 0
    return comb(c + r, c)


def p_closed(l: int, c: int) -> int:
    """Griewank's minimal number of forward steps to reverse l steps with c slots."""
    if l <= 1:
        return 0
    if c < 1:
        raise ValueError("need at least one slot")
    r = 0
    while beta(c, r) < l:
        r += 1
    return r * l - beta(c + 1, r - 1)


def p_recurrence_table(L: int, C: int) -> tuple[np.ndarray, np.ndarray]:
    """Recurrence (3) for all 1 <= l <= L, 1 <= c <= C.

    Returns (p, kmin) with p[c, l] the minimum and kmin[c, l] the smallest
    minimising first advance (0 where undefined)."""
    p = np.zeros((C + 1, L + 1), dtype=np.int64)
    kmin = np.zeros((C + 1, L + 1), dtype=np.int64)
    ls = np.arange(L + 1, dtype=np.int64)
    p[1, :] = ls * (ls - 1) // 2
    for c in range(2, C + 1):
        p[c, 1] = 0
        for l in range(2, L + 1):
            k = np.arange(1, l, dtype=np.int64)
            cost = k + p[c, 1:l] + p[c - 1, l - k]
            j = int(np.argmin(cost))          # first occurrence = smallest k
            p[c, l] = cost[j]
            kmin[c, l] = k[j]
    return p, kmin


def p_recurrence(l: int, c: int) -> int:
    p, _ = p_recurrence_table(l, c)
    return int(p[c, l])


def _closed_vec(ls: np.ndarray, c: int) -> np.ndarray:
    """p_closed over an array of chain lengths (exact integers)."""
    ls = np.asarray(ls, dtype=np.int64)
    if c == 1:
        return ls * (ls - 1) // 2
    top = int(ls.max()) if ls.size else 0
    bet = [beta(c, 0)]
    while bet[-1] < top:                  # beta(c, r) for r = 0.. until it covers every l
        bet.append(beta(c, len(bet)))
    r = np.searchsorted(np.asarray(bet, dtype=np.int64), ls, side="left")   # min r: beta(c, r) >= l
    bet1 = np.asarray([beta(c + 1, j - 1) for j in range(len(bet))], dtype=np.int64)
    return np.where(ls <= 1, 0, r * ls - bet1[r])


def _first_advance(l: int, c: int) -> int:
    """Smallest k minimising k + p(k, c) + p(l-k, c-1) (recurrence (3))."""
    if c >= l - 1:
        return 1
    k = np.arange(1, l, dtype=np.int64)
    cost = k + _closed_vec(k, c) + _closed_vec(l - k, c - 1)
    return int(k[int(np.argmin(cost))])


def write_min_table(L: int, C: int) -> tuple[np.ndarray, np.ndarray]:
    """W[l, c]: the fewest stores of the recursion for a segment of l steps and c slots
    when every split takes an optimal first advance (minimal forward steps); K[l, c]:
    the smallest first advance that attains W[l, c].  A split stores once (unless its
    right part is the single state just reached, which is reversed at once), then the
    right part has c-1 slots and the left part c:
        W[l, c] = min_{k optimal} ( [l-k > 1] + W[l-k, c-1] + W[k, c] ),  W[1, c] = W[l, 1] = 0."""
    W = np.zeros((L + 1, C + 1), dtype=np.int64)
    K = np.ones((L + 1, C + 1), dtype=np.int64)
    ls = np.arange(L + 1, dtype=np.int64)
    for c in range(2, C + 1):
        pc, pc1 = _closed_vec(ls, c), _closed_vec(ls, c - 1)    # p(., c) and p(., c-1)
        for l in range(2, L + 1):
            k = ls[1:l]
            cost = k + pc[k] + pc1[l - k]
            opt = k[cost == cost.min()]
            # a right part of one state is reversed at once from the working state:
            # its checkpoint would never be read, so that split stores nothing
            w = (l - opt > 1) + W[l - opt, c - 1] + W[opt, c]
            j = int(np.argmin(w))
            W[l, c] = w[j]
            K[l, c] = opt[j]
    return W, K


def schedule(N: int, M: int, write_min: bool = False) -> np.ndarray:
    """Action list (int32, shape (n, 3)) reversing N steps with M slots."""
    if N < 0 or M < 1:
        raise ValueError("need N >= 0 and M >= 1")
    if write_min:
        _, K = write_min_table(N + 1, min(M, N + 1))
    acts: list[tuple[int, int, int]] = []
    state = {"wm": 0, "depth": 0}

    def need(s: int, slot: int) -> None:
        if state["wm"] != s:
            acts.append((RESTORE, s, slot))
            state["wm"] = s

    def reverse(k: int) -> None:
        acts.append((REVERSE, k, 0))

    def rev(s: int, l: int, c: int, slot: int) -> None:
        # x_s is held in `slot`; reverse steps s+l-1 .. s (step 0 dropped)
        if l == 1:
            if s > 0:
                need(s, slot)
                reverse(s)
            return
        if c == 1:
            for i in range(l - 1, -1, -1):
                if s + i == 0:
                    break
                need(s, slot)
                if i > 0:
                    acts.append((ADVANCE, s, s + i))
                    state["wm"] = s + i
                reverse(s + i)
            return
        k = int(K[l, min(c, K.shape[1] - 1)]) if write_min else _first_advance(l, c)
        need(s, slot)
        if write_min and l - k == 1:
            # the state reached is reversed at once from the working state: no checkpoint
            acts.append((ADVANCE, s, s + k))
            state["wm"] = s + k
            reverse(s + k)
            rev(s, k, c, slot)
            return
        acts.append((ADVANCE, s, s + k))
        state["wm"] = s + k
        state["depth"] += 1
        ns = state["depth"]
        acts.append((STORE, s + k, ns))
        rev(s + k, l - k, c - 1, ns)
        acts.append((FREE, s + k, ns))
        state["depth"] -= 1
        rev(s, k, c, slot)

    old = sys.getrecursionlimit()
    sys.setrecursionlimit(max(old, 20 * (N + M) + 1000))
    try:
        rev(0, N + 1, M, 0)
    finally:
        sys.setrecursionlimit(old)
    return np.asarray(acts, dtype=np.int32).reshape(-1, 3)


def peak_bytes(acts: np.ndarray, size) -> float:
    """Largest total of the checkpoints held at once when stored state x_k takes size[k]
    bytes (one level per checkpoint; slot 0 holds x_0 and takes nothing)."""
    held = {}
    live = peak = 0.0
    for op, a, b in np.asarray(acts).tolist():
        if op == STORE:
            held[b] = float(size[a])
            live += held[b]
            peak = max(peak, live)
        elif op == FREE:
            live -= held.pop(b)
    return peak


def min_peak(N: int, M: int, size) -> float:
    """The smallest peak_bytes over every schedule whose splits are all optimal in forward
    steps (the minimum of recurrence (3)), by exhaustive dynamic programming over the split
    choices: reversing the segment [a, a + l) with c slots (x_a held below it) and first
    advance k stores x_{a+k} for the whole reversal of the right part [a + k, a + l) (c - 1
    slots) and then frees it before the left part [a, a + k) (c slots), so
        f(a, l, c) = min_{k optimal} max(size[a + k] + f(a + k, l - k, c - 1), f(a, k, c)),
    f(a, 1, c) = f(a, l, 1) = 0.  Exponential memory in nothing, but O(N^2 M) states:
    small N only."""
    from functools import lru_cache

    size = [float(x) for x in size]

    @lru_cache(maxsize=None)
    def opt(l: int, c: int) -> tuple[int, ...]:
        k = np.arange(1, l, dtype=np.int64)
        cost = k + _closed_vec(k, c) + _closed_vec(l - k, c - 1)
        return tuple(int(x) for x in k[cost == cost.min()])

    @lru_cache(maxsize=None)
    def f(a: int, l: int, c: int) -> float:
        if l <= 1 or c <= 1:
            return 0.0
        return min(max(size[a + k] + f(a + k, l - k, c - 1), f(a, k, c)) for k in opt(l, c))

    old = sys.getrecursionlimit()
    sys.setrecursionlimit(max(old, 50 * (N + M) + 1000))
    try:
        return f(0, N + 1, M)
    finally:
        sys.setrecursionlimit(old)


def counts(acts: np.ndarray) -> dict:
    """advances (forward steps), stores, restores, reverses, peak slot depth."""
    a = np.asarray(acts)
    adv = a[a[:, 0] == ADVANCE]
    st = a[a[:, 0] == STORE]
    return {
        "advances": int((adv[:, 2] - adv[:, 1]).sum()) if len(adv) else 0,
        "stores": int(len(st)),
        "restores": int((a[:, 0] == RESTORE).sum()),
        "reverses": int((a[:, 0] == REVERSE).sum()),
        "max_slot": int(st[:, 2].max()) if len(st) else 0,
    }


def brute_force_min_writes(N: int, M: int) -> tuple[int, int]:
    """Exhaustive search over every schedule (tiny N): the fewest forward steps and, among
    schedules with that many, the fewest stores (lexicographic shortest path)."""
    start = (0, frozenset([0]), N)
    dist = {start: (0, 0)}
    heap = [((0, 0), 0, frozenset([0]), N)]
    while heap:
        d, wm, S, nr = heapq.heappop(heap)
        if dist.get((wm, S, nr), (1 << 60, 0)) < d:
            continue
        if nr == 0:
            return d
        moves = []
        if wm == nr:
            moves.append(((0, 0), wm, S, nr - 1))
        if wm < nr:
            moves.append(((1, 0), wm + 1, S, nr))
        if wm not in S and len(S) < M:
            moves.append(((0, 1), wm, S | {wm}, nr))
        for s_ in S:
            if s_ != wm:
                moves.append(((0, 0), s_, S, nr))
            if s_ != 0:
                moves.append(((0, 0), wm, S - {s_}, nr))
        for (da, dw), w2, S2, n2 in moves:
            key = (w2, S2, n2)
            nd = (d[0] + da, d[1] + dw)
            if nd < dist.get(key, (1 << 60, 0)):
                dist[key] = nd
                heapq.heappush(heap, (nd, w2, S2, n2))
    raise RuntimeError("no schedule found")


def brute_force_min(N: int, M: int) -> int:
    """Exhaustive search: fewest forward steps over all schedules that run the
    reverse steps N..1 with at most M checkpoints held (x_0 counts as one)."""
    start = (0, frozenset([0]), N)        # (working state, stored set, next reverse)
    dist = {start: 0}
    heap = [(0, 0, frozenset([0]), N)]
    while heap:
        d, wm, S, nr = heapq.heappop(heap)
        if dist.get((wm, S, nr), 1 << 60) < d:
            continue
        if nr == 0:
            return d
        moves = []
        if wm == nr:
            moves.append((0, wm, S, nr - 1))
        if wm < nr:
            moves.append((1, wm + 1, S, nr))
        if wm not in S and len(S) < M:
            moves.append((0, wm, S | {wm}, nr))
        for s in S:
            if s != wm:
                moves.append((0, s, S, nr))
            if s != 0:
                moves.append((0, wm, S - {s}, nr))
        for cost, w2, S2, n2 in moves:
            key = (w2, S2, n2)
            nd = d + cost
            if nd < dist.get(key, 1 << 60):
                dist[key] = nd
                heapq.heappush(heap, (nd, w2, S2, n2))
    raise RuntimeError("no schedule found")
