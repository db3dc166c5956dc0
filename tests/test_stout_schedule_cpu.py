"""The checkpoint schedule of the reverse pass through a stout chain
(lgt_stout_schedule, host code of the library; no GPU).

Pinned against an independent exhaustive search: Dijkstra over every
strategy of a more general model -- any subset of at most s levels kept by
the forward sweep, any level recomputed from any available one into a slot
or into a one-use transient, slots dropped at any time -- which the DP's
schedule (stack-ordered splits) must match in cost on every small chain.
Also the closed forms n(n-1)/2 (no slot) and 0 (n - 1 slots)."""
import heapq
import itertools

import pytest

import paper_2602_20516_amd as lgt


def exhaustive(n: int, s: int) -> int:
    """Fewest recomputed smearing passes over all strategies (Dijkstra)."""
    if n <= 1:
        return 0
    dist, pq = {}, []
    for k in range(min(s, n - 1) + 1):
        for kept in itertools.combinations(range(1, n), k):
            st = (frozenset(kept), n)  # (kept levels, next adjoint level)
            dist[st] = 0
            pq.append((0, st))
    heapq.heapify(pq)
    while pq:
        d, (kept, lev) = heapq.heappop(pq)
        if d > dist[(kept, lev)]:
            continue
        if lev == 0:
            return d
        avail = [0] + sorted(kept)
        moves = []
        if lev - 1 == 0 or lev - 1 in kept:  # adjoint of level lev with U_{lev-1} at hand
            moves.append(((kept, lev - 1), 0))
        for i in avail:  # U_{lev-1} recomputed from U_i into the transient
            if i < lev - 1:
                moves.append(((kept, lev - 1), lev - 1 - i))
        if len(kept) < s:  # a new checkpoint U_j from U_i
            for i in avail:
                for j in range(i + 1, lev):
                    if j not in kept:
                        moves.append(((kept | {j}, lev), j - i))
        for j in kept:
            moves.append(((kept - {j}, lev), 0))
        for st, c in moves:
            if d + c < dist.get(st, float("inf")):
                dist[st] = d + c
                heapq.heappush(pq, (d + c, st))
    raise AssertionError("unreachable")


@pytest.mark.parametrize("n", range(0, 8))
def test_schedule_is_optimal(n):
    for s in range(0, 5):
        got = lgt.stout_schedule(n, s)
        assert got["recompute_passes"] == exhaustive(n, s), (n, s)


@pytest.mark.parametrize("n", [1, 2, 5, 17, 64, 256])
def test_closed_forms(n):
    assert lgt.stout_schedule(n, 0) == {"recompute_passes": n * (n - 1) // 2, "checkpoints": []}
    full = lgt.stout_schedule(n, n - 1)
    assert full["recompute_passes"] == 0
    assert full["checkpoints"] == list(range(1, n))
    assert lgt.stout_schedule(n, n + 10)["recompute_passes"] == 0  # extra slots unused


@pytest.mark.parametrize("n", [8, 40, 128])
def test_checkpoints_valid_and_cost_monotone(n):
    prev = None
    for s in range(0, 12):
        r = lgt.stout_schedule(n, s)
        cp = r["checkpoints"]
        assert len(cp) <= s and cp == sorted(set(cp)) and all(1 <= c < n for c in cp)
        if prev is not None:
            assert r["recompute_passes"] <= prev
        prev = r["recompute_passes"]


def test_sqrt_storage_is_linear_recompute():
    """With about sqrt(n) slots the reverse pass recomputes O(n) passes."""
    for n in (64, 144, 256):
        s = int(round(n ** 0.5))
        assert lgt.stout_schedule(n, s)["recompute_passes"] <= 2 * n


def test_invalid_arguments():
    for n, s in ((-1, 0), (257, 3), (5, -1)):
        with pytest.raises(lgt.LGTError):
            lgt.stout_schedule(n, s)
