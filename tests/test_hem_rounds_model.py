"""CPU model of the data-parallel matching rounds used by the GPU kernels.

Algorithm 2 visits vertices in ascending order, so it equals the greedy
matching over edges {u < w} (a_uw stored in row u and non-zero) taken in
increasing key (u, -|a_uw|, w).  Greedy matching in a strict total edge order
is reproduced exactly by rounds of locally-dominant edges: every undecided
vertex points along its smallest-key edge to an undecided neighbour, mutual
pointers are matched, and a vertex without undecided neighbours is a
singleton.  Under this key a vertex points to its smallest undecided lower
neighbour if it has one, else to its heaviest undecided higher neighbour
(lowest index on ties).

Only "ready" vertices (no undecided lower neighbour) can start a match, so the
GPU keeps a worklist of ready vertices and a per-vertex count of undecided
lower neighbours; decisions carry the round number so every read in a round
sees the state at the start of that round.  This model runs those exact steps
sequentially and is compared with the oracle bit for bit.  It shares no code
with either implementation.
"""
import numpy as np
import pytest

import oracle
from paper_2007_00056_amd import problems as P

UNDECIDED = 1 << 30


def rounds_model(a):
    n, rp, ci, v = a.n, a.row_ptr, a.col, a.val

    def has_edge(u, w):  # u < w: entry (u, w) stored in row u and non-zero
        lo, hi = rp[u], rp[u + 1]
        k = lo + np.searchsorted(ci[lo:hi], w)
        return k < hi and ci[k] == w and v[k] != 0.0

    dec = np.full(n, UNDECIDED)
    mate = np.full(n, -1)
    lcnt = np.zeros(n, dtype=int)
    for y in range(n):
        for e in range(rp[y], rp[y + 1]):
            if ci[e] < y and has_edge(ci[e], y):
                lcnt[y] += 1
    work = [y for y in range(n) if lcnt[y] == 0]
    r = 0
    rounds = 0
    while work:
        nxt, newly = [], []
        for u in work:
            best, k = -1, -1.0
            for e in range(rp[u], rp[u + 1]):
                j = ci[e]
                if j > u and v[e] != 0.0 and dec[j] >= r and abs(v[e]) > k:
                    best, k = j, abs(v[e])
            if best < 0:
                dec[u] = r
                newly.append(u)
                continue
            s = -1
            for e in range(rp[best], rp[best + 1]):
                x = ci[e]
                if x < best and dec[x] >= r and has_edge(x, best):
                    s = x
                    break
            if s == u:
                dec[u] = dec[best] = r
                mate[u], mate[best] = best, u
                newly += [u, best]
            else:
                nxt.append(u)
        for x in newly:
            for e in range(rp[x], rp[x + 1]):
                y = ci[e]
                if y > x and v[e] != 0.0:
                    lcnt[y] -= 1
                    if lcnt[y] == 0 and dec[y] > r:
                        nxt.append(y)
        work = nxt
        r += 1
        rounds += 1
    assert np.all(dec < UNDECIDED)
    return mate, rounds


def merged_rounds_model(a, rng=None, delay=0.0):
    """One pass per round: the thread that decides a vertex also decrements the
    counters of its higher neighbours and queues newly ready ones for the next
    round; queued vertices that were decided meanwhile (as a match target) are
    skipped.  With `rng`, each round's list is processed in random order and a
    fraction `delay` of ready vertices is deferred to the next round, which
    models arbitrary scheduling: the result must not depend on it."""
    n, rp, ci, v = a.n, a.row_ptr, a.col, a.val

    def has_edge(u, w):
        lo, hi = rp[u], rp[u + 1]
        k = lo + np.searchsorted(ci[lo:hi], w)
        return k < hi and ci[k] == w and v[k] != 0.0

    dec = np.full(n, UNDECIDED)
    mate = np.full(n, -1)
    lcnt = np.zeros(n, dtype=int)
    for y in range(n):
        for e in range(rp[y], rp[y + 1]):
            if ci[e] < y and has_edge(ci[e], y):
                lcnt[y] += 1
    work = [y for y in range(n) if lcnt[y] == 0]
    r = 0

    def release(x, nxt):
        for e in range(rp[x], rp[x + 1]):
            y = ci[e]
            if y > x and v[e] != 0.0:
                lcnt[y] -= 1
                if lcnt[y] == 0:
                    nxt.append(y)

    while work:
        nxt = []
        if rng is not None:
            work = list(rng.permutation(work))
        for u in work:
            if dec[u] < r:  # decided in an earlier round: stale entry
                continue
            if rng is not None and rng.random() < delay:
                nxt.append(u)
                continue
            best, k = -1, -1.0
            for e in range(rp[u], rp[u + 1]):
                j = ci[e]
                if j > u and v[e] != 0.0 and dec[j] >= r and abs(v[e]) > k:
                    best, k = j, abs(v[e])
            if best < 0:
                dec[u] = r
                release(u, nxt)
                continue
            s = -1
            for e in range(rp[best], rp[best + 1]):
                x = ci[e]
                if x < best and dec[x] >= r and has_edge(x, best):
                    s = x
                    break
            if s == u:
                dec[u] = dec[best] = r
                mate[u], mate[best] = best, u
                release(u, nxt)
                release(best, nxt)
            else:
                nxt.append(u)
        work = nxt
        r += 1
        assert r <= n + 2
    assert np.all(dec < UNDECIDED)
    return mate, r


@pytest.mark.parametrize("seed", range(30))
def test_merged_rounds_any_schedule_equal_sequential(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 70))
    a = P.random_symmetric_pattern(n, float(rng.uniform(0.02, 0.4)), seed, weights=(1, 2, 3)[: 1 + seed % 3],
                                   nonsym_values=seed % 2 == 1, explicit_zeros=0.15 * (seed % 4 == 0))
    want = oracle.hem_pass(a)
    np.testing.assert_array_equal(merged_rounds_model(a)[0], want)
    np.testing.assert_array_equal(merged_rounds_model(a, rng, delay=0.3)[0], want)


def test_merged_rounds_grids():
    for a in (P.poisson3d(9, 7, 6), P.convdiff3d(7), P.lognormal_diffusion3d(7, 3)):
        want = oracle.hem_pass(a)
        np.testing.assert_array_equal(merged_rounds_model(a)[0], want)
        np.testing.assert_array_equal(merged_rounds_model(a, np.random.default_rng(1), 0.2)[0], want)


@pytest.mark.parametrize("seed", range(40))
def test_rounds_equal_sequential_random(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 60))
    a = P.random_symmetric_pattern(n, float(rng.uniform(0.02, 0.4)), seed, weights=(1, 2, 3)[: 1 + seed % 3],
                                   nonsym_values=seed % 2 == 1, explicit_zeros=0.15 * (seed % 4 == 0))
    mate, _ = rounds_model(a)
    np.testing.assert_array_equal(mate, oracle.hem_pass(a))


@pytest.mark.parametrize("make", [lambda: P.poisson2d(13, 9), lambda: P.poisson3d(7, 6, 5), lambda: P.convdiff3d(6),
                                  lambda: P.lognormal_diffusion3d(6, 1)])
def test_rounds_equal_sequential_grids_all_levels(make):
    a = make()
    for _ in range(6):  # follow the passes down the hierarchy
        mate, rounds = rounds_model(a)
        np.testing.assert_array_equal(mate, oracle.hem_pass(a))
        agg, nc = oracle.number(mate)
        if nc == a.n or nc < 2:
            break
        rp, ci, cv = oracle.rap(a, agg, nc)
        a = P.CSR(nc, rp, ci, cv)
