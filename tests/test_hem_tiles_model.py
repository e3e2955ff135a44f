"""CPU model of the tiled matching pass (one workgroup per tile of rows).

The vertices are cut into tiles of T consecutive indices.  Every tile runs
rounds of its own (the rounds of the data-parallel matching: a ready vertex
points to its heaviest undecided higher neighbour, lowest index on ties, and
matches when that neighbour's smallest undecided lower edge-neighbour is the
vertex itself), with round stamps, ready counters and worklists private to the
tile.  Decisions reach other tiles only through one published word per vertex
(partner + 2, or 1 for a singleton), which another tile may read late:

* a vertex with lower edge-neighbours in lower tiles starts "pending": it
  counts as undecided but is neither matched inside its tile nor allowed to
  choose until those neighbours read decided; their words then say whether
  one of them took it, and the vertex is settled (free, or decided);
* a vertex whose target lies in a higher tile takes it once the target's lower
  edge-neighbours below it read decided and none of them names the target.

This model runs those steps with tiles advancing at random speeds, words that
become visible to other tiles after random delays (at once to the writing
tile), random visit orders and random deferrals, and is compared with the
oracle's sequential matching bit for bit.  It shares no code with either.
"""
import numpy as np
import pytest

import oracle
from paper_2007_00056_amd import problems as P

UND = 1 << 30      # published word before a decision; LDS stamp "undecided"
PEND = UND - 1     # LDS stamp: pending


def tiled_model(a, T, rng, delay=3, speed=0.7, defer=0.2, lazy=False):
    """lazy: the reads of the LDS-record tiles: a choice reads out-of-tile
    words only for entries before its first undecided in-tile entry, and a
    target of the tile that is no longer pending has its lower-tile
    neighbours taken as decided without reading their words."""
    n, rp, ci, v = a.n, a.row_ptr, a.col, a.val

    def has_edge(u, w):  # u < w: entry (u, w) stored in row u and non-zero
        lo, hi = rp[u], rp[u + 1]
        k = lo + np.searchsorted(ci[lo:hi], w)
        return k < hi and ci[k] == w and v[k] != 0.0

    lower = [[x for x in ci[rp[y]:rp[y + 1]] if x < y and has_edge(x, y)] for y in range(n)]
    higher = []
    for u in range(n):
        hs = [(-abs(v[e]), ci[e]) for e in range(rp[u], rp[u + 1]) if ci[e] > u and v[e] != 0.0]
        higher.append([j for _, j in sorted(hs)])
    tile = lambda x: x // T
    nt = (n + T - 1) // T
    hist = [[] for _ in range(n)]  # published words: (time visible to other tiles, value, writer tile)
    now = [0]

    def word(x, t):
        val = UND
        for vis, w, wt in hist[x]:
            if wt == t or vis <= now[0]:
                val = w
        return val

    def publish(x, partner, t):
        hist[x].append((now[0] + int(rng.integers(0, delay + 1)), partner + 2, t))

    mate = np.full(n, -2)
    stamp = {}
    lcnt = {}
    lists = []
    ndec = [0] * nt
    rnd = [2] * nt
    for t in range(nt):
        lo, hi = t * T, min(n, (t + 1) * T)
        for y in range(lo, hi):
            cross = [x for x in lower[y] if x < lo]
            stamp[y] = PEND if cross else UND
            lcnt[y] = len(lower[y]) - len(cross)
        lists.append([y for y in range(lo, hi) if lcnt[y] == 0])

    for step in range(200 * n + 1000):
        if all(ndec[t] == min(n, (t + 1) * T) - t * T for t in range(nt)):
            break
        now[0] = step
        for t in range(nt):
            lo, hi = t * T, min(n, (t + 1) * T)
            if ndec[t] == hi - lo or rng.random() > speed:
                continue
            r = rnd[t]
            nxt = []

            def get(x):
                if lo <= x < hi:
                    return stamp[x]
                return UND if word(x, t) == UND else -1

            def release(x):
                for y in higher[x]:
                    if lo <= y < hi:
                        lcnt[y] -= 1
                        if lcnt[y] == 0:
                            nxt.append(y)

            def settle(y, taken):
                if stamp[y] == PEND:
                    if taken:
                        stamp[y] = r - 1
                        ndec[t] += 1
                        release(y)
                        return "gone"
                    stamp[y] = UND
                    return "free"
                return "free" if stamp[y] == UND else "gone"

            for u in rng.permutation(lists[t]):
                u = int(u)
                if stamp[u] < r:
                    continue  # decided earlier: stale entry
                if rng.random() < defer:
                    nxt.append(u)
                    continue
                if stamp[u] == PEND:
                    ws = [word(x, t) for x in lower[u] if x < lo]
                    if UND in ws:
                        nxt.append(u)
                        continue
                    if settle(u, u + 2 in ws) != "free":
                        continue
                if lazy:
                    fin = next((k for k, j in enumerate(higher[u]) if lo <= j < hi and stamp[j] >= r),
                               len(higher[u]))
                    best = next((j for k, j in enumerate(higher[u])
                                 if (k == fin) or (k < fin and not lo <= j < hi and get(j) >= r)), -1)
                else:
                    best = next((j for j in higher[u] if get(j) >= r), -1)
                if best < 0:
                    stamp[u] = r
                    mate[u] = -1
                    hist[u].append((now[0] + int(rng.integers(0, delay + 1)), 1, t))
                    ndec[t] += 1
                    release(u)
                    continue
                back, named = -1, False
                settled = lazy and lo <= best < hi and stamp[best] != PEND
                for x in lower[best]:
                    if settled and x < lo:
                        continue
                    if lo <= x < hi:
                        if stamp[x] >= r:
                            back = x
                            break
                    else:
                        w = word(x, t)
                        if w == UND:
                            back = x
                            break
                        named |= w == best + 2
                if back != u:
                    nxt.append(u)
                    continue
                if lo <= best < hi:
                    if stamp[best] == PEND and settle(best, named) != "free":
                        nxt.append(u)
                        continue
                    stamp[u] = stamp[best] = r
                    mate[u], mate[best] = best, u
                    publish(best, u, t)
                    publish(u, best, t)
                    ndec[t] += 2
                    release(u)
                    release(best)
                else:
                    if named:
                        nxt.append(u)
                        continue
                    stamp[u] = r
                    mate[u], mate[best] = best, u
                    publish(best, u, t)
                    publish(u, best, t)
                    ndec[t] += 1
                    release(u)
            lists[t] = nxt
            rnd[t] = r + 1
    assert all(ndec[t] == min(n, (t + 1) * T) - t * T for t in range(nt)), "did not finish"
    assert np.all(mate >= -1)
    return mate


@pytest.mark.parametrize("seed", range(30))
def test_tiles_equal_sequential_random(seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(2, 80))
    a = P.random_symmetric_pattern(n, float(rng.uniform(0.03, 0.4)), seed, weights=(1, 2, 3)[: 1 + seed % 3],
                                   nonsym_values=seed % 2 == 1, explicit_zeros=0.15 * (seed % 4 == 0))
    want = oracle.hem_pass(a)
    for T in (1, 3, int(rng.integers(2, n + 1)), n):
        for lazy in (False, True):
            got = tiled_model(a, T, rng, delay=int(rng.integers(0, 6)), lazy=lazy)
            np.testing.assert_array_equal(got, want, err_msg=f"n={n} T={T} lazy={lazy}")


@pytest.mark.parametrize("make", [lambda: P.poisson3d(6, 5, 4), lambda: P.convdiff3d(5),
                                  lambda: P.lognormal_diffusion3d(5, 2), lambda: P.poisson2d(12, 9)])
def test_tiles_equal_sequential_grids_all_levels(make):
    a = make()
    rng = np.random.default_rng(7)
    for _ in range(4):  # follow the passes down the hierarchy
        want = oracle.hem_pass(a)
        for T in (7, 30, max(1, a.n // 3)):
            for lazy in (False, True):
                np.testing.assert_array_equal(tiled_model(a, T, rng, lazy=lazy), want,
                                              err_msg=f"n={a.n} T={T} lazy={lazy}")
        agg, nc = oracle.number(want)
        if nc == a.n or nc < 2:
            break
        rp, ci, cv = oracle.rap(a, agg, nc)
        a = P.CSR(nc, rp, ci, cv)
