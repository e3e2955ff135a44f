"""Pins of the oracle's aggregation (Algorithm 2) and Galerkin product (Section 2.1.1).

Each test ties the oracle to something other than itself: the worked example
printed in the paper, hand-derived matchings, an independent formulation of the
matching (greedy over the sorted edge list), scipy's sparse product and
algebraic invariants.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2007_00056_amd import problems as P


def prolongation(agg, nc):
    n = agg.size
    return sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, nc))


# ---------------------------------------------------------------- worked example

def test_worked_example_matches_paper(golden):
    g = golden("hem_worked_example.txt")
    A = np.array(g["A"])
    a = P.from_dense(A)
    mate = oracle.hem_pass(a)
    agg, nc = oracle.number(mate)
    Pm = np.zeros((6, nc))
    Pm[np.arange(6), agg] = 1.0
    np.testing.assert_array_equal(Pm, np.array(g["P"]))
    crp, cci, cv = oracle.rap(a, agg, nc)
    Ac = sp.csr_matrix((cv, cci, crp), shape=(nc, nc)).toarray()
    np.testing.assert_array_equal(Ac, np.array(g["Ac"]))


def test_worked_example_diagonal_identity(golden):
    # (A_c)_kk = a_ij + a_ji + a_ii + a_jj for an aggregated pair (i, j)
    A = np.array(golden("hem_worked_example.txt")["A"])
    a = P.from_dense(A)
    mate = oracle.hem_pass(a)
    agg, nc = oracle.number(mate)
    crp, cci, cv = oracle.rap(a, agg, nc)
    Ac = sp.csr_matrix((cv, cci, crp), shape=(nc, nc)).toarray()
    for i in range(6):
        j = mate[i]
        if j > i:
            assert Ac[agg[i], agg[i]] == A[i, j] + A[j, i] + A[i, i] + A[j, j]


# ---------------------------------------------------------------- hand-derived cases

def chain(n):
    d = np.full(n, 2.0)
    o = np.full(n - 1, -1.0)
    return P.from_dense(np.diag(d) + np.diag(o, 1) + np.diag(o, -1))


@pytest.mark.parametrize("n", [1, 2, 5, 8, 9])
def test_chain_pairs_in_order(n):
    mate = oracle.hem_pass(chain(n))
    want = np.full(n, -1)
    for i in range(0, n - 1, 2):
        want[i], want[i + 1] = i + 1, i
    np.testing.assert_array_equal(mate, want)
    agg, nc = oracle.number(mate)
    assert nc == (n + 1) // 2
    np.testing.assert_array_equal(agg, np.arange(n) // 2)


def test_tie_goes_to_lowest_index():
    # vertex 0 has equal-weight neighbours 1, 2, 3 -> picks 1; 2 then picks 3
    A = np.array([[3, -1, -1, -1], [-1, 3, 0, 0], [-1, 0, 3, -1], [-1, 0, -1, 3]], float)
    mate = oracle.hem_pass(P.from_dense(A))
    np.testing.assert_array_equal(mate, [1, 0, 3, 2])


def test_heaviest_by_absolute_value_and_zero_is_not_an_edge():
    A = np.array([[5, 1, -3, 0], [1, 5, 0, 2], [-3, 0, 5, 0], [0, 2, 0, 5]], float)
    a = P.from_dense(A)
    np.testing.assert_array_equal(oracle.hem_pass(a), [2, 3, 0, 1])
    # stored zero: the only neighbour of 0 is an explicit zero -> singleton
    a2 = P.CSR(2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32), np.array([1.0, 0.0, 0.0, 1.0]))
    np.testing.assert_array_equal(oracle.hem_pass(a2), [-1, -1])


def test_unassigned_check_uses_current_state():
    # 0 takes 2 (heavier); 1's heavy neighbour 2 is taken, so 1 falls to 3
    A = np.array([[4, 1, 3, 0], [1, 4, 2, 1], [3, 2, 4, 0], [0, 1, 0, 4]], float)
    np.testing.assert_array_equal(oracle.hem_pass(P.from_dense(A)), [2, 3, 0, 1])


def test_poisson2d_4x4_two_passes_make_boxes():
    a = P.poisson2d(4)
    m1 = oracle.hem_pass(a)
    # pass 1 pairs along x: (0,1),(2,3),(4,5),...
    np.testing.assert_array_equal(m1, np.arange(16) ^ 1)
    agg1, nc1 = oracle.number(m1)
    crp, cci, cv = oracle.rap(a, agg1, nc1)
    a1 = P.CSR(nc1, crp, cci, cv)
    D = sp.csr_matrix((cv, cci, crp), shape=(nc1, nc1)).toarray()
    # coarse 2x4 grid: x-coupling -1, y-coupling -2, diagonal 4+4-1-1
    assert D[0, 1] == -1 and D[0, 2] == -2 and D[0, 0] == 6
    m2 = oracle.hem_pass(a1)
    agg2, nc2 = oracle.number(m2)
    comp = agg2[agg1]
    x, y = np.arange(16) % 4, np.arange(16) // 4
    np.testing.assert_array_equal(comp, (x // 2) + 2 * (y // 2))
    assert nc2 == 4


def test_poisson3d_second_pass_prefers_y_on_y_z_tie():
    a = P.poisson3d(4)
    h = oracle.Hierarchy(a, max_coarse_rows=1, max_levels=2)
    agg = h.level(0).agg
    i = np.arange(64)
    x, y, z = i % 4, (i // 4) % 4, i // 16
    np.testing.assert_array_equal(agg, (x // 2) + 2 * ((y // 2) + 2 * z))


# ---------------------------------------------------------------- independent formulation

def greedy_sorted_edges(A):
    """Greedy matching over edges {i<j} (a_ij stored in row i, non-zero), taken in
    increasing key (i, -|a_ij|, j); an edge is accepted iff both ends are free."""
    n = A.n
    edges = []
    for i in range(n):
        for e in range(A.row_ptr[i], A.row_ptr[i + 1]):
            j = int(A.col[e])
            if j > i and A.val[e] != 0.0:
                edges.append((i, -abs(A.val[e]), j))
    edges.sort()
    mate = [-1] * n
    for i, _, j in edges:
        if mate[i] < 0 and mate[j] < 0:
            mate[i], mate[j] = j, i
    return np.array(mate)


@pytest.mark.parametrize("seed", range(25))
def test_matching_equals_sorted_edge_greedy(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 40))
    a = P.random_symmetric_pattern(n, float(rng.uniform(0.05, 0.5)), seed, weights=(1, 2),
                                   nonsym_values=bool(seed % 2), explicit_zeros=0.1 * (seed % 3 == 0))
    np.testing.assert_array_equal(oracle.hem_pass(a), greedy_sorted_edges(a))


def test_matching_is_maximal_and_consistent():
    a = P.random_symmetric_pattern(60, 0.1, 7, weights=(1, 2, 3))
    mate = oracle.hem_pass(a)
    S = a.to_scipy()
    for i in range(a.n):
        if mate[i] >= 0:
            assert mate[mate[i]] == i and mate[i] != i and S[i, mate[i]] != 0
        else:  # a singleton has no free neighbour left (maximality)
            nb = [j for j in S[[i]].indices if j != i and S[i, j] != 0]
            assert all(mate[j] >= 0 for j in nb)


# ---------------------------------------------------------------- numbering + Galerkin

def test_numbering_follows_minimum_index():
    a = P.random_symmetric_pattern(50, 0.15, 3)
    mate = oracle.hem_pass(a)
    agg, nc = oracle.number(mate)
    first = np.full(nc, -1)
    for i in range(a.n):
        if first[agg[i]] < 0:
            first[agg[i]] = i
    assert np.all(np.diff(first) > 0)  # ids ordered by minimum fine index
    assert np.bincount(agg, minlength=nc).max() <= 2
    assert set(agg) == set(range(nc))


@pytest.mark.parametrize("seed", range(6))
def test_rap_equals_scipy_product_integer_values(seed):
    a = P.random_symmetric_pattern(40, 0.2, seed, weights=(1, 2, 3), nonsym_values=seed % 2 == 1)
    agg, nc = oracle.number(oracle.hem_pass(a))
    crp, cci, cv = oracle.rap(a, agg, nc)
    Pm = prolongation(agg, nc)
    want = (Pm.T @ a.to_scipy() @ Pm).toarray()
    got = sp.csr_matrix((cv, cci, crp), shape=(nc, nc)).toarray()
    np.testing.assert_array_equal(got, want)  # integer sums are exact in any order
    # pattern: every (I, agg(j)) reached by a stored entry, zero sums included
    pat = (Pm.T @ (a.to_scipy() != 0).astype(float) @ Pm).toarray() != 0
    stored = (Pm.T @ sp.csr_matrix((np.ones(a.nnz), a.col, a.row_ptr), shape=(a.n, a.n)) @ Pm).toarray() != 0
    got_pat = sp.csr_matrix((np.ones_like(cv), cci, crp), shape=(nc, nc)).toarray() != 0
    np.testing.assert_array_equal(got_pat, stored)
    assert np.all(pat <= got_pat)
    for I in range(nc):
        assert np.all(np.diff(cci[crp[I]:crp[I + 1]]) > 0)


def test_rap_real_values_close_to_scipy_and_symmetric():
    a = P.lognormal_diffusion3d(6, seed=3)
    agg, nc = oracle.number(oracle.hem_pass(a))
    crp, cci, cv = oracle.rap(a, agg, nc)
    Pm = prolongation(agg, nc)
    want = (Pm.T @ a.to_scipy() @ Pm).toarray()
    got = sp.csr_matrix((cv, cci, crp), shape=(nc, nc)).toarray()
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-13)
    scale = np.abs(want).max()
    assert np.abs(got - got.T).max() <= 8 * np.finfo(float).eps * scale
    # row sums: A_c 1 = P^T A 1
    np.testing.assert_allclose(got.sum(axis=1), Pm.T @ (a.to_scipy() @ np.ones(a.n)), rtol=1e-12, atol=1e-12)
    # SPD is preserved
    assert np.linalg.eigvalsh(0.5 * (got + got.T)).min() > 0


def test_rap_sum_order_is_member_then_column():
    # coarse entries whose float value depends on the summation order
    s = 2.0 ** -53
    A = np.array([[1.0, s, s, s], [s, s, 1.0, s], [s, 1.0, 1.0, 0], [s, s, 0, 1.0]])
    a = P.from_dense(A)
    agg = np.array([0, 0, 1, 1], np.int32)
    crp, cci, cv = oracle.rap(a, agg, 2)
    D = sp.csr_matrix((cv, cci, crp), shape=(2, 2)).toarray()
    # (0,0): members 0 then 1, columns ascending: a00, a01, a10, a11
    assert D[0, 0] == ((1.0 + s) + s) + s == 1.0
    assert (s + s + s) + 1.0 != 1.0  # another order gives another value
    # (0,1): a02, a03, a12, a13
    assert D[0, 1] == ((s + s) + 1.0) + s
    assert D[0, 1] != ((1.0 + s) + s) + s
    # (1,0): members 2 then 3: a20, a21, a30, a31
    assert D[1, 0] == ((s + 1.0) + s) + s


def test_hierarchy_partition_and_sizes():
    a = P.poisson3d(16, 12, 10)
    h = oracle.Hierarchy(a)
    for k in range(h.nlevels - 1):
        L, Cn = h.level(k), h.level(k + 1)
        counts = np.bincount(L.agg, minlength=Cn.n)
        assert counts.min() >= 1 and counts.max() <= 4 and counts.sum() == L.n
    assert h.level(h.nlevels - 1).n <= 64


def test_brute_force_tiny_graphs_all_weight_assignments():
    # every weight assignment in {1,2} on the edges of a 4-cycle plus a chord
    edges = [(0, 1), (1, 2), (2, 3), (0, 3), (0, 2)]
    for ws in itertools.product((1.0, 2.0), repeat=len(edges)):
        A = np.eye(4) * 10
        for (i, j), w in zip(edges, ws):
            A[i, j] = A[j, i] = -w
        a = P.from_dense(A)
        np.testing.assert_array_equal(oracle.hem_pass(a), greedy_sorted_edges(a))


# ---------------------------------------------------------------- edge-based HEM (Algorithm 3)

def edges_of(a):
    """Undirected edges {i, j} with the heavier of |a_ij|, |a_ji| (stored, non-zero)."""
    w = {}
    for i in range(a.n):
        for e in range(a.row_ptr[i], a.row_ptr[i + 1]):
            j = int(a.col[e])
            if j != i and a.val[e] != 0.0:
                k = (min(i, j), max(i, j))
                w[k] = max(w.get(k, 0.0), abs(a.val[e]))
    return w


def random_graph(n, seed, distinct=True, nonsym=False):
    rng = np.random.default_rng(seed)
    mask = np.triu(rng.random((n, n)) < 0.12, 1)
    vals = np.zeros((n, n))
    k = int(mask.sum())
    wts = rng.permutation(np.arange(1, 2 * k + 1))[:k] if distinct else rng.integers(1, 3, k)
    vals[mask] = -wts.astype(float)
    vals = vals + vals.T
    if nonsym:
        m2 = mask.T & (rng.random((n, n)) < 0.5)
        vals[m2] *= 0.5
    np.fill_diagonal(vals, np.abs(vals).sum(axis=1) + 1.0)
    return P.from_dense(vals)


@pytest.mark.parametrize("seed", range(6))
def test_ehem_is_maximal_and_each_unmatched_edge_is_blocked_by_a_heavier_match(seed):
    # under a strict edge order this characterises the greedy matching uniquely
    a = random_graph(40, seed, distinct=seed % 2 == 0, nonsym=seed >= 4)
    mate = oracle.ehem_pass(a)
    W = edges_of(a)

    def key(i, j):
        lo, hi = min(i, j), max(i, j)
        return (-W[(lo, hi)], lo, hi)

    for i in range(a.n):
        if mate[i] >= 0:
            assert mate[mate[i]] == i and (min(i, mate[i]), max(i, mate[i])) in W
    for (i, j) in W:
        if mate[i] == j:
            continue
        assert mate[i] >= 0 or mate[j] >= 0, (i, j)  # maximal
        blockers = [key(x, mate[x]) for x in (i, j) if mate[x] >= 0]
        assert min(blockers) < key(i, j), (i, j)


@pytest.mark.parametrize("seed", range(4))
def test_ehem_is_invariant_to_the_numbering(seed):
    # Section 2.1.1: with distinct weights the aggregates do not depend on the
    # order of the unknowns
    a = random_graph(50, 100 + seed, distinct=True)
    dense = a.to_scipy().toarray()
    perm = np.random.default_rng(seed).permutation(a.n)
    b = P.from_dense(dense[np.ix_(perm, perm)])
    ma, mb = oracle.ehem_pass(a), oracle.ehem_pass(b)
    pairs_a = {frozenset((i, int(ma[i]))) for i in range(a.n) if ma[i] >= 0}
    pairs_b = {frozenset((int(perm[i]), int(perm[mb[i]]))) for i in range(a.n) if mb[i] >= 0}
    assert pairs_a == pairs_b


@pytest.mark.parametrize("make", [lambda: P.poisson2d(9, 7), lambda: P.poisson3d(6, 5, 4)])
def test_ehem_equals_node_based_on_equal_weights(make):
    # equal weights leave the index order (smaller endpoint, then larger), which
    # is the node-based visiting order
    a = make()
    np.testing.assert_array_equal(oracle.ehem_pass(a), oracle.hem_pass(a))


def test_ehem_hierarchy_and_solve():
    a = P.lognormal_diffusion3d(9, 3)
    h = oracle.Hierarchy(a, hem=1)
    assert h.nlevels >= 2
    b = P.rhs_uniform(a.n, 2)
    x, info = h.solve(b, rtol=1e-10)
    assert info["status"] == oracle.OK
    assert np.linalg.norm(a.to_scipy() @ x - b) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-9)
    with pytest.raises(oracle.OracleError):
        oracle.Hierarchy(a, hem=2)


# ---------------------------------------------------------------- matching from the last index

@pytest.mark.parametrize("n", [1, 2, 5, 8, 9])
def test_desc_chain_pairs_from_the_end(n):
    # visiting from the last vertex pairs (n-1, n-2), (n-3, n-4), ... and an odd
    # chain leaves vertex 0 alone
    mate = oracle.hem_pass_desc(chain(n))
    want = np.full(n, -1)
    for i in range(n - 1, 0, -2):
        want[i], want[i - 1] = i - 1, i
    np.testing.assert_array_equal(mate, want)


def test_desc_tie_goes_to_highest_index():
    # vertex 3 is visited first; its neighbours 0 and 1 weigh the same -> it takes 1,
    # and 2 then still finds 0 free.  Taking 0 would leave 1 and 2 alone.
    A = np.array([[3, 0, -1, -1], [0, 3, 0, -1], [-1, 0, 3, 0], [-1, -1, 0, 3]], float)
    np.testing.assert_array_equal(oracle.hem_pass_desc(P.from_dense(A)), [2, 3, 0, 1])


def test_desc_heaviest_and_current_state():
    # 3 takes 1 (heavier than 2); 2's only free neighbour is then 0
    A = np.array([[4, 0, 1, 0], [0, 4, 1, 3], [1, 1, 4, 2], [0, 3, 2, 4]], float)
    np.testing.assert_array_equal(oracle.hem_pass_desc(P.from_dense(A)), [2, 3, 0, 1])


@pytest.mark.parametrize("seed", range(12))
def test_desc_is_the_mirror_image_of_the_ascending_pass(seed):
    # reversing the numbering (i -> n-1-i) turns "from the last index, ties to the
    # highest" into "from the first index, ties to the lowest"
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 50))
    a = P.random_symmetric_pattern(n, float(rng.uniform(0.05, 0.4)), seed, weights=(1, 2),
                                   nonsym_values=bool(seed % 2), explicit_zeros=0.1 * (seed % 3 == 0))
    dense = a.to_scipy().toarray()
    r = P.from_dense(dense[::-1, ::-1].copy())
    # explicit zeros are lost by from_dense; compare on the dense-built pair only
    a2 = P.from_dense(dense)
    m_desc = oracle.hem_pass_desc(a2)
    m_rev = oracle.hem_pass(r)
    want = np.where(m_rev[::-1] >= 0, n - 1 - m_rev[::-1], -1)
    np.testing.assert_array_equal(m_desc, want)
    # and the ascending/descending pair agrees with the sorted-edge greedy under
    # the mirrored key
    np.testing.assert_array_equal(m_rev, greedy_sorted_edges(r))


def test_alternating_passes_on_a_chain():
    # one pass per level: level 0 from the first index pairs (0,1),(2,3),...;
    # level 1 (a 5-chain) from the last pairs (4,3),(2,1) and leaves 0; level 2
    # (a 3-chain) from the first again pairs (0,1)
    a = chain(10)
    h = oracle.Hierarchy(a, passes_per_level=1, max_coarse_rows=1, alternate=1)
    np.testing.assert_array_equal(h.level(0).agg, np.arange(10) // 2)
    np.testing.assert_array_equal(h.level(1).agg, [0, 1, 1, 2, 2])
    np.testing.assert_array_equal(h.level(2).agg, [0, 0, 1])
    g = oracle.Hierarchy(a, passes_per_level=1, max_coarse_rows=1)
    np.testing.assert_array_equal(g.level(1).agg, [0, 0, 1, 1, 2])


@pytest.mark.parametrize("ppl", [1, 2])
def test_alternating_hierarchy_composes_the_passes(ppl):
    # the setup-wide pass index decides the direction: even from the first
    # index, odd from the last
    a = P.lognormal_diffusion3d(7, 5, 1.0)
    h = oracle.Hierarchy(a, passes_per_level=ppl, alternate=1, max_coarse_rows=8)
    cur, g = a, 0
    for k in range(h.nlevels - 1):
        comp = np.arange(cur.n)
        for _ in range(ppl):
            mate = oracle.hem_pass_desc(cur) if g % 2 else oracle.hem_pass(cur)
            agg, nc = oracle.number(mate)
            crp, cci, cv = oracle.rap(cur, agg, nc)
            comp = agg[comp]
            cur, g = P.CSR(nc, crp, cci, cv), g + 1
        L, C = h.level(k), h.level(k + 1)
        np.testing.assert_array_equal(L.agg, comp)
        np.testing.assert_array_equal(C.row_ptr, cur.row_ptr)
        np.testing.assert_array_equal(C.col, cur.col)
        np.testing.assert_array_equal(C.val.view(np.int64), cur.val.view(np.int64))


def test_alternate_parameter_checks():
    a = P.poisson2d(6)
    for kw in (dict(alternate=2), dict(alternate=-1), dict(alternate=1, hem=1)):
        with pytest.raises(oracle.OracleError) as e:
            oracle.Hierarchy(a, **kw)
        assert e.value.status == oracle.EINVAL
