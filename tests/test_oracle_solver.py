"""Pins of the oracle's generators, coarsest LU, V-cycle (Algorithm 1), PCG
(Algorithm 4) and BiCGStab (Algorithm 5) against closed forms, library
routines, dense brute force and invariants."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle
from paper_2007_00056_amd import problems as P


# ---------------------------------------------------------------- generators

@pytest.mark.parametrize("shape", [(5, 7), (3, 4, 5), (6, 6, 6)])
def test_poisson_eigenvalues_closed_form(shape):
    a = P.poisson2d(*shape) if len(shape) == 2 else P.poisson3d(*shape)
    ev = np.sort(np.linalg.eigvalsh(a.to_scipy().toarray()))
    grids = np.meshgrid(*[np.arange(1, s + 1) for s in shape], indexing="ij")
    want = sum(2 - 2 * np.cos(p * np.pi / (s + 1)) for p, s in zip(grids, shape))
    np.testing.assert_allclose(ev, np.sort(want.ravel()), atol=1e-12)


def test_generator_sizes_match_stencil_counts():
    a = P.poisson2d(64)
    assert a.n == 4096 and a.nnz == 5 * 4096 - 4 * 64
    a = P.poisson3d(20)
    assert a.n == 8000 and a.nnz == 7 * 8000 - 6 * 400
    assert np.all(np.diff(a.col[a.row_ptr[5]:a.row_ptr[6]]) > 0)


def test_convdiff_rows_and_upwinding():
    a = P.convdiff3d(6)
    D = a.to_scipy().toarray()
    i = 2 + 6 * (2 + 6 * 2)  # interior cell
    assert D[i, i] == 23.5 and D[i, i - 1] == -11 and D[i, i - 6] == -6 and D[i, i - 36] == -3.5
    assert D[i, i + 1] == -1 and D[i, i + 6] == -1 and D[i, i + 36] == -1
    assert abs(D[i].sum()) == 0.0
    assert not np.allclose(D, D.T)


def test_vardiff_is_spd_and_row_sums_are_boundary_faces():
    n = 8
    a = P.vardiff3d(n, seed=1, corr_len=2.0)
    D = a.to_scipy().toarray()
    np.testing.assert_allclose(D, D.T, rtol=0, atol=0)
    assert np.linalg.eigvalsh(D).min() > 0
    g = P.gaussian_field(n, 1, corr_len=2.0)
    assert abs(g.std() - 1.5) < 1e-12 and abs(g.mean()) < 1e-12
    # interior cells have zero row sum, boundary cells keep their wall faces
    rs = D.sum(axis=1).reshape(n, n, n)
    assert np.abs(rs[1:-1, 1:-1, 1:-1]).max() < 1e-9
    e = np.exp(g)
    np.testing.assert_allclose(rs[1:-1, 1:-1, 0], 2 * e[1:-1, 1:-1, 0], rtol=1e-12)


# ---------------------------------------------------------------- dense LU

def test_lu_matches_lapack_including_pivot_ties():
    rng = np.random.default_rng(0)
    for n in (1, 5, 17, 64):
        A = rng.integers(-3, 4, size=(n, n)).astype(float) + np.eye(n) * 0.5
        lu, piv, st = oracle.lu_factor(A)
        assert st == oracle.OK
        lu_ref, piv_ref = sla.lu_factor(A)
        np.testing.assert_array_equal(piv, piv_ref)  # getrf takes the first max: lowest row on ties
        np.testing.assert_allclose(lu, lu_ref, rtol=1e-12, atol=1e-12)
        b = rng.standard_normal(n)
        np.testing.assert_allclose(oracle.lu_solve(lu, piv, b), sla.lu_solve((lu_ref, piv_ref), b), rtol=1e-10,
                                   atol=1e-12)


def test_lu_singular_detected():
    _, _, st = oracle.lu_factor(np.array([[1.0, 2.0], [2.0, 4.0]]))
    assert st == oracle.ESINGULAR


# ---------------------------------------------------------------- V-cycle

def assembled_preconditioner(h, n):
    return np.stack([h.vcycle(e) for e in np.eye(n)], axis=1)


def test_single_level_vcycle_is_exact_solve():
    a = P.poisson2d(7, 9)  # 63 rows <= 64: the level is solved directly
    h = oracle.Hierarchy(a)
    assert h.nlevels == 1
    b = P.rhs_uniform(a.n, 0)
    np.testing.assert_allclose(h.vcycle(b), np.linalg.solve(a.to_scipy().toarray(), b), rtol=1e-12)
    x, info = h.solve(b, rtol=1e-12)
    assert info["iters"] == 1 and info["status"] == oracle.OK


@pytest.mark.parametrize("make", [lambda: P.poisson2d(12, 10), lambda: P.poisson3d(6, 5, 7),
                                  lambda: P.lognormal_diffusion3d(7, seed=2)])
def test_vcycle_operator_is_symmetric_positive_definite_and_convergent(make):
    a = make()
    h = oracle.Hierarchy(a, max_coarse_rows=8)
    assert h.nlevels >= 3
    M = assembled_preconditioner(h, a.n)
    scale = np.abs(M).max()
    assert np.abs(M - M.T).max() <= 1e-12 * scale
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    E = np.eye(a.n) - M @ a.to_scipy().toarray()
    assert np.abs(np.linalg.eigvals(E)).max() < 1.0


def test_two_level_cycle_matches_dense_formulation():
    # Figure 1 / Algorithm 1 with L = 1, written with dense operators
    a = P.lognormal_diffusion3d(5, seed=4)
    h = oracle.Hierarchy(a, max_coarse_rows=40, max_levels=2)
    assert h.nlevels == 2
    L0 = h.level(0)
    A = a.to_scipy().toarray()
    nc = h.level(1).n
    Pm = np.zeros((a.n, nc))
    Pm[np.arange(a.n), L0.agg] = 1.0
    Ac = Pm.T @ A @ Pm
    w = 2.0 / 3.0
    Dinv = np.diag(1.0 / np.diag(A))
    f = P.rhs_uniform(a.n, 5)
    x = w * Dinv @ f
    x = x + Pm @ np.linalg.solve(Ac, Pm.T @ (f - A @ x))
    x = x + w * Dinv @ (f - A @ x)
    np.testing.assert_allclose(h.vcycle(f), x, rtol=1e-11, atol=1e-13)


def multigrid_operator(A, Ps, omega, pre, post):
    """B_0 with z = B_0 f for the V-cycle, from the textbook error-propagation
    identity of multigrid (not from Algorithm 1's steps): with the Jacobi
    iteration matrix S_k = I - omega D_k^{-1} A_k and the Galerkin operators
    A_{k+1} = P_k^T A_k P_k, the cycle's error propagation is
    E_k = S_k^post (I - P_k B_{k+1} P_k^T A_k) S_k^pre, B_L = A_L^{-1}, and
    B_k = (I - E_k) A_k^{-1}."""
    As = [A]
    for Pm in Ps:
        As.append(Pm.T @ As[-1] @ Pm)
    B = np.linalg.inv(As[-1])
    for k in range(len(Ps) - 1, -1, -1):
        Ak, Pm = As[k], Ps[k]
        S = np.eye(Ak.shape[0]) - omega * np.diag(1.0 / np.diag(Ak)) @ Ak
        E = np.linalg.matrix_power(S, post) @ (np.eye(Ak.shape[0]) - Pm @ B @ Pm.T @ Ak) @ \
            np.linalg.matrix_power(S, pre)
        B = (np.eye(Ak.shape[0]) - E) @ np.linalg.inv(Ak)
    return B


@pytest.mark.parametrize("make,kw", [
    (lambda: P.lognormal_diffusion3d(6, seed=7), dict(omega=0.6, pre=2, post=3)),
    (lambda: P.poisson2d(14, 11), dict(omega=0.8, pre=1, post=2)),
    (lambda: P.convdiff3d(6), dict(omega=0.5, pre=3, post=1)),
])
def test_three_level_cycle_matches_error_propagation_identity(make, kw):
    """Algorithm 1 recursing through two coarse levels (max_levels = 3) with
    non-default damping and sweep counts: the assembled V-cycle operator equals
    the multigrid error-propagation identity built from dense P_k and
    P_k^T A_k P_k (the oracle's coarse matrices are not used)."""
    a = make()
    h = oracle.Hierarchy(a, max_levels=3, max_coarse_rows=8, **kw)
    assert h.nlevels == 3
    A = a.to_scipy().toarray()
    Ps = []
    for k in range(2):
        agg = h.level(k).agg
        Pm = np.zeros((agg.size, h.level(k + 1).n))
        Pm[np.arange(agg.size), agg] = 1.0
        Ps.append(Pm)
    B = multigrid_operator(A, Ps, kw["omega"], kw["pre"], kw["post"])
    M = assembled_preconditioner(h, a.n)
    assert np.abs(M - B).max() <= 1e-10 * np.abs(B).max()
    # a dropped coarse correction or a wrong sweep count is far off
    B_wrong = multigrid_operator(A, Ps, kw["omega"], kw["pre"], kw["post"] + 1)
    assert np.abs(M - B_wrong).max() > 1e-3 * np.abs(B).max()


def poisson_beside_diagonal():
    """A 64x64 Poisson block (coarsens 4:1) beside a 2000-row diagonal block
    (merges nothing): coarsening ends at a level of 1025..4096 rows."""
    return P.block_diag(P.poisson2d(64), P.diagonal(np.arange(1.0, 2001.0)))


def poisson_beside_star():
    """A 64x64 Poisson block beside a 1500-row star (two rows merge per level)."""
    return P.block_diag(P.poisson2d(64), P.star_graph(1500, 2))


@pytest.mark.parametrize("make,kw,coarsest,why", [
    (poisson_beside_diagonal, dict(stall_ratio=1.0), 2001, "no row merged"),
    (poisson_beside_star, dict(stall_ratio=1.0), 1439, "depth limit"),
    (poisson_beside_diagonal, dict(), 2256, "poor progress"),
    (poisson_beside_star, dict(), 1558, "poor progress"),
])
def test_stalled_coarsening_ends_in_a_dense_level_of_up_to_4096_rows(make, kw, coarsest, why):
    """Section 3 setup with the stop readings: a level that stalls (nothing
    merged, or the depth limit) becomes the dense coarsest when it has at most
    max_dense_rows = 4096 rows, and so does one of at most that size whose
    coarsening would keep 90% of its rows; above the limit a stall is an
    error.  The solve with the dense coarsest still reaches a manufactured
    solution."""
    a = make()
    h = oracle.Hierarchy(a, **kw)
    sizes = [h.level(k).n for k in range(h.nlevels)]
    assert sizes[-1] == coarsest and 1024 < coarsest <= 4096, (why, sizes)
    xs = np.random.default_rng(3).standard_normal(a.n)
    b = a.to_scipy() @ xs
    x, info = h.solve(b, rtol=1e-12, maxit=300)
    assert info["status"] == oracle.OK
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    if why != "poor progress":
        with pytest.raises(oracle.OracleError) as e:
            oracle.Hierarchy(a, max_dense_rows=coarsest - 1, **kw)
        assert e.value.status == oracle.ESTALL


def test_dense_level_at_the_4096_row_limit_and_above():
    d = np.linspace(1.0, 7.0, 4096)
    h = oracle.Hierarchy(P.diagonal(d))
    assert h.nlevels == 1
    b = P.rhs_uniform(4096, 2)
    np.testing.assert_allclose(h.vcycle(b), b / d, rtol=1e-15)
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(P.diagonal(np.linspace(1.0, 7.0, 4097)))
    assert e.value.status == oracle.ESTALL


def test_single_dense_level_of_a_star_is_the_exact_solve():
    a = P.star_graph(3000, 2)  # coarsening would keep 2998 of 3000 rows
    h = oracle.Hierarchy(a)
    assert h.nlevels == 1
    b = P.rhs_uniform(a.n, 4)
    np.testing.assert_allclose(h.vcycle(b), sla.solve(a.to_scipy().toarray(), b), rtol=1e-11)


# ---------------------------------------------------------------- PCG / BiCGStab

def test_pcg_manufactured_solution_and_dense_solve():
    a = P.lognormal_diffusion3d(8, seed=0)
    A = a.to_scipy()
    xs = np.random.default_rng(1).standard_normal(a.n)
    b = A @ xs
    h = oracle.Hierarchy(a)
    x, info = h.solve(b, rtol=1e-12)
    assert info["status"] == oracle.OK
    kappa = np.linalg.cond(A.toarray())
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-12
    np.testing.assert_allclose(x, np.linalg.solve(A.toarray(), b), rtol=1e-6)
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-12


def test_pcg_a_norm_error_decreases():
    a = P.poisson3d(10)
    A = a.to_scipy()
    b = P.rhs_uniform(a.n, 3)
    h = oracle.Hierarchy(a)
    xs = np.linalg.solve(A.toarray(), b)
    errs = []
    for k in range(1, 12):
        x, _ = h.solve(b, rtol=0.0, maxit=k)
        e = x - xs
        errs.append(np.sqrt(e @ (A @ e)))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))


class _Count:
    def __init__(self):
        self.n = 0

    def __call__(self, *_):
        self.n += 1


@pytest.mark.parametrize("precond", [True, False])
def test_pcg_iteration_count_matches_scipy_cg(precond):
    a = P.poisson2d(40)
    A = a.to_scipy()
    b = P.rhs_uniform(a.n, 0)
    h = oracle.Hierarchy(a)
    x, info = h.solve(b, rtol=1e-8, precond=precond, maxit=2000)
    M = spla.LinearOperator(A.shape, matvec=h.vcycle) if precond else None
    cnt = _Count()
    xr, st = spla.cg(A, b, rtol=1e-8, M=M, maxiter=2000, callback=cnt)
    assert st == 0 and info["status"] == oracle.OK
    assert abs(info["iters"] - cnt.n) <= 1
    np.testing.assert_allclose(x, xr, rtol=1e-5, atol=1e-7)


def test_bicgstab_matches_scipy_and_manufactured_solution():
    a = P.convdiff3d(10)
    A = a.to_scipy()
    xs = np.random.default_rng(2).uniform(-1, 1, a.n)
    b = A @ xs
    h = oracle.Hierarchy(a)
    x, info = h.solve(b, method="bicgstab", rtol=1e-10)
    assert info["status"] == oracle.OK
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-7
    cnt = _Count()
    xr, st = spla.bicgstab(A, b, rtol=1e-10, M=spla.LinearOperator(A.shape, matvec=h.vcycle), callback=cnt)
    assert st == 0
    assert abs(info["iters"] - cnt.n) <= 1


def test_zero_rhs_and_status_codes():
    a = P.poisson2d(10)
    h = oracle.Hierarchy(a)
    x, info = h.solve(np.zeros(a.n), x0=np.ones(a.n))
    assert info["iters"] == 0 and np.all(x == 0)
    _, info = h.solve(P.rhs_uniform(a.n, 0), rtol=1e-14, maxit=2)
    assert info["status"] == oracle.ENOTCONV and info["iters"] == 2
    b = P.rhs_uniform(a.n, 0)
    b[3] = np.nan
    _, info = h.solve(b)
    assert info["status"] == oracle.ENOTFINITE
    bad = P.poisson2d(3)
    bad.val = bad.val.copy()
    bad.val[0] = 0.0  # zero diagonal
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(bad)
    assert e.value.status == oracle.EINVAL


def test_stall_falls_back_to_dense_or_reports():
    # a diagonal matrix has no edges: no coarsening progress
    a = P.from_dense(np.diag(np.arange(1.0, 101.0)))
    h = oracle.Hierarchy(a)
    assert h.nlevels == 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(a, max_dense_rows=50)
    assert e.value.status == oracle.ESTALL


def test_star_graph_stall_ratio_rule():
    # two pairwise passes on a star merge two leaves into the hub: n -> n - 2
    a = P.star_graph(100, 0)
    h = oracle.Hierarchy(a)  # 98 >= 0.9 * 100 and 100 <= max_dense_rows: dense at once
    assert h.nlevels == 1
    h = oracle.Hierarchy(a, stall_ratio=1.0)  # only a level with no merge stops
    sizes = [h.level(k).row_ptr.size - 1 for k in range(h.nlevels)]
    assert sizes == list(range(100, 63, -2)), sizes
    # a stalling level above max_dense_rows keeps coarsening
    h = oracle.Hierarchy(a, max_dense_rows=90)
    sizes = [h.level(k).row_ptr.size - 1 for k in range(h.nlevels)]
    assert sizes == [100, 98, 96, 94, 92, 90], sizes
    # the V-cycle of the one-level hierarchy is the exact solve
    b = P.rhs_uniform(a.n, 1)
    dense = np.zeros((a.n, a.n))
    for i in range(a.n):
        dense[i, a.col[a.row_ptr[i]:a.row_ptr[i + 1]]] = a.val[a.row_ptr[i]:a.row_ptr[i + 1]]
    np.testing.assert_allclose(oracle.Hierarchy(a).vcycle(b), np.linalg.solve(dense, b), rtol=1e-12)
    for bad in (0.0, -0.5, 1.5):
        with pytest.raises(oracle.OracleError) as e:
            oracle.Hierarchy(a, stall_ratio=bad)
        assert e.value.status == oracle.EINVAL


# ---------------------------------------------------------------- AMG as a solver

def test_stationary_iterates_follow_the_dense_recurrence():
    # x_{k+1} = x_k + M (b - A x_k) with M the assembled V-cycle operator
    a = P.poisson3d(7, 6, 5)
    h = oracle.Hierarchy(a)
    A = a.to_scipy().toarray()
    M = assembled_preconditioner(h, a.n)
    b = P.rhs_uniform(a.n, 4)
    x0 = P.rhs_uniform(a.n, 5)
    x = x0.copy()
    for k in range(1, 7):
        x = x + M @ (b - A @ x)
        xo, info = h.solve(b, x0=x0, method="stationary", rtol=0.0, maxit=k)
        assert info["status"] == oracle.ENOTCONV and info["iters"] == k
        assert np.linalg.norm(xo - x) <= 1e-12 * np.linalg.norm(x)
        r = b - A @ xo
        assert abs(info["true_rel_res"] - np.linalg.norm(r) / np.linalg.norm(b)) <= 1e-12


def test_stationary_converges_at_the_spectral_rate():
    a = P.poisson3d(9, 8, 7)
    h = oracle.Hierarchy(a)
    A = a.to_scipy().toarray()
    M = assembled_preconditioner(h, a.n)
    rho = max(abs(np.linalg.eigvals(np.eye(a.n) - M @ A)))
    assert 0 < rho < 1
    b = P.rhs_uniform(a.n, 6)
    x, info = h.solve(b, method="stationary", rtol=1e-10, maxit=500)
    assert info["status"] == oracle.OK
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-9)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-7 * np.linalg.norm(x)
    # asymptotically the error contracts by rho per sweep
    predicted = np.log(1e-10) / np.log(rho)
    assert 0.5 * predicted <= info["iters"] <= 1.5 * predicted + 5, (info, predicted)


def test_stationary_single_level_is_one_exact_step():
    a = P.poisson2d(6)
    h = oracle.Hierarchy(a)
    assert h.nlevels == 1
    b = P.rhs_uniform(a.n, 1)
    x, info = h.solve(b, method="stationary", rtol=1e-12)
    assert info["status"] == oracle.OK and info["iters"] == 1
    assert np.linalg.norm(x - np.linalg.solve(a.to_scipy().toarray(), b)) <= 1e-13 * np.linalg.norm(x)
