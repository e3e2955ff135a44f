"""GPU tests of the single-precision preconditioner (float V-cycle inside
double-precision PCG / BiCGStab), against the double-precision oracle.

The hierarchy is built in double either way, so aggregates and coarse
operators stay bit-identical to the oracle.  The float V-cycle is a different
(rounded) preconditioner, so its results are compared by what must hold for any
preconditioner of the same quality:
  * one float V-cycle agrees with the oracle's double V-cycle to relative
    2-norm error <= VC32_TOL (a few hundred float unit roundoffs; the cycle is
    a chain of O(levels) stencil sums, each rounded to 24 bits);
  * a solve reaches the same relative true residual rtol, checked again here in
    double on the host;
  * its iteration count is within max(2, 5%) of the oracle's double solve;
  * the difference from the oracle solution x_o is stated and bounded: both
    residuals are <= rtol ||b||, so ||A (x - x_o)|| <= 2 rtol ||b|| at any size,
    and ||x - x_o|| <= 2 rtol ||b|| ||A^{-1}||_2 where ||A^{-1}||_2 is computed
    (sizes up to 10^4 rows).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_2007_00056_amd import hemamg, problems as P

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
VC32_TOL = 256 * U32  # ~1.5e-5


@pytest.fixture(scope="module")
def torch():
    import torch as _t

    assert _t.cuda.is_available(), "GPU tests need a ROCm GPU"
    return _t


def say(*a):
    print(*a, flush=True)


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def bits(x):
    return np.ascontiguousarray(x, dtype=np.float64).view(np.int64)


def scipy_csr(a):
    return sp.csr_matrix((a.val, a.col, a.row_ptr), shape=(a.n, a.n))


def inv_norm2(a):
    """||A^{-1}||_2 = 1 / sigma_min(A), by shift-invert Lanczos at zero."""
    M = scipy_csr(a)
    if abs(M - M.T).max() == 0:
        lam = spla.eigsh(M.tocsc(), k=1, sigma=0.0, which="LM", return_eigenvectors=False)
        return 1.0 / abs(lam[0])
    N = (M.T @ M).tocsc()
    lam = spla.eigsh(N, k=1, sigma=0.0, which="LM", return_eigenvectors=False)
    return 1.0 / np.sqrt(abs(lam[0]))


def fp32_hierarchy(a, **kw):
    A = hemamg.DeviceCSR.from_host(a)
    return hemamg.Hierarchy(A, hemamg.amg_params_default(precond_fp32=1, **kw))


CASES = {
    "poisson2d_64": lambda: P.poisson2d(64),
    "poisson3d_17x13x11": lambda: P.poisson3d(17, 13, 11),
    "convdiff3d_13": lambda: P.convdiff3d(13),
    "lognormal3d_11": lambda: P.lognormal_diffusion3d(11, 5),
    "vardiff3d_20": lambda: P.vardiff3d(20, seed=1, corr_len=4.0),
    "random_ties_300": lambda: P.random_symmetric_pattern(300, 0.02, 3, weights=(1, 2)),
    "random_nonsym_zeros_400": lambda: P.random_symmetric_pattern(400, 0.015, 4, weights=(1, 2, 3),
                                                                  nonsym_values=True, explicit_zeros=0.1),
}
NONSYM = {"convdiff3d_13", "random_nonsym_zeros_400"}


def assert_same_hierarchy(g, o):
    assert g.nlevels == o.nlevels
    for k in range(o.nlevels):
        ol = o.level(k)
        rp, ci, v, agg = g.level(k)
        np.testing.assert_array_equal(rp, ol.row_ptr, err_msg=f"level {k} row_ptr")
        np.testing.assert_array_equal(ci, ol.col, err_msg=f"level {k} col_idx")
        np.testing.assert_array_equal(bits(v), bits(ol.val), err_msg=f"level {k} values")
        if ol.agg is not None:
            np.testing.assert_array_equal(agg, ol.agg, err_msg=f"level {k} aggregates")


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_setup_is_the_double_hierarchy(torch, name):
    say("case", name)
    a = CASES[name]()
    with fp32_hierarchy(a) as g:
        assert_same_hierarchy(g, oracle.Hierarchy(a))


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_vcycle_close_to_double(torch, name):
    say("case", name)
    a = CASES[name]()
    f = P.rhs_uniform(a.n, 11)
    with fp32_hierarchy(a) as g:
        z = g.vcycle(dev(torch, f)).cpu().numpy()
    err = rel(z, oracle.Hierarchy(a).vcycle(f))
    say("float V-cycle relative error", err)
    assert err <= VC32_TOL, err


def mixed_solve_check(torch, a, method, rtol, seed=0, inv_norm=None):
    b = P.rhs_uniform(a.n, seed)
    o = oracle.Hierarchy(a)
    xo, io = o.solve(b, method=method, rtol=rtol, maxit=1000)
    assert io["status"] == oracle.OK
    with fp32_hierarchy(a) as g:
        xg, ig = g.solve(dev(torch, b), method=method, rtol=rtol, maxit=1000)
        xg = xg.cpu().numpy()
    assert ig["status"] == hemamg.AMG_OK, ig
    M = scipy_csr(a)
    nb = np.linalg.norm(b)
    true_res = np.linalg.norm(b - M @ xg) / nb
    assert true_res <= rtol * (1 + 1e-6), (true_res, ig)
    assert abs(ig["iters"] - io["iters"]) <= max(2, int(0.05 * io["iters"])), (ig, io)
    dres = np.linalg.norm(M @ (xg - xo)) / nb
    assert dres <= 2 * rtol * (1 + 1e-6), dres
    err = rel(xg, xo)
    line = dict(iters=ig["iters"], oracle_iters=io["iters"], true_res=true_res, diff_res=dres, rel_err=err)
    if inv_norm is not None:
        bound = 2 * rtol * nb * inv_norm / np.linalg.norm(xo)
        line["rel_err_bound"] = bound
        assert err <= bound, line
    say("float preconditioner vs double oracle:", line)
    return ig, io


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_solve_against_double_oracle(torch, name):
    say("case", name)
    a = CASES[name]()
    method = "bicgstab" if name in NONSYM else "pcg"
    mixed_solve_check(torch, a, method, 1e-8, inv_norm=inv_norm2(a))


def test_fp32_rtol_near_double_limit(torch):
    # the float preconditioner does not limit the attainable accuracy: the
    # outer iteration and its true residual stay in double
    a = P.poisson3d(20, 18, 16)
    mixed_solve_check(torch, a, "pcg", 1e-12, inv_norm=inv_norm2(a))


@pytest.mark.parametrize("name", ["poisson3d_17x13x11", "lognormal3d_11"])
def test_fp32_stationary_solver(torch, name):
    # iterative refinement with a float V-cycle: the update and the residual
    # are double, so the double tolerance is reached
    say("case", name)
    a = CASES[name]()
    mixed_solve_check(torch, a, "stationary", 1e-10, inv_norm=inv_norm2(a))


def test_fp32_parameter_rules(torch):
    a = P.poisson3d(10, 9, 8)
    A = hemamg.DeviceCSR.from_host(a)
    for kw in (dict(precond_fp32=1, pre=2, post=1), dict(precond_fp32=1, pre=1, post=0), dict(precond_fp32=2)):
        with pytest.raises(hemamg.AmgError) as e:
            hemamg.Hierarchy(A, hemamg.amg_params_default(**kw))
        assert e.value.status == hemamg.AMG_EINVAL, kw


def test_fp32_single_level_is_exact(torch):
    # a matrix at or below the coarsest size is solved directly in double
    a = P.poisson2d(7)
    b = P.rhs_uniform(a.n, 3)
    with fp32_hierarchy(a) as g:
        assert g.nlevels == 1
        z = g.vcycle(dev(torch, b)).cpu().numpy()
    x = np.linalg.solve(scipy_csr(a).toarray(), b)
    assert rel(z, x) <= 1e-13


def test_fp32_deterministic_bitwise(torch):
    a = P.lognormal_diffusion3d(14, 2)
    b = dev(torch, P.rhs_uniform(a.n, 0))
    with fp32_hierarchy(a) as g:
        x1, i1 = g.solve(b, rtol=1e-9)
        x2, i2 = g.solve(b, rtol=1e-9)
    assert i1["iters"] == i2["iters"]
    np.testing.assert_array_equal(bits(x1.cpu().numpy()), bits(x2.cpu().numpy()))


# ---------------------------------------------------------------- full size

def test_vardiff3d_160_fp32(torch):
    """3-D variable-coefficient diffusion, 160^3, float preconditioner, PCG."""
    say("case vardiff3d_160 fp32")
    a, _, spec = P.make_workload("vardiff3d_160")
    with fp32_hierarchy(a) as g:
        assert_same_hierarchy(g, oracle.Hierarchy(a))
    ig, io = mixed_solve_check(torch, a, spec["kind"], spec["rtol"])
    say("gpu", ig, "oracle", io)


def test_convdiff3d_96_bicgstab_double(torch):
    """3-D convection-diffusion, 96^3, BiCGStab, double throughout."""
    say("case convdiff3d_96 fp64")
    a, _, spec = P.make_workload("convdiff3d_96")
    b = P.rhs_uniform(a.n, 0)
    o = oracle.Hierarchy(a)
    xo, io = o.solve(b, method="bicgstab", rtol=spec["rtol"], maxit=500)
    assert io["status"] == oracle.OK
    with hemamg.Hierarchy(hemamg.DeviceCSR.from_host(a)) as g:
        assert_same_hierarchy(g, o)
        xg, ig = g.solve(dev(torch, b), method="bicgstab", rtol=spec["rtol"], maxit=500)
        assert ig["status"] == hemamg.AMG_OK and abs(ig["iters"] - io["iters"]) <= 1, (ig, io)
        xg2, ig2 = g.solve(dev(torch, b), method="bicgstab", rtol=0.0, maxit=io["iters"], check=False)
        assert ig2["iters"] == io["iters"]
        err = rel(xg2.cpu().numpy(), xo)
        emax = np.abs(xg2.cpu().numpy() - xo).max() / np.abs(xo).max()
    say("gpu", ig, "oracle", io, "rel err at equal iterations", err, "max element err", emax)
    assert err <= 1e-9 and emax <= 1e-9, (err, emax)


def test_convdiff3d_96_fp32(torch):
    """3-D convection-diffusion, 96^3, float preconditioner, BiCGStab."""
    say("case convdiff3d_96 fp32")
    a, _, spec = P.make_workload("convdiff3d_96")
    ig, io = mixed_solve_check(torch, a, spec["kind"], spec["rtol"])
    say("gpu", ig, "oracle", io)
