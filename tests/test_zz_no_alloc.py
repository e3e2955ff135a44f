"""krylov_solve_noalloc: the allocation-free form of krylov_solve (work
vectors in the library's static scratch) gives bit for bit the result of
krylov_solve on the same handle, draws nothing through the handle's
allocator, and keeps doing so on consecutive calls whose sizes shrink (the
scratch keeps the previous call's contents)."""
import numpy as np
import pytest

from conftest import CountingAllocator
from paper_2007_00056_amd import hemamg, problems as P

pytestmark = pytest.mark.gpu

NOALLOC_MAX_ROWS = 1 << 20


@pytest.fixture(scope="module")
def torch():
    import torch as _t

    assert _t.cuda.is_available(), "GPU tests need a ROCm GPU"
    return _t


def say(*a):
    print(*a, flush=True)


def bits(x):
    return np.ascontiguousarray(x, dtype=np.float64).view(np.int64)


def both_forms(torch, a, method, rtol, **kw):
    """Solve one system with krylov_solve_noalloc first (on a fresh handle,
    so its workspace has never been drawn), then with krylov_solve; returns
    both results and the allocator's call counts around the no-alloc call."""
    A = hemamg.DeviceCSR.from_host(a)
    b = torch.from_numpy(P.rhs_uniform(a.n, 3)).cuda()
    ca = CountingAllocator(torch)
    g = hemamg.Hierarchy(A, alloc=ca, **kw)
    try:
        torch.cuda.synchronize()
        calls0 = ca.calls
        x_na = torch.zeros_like(b)
        info_na = hemamg.krylov_solve_noalloc(g.h, method, b, x_na, rtol, 500)
        calls1 = ca.calls
        x_ref = torch.zeros_like(b)
        info_ref = hemamg.krylov_solve(g.h, method, b, x_ref, rtol, 500)
        return x_na.cpu().numpy(), info_na, x_ref.cpu().numpy(), info_ref, calls1 - calls0, ca.calls - calls1
    finally:
        g.close()


def check_same(x_na, info_na, x_ref, info_ref):
    assert info_na["status"] == info_ref["status"] == hemamg.AMG_OK
    assert info_na["iters"] == info_ref["iters"]
    assert info_na["rel_res"] == info_ref["rel_res"]
    assert info_na["true_rel_res"] == info_ref["true_rel_res"]
    assert np.array_equal(bits(x_na), bits(x_ref))


def test_noalloc_equals_krylov_solve_on_consecutive_calls_of_decreasing_size(torch):
    # first a larger system, then a smaller one: the second call finds the
    # first one's vectors in the scratch and must not depend on them
    for a in (P.poisson3d(48, 44, 40), P.poisson3d(21, 17, 13)):
        say("noalloc PCG n =", a.n)
        x_na, info_na, x_ref, info_ref, drawn_na, drawn_ref = both_forms(torch, a, hemamg.PCG, 1e-10)
        check_same(x_na, info_na, x_ref, info_ref)
        assert drawn_na == 0  # the no-alloc call drew nothing through the handle's allocator
        assert drawn_ref > 0  # while krylov_solve drew the workspace on its first call
        say("  iters", info_na["iters"], "rel_res", info_na["rel_res"])


def test_noalloc_bicgstab_and_float_preconditioner(torch):
    cases = [(P.convdiff3d(30), hemamg.BICGSTAB, dict(precond_fp32=1)),
             (P.lognormal_diffusion3d(26, 7, 1.0), hemamg.PCG, dict(precond_fp32=1)),
             (P.convdiff3d(18), hemamg.BICGSTAB, dict())]
    for a, method, kw in cases:
        say("noalloc method", method, "n =", a.n, kw)
        x_na, info_na, x_ref, info_ref, drawn_na, _ = both_forms(torch, a, method, 1e-8, **kw)
        check_same(x_na, info_na, x_ref, info_ref)
        assert drawn_na == 0


def test_noalloc_rejects_systems_beyond_the_scratch(torch):
    side = 102  # 102^3 = 1,061,208 rows > 2^20
    a = P.poisson3d(side, side, side)
    assert a.n > NOALLOC_MAX_ROWS
    A = hemamg.DeviceCSR.from_host(a)
    b = torch.from_numpy(P.rhs_uniform(a.n, 0)).cuda()
    with hemamg.Hierarchy(A) as g:
        x = torch.zeros_like(b)
        info = hemamg.krylov_solve_noalloc(g.h, hemamg.PCG, b, x, 1e-8, 10, check=False)
        assert info["status"] == hemamg.AMG_EINVAL
        assert "scratch" in hemamg.amg_last_error()
        assert not bool(x.abs().sum().item())  # nothing ran
