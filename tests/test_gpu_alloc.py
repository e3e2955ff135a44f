"""The caller's device allocator (amg_allocator) on the setup entry points:
every buffer a handle or batch owns, and every temporary of its setup, is
drawn through it; an allocation that fails at any point gives AMG_ENOMEM with
nothing left allocated, and the next setup succeeds with results unchanged."""
import numpy as np
import pytest

from conftest import CountingAllocator
from paper_2007_00056_amd import hemamg, problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t

    assert _t.cuda.is_available(), "GPU tests need a ROCm GPU"
    return _t


def say(*a):
    print(*a, flush=True)


def bits(x):
    return np.ascontiguousarray(x, dtype=np.float64).view(np.int64)


def setup_and_solve(torch, A, b, alloc, **kw):
    """Setup + PCG (the first solve draws the Krylov workspace); returns
    (status, solution or None)."""
    try:
        g = hemamg.Hierarchy(A, alloc=alloc, **kw)
    except hemamg.AmgError as e:
        return e.status, None
    try:
        x, info = g.solve(b, rtol=1e-8, maxit=300, check=False)
        return info["status"], x.cpu().numpy()
    finally:
        g.close()


@pytest.mark.parametrize("kw", [dict(), dict(precond_fp32=1), dict(alternate=1), dict(hem=1)])
def test_every_allocation_failure_is_enomem_without_leak(torch, kw):
    a = P.lognormal_diffusion3d(24, 5, 1.0)
    A = hemamg.DeviceCSR.from_host(a)
    b = torch.from_numpy(P.rhs_uniform(a.n, 1)).cuda()
    ref = CountingAllocator(torch)
    st, xref = setup_and_solve(torch, A, b, ref, **kw)
    assert st == hemamg.AMG_OK and ref.live == 0
    say(kw, "allocation calls of setup + first solve:", ref.calls, "peak MB", ref.peak / 1e6)
    assert ref.calls >= 3
    for k in range(1, ref.calls + 1):
        ca = CountingAllocator(torch, fail_at=k)
        st, _ = setup_and_solve(torch, A, b, ca, **kw)
        assert st == hemamg.AMG_ENOMEM, (k, st)
        assert ca.live == 0, (k, ca.live)
        ok = CountingAllocator(torch)
        st, x = setup_and_solve(torch, A, b, ok, **kw)
        assert st == hemamg.AMG_OK and ok.live == 0
        np.testing.assert_array_equal(bits(x), bits(xref))


def test_library_pool_and_caller_allocator_give_the_same_result(torch):
    a = P.poisson3d(30, 26, 22)
    A = hemamg.DeviceCSR.from_host(a)
    b = torch.from_numpy(P.rhs_uniform(a.n, 2)).cuda()
    st0, x0 = setup_and_solve(torch, A, b, None)
    ta = hemamg.TorchAllocator()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    with hemamg.Hierarchy(A, alloc=ta) as g:
        owned = g.stats()["owned_bytes"]
        during = torch.cuda.memory_allocated()
        x1, info = g.solve(b, rtol=1e-8, maxit=300)
        owned_after_solve = g.stats()["owned_bytes"]
        during_solve = torch.cuda.memory_allocated()
    torch.cuda.synchronize()
    after = torch.cuda.memory_allocated()
    say("owned", owned, "torch sees", during - before, "after first solve", owned_after_solve, during_solve - before)
    # torch's allocator sees the handle's bytes (it rounds each chunk up to 512
    # bytes; x1 is a torch tensor too)
    slack = 512 * 64
    xb = x1.numel() * 8
    assert owned <= during - before <= owned + slack
    assert owned_after_solve <= during_solve - before - xb <= owned_after_solve + slack
    assert owned_after_solve > owned  # the Krylov workspace came through it at the first solve
    assert xb <= after - before <= xb + 512
    assert st0 == hemamg.AMG_OK
    np.testing.assert_array_equal(bits(x1.cpu().numpy()), bits(x0))


def test_half_set_allocator_is_rejected(torch):
    a = P.poisson2d(20)
    A = hemamg.DeviceCSR.from_host(a)
    bad = hemamg.amg_allocator()
    bad.alloc = hemamg.ALLOC_FN(lambda n, c, s: None)
    h = hemamg.C.c_void_p()
    st = hemamg.lib().amg_setup(hemamg.C.byref(A.c), None, hemamg.C.byref(bad), None, hemamg.C.byref(h))
    assert st == hemamg.AMG_EINVAL and not h.value


@pytest.mark.parametrize("fp32", [0, 1])
def test_batched_setup_allocation_failures(torch, fp32):
    systems = [P.lognormal_diffusion3d(m, 40 + m, 1.0) for m in (9, 14, 20)] + [P.poisson3d(12)]
    Ds = [hemamg.DeviceCSR.from_host(a) for a in systems]
    params = hemamg.amg_params_default(precond_fp32=fp32)
    rhs = torch.from_numpy(np.concatenate([P.rhs_uniform(a.n, 3) for a in systems])).cuda()

    def run(alloc):
        try:
            bt = hemamg.Batch.setup(Ds, params, alloc=alloc)
        except hemamg.AmgError as e:
            return e.status, None
        try:
            x, infos = bt.solve(rhs, rtol=1e-8, maxit=300)
            assert all(i["status"] == hemamg.AMG_OK for i in infos)
            assert all(i["levels"] >= 2 and i["setup_ms"] > 0 for i in infos)
            return hemamg.AMG_OK, x.cpu().numpy()
        finally:
            bt.close()

    ref = CountingAllocator(torch)
    st, xref = run(ref)
    assert st == hemamg.AMG_OK and ref.live == 0
    say("batched setup allocation calls", ref.calls)
    for k in range(1, ref.calls + 1):
        ca = CountingAllocator(torch, fail_at=k)
        st, _ = run(ca)
        assert st == hemamg.AMG_ENOMEM and ca.live == 0, (k, st, ca.live)
    st, x = run(CountingAllocator(torch))
    np.testing.assert_array_equal(bits(x), bits(xref))


def test_kept_chunks_are_reused_and_released(torch):
    """The library pool keeps the chunks of a destroyed handle: a second setup
    of the same system draws exactly those chunks again (the kept bytes do not
    grow), amg_release_cached frees them and gives the pool's memory back to
    the driver, and setups afterwards give the same bits."""
    a = P.poisson3d(64)
    A = hemamg.DeviceCSR.from_host(a)
    b = torch.from_numpy(P.rhs_uniform(a.n, 2)).cuda()
    hemamg.amg_release_cached()
    assert hemamg.amg_cached_bytes() == 0
    st, x1 = setup_and_solve(torch, A, b, None)
    assert st == hemamg.AMG_OK
    torch.cuda.synchronize()
    kept = hemamg.amg_cached_bytes()
    say("kept after one setup + solve:", kept / 1e6, "MB")
    assert kept >= 1 << 20
    st, x2 = setup_and_solve(torch, A, b, None)
    assert st == hemamg.AMG_OK
    assert hemamg.amg_cached_bytes() == kept
    np.testing.assert_array_equal(bits(x2), bits(x1))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    hemamg.amg_release_cached()
    assert hemamg.amg_cached_bytes() == 0
    free1 = torch.cuda.mem_get_info()[0]
    say("device memory freed by the release:", (free1 - free0) / 1e6, "MB")
    assert free1 - free0 >= kept // 2
    st, x3 = setup_and_solve(torch, A, b, None)
    assert st == hemamg.AMG_OK
    np.testing.assert_array_equal(bits(x3), bits(x1))
