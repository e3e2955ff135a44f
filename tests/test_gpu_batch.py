"""GPU tests of batched solves (amg_batch_*): systems of different sizes and
depths advanced together.  Each system must follow the oracle (same stop
iteration within one, the same iterate at equal iteration count), and its
result must be bit-identical whether it is solved alone or in a mix, with or
without graph replay."""
import numpy as np
import pytest

import oracle
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


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def maxrel(a, b):
    """Largest element-wise difference relative to the largest element of b."""
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def mix():
    """SPD systems of several sizes and hierarchy depths (a ragged mix), one with
    many tied weights and explicit zeros."""
    out = [P.lognormal_diffusion3d(m, 1000 + m, 1.0) for m in (5, 9, 16, 23, 12, 31)]
    out.append(P.poisson3d(21, 17, 13))
    out.append(P.poisson2d(40))
    out.append(P.vardiff3d(14, seed=2, corr_len=3.0))
    out.append(P.random_symmetric_pattern(300, 0.02, 3, weights=(1, 2), explicit_zeros=0.1))
    return out


def make_batch(torch, systems, params, seeds):
    hs = [hemamg.Hierarchy(hemamg.DeviceCSR.from_host(a), params) for a in systems]
    bt = hemamg.Batch(hs)
    off = bt.offsets
    rhs = np.concatenate([P.rhs_uniform(a.n, s) for a, s in zip(systems, seeds)])
    assert off[-1] == rhs.size
    return hs, bt, torch.from_numpy(rhs).cuda()


def run(torch, systems, params, seeds, rtol=1e-8, maxit=500, x0=None):
    hs, bt, rhs = make_batch(torch, systems, params, seeds)
    try:
        x = torch.zeros_like(rhs) if x0 is None else torch.from_numpy(x0).cuda()
        x, infos = bt.solve(rhs, x, rtol=rtol, maxit=maxit)
        off = bt.offsets
        xs = x.cpu().numpy()
        return [xs[off[i]:off[i + 1]] for i in range(len(systems))], infos
    finally:
        bt.close()
        for h in hs:
            h.close()


@pytest.mark.parametrize("fp32", [0, 1])
def test_batch_follows_the_oracle(torch, fp32):
    systems = mix()
    seeds = list(range(len(systems)))
    params = hemamg.amg_params_default(precond_fp32=fp32)
    xs, infos = run(torch, systems, params, seeds)
    for i, (a, x, inf) in enumerate(zip(systems, xs, infos)):
        say("system", i, "n", a.n, inf)
        assert inf["status"] == hemamg.AMG_OK
        b = P.rhs_uniform(a.n, seeds[i])
        assert np.linalg.norm(b - a.to_scipy() @ x) <= 1e-8 * np.linalg.norm(b) * (1 + 1e-6)
        o = oracle.Hierarchy(a)
        xo, io = o.solve(b, rtol=1e-8, maxit=500)
        if fp32:
            assert abs(inf["iters"] - io["iters"]) <= max(2, int(0.05 * io["iters"])), (inf, io)
        else:
            assert abs(inf["iters"] - io["iters"]) <= 1, (inf, io)


def test_batch_equal_iterations_match_the_oracle(torch):
    systems = mix()
    seeds = [7 + i for i in range(len(systems))]
    K = 12
    xs, infos = run(torch, systems, hemamg.amg_params_default(), seeds, rtol=0.0, maxit=K)
    for i, (a, x, inf) in enumerate(zip(systems, xs, infos)):
        assert inf["status"] == hemamg.AMG_ENOTCONV and inf["iters"] == K, inf
        xo, io = oracle.Hierarchy(a).solve(P.rhs_uniform(a.n, seeds[i]), rtol=0.0, maxit=K)
        assert io["iters"] == K
        err, emax = rel(x, xo), maxrel(x, xo)
        say("system", i, "n", a.n, "rel err", err, "max element err", emax)
        assert err <= 1e-9 and emax <= 1e-9


@pytest.mark.parametrize("fp32", [0, 1])
def test_alone_and_in_the_mix_bit_identical(torch, fp32, monkeypatch):
    systems = mix()
    seeds = list(range(len(systems)))
    params = hemamg.amg_params_default(precond_fp32=fp32)
    xs, infos = run(torch, systems, params, seeds)
    # reversed order, and without graph replay
    monkeypatch.setenv("HEMAMG_BATCH_GRAPHS", "0")
    xr, ir = run(torch, systems[::-1], params, seeds[::-1])
    monkeypatch.delenv("HEMAMG_BATCH_GRAPHS")
    for i in (0, 3, 6, 8):
        xa, ia = run(torch, [systems[i]], params, [seeds[i]])
        assert ia[0]["iters"] == infos[i]["iters"] == ir[len(systems) - 1 - i]["iters"]
        np.testing.assert_array_equal(bits(xa[0]), bits(xs[i]), err_msg=f"system {i}")
        np.testing.assert_array_equal(bits(xr[len(systems) - 1 - i]), bits(xs[i]), err_msg=f"system {i} reversed")


def test_batch_iterations_equal_the_single_solver(torch):
    systems = mix()
    params = hemamg.amg_params_default()
    xs, infos = run(torch, systems, params, list(range(len(systems))))
    for i, a in enumerate(systems):
        with hemamg.Hierarchy(hemamg.DeviceCSR.from_host(a), params) as g:
            x1, i1 = g.solve(torch.from_numpy(P.rhs_uniform(a.n, i)).cuda(), rtol=1e-8, maxit=500)
        assert abs(i1["iters"] - infos[i]["iters"]) <= 1
        assert rel(xs[i], x1.cpu().numpy()) <= 1e-8


def test_initial_guess_zero_rhs_and_limits(torch):
    systems = [P.lognormal_diffusion3d(10, 3, 1.0), P.poisson3d(9), P.lognormal_diffusion3d(13, 4, 1.0)]
    params = hemamg.amg_params_default()
    hs, bt, rhs = make_batch(torch, systems, params, [1, 2, 3])
    try:
        off = bt.offsets
        rhs[off[1]:off[2]] = 0.0  # system 1: b = 0 -> x = 0
        x0 = torch.ones_like(rhs)
        x, infos = bt.solve(rhs, x0.clone(), rtol=1e-8, maxit=500)
        assert [i["status"] for i in infos] == [hemamg.AMG_OK] * 3
        assert infos[1]["iters"] == 0
        xs = x.cpu().numpy()
        assert np.all(xs[off[1]:off[2]] == 0.0)
        for i in (0, 2):
            a = systems[i]
            b = rhs[off[i]:off[i + 1]].cpu().numpy()
            assert np.linalg.norm(b - a.to_scipy() @ xs[off[i]:off[i + 1]]) <= 1e-8 * np.linalg.norm(b) * 1.000001
        # iteration limit: every live system reports it, x keeps the last iterate
        _, lim = bt.solve(rhs, x0.clone(), rtol=1e-14, maxit=3)
        assert [i["status"] for i in lim] == [hemamg.AMG_ENOTCONV, hemamg.AMG_OK, hemamg.AMG_ENOTCONV]
        assert lim[0]["iters"] == 3 and lim[2]["iters"] == 3
        # non-finite input is refused
        bad = rhs.clone()
        bad[off[2]] = float("nan")
        _, nf = bt.solve(bad, x0.clone())
        assert all(i["status"] == hemamg.AMG_ENOTFINITE for i in nf)
    finally:
        bt.close()
        for h in hs:
            h.close()


def test_batch_argument_checks(torch):
    a = P.lognormal_diffusion3d(8, 1, 1.0)
    with hemamg.Hierarchy(hemamg.DeviceCSR.from_host(a)) as g64, \
            hemamg.Hierarchy(hemamg.DeviceCSR.from_host(a), precond_fp32=1) as g32, \
            hemamg.Hierarchy(hemamg.DeviceCSR.from_host(P.poisson2d(5))) as tiny:
        assert tiny.nlevels == 1
        for hs in ([g64, g32], [g64, tiny], []):
            with pytest.raises(hemamg.AmgError) as e:
                hemamg.Batch(hs)
            assert e.value.status == hemamg.AMG_EINVAL
        with hemamg.Batch([g64]) as bt:
            rhs = torch.ones(a.n, dtype=torch.float64, device="cuda")
            st = hemamg.lib().amg_batch_solve(bt.b, hemamg.STATIONARY, rhs.data_ptr(), rhs.data_ptr(), 1e-8, 10,
                                              hemamg._stream_ptr(None), (hemamg.amg_info * 1)())
            assert st == hemamg.AMG_EINVAL


def test_batch_of_many_with_a_large_system(torch):
    """A 64^3 system with 40 small ones: deep and shallow hierarchies side by
    side, many reduction blocks, solved alone and in the batch."""
    systems = [P.poisson3d(64)] + [P.lognormal_diffusion3d(6 + (i % 9), 50 + i, 1.0) for i in range(40)]
    seeds = list(range(len(systems)))
    params = hemamg.amg_params_default()
    xs, infos = run(torch, systems, params, seeds)
    assert all(i["status"] == hemamg.AMG_OK for i in infos)
    xa, ia = run(torch, [systems[0]], params, [0])
    assert ia[0]["iters"] == infos[0]["iters"]
    np.testing.assert_array_equal(bits(xa[0]), bits(xs[0]))
    for i in (1, 17, 40):
        xo, io = oracle.Hierarchy(systems[i]).solve(P.rhs_uniform(systems[i].n, seeds[i]), rtol=1e-8, maxit=500)
        assert abs(io["iters"] - infos[i]["iters"]) <= 1


@pytest.mark.parametrize("fp32", [0, 1])
def test_batch_autotune_keeps_every_bit(torch, fp32):
    """Tuning the rows per block of the concatenated levels changes launch
    shapes only: results before and after are bit-identical."""
    systems = mix()
    seeds = list(range(len(systems)))
    params = hemamg.amg_params_default(precond_fp32=fp32)
    hs, bt, rhs = make_batch(torch, systems, params, seeds)
    try:
        x0, i0 = bt.solve(rhs, rtol=1e-8, maxit=500)
        sched = bt.autotune()
        say("batch schedule", sched)
        assert len(sched) == hemamg.amg_batch_levels(bt.b)
        assert all(v in (128, 256, 512) for v in sched[:-1]) and sched[-1] == 0
        x1, i1 = bt.solve(rhs, rtol=1e-8, maxit=500)
        assert [a["iters"] for a in i0] == [a["iters"] for a in i1]
        np.testing.assert_array_equal(bits(x0.cpu().numpy()), bits(x1.cpu().numpy()))
    finally:
        bt.close()
        for h in hs:
            h.close()


def separate(torch, systems, params, seeds):
    xs, infos = run(torch, systems, params, seeds)
    return xs, infos


def setup_batch(torch, systems, params, seeds):
    devs = [hemamg.DeviceCSR.from_host(a) for a in systems]
    bt = hemamg.Batch.setup(devs, params)
    return bt, devs


@pytest.mark.parametrize("kw", [dict(), dict(precond_fp32=1), dict(alternate=1), dict(hem=1),
                                dict(passes_per_level=1, max_coarse_rows=16),
                                dict(passes_per_level=1, alternate=1, max_coarse_rows=16)])
def test_batched_setup_equals_separate_setups(torch, kw):
    """Building the hierarchies together (block-diagonal concatenations, one
    matching round for all) gives every system the hierarchy amg_setup
    builds: the batched solve is bit-identical to the batch assembled from
    separate hierarchies."""
    say("params", kw)
    systems = mix()
    seeds = list(range(len(systems)))
    params = hemamg.amg_params_default(**kw)
    xs, infos = separate(torch, systems, params, seeds)
    bt, devs = setup_batch(torch, systems, params, seeds)
    try:
        assert bt.status == [hemamg.AMG_OK] * len(systems)
        off = bt.offsets
        rhs = torch.from_numpy(np.concatenate([P.rhs_uniform(a.n, s) for a, s in zip(systems, seeds)])).cuda()
        x, inf2 = bt.solve(rhs, rtol=1e-8, maxit=500)
        xh = x.cpu().numpy()
        for i in range(len(systems)):
            assert inf2[i]["iters"] == infos[i]["iters"], (i, inf2[i], infos[i])
            np.testing.assert_array_equal(bits(xh[off[i]:off[i + 1]]), bits(xs[i]), err_msg=f"system {i}")
    finally:
        bt.close()


def test_batched_setup_reports_failing_systems(torch):
    good = [P.lognormal_diffusion3d(10, 5, 1.0), P.poisson3d(12), P.lognormal_diffusion3d(14, 6, 1.0)]
    zero_diag = P.poisson3d(6)
    zero_diag.val = zero_diag.val.copy()
    row = slice(zero_diag.row_ptr[7], zero_diag.row_ptr[8])
    zero_diag.val[row][zero_diag.col[row] == 7] = 0.0
    tiny = P.poisson2d(5)  # one level: not batched
    systems = [good[0], zero_diag, good[1], tiny, good[2]]
    params = hemamg.amg_params_default()
    bt, devs = setup_batch(torch, systems, params, None)
    try:
        assert bt.status == [hemamg.AMG_OK, hemamg.AMG_EINVAL, hemamg.AMG_OK, hemamg.AMG_EINVAL, hemamg.AMG_OK]
        off = bt.offsets
        assert off[2] - off[1] == 0 and off[4] - off[3] == 0
        rhs = torch.from_numpy(np.concatenate([P.rhs_uniform(a.n, 3) if bt.status[i] == 0 else np.zeros(0)
                                               for i, a in enumerate(systems)])).cuda()
        x, infos = bt.solve(rhs, rtol=1e-8, maxit=500)
        assert [i["status"] for i in infos] == bt.status
        xh = x.cpu().numpy()
        for i, a in ((0, good[0]), (2, good[1]), (4, good[2])):
            xa, ia = run(torch, [a], params, [3])
            assert ia[0]["iters"] == infos[i]["iters"]
            np.testing.assert_array_equal(bits(xh[off[i]:off[i + 1]]), bits(xa[0]))
    finally:
        bt.close()


def test_batched_setup_stall_and_depths(torch):
    """Systems of very different depths and a high-contrast one whose coarse
    levels stall (stall-ratio stop): every system stops where amg_setup
    stops, and systems leave the concatenation at different levels."""
    systems = [P.vardiff3d(24, seed=3), P.lognormal_diffusion3d(7, 2, 1.0), P.poisson3d(40),
               P.lognormal_diffusion3d(20, 9, 2.0)]
    params = hemamg.amg_params_default()
    for a in systems:
        with hemamg.Hierarchy(hemamg.DeviceCSR.from_host(a), params) as g:
            say("n", a.n, "levels", g.nlevels, [hemamg.amg_level_size(g.h, k)[0] for k in range(g.nlevels)])
    seeds = [11, 12, 13, 14]
    xs, infos = separate(torch, systems, params, seeds)
    bt, devs = setup_batch(torch, systems, params, seeds)
    try:
        assert bt.status == [hemamg.AMG_OK] * 4
        assert hemamg.amg_batch_levels(bt.b) == max(hemamg.Hierarchy(d, params).nlevels for d in devs)
        off = bt.offsets
        rhs = torch.from_numpy(np.concatenate([P.rhs_uniform(a.n, s) for a, s in zip(systems, seeds)])).cuda()
        x, inf2 = bt.solve(rhs, rtol=1e-8, maxit=500)
        xh = x.cpu().numpy()
        for i in range(4):
            assert inf2[i]["iters"] == infos[i]["iters"]
            np.testing.assert_array_equal(bits(xh[off[i]:off[i + 1]]), bits(xs[i]), err_msg=f"system {i}")
    finally:
        bt.close()


def nonsym_mix():
    """Nonsymmetric systems of several sizes: upwind convection-diffusion and
    random patterns with unsymmetric values."""
    out = [P.convdiff3d(m) for m in (7, 11, 16, 24)]
    out.append(P.random_symmetric_pattern(400, 0.015, 4, weights=(1, 2, 3), nonsym_values=True))
    for a in out[-1:]:  # diagonally dominant so that the method converges
        d = a.to_scipy()
        import scipy.sparse as sp
        rows = np.abs(d).sum(axis=1).A.ravel()
        a2 = (d + sp.diags(rows + 1.0)).tocsr()
        a2.sort_indices()
        out[-1] = P.CSR(a2.shape[0], a2.indptr.astype(np.int32), a2.indices.astype(np.int32), a2.data)
    return out


@pytest.mark.parametrize("fp32", [0, 1])
def test_batched_bicgstab_follows_the_oracle_and_is_composition_independent(torch, fp32):
    systems = nonsym_mix()
    seeds = [20 + i for i in range(len(systems))]
    params = hemamg.amg_params_default(precond_fp32=fp32)
    hs, bt, rhs = make_batch(torch, systems, params, seeds)
    try:
        x, infos = bt.solve(rhs, rtol=1e-8, maxit=500, method="bicgstab")
        off = bt.offsets
        xh = x.cpu().numpy()
    finally:
        bt.close()
        for h in hs:
            h.close()
    for i, (a, inf) in enumerate(zip(systems, infos)):
        say("system", i, "n", a.n, inf)
        assert inf["status"] == hemamg.AMG_OK
        b = P.rhs_uniform(a.n, seeds[i])
        xi = xh[off[i]:off[i + 1]]
        assert np.linalg.norm(b - a.to_scipy() @ xi) <= 1e-8 * np.linalg.norm(b) * (1 + 1e-6)
        xo, io = oracle.Hierarchy(a).solve(b, method="bicgstab", rtol=1e-8, maxit=500)
        tol = max(2, int(0.05 * io["iters"])) if fp32 else 1
        assert abs(inf["iters"] - io["iters"]) <= tol, (inf, io)
        # alone (a batch of one, from the batched setup) gives the same bits
        bt1 = hemamg.Batch.setup([hemamg.DeviceCSR.from_host(a)], params)
        try:
            x1, i1 = bt1.solve(torch.from_numpy(b).cuda(), rtol=1e-8, maxit=500, method="bicgstab")
        finally:
            bt1.close()
        assert i1[0]["iters"] == inf["iters"]
        np.testing.assert_array_equal(bits(x1.cpu().numpy()), bits(xi))


def test_batched_bicgstab_equal_iterations_match_the_oracle(torch):
    systems = nonsym_mix()
    seeds = [30 + i for i in range(len(systems))]
    K = 6
    hs, bt, rhs = make_batch(torch, systems, hemamg.amg_params_default(), seeds)
    try:
        x, infos = bt.solve(rhs, rtol=0.0, maxit=K, method="bicgstab")
        off = bt.offsets
        xh = x.cpu().numpy()
    finally:
        bt.close()
        for h in hs:
            h.close()
    for i, a in enumerate(systems):
        assert infos[i]["iters"] == K and infos[i]["status"] == hemamg.AMG_ENOTCONV
        xo, io = oracle.Hierarchy(a).solve(P.rhs_uniform(a.n, seeds[i]), method="bicgstab", rtol=0.0, maxit=K)
        err, emax = rel(xh[off[i]:off[i + 1]], xo), maxrel(xh[off[i]:off[i + 1]], xo)
        say("system", i, "rel err", err, "max element err", emax)
        assert err <= 1e-9 and emax <= 1e-9


def test_batched_setup_at_served_sizes(torch):
    """A group as the server forms it from the served stream: 96^3 (the
    largest side) with smaller lognormal systems, float preconditioner; the
    batched setup and solve equal the separate hierarchies' batch bit for
    bit, and every system meets the tolerance."""
    sides = [96, 16, 41, 23, 64, 18, 30, 55]
    systems = [P.lognormal_diffusion3d(m, 2000 + m, 1.0) for m in sides]
    seeds = [2000 + m for m in sides]
    params = hemamg.amg_params_default(precond_fp32=1)
    xs, infos = separate(torch, systems, params, seeds)
    bt, devs = setup_batch(torch, systems, params, seeds)
    try:
        assert bt.status == [hemamg.AMG_OK] * len(systems)
        off = bt.offsets
        rhs = torch.from_numpy(np.concatenate([P.rhs_uniform(a.n, s) for a, s in zip(systems, seeds)])).cuda()
        x, inf2 = bt.solve(rhs, rtol=1e-8, maxit=1000)
        xh = x.cpu().numpy()
        for i, a in enumerate(systems):
            say("side", sides[i], inf2[i])
            assert inf2[i]["status"] == hemamg.AMG_OK and inf2[i]["iters"] == infos[i]["iters"]
            np.testing.assert_array_equal(bits(xh[off[i]:off[i + 1]]), bits(xs[i]), err_msg=f"side {sides[i]}")
            b = P.rhs_uniform(a.n, seeds[i])
            assert np.linalg.norm(b - a.to_scipy() @ xh[off[i]:off[i + 1]]) <= 1e-8 * np.linalg.norm(b) * 1.000001
    finally:
        bt.close()


@pytest.mark.parametrize("compact", [0, 1])
@pytest.mark.parametrize("alternate", [0, 1])
def test_batched_setup_tiles_across_systems(torch, alternate, compact, monkeypatch):
    """Tiled matching inside a batched setup: with the per-system LDS limit at
    200 rows and tiles of 37 rows, the small systems are matched one
    workgroup each and marked decided, and the others by tiles that straddle
    system boundaries and those decided rows.  The batch must equal the
    hierarchies set up one by one (which use the same drivers alone)."""
    say("alternate", alternate, "compact", compact)
    monkeypatch.setenv("HEMAMG_HEM_LDS", "200")
    monkeypatch.setenv("HEMAMG_HEM_TILE", "37")
    monkeypatch.setenv("HEMAMG_HEM_TILE_C", "37" if compact else "0")
    monkeypatch.setenv("HEMAMG_TILE_STRICT", "1")
    systems = mix()
    seeds = list(range(len(systems)))
    params = hemamg.amg_params_default(alternate=alternate)
    xs, infos = separate(torch, systems, params, seeds)
    bt, devs = setup_batch(torch, systems, params, seeds)
    try:
        assert bt.status == [hemamg.AMG_OK] * len(systems)
        off = bt.offsets
        rhs = torch.from_numpy(np.concatenate([P.rhs_uniform(a.n, s) for a, s in zip(systems, seeds)])).cuda()
        x, inf2 = bt.solve(rhs, rtol=1e-8, maxit=500)
        xh = x.cpu().numpy()
        for i in range(len(systems)):
            assert inf2[i]["iters"] == infos[i]["iters"], (i, inf2[i], infos[i])
            np.testing.assert_array_equal(bits(xh[off[i]:off[i + 1]]), bits(xs[i]), err_msg=f"system {i}")
    finally:
        bt.close()
