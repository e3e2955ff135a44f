"""Benchmark: AMG-preconditioned Krylov solve on one MI355X.

One step = the whole hot path on one synthetic system already resident in GPU
memory: amg_setup (matching, Galerkin products, coarsest LU) + krylov_solve
to the workload's relative tolerance + amg_destroy.  After the timed steps
the same run measures the served stream (1024 requests of lognormal
diffusion, plain double form against the batched float-preconditioned form
at the plain form's capacity, and the batched form in closed loop) and the
CPU oracle on a bounded sample.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--gpus 1]
                  [--no-serve] [--no-cpu-baseline]
  python bench.py --serve-only   (the served stream alone, with more rates)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "AMG-PCG time to 1e-8 residual + HBM GB/s; served solves/s, p50/p99 latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2007_00056_amd", "csrc", "k_vcycle.hip")
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash() -> str:
    import hashlib

    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, precond: str):
    """HBM bytes per launch from the committed counter summary of this kernel
    and workload, if it was taken on the current kernel source (else None)."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_{precond}_traffic.txt")
    try:
        # "key: value" lines; keys may hold a colon themselves, values do not
        kv = dict(line.rsplit(":", 1) for line in open(path) if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel") != kernel or kv.get("k_vcycle.hip sha256[:16]") != kernel_source_hash():
        return None
    return float(kv["hbm_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def level_sizes(h, hemamg):
    L = hemamg.amg_num_levels(h)
    return [hemamg.amg_level_size(h, k) for k in range(L)]


STREAM_MIN = 262144  # levels with at least this many rows use the CSR-stream kernels


def kernel_bytes(sizes, e, method):
    """Bytes each timed level-0 kernel moves as implemented: preconditioner
    values and vectors of e bytes (8 double, 4 float), int32 indices, the
    level-0 right-hand side and result in double; every array counted once."""
    (n, nnz) = sizes[0]
    csr = (e + 4) * nnz + 4 * (n + 1)
    return {
        # postsmoothing from the prolongated iterate xp: xp gather and D^{-1}
        # (2e n), z write (8 n), and g = D^{-1} f: a double level 0 forms it from
        # f (8 n read), a float one reads it (4 n); PCG's fused (r, z) reads r = f
        0: csr + 2 * e * n + 8 * n + (8 * n if e == 8 else 4 * n + (8 * n if method == "pcg" else 0)),
        # presmoothing + residual: g gather, r read (8 n), residual write
        1: csr + 2 * e * n + 8 * n,
        # outer SpMV + dot, always double: p read + q write
        2: 12 * nnz + 4 * (n + 1) + 16 * n,
    }


def model_bytes(sizes, e):
    """The per-launch byte model of the fused prolongation + postsmoothing on
    level 0 (values of e bytes, int32 columns): (e + 4) nnz + 32 N + 8 N_c,
    i.e. 12 nnz + 32 N + 8 N_c in double."""
    (n, nnz), nc = sizes[0], sizes[1][0]
    return (e + 4) * nnz + 32 * n + 8 * nc


def host_cpu():
    """Host description for the CPU baseline: logical CPUs and model name."""
    import subprocess

    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        nproc = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout.strip())
    except (OSError, ValueError, subprocess.SubprocessError):
        nproc = os.cpu_count()
    return {"nproc": nproc, "model": model}


def level_bytes(k, sizes, e):
    """One V-cycle level k (down + up sweep) in the fused form, values and
    vectors of e bytes; level 0 reads its right-hand side in double."""
    n, nnz = sizes[k]
    nc = sizes[k + 1][0]
    nf = sizes[k - 1][0] if k > 0 else 0
    csr = (e + 4) * nnz + 4 * (n + 1)
    fin = 8 if k == 0 else e
    scatter = (16 * n + 2 * e * nf) if k > 0 else 0  # members + finer g read + finer xp write
    if n >= STREAM_MIN:
        down = (csr + (fin + 2 * e) * n) + (e * n + (16 + 3 * e) * nc)  # residual, restriction (+ g_c)
    else:
        down = csr + (fin + e) * n + (16 + 3 * e) * nc  # fused residual + restriction
    up = csr + 4 * e * n + scatter
    return down + up


def iteration_bytes(sizes, method, e):
    """Algorithmic bytes of one Krylov iteration (V-cycle + outer kernels)."""
    vc = sum(level_bytes(k, sizes, e) for k in range(len(sizes) - 1))
    m = sizes[-1][0]
    vc += 8 * m * m + 2 * e * m + (16 * m + 2 * e * sizes[-2][0] if len(sizes) > 1 else 0)
    n, nnz = sizes[0]
    vc += (8 - e) * n  # level-0 result in double
    spmv = 12 * nnz + 4 * (n + 1) + 16 * n
    if method == "pcg":
        # spmv+dot, update (x,r,p,q,dinv read; x,r write; g write), (r,z) in the V-cycle, direction (z,p read; p write)
        return vc + spmv + 8 * n + 56 * n + e * n + 24 * n
    # BiCGStab: 2 V-cycles (+ D^{-1} scaling of their inputs), 2 SpMVs, s, update, direction
    return 2 * vc + 2 * (16 + e) * n + 2 * spmv + 24 * n + 72 * n + 32 * n


def cpu_baseline(a, b, spec, gpu_iters, hem=0, alternate=0, budget_s=25.0):
    """The oracle (single-threaded C) on the same input: setup + solve, with
    the solve cut to fit `budget_s` and scaled to the GPU's iteration count."""
    import oracle

    t0 = time.perf_counter()
    h = oracle.Hierarchy(a, hem=hem, alternate=alternate)
    t_setup = time.perf_counter() - t0
    # time a few iterations first to size the sample
    t0 = time.perf_counter()
    _, info = h.solve(b, method=spec["kind"], rtol=spec["rtol"], maxit=2)
    per_it = (time.perf_counter() - t0) / max(info["iters"], 1)
    cap = max(1, int((budget_s - t_setup) / per_it)) if per_it > 0 else gpu_iters
    t0 = time.perf_counter()
    _, info = h.solve(b, method=spec["kind"], rtol=spec["rtol"], maxit=min(cap, 10 * gpu_iters + 10))
    t_solve = time.perf_counter() - t0
    done = max(info["iters"], 1)
    full = info["status"] == oracle.OK
    est_solve = t_solve if full else t_solve * gpu_iters / done
    total = t_setup + est_solve
    h.close()
    return dict({
        "value": 1.0 / total, "unit": "solves/s", "cores": 1, "kind": "oracle",
        "sample": (f"one setup ({t_setup:.2f} s) + {'full solve' if full else 'partial solve'} of {done} "
                   f"iterations ({t_solve:.2f} s)" + ("" if full else f", scaled to {gpu_iters} iterations")),
        "setup_s": t_setup, "solve_s": est_solve, "oracle_iters": info["iters"],
    }, **host_cpu())


def gen_request(item):
    """Matrix and right-hand side of one served request (side, seed)."""
    from paper_2007_00056_amd import problems as P

    side, seed = item
    a = P.lognormal_diffusion3d(side, seed, 1.0)
    return a, P.rhs_uniform(a.n, seed)


def served_stream(args, rates, closed_streams=False):
    """Served stream: requests of side log-uniform in [16, 96] with lognormal
    coefficients arrive as a Poisson process.  The plain form solves them one
    at a time in double; the batched form runs `--workers` workers that group
    queued requests (up to `--batch`) into batched setups and solves with the
    float preconditioner.  Both see the same arrival trace, at rates that are
    fractions of the plain form's measured capacity.  Returns a dict."""
    from concurrent.futures import ProcessPoolExecutor

    import torch

    from paper_2007_00056_amd import hemamg, problems as P

    t_gen = time.perf_counter()
    stream = P.served_stream(args.requests, seed=0)
    log(f"generating {len(stream)} requests")
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        reqs = list(ex.map(gen_request, stream, chunksize=4))
    dev = []
    for a, b in reqs:
        A = hemamg.DeviceCSR.from_host(a)
        dev.append((A, torch.from_numpy(b).cuda(), torch.zeros(a.n, dtype=torch.float64, device="cuda")))
    torch.cuda.synchronize()
    rows = sum(a.n for a, _ in reqs)
    del reqs
    log(f"{len(dev)} requests, {rows} rows in total, ready in {time.perf_counter() - t_gen:.1f} s")

    def run(workers, fp32, arrivals, batch=0, limit=None):
        cfg = hemamg.amg_server_config_default(workers=workers, batch=batch)
        cfg.params.precond_fp32 = fp32
        srv = hemamg.amg_server_create(cfg)
        items = dev if limit is None else dev[:limit]
        for _, _, x in items:
            x.zero_()
        torch.cuda.synchronize()
        tickets = []
        t0 = time.perf_counter()
        for i, (A, b, x) in enumerate(items):
            if arrivals is not None:
                dt = t0 + arrivals[i] - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            tickets.append((time.perf_counter() - t0, hemamg.amg_server_submit(srv, A, b, x, hemamg.PCG, 1e-8, 1000)))
        res = [hemamg.amg_server_wait(srv, t) for _, t in tickets]
        hemamg.amg_server_destroy(srv)
        bad = [r for r in res if r["status"] != hemamg.AMG_OK]
        if bad:
            raise RuntimeError(f"{len(bad)} requests failed, e.g. {bad[0]}")
        lat = np.array([r["latency_ms"] for r in res])
        done = max(ts + l / 1e3 for (ts, _), l in zip(tickets, lat))
        return dict(solves_per_s=len(res) / done, p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)), mean_iters=float(np.mean([r["iters"] for r in res])))

    run(1, 0, None, limit=32)  # warm-up
    run(args.workers, 1, None, args.batch, limit=64)
    cap = run(1, 0, None)
    log(f"plain capacity {cap['solves_per_s']:.1f} solves/s")
    rng = np.random.default_rng(0)
    gaps = rng.exponential(1.0, len(dev))
    out_rates = {}
    for f in rates:
        lam = f * cap["solves_per_s"]
        arr = np.cumsum(gaps) / lam
        r = {"plain": run(1, 0, arr), "batched": run(args.workers, 1, arr, args.batch)}
        if closed_streams:
            r["served"] = run(args.workers, 1, arr)
        out_rates[str(f)] = r
        log(f"rate {f}: {r}")
    closed_b = run(args.workers, 1, None, args.batch)
    log(f"closed loop, batched: {closed_b}")
    out = {"workload": "served lognormal diffusion stream", "requests": len(dev), "rows": rows, "side": [16, 96],
           "sigma": 1.0, "rtol": 1e-8, "method": "pcg", "workers": args.workers, "batch": args.batch,
           "plain": "one request at a time, double", "batched": "grouped batched setup + solve, float preconditioner",
           "plain_capacity": cap, "rates": out_rates, "batched_closed_loop": closed_b}
    if closed_streams:
        out["served_closed_loop"] = run(args.workers, 1, None)
    del dev
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def serve_main(args):
    """The served stream alone (--serve-only): one JSON line."""
    out = served_stream(args, args.rates, closed_streams=True)
    best = out["batched_closed_loop"]
    print(json.dumps({
        "metric": "served solves/s, p50/p99 latency", "value": best["solves_per_s"], "unit": "solves/s",
        "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "dtype": "f32+f64",
        "config": {k: out[k] for k in ("workload", "requests", "rows", "side", "sigma", "rtol", "method", "workers",
                                       "batch")},
        "served": out,
    }), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="poisson3d_128")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precond", choices=["fp64", "fp32"], default=None,
                    help="preconditioner precision (default: the workload's)")
    ap.add_argument("--hem", choices=["node", "edge"], default="node",
                    help="matching: node-based (Algorithm 2) or edge-based (Algorithm 3)")
    ap.add_argument("--alternate", action="store_true",
                    help="node-based passes alternate between the first and the last index")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="no HIP events in the timed region (roofline fields are then null)")
    ap.add_argument("--time-all-kernels", action="store_true",
                    help="also time the level-0 residual and the outer SpMV (more events in the timed region)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, copy 256 MiB device-to-device (counter calibration for profiles)")
    ap.add_argument("--serve-only", action="store_true", help="the served stream of solve requests alone")
    ap.add_argument("--no-serve", action="store_true", help="skip the served stream after the timed steps")
    ap.add_argument("--requests", type=int, default=1024)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--batch", type=int, default=32, help="batched serving: most requests per batched solve")
    ap.add_argument("--rates", type=lambda t: [float(v) for v in t.split(",")], default=[0.5, 1.0, 2.0],
                    help="arrival rates (fractions of the plain capacity) of --serve-only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solver runs on one "
              "GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2007_00056_amd import hemamg, problems as P

    if not torch.cuda.is_available():
        log("bench.py needs a ROCm GPU")
        sys.exit(1)
    if args.serve_only:
        serve_main(args)
        return
    torch.cuda.set_device(0)
    log(f"generating {args.workload} (seed {args.seed})")
    a, b_host, spec = P.make_workload(args.workload, args.seed)
    method = spec["kind"]
    A = hemamg.DeviceCSR.from_host(a)
    b = torch.from_numpy(b_host).cuda()
    x = torch.zeros_like(b)
    precond = args.precond or spec["precond"]
    params = hemamg.amg_params_default(precond_fp32=int(precond == "fp32"), hem=int(args.hem == "edge"),
                                        alternate=int(args.alternate))
    esz = 4 if precond == "fp32" else 8
    mcode = hemamg.PCG if method == "pcg" else hemamg.BICGSTAB
    torch.cuda.synchronize()

    # HIP events bracket the timed kernels on the library's stream; by default only
    # the dominant one (level-0 prolongation + postsmoothing) is timed
    kern_tot = {0: [0, 0.0], 1: [0, 0.0], 2: [0, 0.0]} if args.time_all_kernels else {0: [0, 0.0]}
    if args.no_kernel_timing:
        kern_tot = {}

    def step(timed):
        t0 = time.perf_counter()
        h = hemamg.amg_setup(A, params)
        t1 = time.perf_counter()
        if timed:
            for k in kern_tot:
                hemamg.amg_timing_enable(h, k, True)
        x.zero_()
        info = hemamg.krylov_solve(h, mcode, b, x, spec["rtol"], 1000)
        t2 = time.perf_counter()
        if timed:
            for k in kern_tot:
                c, ms = hemamg.amg_timing_read(h, k)
                kern_tot[k][0] += c
                kern_tot[k][1] += ms
        sizes = level_sizes(h, hemamg)
        stats = hemamg.amg_setup_stats(h)
        t3 = time.perf_counter()
        hemamg.amg_destroy(h)
        t4 = time.perf_counter()
        return dict(setup_ms=(t1 - t0) * 1e3, solve_ms=(t2 - t1) * 1e3, destroy_ms=(t4 - t3) * 1e3,
                    other_ms=(t3 - t2) * 1e3, iters=info["iters"], true_rel_res=info["true_rel_res"], sizes=sizes,
                    stats=stats)

    for i in range(args.warmup):
        r = step(False)
        log(f"warmup {i}: setup {r['setup_ms']:.2f} ms, solve {r['solve_ms']:.2f} ms, iters {r['iters']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for i in range(args.steps):
        r = step(True)
        recs.append(r)
        log(f"step {i}: setup {r['setup_ms']:.2f} ms, solve {r['solve_ms']:.2f} ms, destroy {r['destroy_ms']:.2f} ms, "
            f"stats {r['other_ms']:.2f} ms, iters {r['iters']}, true rel res {r['true_rel_res']:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    sizes = recs[-1]["sizes"]
    iters = recs[-1]["iters"]
    setup_ms = float(np.median([r["setup_ms"] for r in recs]))
    solve_ms = float(np.median([r["solve_ms"] for r in recs]))
    it_bytes = iteration_bytes(sizes, method, esz)
    kb = kernel_bytes(sizes, esz, method)
    names = {0: "k_vc_post (level 0)", 1: "k_vc_resid (level 0)", 2: "k_stream_spmv_dot (outer SpMV)"}
    kernels = {}
    for k, (c, ms) in kern_tot.items():
        if c:
            avg = ms / c
            kernels[names[k]] = {"launches": c, "avg_us": avg * 1e3, "bytes": kb[k],
                                 "gbs": kb[k] / (avg * 1e-3) / 1e9}
    dom = max(kern_tot, key=lambda k: kern_tot[k][1]) if kern_tot else 0
    c, ms = kern_tot.get(dom, (0, 0.0))
    # the roofline of the dominant kernel (level-0 prolongation + postsmoothing)
    # uses the byte model; the implementation's own count is reported beside it
    mb = model_bytes(sizes, esz)
    avg_s = ms / c * 1e-3 if c else None
    achieved = mb / avg_s / 1e9 if c and dom == 0 else (kb[dom] / avg_s / 1e9 if c else None)
    # setup: matching passes (GPU time of each pass from its own events)
    st = recs[-1]["stats"]
    m_ms = [float(np.median([r["stats"]["match_ms"][i] for r in recs])) for i in range(len(st["rounds"]))]
    passes = []
    for i, (rd, mm, pn, pz) in enumerate(zip(st["rounds"], m_ms, st["pass_n"], st["pass_nnz"])):
        rb = 12 * pz + 4 * (pn + 1)  # one read of the matched operator
        passes.append({"n": pn, "nnz": pz, "rounds": rd, "ms": mm, "us_per_round": mm * 1e3 / max(rd, 1),
                       "read_bytes": rb, "hbm_frac": rb / (mm * 1e-3) / (HBM_PEAK_GBS * 1e9) if mm > 0 else None})
    match_total = sum(m_ms)
    setup_block = {"setup_ms": setup_ms, "matching_ms": match_total, "matching_share_of_setup": match_total / setup_ms,
                   "rounds_total": int(sum(st["rounds"])),
                   "us_per_round": match_total * 1e3 / max(sum(st["rounds"]), 1),
                   "matching_hbm_frac": (sum(p["read_bytes"] for p in passes) / (match_total * 1e-3)
                                         / (HBM_PEAK_GBS * 1e9)) if match_total > 0 else None,
                   "passes": passes}
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precond == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "desc": spec["desc"], "n": a.n, "nnz": a.nnz, "rtol": spec["rtol"],
                   "method": method, "precond": precond, "hem": args.hem,
                   "alternate": int(args.alternate), "levels": len(sizes), "seed": args.seed},
        "setup_ms": setup_ms,
        "solve_ms": solve_ms,
        "destroy_ms": float(np.median([r["destroy_ms"] for r in recs])),
        "between_ms": float(np.median([r["other_ms"] for r in recs])),
        "iters": iters,
        "ms_per_iter": solve_ms / max(iters, 1),
        "solve_gbs": it_bytes * iters / (solve_ms * 1e-3) / 1e9,
        "matching_rounds": st["rounds"],
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": measured_traffic(names[dom].split()[0], args.workload, precond),
                     "algorithmic_bytes": mb if dom == 0 else kb[dom],
                     "bytes_model": f"({esz}+4) nnz + 32 N + 8 N_c" if dom == 0 else "as implemented",
                     "impl_bytes": kb[dom], "avg_us": avg_s * 1e6 if avg_s else None,
                     "impl_frac": kb[dom] / avg_s / 1e9 / HBM_PEAK_GBS if avg_s else None},
        "setup": setup_block,
    }
    if args.copy_calibration:
        src = torch.empty(1 << 25, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 268435456 bytes device-to-device for counter calibration")
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on the same input")
        out["cpu_baseline"] = cpu_baseline(a, b_host, spec, iters, hem=int(args.hem == "edge"),
                                           alternate=int(args.alternate))
    if not args.no_serve:
        del A, b, x
        torch.cuda.empty_cache()
        log("served stream")
        out["served"] = served_stream(args, [1.0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
