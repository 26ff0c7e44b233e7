"""Benchmarks of the C-A / CUR library on one MI355X.

Default (the headline line): C-A / CUR of a dense 16384 x 16384 float32
matrix.  A = G1 G2 D + 1e-4-scaled Gaussian noise (G1 16384x32, G2 32x16384,
D log-uniform column scales in [0.1, 10]), stored float32 row-major in HBM;
rank k = 32, 4 C-A sweeps from 32 seeded columns, maxvol tau = 0.01, 64 x 64
sampled residual.  Only the gathered strips, the generator and the sample
are read.  One step = one complete C-A / CUR (sweeps, nucleus, residual
estimate) with the matrix resident.

Other workloads (--workload):
  plain      dense binary64 512 x 512, W = G1 G2 + 1e-8 E, k = 8, 3 sweeps
  cauchy     implicit a_ij = 1/(s_i - t_j), m = n = 2^20, adaptive k 8..40 to
             tol 1e-10 (binary64) or 1e-6 (--precision mixed)
  multipole  every far-field block of a 1D adaptive tree over 2^20 mixture
             points, kernel 1/|x - y|, adaptive k 8..48 to tol 1e-8, all
             blocks in one batched launch vs one block per call
  serve      a stream of dense and Cauchy requests (m, n log-uniform in
             [1024, 65536], k in {8, 16, 32, 64}, tol log-uniform in
             [1e-10, 1e-4], binary32 or binary64): served (continuous
             batching) vs plain sequential calls, throughput at saturation
             and p50 / p99 latency under Poisson arrivals

Prints one JSON line.  --gpus N > 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CUR LRAs/s + HBM GB/s, served/batched vs plain at equal err; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# binary64 VALU issue rate: 256 CUs x 64 lanes per clock x 2.4 GHz
VALU64_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# binary64 VALU instructions per generated entry in the engine (one
# subtraction of coordinates and the correctly rounded division sequence:
# 2 div_scale, rcp, 5 fma, mul, div_fmas, div_fixup), from the gfx950 assembly
OPS_PER_ENTRY = 12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu": model}


def _profiled_traffic(summary, kernel_src="paper_1611_01391_amd/csrc/lra_engine.hip"):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None when the engine source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(os.path.join(ROOT, kernel_src), "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    vals = dict(l.split(":", 1) for l in text.splitlines()
                if l.startswith(("traffic_bytes_per_launch:", "engine_source_sha256_prefix:")))
    if vals.get("engine_source_sha256_prefix", "").strip() != sha:
        return None
    return float(vals["traffic_bytes_per_launch"])


def _median_time(fn, reps):
    ts = []
    out = None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), out


def _timed_steps(ctx, torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ctx.set_timing(True, reset=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    st = ctx.stats()
    ctx.set_timing(False, reset=False)
    return t2 - t1, st, out


def _base(args, value, unit, ms_per_step, dtype, config, higher=True):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": higher,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


# ---------------------------------------------------------------------------
# dense workloads (default: 16384^2 float32; plain: 512^2 binary64)
# ---------------------------------------------------------------------------

def _dense_alg_bytes(m, n, k, sweeps, q, s, esz):
    """Entries the method must read, times the element size: per sweep one
    m x k column strip and one k x n row strip, then the k x k generator, the
    q x k, k x s and q x s sample blocks."""
    entries = sweeps * (m * k + k * n) + k * k + q * k + k * s + q * s
    return entries * esz


def bench_dense(args, plain=False):
    import torch

    import synth
    from paper_1611_01391_amd import lra

    if plain:
        n, k, sweeps = 512, 8, 3
        A, d = synth.plain_fp64(args.seed)
        esz = 8
        prec = lra.PREC_FP64
        desc = "dense binary64 512x512 (W = G1 G2 + 1e-8 E, rank 8), k=8, 3 C-A sweeps, 64x64 residual sample"
    else:
        n, k, sweeps = args.n, args.k, args.sweeps
        t0 = time.time()
        A, d = synth.dense_scaled(args.seed, n=n, r=32, k=k)
        log(f"# generated {n}x{n} float32 input in {time.time() - t0:.1f}s")
        esz = 4
        prec = lra.PREC_FP64 if args.precision == "fp64" else lra.PREC_MIXED
        desc = (f"dense float32 {n}x{n} (rank-32 scaled factor-Gaussian + 1e-4 noise), k={k}, "
                f"{sweeps} C-A sweeps, 64x64 residual sample, {args.precision} path")
    dev = torch.device("cuda:0")
    At = torch.from_numpy(A).to(dev)
    torch.cuda.synchronize()
    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        src_t = torch.empty(nb // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst_t = torch.empty_like(src_t)
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t

    ctx = lra.Context()
    src = lra.dense(At)
    kw = dict(init_cols=d.cand_cols, sample_rows=d.sample_rows, sample_cols=d.sample_cols,
              precision=prec, team_wgs=args.team)
    tuned = None
    if args.autotune and not args.team:
        team, tms = ctx.autotune_team(src, k, sweeps, 0.0, init_cols=d.cand_cols, sample_rows=d.sample_rows,
                                      sample_cols=d.sample_cols, precision=prec)
        tuned = {"team_wgs": team, "kernel_ms": tms}
        log(f"# autotuned team: {team} workgroups ({tms:.3f} ms)")
    el, st, res = _timed_steps(ctx, torch, lambda: ctx.ca_cur(src, k, sweeps, 0.0, **kw), args.steps, args.warmup)
    ms_per_step = el * 1e3 / args.steps
    kernel_ms = st["engine_ms_total"] / max(1, st["launches"])
    alg_bytes = _dense_alg_bytes(n, n, k, sweeps, 64, 64, esz)
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    log(f"# gpu: status {res.status} k {res.k} swaps {res.swaps_total} est_rel {res.err_est_rel:.3e} "
        f"kernel {kernel_ms:.3f} ms grid {st['last_grid']}")

    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle
        osrc = oracle.dense(A)
        reps = max(1, args.cpu_samples)
        med, ref = _median_time(lambda: oracle.ca_cur(osrc, k, sweeps, 0.0, d.cand_cols, d.sample_rows,
                                                      d.sample_cols,
                                                      precision="f64" if prec == lra.PREC_FP64 else "f32"),
                                reps)
        cpu = {"value": 1.0 / med, "unit": "CUR LRAs/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} full C-A/CUR runs of the same {n}x{n} workload, single-threaded, "
                         f"median {med:.3f}s", "host": host_info()}
        parity = {"oracle_status": int(ref.status), "same_I": bool(np.array_equal(ref.I, res.I)),
                  "same_J": bool(np.array_equal(ref.J, res.J)),
                  "est_rel_gpu": res.err_est_rel, "est_rel_oracle": ref.err_est_rel,
                  "oracle_min_gap": ref.min_gap()}
    out = _base(args, args.steps / el, "CUR LRAs/s", ms_per_step,
                "f64" if prec == lra.PREC_FP64 else "f32",
                {"workload": desc, "m": n, "n": n, "k": k, "sweeps": sweeps,
                 "precision": "fp64" if prec == lra.PREC_FP64 else "mixed", "autotuned": tuned})
    traffic = None
    if not plain and (n, k, sweeps, args.precision) == (16384, 32, 4, "fp64"):
        traffic = _profiled_traffic("engine_kernel_dense16384_k32.md")
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "engine_kernel",
                       "kernel_ms": kernel_ms, "algorithmic_bytes": alg_bytes}
    if traffic:
        out["roofline"]["traffic_GBps"] = traffic / (kernel_ms * 1e-3) / 1e9
    out["cpu_baseline"] = cpu
    out["parity"] = parity
    out["result"] = {"status": int(res.status), "k": int(res.k), "swaps": int(res.swaps_total),
                     "est_rel": res.err_est_rel, "entries_read": int(res.entries_read)}
    ctx.close()
    return out


# ---------------------------------------------------------------------------
# implicit Cauchy kernel, 2^20 x 2^20
# ---------------------------------------------------------------------------

def _alu_roofline(entries, kernel_ms, kernel="engine_kernel"):
    achieved = entries * OPS_PER_ENTRY / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": VALU64_PEAK_TOPS, "unit": "T VALU op/s (binary64)",
            "frac": achieved / VALU64_PEAK_TOPS, "traffic": None, "kernel": kernel, "kernel_ms": kernel_ms,
            "entries_generated": int(entries), "ops_per_entry": OPS_PER_ENTRY}


def bench_cauchy(args):
    import torch

    import synth
    from paper_1611_01391_amd import lra

    m = 1 << 20
    f64 = args.precision == "fp64"
    dt = np.float64 if f64 else np.float32
    tol = 1e-10 if f64 else 1e-6
    s, t, d = synth.cauchy_points(args.seed, m=m, k=8, k_max=40, dtype=dt)
    ctx = lra.Context()
    src = lra.cauchy(torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda())
    kw = dict(init_cols=d.cand_cols, sample_rows=d.sample_rows, sample_cols=d.sample_cols, k_max=40,
              precision=lra.PREC_FP64 if f64 else lra.PREC_MIXED, raise_on_error=False)
    el, st, res = _timed_steps(ctx, torch, lambda: ctx.ca_cur(src, 8, 4, tol, **kw), args.steps, args.warmup)
    kernel_ms = st["engine_ms_total"] / max(1, st["launches"])
    log(f"# gpu: status {res.status} k {res.k} sweeps {res.sweeps_done} swaps {res.swaps_total} "
        f"est_rel {res.err_est_rel:.3e} kernel {kernel_ms:.3f} ms grid {st['last_grid']}")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        osrc = oracle.cauchy(s, t)
        reps = max(1, min(args.cpu_samples, 5))
        med, ref = _median_time(lambda: oracle.ca_cur(osrc, 8, 4, tol, d.cand_cols, d.sample_rows, d.sample_cols,
                                                      k_max=40, precision="f64" if f64 else "f32"), reps)
        cpu = {"value": 1.0 / med, "unit": "CUR LRAs/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} full adaptive C-A/CUR runs of the same 2^20 x 2^20 Cauchy workload, "
                         f"single-threaded, median {med:.3f}s (oracle status {ref.status}, k {ref.k}, "
                         f"est {ref.err_est_rel:.3e})", "host": host_info()}
    out = _base(args, args.steps / el, "CUR LRAs/s", el * 1e3 / args.steps, "f64" if f64 else "f32",
                {"workload": f"implicit Cauchy 1/(s_i - t_j), s ~ U[0,1], t ~ U[2,3], m = n = 2^20, adaptive k "
                             f"8..40 step 8, tol {tol:g}, up to 4 sweeps per rank",
                 "m": m, "n": m, "k0": 8, "k_max": 40, "tol": tol, "precision": args.precision})
    out["roofline"] = _alu_roofline(res.entries_read, kernel_ms)
    out["cpu_baseline"] = cpu
    out["result"] = {"status": int(res.status), "k": int(res.k), "sweeps": int(res.sweeps_done),
                     "swaps": int(res.swaps_total), "est_rel": res.err_est_rel,
                     "entries_read": int(res.entries_read)}
    ctx.close()
    return out


# ---------------------------------------------------------------------------
# batched far-field blocks
# ---------------------------------------------------------------------------

def bench_multipole(args):
    import torch

    import synth
    from paper_1611_01391_amd import lra

    N = args.points
    tol, kmax = 1e-8, 48
    f64 = args.precision == "fp64"
    t0 = time.time()
    x, blocks, dense_blocks = synth.multipole(args.seed, N, 4096, 96)
    log(f"# {len(blocks)} far-field blocks ({len(dense_blocks)} left dense) in {time.time() - t0:.1f}s")
    xd = torch.from_numpy(x if f64 else x.astype(np.float32)).cuda()
    if not f64:
        tol = 1e-5
    prec = lra.PREC_FP64 if f64 else lra.PREC_MIXED
    jobs = [(lra.invdist(xd[a0:a1], xd[b0:b1]), 8, 4, tol) for (a0, a1, b0, b1) in blocks]
    ctx = lra.Context()
    tuned = None
    if args.autotune:
        floor, fms = ctx.autotune_batched(jobs, k_max=kmax, precision=prec, seed=args.seed)
        tuned = {"floor_rows": floor, "kernel_ms": fms}
        log(f"# autotuned planning floor: {floor} rows ({fms:.2f} ms)")
    el, st, (bst, out_b) = _timed_steps(
        ctx, torch, lambda: ctx.ca_cur_batched(jobs, raise_on_error=False, k_max=kmax, precision=prec,
                                               seed=args.seed),
        args.steps, args.warmup)
    kernel_ms = st["engine_ms_total"] / max(1, st["launches"])
    batched_s = el / args.steps
    entries = sum(r.entries_read for r in out_b)
    log(f"# batched: {batched_s * 1e3:.2f} ms per pass, kernel {kernel_ms:.2f} ms, grid {st['last_grid']}, "
        f"teams {st['last_teams']}")
    # plain: one block per call, same draws (stream seed + block index)
    for b in range(min(8, len(jobs))):
        src, k, sw, tl = jobs[b]
        ctx.ca_cur(src, k, sw, tl, raise_on_error=False, k_max=kmax, precision=prec,
                   seed=synth.block_draws(args.seed, b))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out_p = []
    for b, (src, k, sw, tl) in enumerate(jobs):
        out_p.append(ctx.ca_cur(src, k, sw, tl, raise_on_error=False, k_max=kmax, precision=prec,
                                seed=synth.block_draws(args.seed, b)))
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t1
    same = sum(1 for a, b in zip(out_b, out_p)
               if a.status == b.status and a.err_est_rel == b.err_est_rel and np.array_equal(a.I, b.I)
               and np.array_equal(a.J, b.J))
    from collections import Counter
    statuses = dict(Counter(int(r.status) for r in out_b))
    ks = dict(Counter(int(r.k) for r in out_b))
    met = sum(1 for r in out_b if r.status >= 0 and r.err_est_rel <= tol)
    log(f"# plain: {plain_s * 1e3:.1f} ms for {len(jobs)} calls; identical results {same}/{len(jobs)}")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        step = max(1, len(blocks) // 128)
        sample = list(range(0, len(blocks), step))
        c0 = time.perf_counter()
        for b in sample:
            a0, a1, b0, b1 = blocks[b]
            m, n = a1 - a0, b1 - b0
            kc = max(8, min(kmax, m, n))
            sd = synth.block_draws(args.seed, b)
            cand = oracle.draw_distinct(sd, n, min(n, 2 * kc))
            Q = np.sort(oracle.draw_distinct(sd + 1, m, min(64, m)))
            S = np.sort(oracle.draw_distinct(sd + 2, n, min(64, n)))
            oracle.ca_cur(oracle.invdist(x[a0:a1], x[b0:b1]), 8, 4, tol, cand, Q, S, k_max=kmax,
                          precision="f64" if f64 else "f32")
        cs = time.perf_counter() - c0
        frac = sum((blocks[b][1] - blocks[b][0]) + (blocks[b][3] - blocks[b][2]) for b in sample) / \
            sum((b[1] - b[0]) + (b[3] - b[2]) for b in blocks)
        cpu = {"value": len(sample) / cs, "unit": "CUR LRAs/s (blocks/s)", "cores": 1, "kind": "oracle",
               "sample": f"every {step}th block ({len(sample)} blocks, {frac:.1%} of the rows+columns), "
                         f"single-threaded, {cs:.2f}s", "host": host_info()}
    out = _base(args, len(blocks) / batched_s, "CUR LRAs/s (blocks/s)", batched_s * 1e3, "f64" if f64 else "f32",
                {"workload": f"1D multipole far field: N = {N} mixture points, adaptive binary tree (leaves <= 4096), "
                             f"{len(blocks)} admissible blocks (dist >= width, min side 96), kernel 1/|x-y|, "
                             f"adaptive k 8..{kmax} step 8 to tol {tol:g}, one batched launch",
                 "points": N, "blocks": len(blocks), "tol": tol, "k_max": kmax, "precision": args.precision,
                 "autotuned": tuned})
    out["roofline"] = _alu_roofline(entries, kernel_ms)
    out["cpu_baseline"] = cpu
    out["batched_vs_plain"] = {"batched_blocks_per_s": len(blocks) / batched_s,
                               "plain_blocks_per_s": len(blocks) / plain_s,
                               "speedup": plain_s / batched_s, "identical_results": same,
                               "blocks": len(blocks)}
    out["result"] = {"statuses": statuses, "k_hist": ks, "tol_met": met, "entries_read": int(entries)}
    ctx.close()
    return out


# ---------------------------------------------------------------------------
# served stream
# ---------------------------------------------------------------------------

def _pool(torch, specs, seed, maxdim):
    """Dense pool: one maxdim x maxdim matrix per (rank, dtype) in use; a
    request of shape m x n reads the leading m x n window.  Each is a Gaussian
    rank-r product plus Gaussian noise at a log-uniform 1e-6..1e-3 relative
    level, generated on the device from a seeded generator."""
    want = sorted({(s.k, s.dtype) for s in specs if s.kind == "dense"}, key=lambda v: (v[1] == "f64", v[0]))
    rng = np.random.default_rng(seed + 7)
    pool = {}
    for idx, (r, dt) in enumerate(want):
        tdt = torch.float64 if dt == "f64" else torch.float32
        g = torch.Generator(device="cuda")
        g.manual_seed(seed * 1000 + idx)
        noise = float(np.exp(rng.uniform(np.log(1e-6), np.log(1e-3))))
        G1 = torch.randn(maxdim, r, generator=g, device="cuda", dtype=tdt)
        G2 = torch.randn(r, maxdim, generator=g, device="cuda", dtype=tdt)
        A = G1 @ G2
        del G1, G2
        E = torch.randn(maxdim, maxdim, generator=g, device="cuda", dtype=tdt)
        c = noise * float(torch.linalg.vector_norm(A)) / float(torch.linalg.vector_norm(E))
        A.add_(E, alpha=c)
        del E
        torch.cuda.synchronize()
        pool[(r, dt)] = A
    return pool


def _sources(torch, lra, specs, pool, seed):
    srcs = []
    for i, sp in enumerate(specs):
        if sp.kind == "dense":
            A = pool[(sp.k, sp.dtype)]
            srcs.append(lra.dense(A[:sp.m, :sp.n]))
        else:
            rng = np.random.default_rng(seed * 100003 + i)
            dt = np.float64 if sp.dtype == "f64" else np.float32
            s = torch.from_numpy(rng.uniform(0, 1, sp.m).astype(dt)).cuda()
            t = torch.from_numpy(rng.uniform(2, 3, sp.n).astype(dt)).cuda()
            srcs.append(lra.cauchy(s, t))
    return srcs


def bench_serve(args):
    import torch

    import synth
    from paper_1611_01391_amd import lra

    count = args.requests
    specs = synth.request_stream(args.seed, count, rate=0.0, hi=args.max_dim)
    t0 = time.time()
    pool = _pool(torch, specs, args.seed, args.max_dim)
    srcs = _sources(torch, lra, specs, pool, args.seed)
    torch.cuda.synchronize()
    log(f"# {count} requests; dense pool of {len(pool)} matrices ({args.max_dim}^2) in {time.time() - t0:.1f}s")
    sweeps = 4

    def kw(i):
        sp = specs[i]
        return dict(precision=lra.PREC_FP64 if sp.dtype == "f64" else lra.PREC_MIXED, seed=i)

    ctx = lra.Context()
    # plain: sequential blocking calls
    for i in range(min(4, count)):
        ctx.ca_cur(srcs[i], specs[i].k, sweeps, specs[i].tol, raise_on_error=False, **kw(i))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plain = [ctx.ca_cur(srcs[i], specs[i].k, sweeps, specs[i].tol, raise_on_error=False, **kw(i))
             for i in range(count)]
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t1
    thr_plain = count / plain_s
    log(f"# plain sequential: {plain_s:.2f}s, {thr_plain:.1f} requests/s")

    # served, saturation: everything arrives at t = 0
    sctx = lra.Context(hbm_budget_bytes=args.budget_gib << 30)
    sctx.serve_config(arena_bytes=(args.budget_gib << 30) // 2, phases_per_tick=args.phases)
    t1 = time.perf_counter()
    tickets = [sctx.submit(srcs[i], specs[i].k, sweeps, specs[i].tol, **kw(i)) for i in range(count)]
    served = [sctx.wait(t) for t in tickets]
    torch.cuda.synchronize()
    served_s = time.perf_counter() - t1
    thr_served = count / served_s
    ticks = sctx.stats()["ticks"]
    log(f"# served at saturation: {served_s:.2f}s, {thr_served:.1f} requests/s, {ticks} ticks")
    same = sum(1 for a, b in zip(plain, served)
               if a.status == b.status and a.err_est_rel == b.err_est_rel and np.array_equal(a.I, b.I)
               and np.array_equal(a.J, b.J))

    # latency under Poisson arrivals at 0.7 x the plain saturated throughput
    lam = 0.7 * thr_plain
    arr = np.array([s.arrival for s in synth.request_stream(args.seed, count, rate=lam, hi=args.max_dim)])
    lat_plain = []
    t1 = time.perf_counter()
    for i in range(count):
        now = time.perf_counter() - t1
        if now < arr[i]:
            time.sleep(arr[i] - now)
        ctx.ca_cur(srcs[i], specs[i].k, sweeps, specs[i].tol, raise_on_error=False, **kw(i))
        lat_plain.append(time.perf_counter() - t1 - arr[i])
    lat_served = [0.0] * count
    pending = {}
    nxt = 0
    t1 = time.perf_counter()
    while nxt < count or pending:
        now = time.perf_counter() - t1
        while nxt < count and arr[nxt] <= now:
            pending[sctx.submit(srcs[nxt], specs[nxt].k, sweeps, specs[nxt].tol, **kw(nxt))] = nxt
            nxt += 1
        for tk in list(pending):
            r = sctx.poll(tk)
            if r is not None:
                i = pending.pop(tk)
                lat_served[i] = time.perf_counter() - t1 - arr[i]
        if not pending and nxt < count:
            time.sleep(max(0.0, min(arr[nxt] - (time.perf_counter() - t1), 0.001)))
    lp = np.percentile(np.array(lat_plain) * 1e3, [50, 99])
    ls = np.percentile(np.array(lat_served) * 1e3, [50, 99])
    log(f"# latency at {lam:.1f}/s: plain p50 {lp[0]:.2f} ms p99 {lp[1]:.2f} ms; "
        f"served p50 {ls[0]:.2f} ms p99 {ls[1]:.2f} ms")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        sample = [i for i, s in enumerate(specs) if s.kind == "cauchy"][:20]
        c0 = time.perf_counter()
        for i in sample:
            sp = specs[i]
            rng = np.random.default_rng(args.seed * 100003 + i)
            dt = np.float64 if sp.dtype == "f64" else np.float32
            sx = rng.uniform(0, 1, sp.m).astype(dt)
            tx = rng.uniform(2, 3, sp.n).astype(dt)
            kc = sp.k
            sd = i
            cand = oracle.draw_distinct(sd, sp.n, min(sp.n, 2 * kc))
            Q = np.sort(oracle.draw_distinct(sd + 1, sp.m, min(64, sp.m)))
            S = np.sort(oracle.draw_distinct(sd + 2, sp.n, min(64, sp.n)))
            oracle.ca_cur(oracle.cauchy(sx, tx), sp.k, sweeps, sp.tol, cand, Q, S,
                          precision=sp.dtype)
        cs = time.perf_counter() - c0
        cpu = {"value": len(sample) / cs, "unit": "requests/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {len(sample)} Cauchy requests of the stream, single-threaded, {cs:.2f}s "
                         f"(dense requests need host copies of the pool and are not sampled)",
               "host": host_info()}
    out = _base(args, thr_served, "requests/s (CUR LRAs/s)", served_s * 1e3 / count, "f64+f32",
                {"workload": f"served stream of {count} requests (dense pool windows and Cauchy kernels, m, n "
                             f"log-uniform [1024, {args.max_dim}], k in {{8,16,32,64}}, tol log-uniform "
                             f"[1e-10, 1e-4], binary32/binary64, up to 4 sweeps), continuous batching",
                 "requests": count, "max_dim": args.max_dim, "phases_per_tick": args.phases})
    out["steps"] = 1
    out["roofline"] = None
    out["cpu_baseline"] = cpu
    out["served_vs_plain"] = {"served_requests_per_s": thr_served, "plain_requests_per_s": thr_plain,
                              "speedup": thr_served / thr_plain, "identical_results": same,
                              "offered_load_per_s": lam,
                              "latency_ms": {"plain_p50": lp[0], "plain_p99": lp[1],
                                             "served_p50": ls[0], "served_p99": ls[1]},
                              "ticks": int(ticks)}
    from collections import Counter
    out["result"] = {"statuses": dict(Counter(int(r.status) for r in served))}
    ctx.close()
    sctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["dense", "plain", "cauchy", "multipole", "serve"], default="dense")
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--sweeps", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--points", type=int, default=1 << 20, help="multipole: number of points")
    ap.add_argument("--requests", type=int, default=1000, help="serve: number of requests")
    ap.add_argument("--max-dim", type=int, default=65536, help="serve: largest m, n")
    ap.add_argument("--phases", type=int, default=4, help="serve: phases per request per tick")
    ap.add_argument("--budget-gib", type=int, default=64, help="serve: HBM budget of the serving context")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=20)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--team", type=int, default=0)
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="skip the team / planning-floor search before the timed steps")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    if args.workload == "dense":
        out = bench_dense(args)
    elif args.workload == "plain":
        out = bench_dense(args, plain=True)
    elif args.workload == "cauchy":
        out = bench_cauchy(args)
    elif args.workload == "multipole":
        out = bench_multipole(args)
    else:
        out = bench_serve(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
