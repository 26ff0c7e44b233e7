"""Benchmarks of the C-A / CUR library on one MI355X.

Default (no --workload): every leg of the metric in one run, one JSON line.
The headline `value` is C-A / CUR of a dense 16384 x 16384 float32 matrix
on the binary64 path: A = G1 G2 D + 1e-4-scaled Gaussian noise (G1
16384x32, G2 32x16384, D log-uniform column scales in [0.1, 10]), stored
float32 row-major in HBM; rank k = 32, 4 C-A sweeps from 32 seeded columns,
maxvol tau = 0.01, 64 x 64 sampled residual.  Only the gathered strips, the
generator and the sample are read.  One step = one complete C-A / CUR
(sweeps, nucleus, residual estimate) with the matrix resident.  The other
legs ride along as objects of the same line:
  mixed_path        the same matrix on the binary32 path, parity against the
                    binary32 oracle and error against the binary64 oracle
  bf16_select_path  the same with the BF16-shortlist selection (binary32
                    recheck), against the same two oracles
  top_svd           the LRA -> top SVD transition on the headline CUR
  ca_test_algorithms_and_preprocessing
                    Tests 1, 3, 4, the truncated-nucleus Primitive CUR and
                    C-A on F A H (abridged Hadamard, depth 3) at 16384^2
  plain_512         dense binary64 512 x 512, W = G1 G2 + 1e-8 E, k = 8,
                    3 sweeps
  cauchy_2p20       implicit a_ij = 1/(s_i - t_j), m = n = 2^20, adaptive k
                    8..40 to tol 1e-10
  batched_vs_plain  every far-field block of a 1D adaptive tree over 2^20
                    mixture points, kernel 1/|x - y|, adaptive k 8..48 to
                    tol 1e-8: one batched launch vs one block per call
  served_vs_plain   a stream of dense and Cauchy requests (m, n log-uniform
                    in [1024, 65536], k in {8, 16, 32, 64} growing up to 64,
                    tol log-uniform in [1e-10, 1e-4], binary32 or binary64):
                    continuous batching vs sequential calls, throughput at
                    saturation, p50 / p99 latency under Poisson arrivals
Every leg carries its own oracle baseline: the CPU oracle as it stands,
run on the host's cores (independent problems on a thread pool; the
oracle's C calls release the interpreter lock).

--workload X runs one leg alone with its own line.  --gpus N > 1 is
refused: this build runs on one GPU.
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
# VALU issue peak: 256 CUs, four 16-lane SIMDs each (one wave64 instruction
# per CU per cycle; binary64 FMA at that rate is the 78.6 TFLOP/s peak), 2.4 GHz
VALU_WAVE_INSTR_PEAK_G = 256 * 2.4


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


def host_threads(args):
    """Threads for the oracle baselines: --threads, else the host's cores
    (at most 16, the CPU share of one GPU on the box)."""
    return max(1, args.threads or min(16, os.cpu_count() or 1))


def pool_map(fn, items, threads):
    """fn over items on a thread pool (the oracle's ctypes calls release the
    interpreter lock, so independent problems run on separate cores)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, items))


def _profiled(summary, key, kernel_src="paper_1611_01391_amd/csrc/lra_engine.hip"):
    """A figure from a committed rocprofv3 summary, or None when the engine
    source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(os.path.join(ROOT, kernel_src), "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    vals = dict(l.split(":", 1) for l in text.splitlines() if ":" in l and not l.startswith((" ", "#", "|")))
    if vals.get("engine_source_sha256_prefix", "").strip() != sha:
        return None
    v = vals.get(key)
    return float(v) if v is not None else None


def _median_time(fn, reps):
    ts = []
    out = None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), out


def _cpu_throughput(fn, runs, threads, unit, what):
    """The oracle run `runs` times on `threads` threads: throughput over the
    wall clock, with the single-thread median of the first runs beside it."""
    t1 = time.perf_counter()
    _, ref = _median_time(fn, 1)
    single = time.perf_counter() - t1
    t0 = time.perf_counter()
    pool_map(lambda _: fn(), range(runs), threads)
    wall = time.perf_counter() - t0
    return {"value": runs / wall, "unit": unit, "cores": threads, "kind": "oracle",
            "sample": f"{runs} independent runs of {what} on {threads} host threads in {wall:.2f}s "
                      f"(one run alone: {single:.3f}s)",
            "single_thread_value": 1.0 / single, "host": host_info()}, ref


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


_DENSE_CACHE = {}


def _dense_input(args):
    key = (args.seed, args.n, args.k)
    if key not in _DENSE_CACHE:
        import synth
        t0 = time.time()
        _DENSE_CACHE.clear()
        _DENSE_CACHE[key] = synth.dense_scaled(args.seed, n=args.n, r=32, k=args.k)
        log(f"# generated {args.n}x{args.n} float32 input in {time.time() - t0:.1f}s")
    return _DENSE_CACHE[key]


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
        A, d = _dense_input(args)
        esz = 4
        prec = {"fp64": lra.PREC_FP64, "mixed": lra.PREC_MIXED, "bf16sel": lra.PREC_BF16SEL}[args.precision]
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
        oprec = "f64" if prec == lra.PREC_FP64 else "f32"
        threads = host_threads(args)
        runs = max(2 * threads, args.cpu_samples) if not plain else 1000 * threads
        cpu, ref = _cpu_throughput(
            lambda: oracle.ca_cur(osrc, k, sweeps, 0.0, d.cand_cols, d.sample_rows, d.sample_cols, precision=oprec),
            runs, threads, "CUR LRAs/s", f"the full C-A/CUR of the same {n}x{n} workload")
        parity = {"oracle_precision": oprec, "oracle_status": int(ref.status),
                  "same_I": bool(np.array_equal(ref.I, res.I)), "same_J": bool(np.array_equal(ref.J, res.J)),
                  "est_rel_gpu": res.err_est_rel, "est_rel_oracle": ref.err_est_rel,
                  "oracle_min_gap": ref.min_gap()}
        if oprec == "f32":
            # the binary32 path's error against the binary64 oracle's
            ref64 = oracle.ca_cur(osrc, k, sweeps, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
            parity["est_rel_oracle_f64"] = ref64.err_est_rel
            parity["est_rel_ratio_vs_f64"] = res.err_est_rel / ref64.err_est_rel if ref64.err_est_rel else None
            parity["same_I_as_f64"] = bool(np.array_equal(ref64.I, res.I))
            parity["same_J_as_f64"] = bool(np.array_equal(ref64.J, res.J))
    out = _base(args, args.steps / el, "CUR LRAs/s", ms_per_step,
                "f64" if prec == lra.PREC_FP64 else "f32",
                {"workload": desc, "m": n, "n": n, "k": k, "sweeps": sweeps,
                 "precision": args.precision if not plain else "fp64", "autotuned": tuned})
    traffic = None
    if not plain and (n, k, sweeps, args.precision) == (16384, 32, 4, "fp64"):
        traffic = _profiled("engine_kernel_dense16384_k32.md", "traffic_bytes_per_launch")
    if plain:
        # one workgroup, all in LDS: a latency-bound launch (no roofline binds)
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "engine_kernel",
                           "kernel_ms": kernel_ms, "algorithmic_bytes": alg_bytes,
                           "note": "latency-bound: one workgroup, the strips live in LDS"}
    else:
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "engine_kernel",
                           "kernel_ms": kernel_ms, "algorithmic_bytes": alg_bytes}
    if traffic:
        out["roofline"]["traffic_GBps"] = traffic / (kernel_ms * 1e-3) / 1e9
    out["cpu_baseline"] = cpu
    out["parity"] = parity
    out["result"] = {"status": int(res.status), "k": int(res.k), "swaps": int(res.swaps_total),
                     "est_rel": res.err_est_rel, "entries_read": int(res.entries_read)}
    if not plain:
        out["strip_gather"] = _strip_gather(ctx, torch, src, n, n, res, esz)
        if args.precision == "fp64" or args.top_svd:
            out["top_svd"] = _top_svd_leg(ctx, torch, src, n, n, res, esz, cpu=not args.no_cpu_baseline)
    ctx.close()
    del At
    return out


def _strip_gather(ctx, torch, src, m, n, res, esz, reps=50):
    """The strip gather on its own: lra_cur_factors writes C = A[:, J] and
    R = A[I, :] for the run's final sets (one column strip and one row strip
    of the workload, in the source precision), timed with HIP events.  The
    algorithmic bytes are the strips read and written; the DRAM bytes come
    from the committed FETCH_SIZE / WRITE_SIZE counters of the same kernel."""
    dt = torch.float32 if esz == 4 else torch.float64
    k = res.k
    Cb = torch.empty(k * m, dtype=dt, device="cuda")
    Rb = torch.empty(k * n, dtype=dt, device="cuda")
    for _ in range(3):
        ctx.cur_factors(src, res.I, res.J, dtype=dt, C_out=Cb, R_out=Rb)
    torch.cuda.synchronize()
    ctx.set_timing(True, reset=True)
    for _ in range(reps):
        ctx.cur_factors(src, res.I, res.J, dtype=dt, C_out=Cb, R_out=Rb)
    st = ctx.stats()
    ctx.set_timing(False, reset=False)
    kms = st["engine_ms_total"] / max(1, st["launches"])
    alg = 2 * (m * k + k * n) * esz
    dram = _profiled("factors_kernel_dense16384_k32.md", "traffic_bytes_per_launch")
    g = {"kernel": "factors_kernel", "kernel_ms": kms, "algorithmic_bytes": alg,
         "achieved_GBps": alg / (kms * 1e-3) / 1e9, "frac_algorithmic": alg / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
         "dram_bytes": dram, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "note": "one m x k column strip and one k x n row strip of the workload, read and written"}
    if dram:
        g["dram_GBps"] = dram / (kms * 1e-3) / 1e9
        g["frac_dram"] = g["dram_GBps"] / HBM_PEAK_GBS
    log(f"# strip gather: {kms * 1e3:.1f} us, {g['achieved_GBps']:.0f} GB/s algorithmic"
        + (f", {g['dram_GBps']:.0f} GB/s DRAM" if dram else ""))
    return g


def _top_svd_leg(ctx, torch, src, m, n, res, esz, reps=20, cpu=True):
    """The LRA -> top SVD transition (Appendix D, Algorithm D.1) on the run's
    own CUR: lra_cur_factors gives C and R in the source precision, then
    lra_top_svd at r = k and r = k / 2, timed with HIP events around all of
    its launches (TSQR levels, core, apply).  Parity: sigma and sampled
    entries of S diag(sigma) T^T against the oracle on the same factors.
    Algorithmic bytes: C and R read twice (QR and output), S and T^T written
    in binary64."""
    Cd, Rd = ctx.cur_factors(src, res.I, res.J)
    k = res.k
    out = {}
    for r in (k, k // 2):
        S = torch.empty(r * m, dtype=torch.float64, device="cuda")
        T = torch.empty(r * n, dtype=torch.float64, device="cuda")
        for _ in range(3):
            ctx.top_svd(Cd, res.U, Rd, r, S_out=S, Tt_out=T)
        torch.cuda.synchronize()
        ctx.set_timing(True, reset=True)
        for _ in range(reps):
            Sv, sigma, Tv, pc, pr = ctx.top_svd(Cd, res.U, Rd, r, S_out=S, Tt_out=T)
        st = ctx.stats()
        ctx.set_timing(False, reset=False)
        ms = st["engine_ms_total"] / reps
        alg = 2 * (m * k + k * n) * esz + 8 * r * (m + n)
        leg = {"r": r, "ms": ms, "launches_per_call": st["launches"] / reps, "algorithmic_bytes": alg,
               "achieved_GBps": alg / (ms * 1e-3) / 1e9, "frac_hbm": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "bound": "latency (k-step Householder and Jacobi chains on one workgroup)"}
        if cpu:
            from oracle.top_svd import top_svd as oracle_top_svd
            Ch = Cd.cpu().numpy().astype(np.float64)
            Rh = Rd.cpu().numpy().astype(np.float64)
            t0 = time.perf_counter()
            ref = oracle_top_svd(Ch, res.U, Rh, r)
            leg["cpu_oracle_s"] = time.perf_counter() - t0
            rng = np.random.default_rng(3)
            ii, jj = rng.integers(0, m, 256), rng.integers(0, n, 256)
            Sh, Th = Sv.cpu().numpy(), Tv.cpu().numpy()
            got = np.einsum("ia,a,ai->i", Sh[ii], sigma, Th[:, jj])
            want = np.einsum("ia,a,ai->i", ref.S[ii], ref.sigma, ref.Tt[:, jj])
            leg["parity"] = {"pivots_equal": bool(np.array_equal(pc[:r], ref.piv_c[:r])
                                                  and np.array_equal(pr[:r], ref.piv_r[:r])),
                             "min_pivot_margin": ref.min_margin(r),
                             "sigma_max_rel_diff": float(np.max(np.abs(sigma - ref.sigma)) / ref.sigma[0]),
                             "lra_max_rel_diff_sampled": float(np.max(np.abs(got - want)) / ref.sigma[0])}
        log(f"# top SVD r={r}: {ms * 1e3:.1f} us per call")
        out[f"r{r}"] = leg
    return out


# ---------------------------------------------------------------------------
# the fixed-rank algorithms of the C-A tests and pre-processed C-A, at the
# dense 16384^2 float32 shape
# ---------------------------------------------------------------------------

def bench_variants(args, reps=10):
    """On the headline matrix: Tests 1 (random I, J, U = A[I,J]^-1; Section
    12.2), Tests 3 (random 64 x 64 generator -> Cynical 16 x 16) and Tests 4
    (one C-A loop at width 64, then Cynical 16 x 16; Section 6.5), the
    Primitive CUR with the nucleus truncated to rank 32 of a 64 x 64
    generator (Section 6.5), and 4 C-A sweeps at k = 32 on F A H with depth-3
    abridged scaled Hadamard multipliers (Section 8.3).  Each is timed with HIP
    events (kernel time per call) and, in the CPU leg, run once by the oracle
    (single thread) for the parity figures and the baseline."""
    import torch

    from paper_1611_01391_amd import lra

    A, d = _dense_input(args)
    n = A.shape[0]
    At = torch.from_numpy(A).cuda()
    torch.cuda.synchronize()
    rng = np.random.default_rng(args.seed + 11)
    cols64 = rng.choice(n, 64, replace=False).astype(np.int64)
    rows64 = rng.choice(n, 64, replace=False).astype(np.int64)
    base = dict(sample_rows=d.sample_rows, sample_cols=d.sample_cols)
    dense_src = lra.dense(At)
    pre_src = lra.preprocessed(At, 3, args.seed + 5)
    cases = [
        ("tests1_random_k32", dense_src, 32, 0, dict(init_cols=cols64[:32], init_rows=rows64[:32])),
        ("tests3_cynical_64_to_16", dense_src, 64, 0, dict(init_cols=cols64, init_rows=rows64, cur_rank=16)),
        ("tests4_loop_then_cynical_64_to_16", dense_src, 64, 1, dict(init_cols=cols64, cur_rank=16)),
        ("primitive_64_nucleus_rank_32", dense_src, 64, 0, dict(init_cols=cols64, init_rows=rows64, nucleus_rank=32)),
        ("preprocessed_depth3_k32", pre_src, 32, 4, dict(init_cols=d.cand_cols)),
    ]
    ctx = lra.Context()
    out = {}
    for name, src, k, sw, extra in cases:
        kw = dict(base, **extra)
        el, st, res = _timed_steps(ctx, torch, lambda: ctx.ca_cur(src, k, sw, 0.0, **kw), reps, 2)
        kms = st["engine_ms_total"] / max(1, st["launches"])
        leg = {"k": k, "sweeps": sw, "options": {a: b for a, b in extra.items() if a in ("cur_rank", "nucleus_rank")},
               "kernel_ms": kms, "calls_per_s": reps / el, "status": int(res.status), "k_out": int(res.k),
               "est_rel": res.err_est_rel, "entries_read": int(res.entries_read)}
        # bytes of A read: 4 per entry, 4^3 entries of A per entry of F A H
        per_entry = 4 * (64 if src is pre_src else 1)
        leg["bytes_read_of_A"] = int(res.entries_read) * per_entry
        leg["achieved_GBps"] = leg["bytes_read_of_A"] / (kms * 1e-3) / 1e9
        leg["frac_hbm"] = leg["achieved_GBps"] / HBM_PEAK_GBS
        log(f"# {name}: kernel {kms:.3f} ms, status {res.status}, k {res.k}, est_rel {res.err_est_rel:.3e}")
        if not args.no_cpu_baseline:
            import oracle
            hs = oracle.abridged(A, 3, args.seed + 5) if src is pre_src else oracle.dense(A)
            t0 = time.perf_counter()
            if src is pre_src:
                ref = oracle.ca_cur(hs, k, sw, 0.0, d.cand_cols, d.sample_rows, d.sample_cols)
            else:
                ref = oracle.cur_variant(hs, k, sw, kw["init_cols"], d.sample_rows, d.sample_cols,
                                         init_rows=kw.get("init_rows"), cur_rank=kw.get("cur_rank", 0),
                                         nucleus_rank=kw.get("nucleus_rank", 0))
            t_cpu = time.perf_counter() - t0
            leg["cpu_baseline"] = {"value": 1.0 / t_cpu, "unit": "calls/s", "cores": 1, "kind": "oracle",
                                   "sample": "one call of the same algorithm on the same matrix"}
            leg["parity"] = {"same_status_k": (int(ref.status), int(ref.k)) == (int(res.status), int(res.k)),
                             "same_I": bool(np.array_equal(np.sort(ref.I), np.sort(res.I))),
                             "same_J": bool(np.array_equal(np.sort(ref.J), np.sort(res.J))),
                             "est_rel_oracle": ref.err_est_rel,
                             "est_rel_abs_diff": abs(ref.err_est_rel - res.err_est_rel)}
        out[name] = leg
    ctx.close()
    del At
    return {"workload": f"dense float32 {n}x{n} (the headline matrix)", "cases": out}


# ---------------------------------------------------------------------------
# implicit Cauchy kernel, 2^20 x 2^20
# ---------------------------------------------------------------------------

def _alu_roofline(entries, kernel_ms, summary, kernel="engine_kernel"):
    """VALU roofline of a generated-entry workload: the engine's binary64
    VALU issue rate against the chip's (256 CUs x one wave64 instruction per
    cycle x 2.4 GHz), from the VALU instructions per launch that rocprofv3
    counted (SQ_INSTS_VALU, committed under profiles/) over the live kernel
    time; None while the engine source differs from the profiled one.  The
    generated entries per second ride along."""
    insts = _profiled(summary, "valu_insts_per_launch")
    out = {"bound": "alu", "achieved": None, "peak": VALU_WAVE_INSTR_PEAK_G, "unit": "G VALU wave-instructions/s",
           "frac": None, "traffic": None, "kernel": kernel, "kernel_ms": kernel_ms,
           "entries_generated": int(entries), "entries_per_s": entries / (kernel_ms * 1e-3)}
    if insts:
        ach = insts / (kernel_ms * 1e-3) / 1e9
        out.update(achieved=ach, frac=ach / VALU_WAVE_INSTR_PEAK_G, valu_insts_per_launch=insts,
                   counters=f"profiles/{summary}")
    return out


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
              precision=lra.PREC_FP64 if f64 else lra.PREC_MIXED, raise_on_error=False, team_wgs=args.team)
    tuned = None
    if args.autotune and not args.team:
        team, tms = ctx.autotune_team(src, 8, 4, tol, init_cols=d.cand_cols, sample_rows=d.sample_rows,
                                      sample_cols=d.sample_cols, k_max=40,
                                      precision=lra.PREC_FP64 if f64 else lra.PREC_MIXED)
        tuned = {"team_wgs": team, "kernel_ms": tms}
        kw["team_wgs"] = team
        log(f"# autotuned team: {team} workgroups ({tms:.3f} ms)")
    el, st, res = _timed_steps(ctx, torch, lambda: ctx.ca_cur(src, 8, 4, tol, **kw), args.steps, args.warmup)
    kernel_ms = st["engine_ms_total"] / max(1, st["launches"])
    log(f"# gpu: status {res.status} k {res.k} sweeps {res.sweeps_done} swaps {res.swaps_total} "
        f"est_rel {res.err_est_rel:.3e} kernel {kernel_ms:.3f} ms grid {st['last_grid']}")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        osrc = oracle.cauchy(s, t)
        threads = host_threads(args)
        cpu, ref = _cpu_throughput(
            lambda: oracle.ca_cur(osrc, 8, 4, tol, d.cand_cols, d.sample_rows, d.sample_cols, k_max=40,
                                  precision="f64" if f64 else "f32"),
            threads, threads, "CUR LRAs/s", "the full adaptive C-A/CUR of the same 2^20 x 2^20 Cauchy workload")
        cpu["oracle_result"] = {"status": int(ref.status), "k": int(ref.k), "est_rel": ref.err_est_rel}
    out = _base(args, args.steps / el, "CUR LRAs/s", el * 1e3 / args.steps, "f64" if f64 else "f32",
                {"workload": f"implicit Cauchy 1/(s_i - t_j), s ~ U[0,1], t ~ U[2,3], m = n = 2^20, adaptive k "
                             f"8..40 step 8, tol {tol:g}, up to 4 sweeps per rank",
                 "m": m, "n": m, "k0": 8, "k_max": 40, "tol": tol, "precision": args.precision,
                 "autotuned": tuned})
    out["roofline"] = _alu_roofline(res.entries_read, kernel_ms,
                                    f"engine_kernel_cauchy_2p20_{'fp64' if f64 else 'fp32'}.md")
    # the basis passes over the 2^20-row strips in HBM (counted by FETCH_SIZE / WRITE_SIZE)
    tr = _profiled(f"engine_kernel_cauchy_2p20_{'fp64' if f64 else 'fp32'}.md", "traffic_bytes_per_launch")
    if tr:
        out["roofline"]["traffic"] = tr
        out["roofline"]["traffic_GBps"] = tr / (kernel_ms * 1e-3) / 1e9
        out["roofline"]["traffic_frac_hbm"] = out["roofline"]["traffic_GBps"] / HBM_PEAK_GBS
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
    tol, kmax = args.mp_tol, 48
    f64 = args.precision == "fp64"
    t0 = time.time()
    x, blocks, dense_blocks = synth.multipole(args.seed, N, 4096, 96)
    log(f"# {len(blocks)} far-field blocks ({len(dense_blocks)} left dense) in {time.time() - t0:.1f}s")
    xd = torch.from_numpy(x if f64 else x.astype(np.float32)).cuda()
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
        threads = host_threads(args)
        xo = x if f64 else x.astype(np.float32)

        def one(b):
            a0, a1, b0, b1 = blocks[b]
            m, n = a1 - a0, b1 - b0
            kc = max(8, min(kmax, m, n))
            sd = synth.block_draws(args.seed, b)
            cand = oracle.draw_distinct(sd, n, min(n, 2 * kc))
            Q = np.sort(oracle.draw_distinct(sd + 1, m, min(64, m)))
            S = np.sort(oracle.draw_distinct(sd + 2, n, min(64, n)))
            r = oracle.ca_cur(oracle.invdist(xo[a0:a1], xo[b0:b1]), 8, 4, tol, cand, Q, S, k_max=kmax,
                              precision="f64" if f64 else "f32")
            return r.status >= 0 and r.err_est_rel <= tol
        # every block, largest first (dynamic assignment to the threads)
        order = sorted(range(len(blocks)), key=lambda b: -((blocks[b][1] - blocks[b][0]) + (blocks[b][3] - blocks[b][2])))
        c0 = time.perf_counter()
        met_cpu = sum(pool_map(one, order, threads))
        cs = time.perf_counter() - c0
        cpu = {"value": len(blocks) / cs, "unit": "CUR LRAs/s (blocks/s)", "cores": threads, "kind": "oracle",
               "sample": f"all {len(blocks)} blocks of the same pass, largest first on {threads} host threads, "
                         f"{cs:.2f}s; {met_cpu} meet tol", "host": host_info()}
    out = _base(args, len(blocks) / batched_s, "CUR LRAs/s (blocks/s)", batched_s * 1e3, "f64" if f64 else "f32",
                {"workload": f"1D multipole far field: N = {N} mixture points, adaptive binary tree (leaves <= 4096), "
                             f"{len(blocks)} admissible blocks (dist >= width, min side 96), kernel 1/|x-y|, "
                             f"adaptive k 8..{kmax} step 8 to tol {tol:g}, one batched launch",
                 "points": N, "blocks": len(blocks), "tol": tol, "k_max": kmax, "precision": args.precision,
                 "autotuned": tuned})
    out["roofline"] = _alu_roofline(entries, kernel_ms, "engine_kernel_multipole_2p20.md")
    out["cpu_baseline"] = cpu
    met_plain = sum(1 for r in out_p if r.status >= 0 and r.err_est_rel <= tol)
    out["batched_vs_plain"] = {"batched_blocks_per_s": len(blocks) / batched_s,
                               "plain_blocks_per_s": len(blocks) / plain_s,
                               "speedup": plain_s / batched_s, "identical_results": same,
                               "tol_met_batched": met, "tol_met_plain": met_plain,
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
        return dict(precision=lra.PREC_FP64 if sp.dtype == "f64" else lra.PREC_MIXED, seed=i,
                    k_max=min(args.serve_kmax, sp.m, sp.n))

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
        threads = host_threads(args)
        cau = [i for i, sp in enumerate(specs) if sp.kind == "cauchy"][:40]
        den = [i for i, sp in enumerate(specs) if sp.kind == "dense" and sp.m * sp.n <= (1 << 24)][:40]
        hosts = {}
        for i in den:
            # host copy of the request's window of its pool matrix
            sp = specs[i]
            hosts[i] = pool[(sp.k, sp.dtype)][:sp.m, :sp.n].cpu().numpy()

        def one(i):
            sp = specs[i]
            if sp.kind == "dense":
                osrc = oracle.dense(hosts[i])
            else:
                rng = np.random.default_rng(args.seed * 100003 + i)
                dt = np.float64 if sp.dtype == "f64" else np.float32
                osrc = oracle.cauchy(rng.uniform(0, 1, sp.m).astype(dt), rng.uniform(2, 3, sp.n).astype(dt))
            km = min(args.serve_kmax, sp.m, sp.n)
            kc = max(sp.k, km)
            cand = oracle.draw_distinct(i, sp.n, min(sp.n, 2 * kc))
            Q = np.sort(oracle.draw_distinct(i + 1, sp.m, min(64, sp.m)))
            S = np.sort(oracle.draw_distinct(i + 2, sp.n, min(64, sp.n)))
            r = oracle.ca_cur(osrc, sp.k, sweeps, sp.tol, cand, Q, S, k_max=km, precision=sp.dtype)
            return r.status >= 0 and r.err_est_rel <= sp.tol
        sample = cau + den
        c0 = time.perf_counter()
        met_cpu = sum(pool_map(one, sample, threads))
        cs = time.perf_counter() - c0
        del hosts
        cpu = {"value": len(sample) / cs, "unit": "requests/s", "cores": threads, "kind": "oracle",
               "sample": f"the first {len(cau)} Cauchy requests and the first {len(den)} dense requests with "
                         f"m n <= 2^24 (host copies of their pool windows) on {threads} host threads, "
                         f"{cs:.2f}s; {met_cpu} meet tol", "host": host_info()}
    dense_bytes = sum(r.entries_read * (8 if sp.dtype == "f64" else 4)
                      for r, sp in zip(served, specs) if sp.kind == "dense" and r.status >= 0)
    met_plain = sum(1 for r, sp in zip(plain, specs) if r.status >= 0 and r.err_est_rel <= sp.tol)
    met_served = sum(1 for r, sp in zip(served, specs) if r.status >= 0 and r.err_est_rel <= sp.tol)
    out = _base(args, thr_served, "requests/s (CUR LRAs/s)", served_s * 1e3 / count, "f64+f32",
                {"workload": f"served stream of {count} requests (dense pool windows and Cauchy kernels, m, n "
                             f"log-uniform [1024, {args.max_dim}], k in {{8,16,32,64}}, tol log-uniform "
                             f"[1e-10, 1e-4], rank growth up to {args.serve_kmax}, binary32/binary64, up to 4 sweeps per "
                             f"rank), continuous batching",
                 "requests": count, "k_max": args.serve_kmax, "max_dim": args.max_dim, "phases_per_tick": args.phases})
    out["steps"] = 1
    ach = dense_bytes / served_s / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": "engine_kernel_all",
                       "algorithmic_bytes": dense_bytes,
                       "note": "entries read by the dense requests over the served makespan (the Cauchy "
                               "requests generate theirs)"}
    out["cpu_baseline"] = cpu
    out["served_vs_plain"] = {"served_requests_per_s": thr_served, "plain_requests_per_s": thr_plain,
                              "speedup": thr_served / thr_plain, "identical_results": same,
                              "tol_met_plain": met_plain, "tol_met_served": met_served,
                              "offered_load_per_s": lam,
                              "latency_ms": {"plain_p50": lp[0], "plain_p99": lp[1],
                                             "served_p50": ls[0], "served_p99": ls[1]},
                              "ticks": int(ticks)}
    from collections import Counter
    out["result"] = {"statuses": dict(Counter(int(r.status) for r in served))}
    ctx.close()
    sctx.close()
    return out


def _leg(name, fn, args, **over):
    """Run one leg with its own step counts; returns its line and wall time."""
    import copy
    a = copy.copy(args)
    for key, val in over.items():
        setattr(a, key, val)
    t0 = time.time()
    out = fn(a)
    wall = time.time() - t0
    log(f"# leg {name}: {wall:.1f}s")
    import gc
    import torch
    gc.collect()
    torch.cuda.empty_cache()
    out["wall_s"] = wall
    return out


def _summary(leg, keys):
    return {key: leg.get(key) for key in keys if key in leg}


def bench_all(args):
    """The headline dense leg, with every other leg of the metric attached."""
    t0 = time.time()
    out = _leg("dense fp64", bench_dense, args)
    keep = ("value", "unit", "ms_per_step", "steps", "warmup", "dtype", "config", "roofline", "cpu_baseline",
            "parity", "result", "strip_gather", "wall_s")
    mixed = _leg("dense mixed", bench_dense, args, precision="mixed", steps=10, warmup=2)
    out["mixed_path"] = _summary(mixed, keep)
    bsel = _leg("dense bf16-select", bench_dense, args, precision="bf16sel", steps=10, warmup=2)
    out["bf16_select_path"] = _summary(bsel, keep)
    plain = _leg("plain 512", lambda a: bench_dense(a, plain=True), args, steps=50, warmup=5)
    out["plain_512"] = _summary(plain, keep)
    cau = _leg("cauchy 2^20", bench_cauchy, args, steps=10, warmup=2)
    out["cauchy_2p20"] = _summary(cau, keep)
    mp = _leg("multipole", bench_multipole, args, steps=3, warmup=1)
    out["batched_vs_plain"] = dict(mp["batched_vs_plain"], config=mp["config"], roofline=mp["roofline"],
                                   cpu_baseline=mp["cpu_baseline"], result=mp["result"], wall_s=mp["wall_s"],
                                   kernel_ms=mp["roofline"]["kernel_ms"])
    var = _leg("variants", bench_variants, args)
    out["ca_test_algorithms_and_preprocessing"] = var
    sv = _leg("serve", bench_serve, args)
    out["served_vs_plain"] = dict(sv["served_vs_plain"], config=sv["config"], roofline=sv["roofline"],
                                  cpu_baseline=sv["cpu_baseline"], result=sv["result"], wall_s=sv["wall_s"])
    out["wall_s_total"] = time.time() - t0
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["all", "dense", "plain", "cauchy", "multipole", "serve", "variants"],
                    default="all")
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--sweeps", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", choices=["fp64", "mixed", "bf16sel"], default="fp64")
    ap.add_argument("--top-svd", action="store_true", help="dense: time lra_top_svd also without the CPU legs")
    ap.add_argument("--points", type=int, default=1 << 20, help="multipole: number of points")
    ap.add_argument("--mp-tol", type=float, default=1e-8, help="multipole: tolerance")
    ap.add_argument("--requests", type=int, default=1000, help="serve: number of requests")
    ap.add_argument("--max-dim", type=int, default=65536, help="serve: largest m, n")
    ap.add_argument("--serve-kmax", type=int, default=64, help="serve: rank cap of the adaptive growth")
    ap.add_argument("--phases", type=int, default=4, help="serve: phases per request per tick")
    ap.add_argument("--budget-gib", type=int, default=64, help="serve: HBM budget of the serving context")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=20)
    ap.add_argument("--threads", type=int, default=0, help="host threads of the oracle baselines (0: cores, <= 16)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--team", type=int, default=0)
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="skip the team / planning-floor search before the timed steps")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    if args.workload == "all":
        out = bench_all(args)
    elif args.workload == "dense":
        out = bench_dense(args)
    elif args.workload == "plain":
        out = bench_dense(args, plain=True)
    elif args.workload == "cauchy":
        out = bench_cauchy(args)
    elif args.workload == "multipole":
        out = bench_multipole(args)
    elif args.workload == "variants":
        out = bench_variants(args)
    else:
        out = bench_serve(args)
    print(json.dumps(out), flush=True)
    # explicit teardown before the interpreter exits: every context is closed
    # inside its leg; drop the cached input and torch's cached device memory
    import gc
    import torch
    torch.cuda.synchronize()
    _DENSE_CACHE.clear()
    gc.collect()
    torch.cuda.empty_cache()
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
