"""Benchmark: C-A / CUR of a dense 16384 x 16384 float32 matrix on one MI355X.

Workload (the dense-strip configuration): A = G1 G2 D + 1e-4-scaled Gaussian
noise (G1 16384x32, G2 32x16384, D log-uniform column scales in [0.1, 10]),
stored float32 row-major in HBM; rank k = 32, 4 C-A sweeps from 32 seeded
columns, maxvol tau = 0.01, 64 x 64 sampled residual.  Only the gathered
strips, the generator and the sample are read.  One step = one complete
C-A / CUR (sweeps, nucleus, residual estimate) with the matrix resident.

Prints one JSON line (metric, value = CUR LRAs/s, roofline of the engine
kernel, oracle CPU baseline).  --gpus N > 1 is refused: this build runs on
one GPU.
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

METRIC = "CUR LRAs/s + HBM GB/s, served/batched vs plain at equal err; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def _algorithmic_bytes(m, n, k, sweeps, q, s, esz):
    """Entries the method must read, times the element size: per sweep one
    m x k column strip and one k x n row strip, then the k x k generator, the
    q x k, k x s and q x s sample blocks (the residual's binary64 entries are
    read from the same float32 matrix)."""
    entries = sweeps * (m * k + k * n) + k * k + q * k + k * s + q * s
    return entries * esz


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--sweeps", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=20)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--team", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import synth
    from paper_1611_01391_amd import lra

    t0 = time.time()
    A, d = synth.dense_scaled(args.seed, n=args.n, r=32, k=args.k)
    gen_s = time.time() - t0
    print(f"# generated {args.n}x{args.n} float32 input in {gen_s:.1f}s", file=sys.stderr, flush=True)
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

    prec = lra.PREC_FP64 if args.precision == "fp64" else lra.PREC_MIXED
    ctx = lra.Context()
    src = lra.dense(At)
    kw = dict(init_cols=d.cand_cols, sample_rows=d.sample_rows, sample_cols=d.sample_cols,
              precision=prec, team_wgs=args.team)

    res = None
    for _ in range(args.warmup):
        res = ctx.ca_cur(src, args.k, args.sweeps, 0.0, **kw)
    torch.cuda.synchronize()
    ctx.set_timing(True, reset=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        res = ctx.ca_cur(src, args.k, args.sweeps, 0.0, **kw)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    st = ctx.stats()
    ms_per_step = (t2 - t1) * 1e3 / args.steps
    value = args.steps / (t2 - t1)
    kernel_ms = st["engine_ms_total"] / max(1, st["launches"])
    esz = 4
    alg_bytes = _algorithmic_bytes(args.n, args.n, args.k, args.sweeps, 64, 64, esz)
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    print(f"# gpu: status {res.status} k {res.k} swaps {res.swaps_total} est_rel {res.err_est_rel:.3e} "
          f"kernel {kernel_ms:.3f} ms grid {st['last_grid']}", file=sys.stderr, flush=True)

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        osrc = oracle.dense(A)
        times = []
        ref = None
        for _ in range(max(1, args.cpu_samples)):
            c0 = time.perf_counter()
            ref = oracle.ca_cur(osrc, args.k, args.sweeps, 0.0, d.cand_cols, d.sample_rows,
                                d.sample_cols, precision="f64" if prec == lra.PREC_FP64 else "f32")
            times.append(time.perf_counter() - c0)
        cpu = {"value": 1.0 / float(np.median(times)), "unit": "CUR LRAs/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{len(times)} full C-A/CUR runs of the same {args.n}x{args.n} workload, "
                         f"single-threaded, median {np.median(times):.2f}s"}
        parity = {"oracle_status": int(ref.status), "same_I": bool(np.array_equal(ref.I, res.I)),
                  "same_J": bool(np.array_equal(ref.J, res.J)),
                  "est_rel_gpu": res.err_est_rel, "est_rel_oracle": ref.err_est_rel,
                  "oracle_min_gap": ref.min_gap()}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "CUR LRAs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == lra.PREC_FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"dense float32 {args.n}x{args.n} (rank-32 scaled factor-Gaussian "
                               f"+ 1e-4 noise), k={args.k}, {args.sweeps} C-A sweeps, 64x64 residual "
                               f"sample, {args.precision} path",
                   "m": args.n, "n": args.n, "k": args.k, "sweeps": args.sweeps,
                   "precision": args.precision},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "engine_kernel", "kernel_ms": kernel_ms,
                     "algorithmic_bytes": alg_bytes},
        "cpu_baseline": cpu,
        "parity": parity,
        "result": {"status": int(res.status), "k": int(res.k), "swaps": int(res.swaps_total),
                   "est_rel": res.err_est_rel, "entries_read": int(res.entries_read)},
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
