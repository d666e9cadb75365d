"""Benchmark of the exhaustive Axilrod-Teller Phi on one MI355X.

Workload: Phi for all N = 32768 points of the 32^3 jittered cubic lattice
(spacing 1.0, per-coordinate jitter +-0.25, seed 2), the configuration the
headline metric is quoted on.  A step is one full evaluation through the C
ABI (validation + exhaustive sum) with the points already in HBM.

Metric: effective unordered triples per second, C(N, 3) per step, counted
only for a precision whose relative error against the binary64 CPU oracle
is <= 1e-6 on sampled particles.  Both precisions are timed; the faster one
that meets the bar is reported.

Extra fields:
  roofline     - the exhaustive-sum kernel (19 flops per unordered triple,
                 FMA = 2) against the MI355X FP64 (or FP32) vector peak; its
                 duration is measured with HIP events around enqueue-only
                 calls (mb_eval_direct_unchecked) on the stream the kernel
                 runs on.
  cpu_baseline - the CPU oracle timed on the host's cores on a bounded
                 sample of the same workload (a few particles' full sums);
                 its values also give the accuracy check above.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_TRIPLE = 19
PEAK_TFLOPS = {"fp64": 78.6, "fp32c": 157.3}
DTYPE = {"fp64": "f64", "fp32c": "f32"}


def comb3(n: int) -> int:
    return n * (n - 1) * (n - 2) // 6


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="particles for the CPU-oracle leg (0: two per host thread)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prec", choices=["fp64", "fp32c", "both"], default="both")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (the "
                         "reference kernel for scaling HBM byte counters), then exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the path has no multi-GPU implementation "
              "(see the sharding notes in DESIGN.md); use --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1105_2769_amd as mb
    import workloads

    dev = torch.device("cuda:0")
    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 3}), flush=True)
        return 0
    n = args.n
    x_np = workloads.jittered_lattice(n, seed=2)
    x = torch.from_numpy(x_np).to(dev)
    stream = torch.cuda.current_stream(dev)
    triples = comb3(n)

    # CPU oracle leg: bounded sample of particles (also the accuracy reference)
    cpu = None
    sample_idx = workloads.sample_indices(n, 8, seed=1002)
    ref = None
    if not args.no_cpu_baseline:
        from oracle import direct as oracle_direct

        threads = oracle_direct.max_threads()
        m = args.cpu_sample or 2 * threads
        sample_idx = workloads.sample_indices(n, m, seed=1002)
        print(f"cpu oracle: {m} particles of N={n} on {threads} threads", flush=True)
        t0 = time.perf_counter()
        ref = oracle_direct.phi(x_np, sample_idx)
        dt = time.perf_counter() - t0
        evals = m * (n - 1) * (n - 2) // 2  # phi evaluations (one per (j, k) pair)
        # a full evaluation needs 3 C(N,3) such evaluations: effective triples/s = evals/3/dt
        cpu = {"value": evals / 3.0 / dt, "unit": "triples/s", "cores": threads, "kind": "oracle",
               "sample": f"full sums of {m} seeded-sampled particles of the N={n} workload "
                         f"({evals:.3e} phi evaluations, {dt:.1f} s); triples/s = evaluations/3/s "
                         f"since all-particle Phi takes 3 C(N,3) evaluations by this loop"}

    results = {}
    precs = ["fp64", "fp32c"] if args.prec == "both" else [args.prec]
    for prec in precs:
        print(f"gpu {prec}: warmup {args.warmup}", flush=True)
        phi = torch.empty(n, dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            mb.eval_direct(x, prec=prec, out=phi)
        torch.cuda.synchronize()
        # whole-step timing (validation + evaluation), K steps
        t0 = time.perf_counter()
        for _ in range(args.steps):
            mb.eval_direct(x, prec=prec, out=phi)
        torch.cuda.synchronize()
        step_s = (time.perf_counter() - t0) / args.steps
        # kernel timing with HIP events on the launch stream (enqueue-only calls)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            mb.eval_direct(x, prec=prec, out=phi, checked=False)
        ev1.record(stream)
        ev1.synchronize()
        kern_s = ev0.elapsed_time(ev1) / 1e3 / args.steps
        got = phi.cpu().numpy()
        rel = None
        if ref is not None:
            rel = float(np.max(np.abs(got[sample_idx] - ref) / np.abs(ref)))
        print(f"gpu {prec}: step {step_s * 1e3:.1f} ms, kernel {kern_s * 1e3:.1f} ms, "
              f"max rel err {rel}", flush=True)
        results[prec] = dict(step_s=step_s, kern_s=kern_s, rel=rel)

    ok = [p for p in precs if results[p]["rel"] is None or results[p]["rel"] <= 1e-6]
    best = min(ok, key=lambda p: results[p]["step_s"]) if ok else None
    if best is None:
        print("no precision met the 1e-6 accuracy bar", file=sys.stderr)
        best = min(precs, key=lambda p: results[p]["step_s"])
    r = results[best]
    achieved = FLOPS_PER_TRIPLE * triples / r["kern_s"] / 1e12
    out = {
        "metric": "triples/sec (effective) at rel err <=1e-6 vs FP64; p50/p99 request latency",
        "value": triples / r["step_s"] if best in ok else 0.0,
        "unit": "triples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["step_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[best],
        "data": "synthetic",
        "config": {"workload": f"direct Phi for all N={n} points, jittered 32^3 lattice "
                               f"(spacing 1.0, jitter 0.25, seed 2)",
                   "n": n, "prec": best, "triples_per_step": triples},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[best],
                     "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[best], "traffic": None,
                     "kernel": "direct_kernel", "kernel_ms": r["kern_s"] * 1e3},
        "cpu_baseline": cpu,
        "accuracy": {p: results[p]["rel"] for p in precs},
        "paths": {p: {"triples_per_s": triples / results[p]["step_s"],
                      "kernel_ms": results[p]["kern_s"] * 1e3,
                      "max_rel_err": results[p]["rel"]} for p in precs},
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
