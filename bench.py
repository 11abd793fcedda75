"""Benchmark of the hybrid-symplectic hot path on one MI355X.

One "step" is a full B(dt/2) C(dt/2) A(dt) C(dt/2) B(dt/2) step of the N = 32768 planetesimal disk
(a = 0.3-4 AU, 5 Earth masses, dt = 6 days): the changeover-weighted all-pairs kick with fused
close-encounter detection, the momentum jumps and the Kepler drift; the encounter list at the
final positions is emitted. K steps run as one nbody_step call, so consecutive half kicks share
one force evaluation: K + 1 evaluations of N(N-1) pair interactions.

Prints one JSON line:
  value      pair interactions per second of the timed K steps (inputs resident in HBM),
  roofline   the pair kernel's algorithmic binary64 rate (20 flop per pair) against the MI355X
             binary64 vector peak, from the kernel's mean launch time measured with HIP events,
  cpu_baseline  the CPU oracle on a bounded sample of the same workload (host cores),
  variants   split-precision kick, batched ensembles and the adjoint where available.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 20                 # N-body convention: 3 sub, 5 for r^2, rsqrt, 3 for m r^-3, 6 accumulate, 2 slack
FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X: 256 CU x 128 flop/clk x 2.4 GHz
METRIC = "pair interactions/s & % FP64 peak: plain vs split-prec/batched/adjoint"


def cpu_baseline(budget_s=25.0):
    """The oracle (plain C++, OpenMP) on the first steps of the same N = 32768 disk."""
    import numpy as np

    import diskgen
    import oracle
    p = diskgen.PARAMS
    d = diskgen.workload("disk32768")
    n = len(d["m"])
    thr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    x, v = d["x"], d["v"]
    steps = 0
    t0 = time.perf_counter()
    while steps < 10:
        x, v, _ = oracle.step(x, v, d["m"], p, 1, thr=thr)
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    evals = 2 * steps                # the oracle evaluates both half kicks of every step
    return {"value": evals * n * (n - 1) / el, "unit": "pair-interactions/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"first {steps} steps of the N={n} disk ({evals} force evaluations, "
                      f"{el:.1f} s), full step incl. drift and jumps"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import diskgen
    import paper_2604_09184_amd as nb

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    p = diskgen.PARAMS
    d = diskgen.workload("disk32768")
    n = len(d["m"])
    xm, v4 = diskgen.pack4(d["x"], d["v"], d["m"])
    X = torch.tensor(xm, device=dev)
    V = torch.tensor(v4, device=dev)
    ctx = nb.Context(nb.Params(**p))
    thr = ctx.rcrit(X, V)
    torch.cuda.synchronize()
    print(f"[bench] N={n} warmup {args.warmup} steps", file=sys.stderr, flush=True)
    if args.warmup:
        ctx.step(X, V, args.warmup, thr=thr)
    torch.cuda.synchronize()

    K = args.steps
    print(f"[bench] timing {K} steps", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    pairs, count = ctx.step(X, V, K, thr=thr, pairs_cap=1 << 22)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    evals = K + 1
    value = evals * n * (n - 1) / (ms / 1e3)

    # the dominant kernel alone: mean launch time of the pair kernel (HIP events on the stream)
    kernel_ms = ctx.bench_pairs(X, thr, reps=20)
    achieved = FLOP_PER_PAIR * n * (n - 1) / (kernel_ms / 1e3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4),
                "traffic": None, "kernel": "k_pairs (binary64)",
                "kernel_ms": round(kernel_ms, 4),
                "pairs_per_s_kernel": n * (n - 1) / (kernel_ms / 1e3)}

    variants = {}
    if not args.no_variants:
        print("[bench] variants", file=sys.stderr, flush=True)
        ctx_s = nb.Context(nb.Params(**p, precision=nb.PREC_SPLIT))
        ms_s = ctx_s.bench_pairs(X, thr, reps=20)
        variants["split_precision_kick"] = {"pairs_per_s": n * (n - 1) / (ms_s / 1e3),
                                            "kernel_ms": round(ms_s, 4),
                                            "speedup_vs_f64": round(kernel_ms / ms_s, 3)}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "disk32768", "n": n, "steps": K, "force_evaluations": evals,
                   "dt_days": 6, "a_au": [0.3, 4.0], "total_mass_earth": 5.0,
                   "encounter_pairs_final": count, "wall_s": round(wall, 3)},
        "roofline": roofline,
        "variants": variants,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
