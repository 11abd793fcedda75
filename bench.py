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
import warnings

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HBM bytes per launch of the binary64 pair kernel from the FETCH_SIZE / WRITE_SIZE passes
# (calibrated with a plain copy; see profiles/k_pairs_disk32768.md), valid for the kernel source
# whose hash is stored beside it.
PAIR_KERNEL_TRAFFIC = {"bytes": 84916510, "source_sha256": "e27177fb31e16e1a8b140103e76930b8ad60da34a747f9fc804dd90a7785dd06"}
PAIR_KERNEL_SOURCES = ["paper_2604_09184_amd/csrc/pairs.hip", "paper_2604_09184_amd/csrc/device.hpp"]
# Binary64 flop the hardware executes per pair, 64 x (ADD + MUL + TRANS + 2 FMA) from the
# SQ_INSTS_VALU_*_F64 counters of the same profile, for the same kernel source.
PAIR_KERNEL_HW_FLOP = {"per_pair": 22.42, "source_sha256": PAIR_KERNEL_TRAFFIC["source_sha256"]}
HBM_PEAK_GBPS = 8000.0             # MI355X HBM3E

FLOP_PER_PAIR = 20                 # N-body convention: 3 sub, 5 for r^2, rsqrt, 3 for m r^-3, 6 accumulate, 2 slack
FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X: 256 CU x 128 flop/clk x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3    # MI355X binary32 vector
METRIC = "pair interactions/s & % FP64 peak: plain vs split-prec/batched/adjoint"


def pair_kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for f in PAIR_KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def traffic_bytes():
    t = PAIR_KERNEL_TRAFFIC
    return t["bytes"] if t["source_sha256"] == pair_kernel_sha() else None


def hw_flop_per_pair():
    t = PAIR_KERNEL_HW_FLOP
    return t["per_pair"] if t["source_sha256"] == pair_kernel_sha() else None


def timed(fn):
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    s = torch.cuda.current_stream()
    e0.record(s)
    r = fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, r


def variant_split(nb, p):
    """Split-precision kick on the 131072-body narrow ring, 100 steps, against binary64: the
    accelerations at t0 against the CPU oracle on sampled bodies, the state after 100 steps, the
    K-weighted energy drift and the final encounter lists against the binary64 GPU run."""
    import numpy as np
    import torch

    import diskgen
    import oracle
    d = diskgen.workload("ring131072")
    n = len(d["m"])
    xm, v4 = diskgen.pack4(d["x"], d["v"], d["m"])
    rows = np.random.default_rng(11).choice(n, 1024, replace=False)
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    oacc, ol1 = oracle.kick_acc_rows(d["x"], d["m"], othr, p, rows)
    out = {"workload": "ring131072", "n": n, "steps": 100}
    res = {}
    for name, prec in (("f64", nb.PREC_F64), ("split", nb.PREC_SPLIT)):
        ctx = nb.Context(nb.Params(**p, precision=prec))
        X = torch.tensor(xm, device="cuda:0")
        V = torch.tensor(v4, device="cuda:0")
        thr = ctx.rcrit(X, V)
        acc = ctx.accelerations(X, thr)[:, :3].cpu().numpy()
        e0 = ctx.energy(X, V, thr)
        ctx.step(X, V, 2, thr=thr)                      # warm-up
        X = torch.tensor(xm, device="cuda:0")
        V = torch.tensor(v4, device="cuda:0")
        sec, (pairs, count) = timed(lambda: ctx.step(X, V, 100, thr=thr, pairs_cap=1 << 26))
        e1 = ctx.energy(X, V, thr)
        kms = ctx.bench_pairs(X, thr, reps=3)
        err = np.abs(acc[rows] - oacc).max(1) / np.maximum(np.abs(oacc).max(1), ol1)
        res[name] = (sec, X, pairs.cpu().numpy(), count)
        kpps = n * (n - 1) / (kms / 1e3)
        out[name] = {"pairs_per_s": 101 * n * (n - 1) / sec, "kernel_ms": round(kms, 3),
                     "kernel_pairs_per_s": kpps,
                     "acc_err_vs_oracle_1024_rows": {"max": float(err.max()), "p99": float(np.percentile(err, 99)),
                                                     "median": float(np.median(err))},
                     "Eprime_rel_drift_100_steps": float(abs(e1["Eprime"] - e0["Eprime"]) / abs(e0["Eprime"])),
                     "encounter_pairs_final": count}
    out["speedup_vs_f64"] = round(res["f64"][0] / res["split"][0], 3)
    # fraction of the mixed peak: of the 20 flop per pair, r^-1 and the two products forming r^-3
    # run in binary32 (157.3 TFLOP/s), the other 17 in binary64 (78.6 TFLOP/s)
    kp = out["split"]["kernel_pairs_per_s"]
    out["split"]["mixed_peak_frac"] = round(kp * (17 / (FP64_VECTOR_PEAK_TFLOPS * 1e12)
                                                  + 3 / (FP32_VECTOR_PEAK_TFLOPS * 1e12)), 4)
    out["f64"]["fp64_peak_frac"] = round(FLOP_PER_PAIR * out["f64"]["kernel_pairs_per_s"]
                                         / (FP64_VECTOR_PEAK_TFLOPS * 1e12), 4)
    dx = (res["split"][1][:, :3] - res["f64"][1][:, :3]).norm(dim=1) / res["f64"][1][:, :3].norm(dim=1)
    out["state_rel_diff_vs_f64_after_100_steps"] = {"max": float(dx.max()), "median": float(dx.median())}
    keys = [r[2][:, 0].astype(np.int64) << 32 | r[2][:, 1].astype(np.int64) for r in (res["f64"], res["split"])]
    out["final_pairs_only_in_one_run"] = int(np.setxor1d(keys[0], keys[1], assume_unique=True).size)
    return out


def variant_batched(nb, p):
    """4096 independent disks, N log-uniform in 64..2048, 100 steps in one persistent launch."""
    import torch

    import diskgen
    offs, x, v, m = diskgen.ensemble()
    xm, v4 = diskgen.pack4(x, v, m)
    X = torch.tensor(xm, device="cuda:0")
    V = torch.tensor(v4, device="cuda:0")
    ctx = nb.Context(nb.Params(**p))
    # every tile code applied to all classes, 20 steps each (on copies): what the autotuner chooses
    # from; codes in order and then in reverse order (the clock drifts during the first runs), the
    # mean of the two runs of each
    per_code = {code: 0.0 for code in range(4)}
    ctx.set_batched_tiles([0] * 6)
    Xc, Vc = X.clone(), V.clone()
    ctx.step_batched(offs, Xc, Vc, 2)
    for code in [0, 1, 2, 3, 3, 2, 1, 0]:
        ctx.set_batched_tiles([code] * 6)
        Xc, Vc = X.clone(), V.clone()
        t_code, _ = timed(lambda: ctx.step_batched(offs, Xc, Vc, 20))
        per_code[code] += t_code * 1e3 / 2
    per_code = {code: round(t, 2) for code, t in per_code.items()}
    ctx.set_batched_tiles([0] * 6)
    t_tune, tiles = timed(lambda: ctx.autotune_batched(offs, X, V, nsteps=10))
    sec, _ = timed(lambda: ctx.step_batched(offs, X, V, 100))
    sizes = offs[1:] - offs[:-1]
    pairs = 101 * float((sizes * (sizes - 1)).sum())
    ach = FLOP_PER_PAIR * pairs / sec / 1e12
    return {"workload": "ensemble4096", "systems": len(sizes), "bodies": int(offs[-1]), "steps": 100,
            "pairs_per_s": pairs / sec, "seconds": round(sec, 4), "tiles": tiles,
            "autotune_seconds": round(t_tune, 3),
            "ms_20_steps_per_uniform_code": per_code,
            "roofline": {"bound": "alu", "kernel": "k_batched (binary64, one launch)",
                         "achieved": round(ach, 3), "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(ach / FP64_VECTOR_PEAK_TFLOPS, 4)}}


def variant_adjoint(nb, p):
    """Gradient of |x(T) - target|^2 after 100 steps of the 8192-body disk, checkpoint every 10."""
    import torch

    import diskgen
    from paper_2604_09184_amd.autograd import trajectory
    d = diskgen.workload("adjoint8192")
    n = len(d["m"])
    xm, v4 = diskgen.pack4(d["x"], d["v"], d["m"])
    ctx = nb.Context(nb.Params(**p))
    X0 = torch.tensor(xm, device="cuda:0")
    V0 = torch.tensor(v4, device="cuda:0")
    thr = ctx.rcrit(X0, V0)
    target = None
    res = {}
    for rep in range(2):
        X = X0.clone().requires_grad_(True)
        V = V0.clone().requires_grad_(True)
        fsec, (xT, vT) = timed(lambda: trajectory(ctx, X, V, 100, every=10, thr=thr))
        if target is None:
            target = (xT[:, :3] + 1e-4).detach()
        loss = ((xT[:, :3] - target) ** 2).sum()
        bsec, _ = timed(lambda: loss.backward())
        res = {"forward_s": fsec, "backward_s": bsec}
    # pair evaluations in the backward, per segment of 10 steps: the replay (11 kick evaluations)
    # and the kick derivatives (11 evaluations, two half kicks at the same positions sharing one)
    evals = 10 * (11 + 11)
    return {"workload": "adjoint8192", "n": n, "steps": 100, "checkpoint_every": 10,
            "forward_s": round(res["forward_s"], 4), "backward_s": round(res["backward_s"], 4),
            "backward_over_forward": round(res["backward_s"] / res["forward_s"], 2),
            "forward_pairs_per_s": 101 * n * (n - 1) / res["forward_s"],
            "backward_pair_evals_per_s": evals * n * (n - 1) / res["backward_s"]}


def variant_hybrid(nb, p):
    """Hybrid step (close-encounter groups integrated in full in the drift) against the plain step on
    the 2048-body disk, 100 steps each: time and the drift of the full energy E and of E'; then the
    hybrid step with collisions as perfect mergers (f = 300)."""
    import torch

    import diskgen
    d = diskgen.workload("disk2048")
    n = len(d["m"])
    xm, v4 = diskgen.pack4(d["x"], d["v"], d["m"])
    ctx = nb.Context(nb.Params(**p))
    out = {"workload": "disk2048", "n": n, "steps": 100}
    for name in ("plain", "hybrid"):
        X = torch.tensor(xm, device="cuda:0")
        V = torch.tensor(v4, device="cuda:0")
        thr = ctx.rcrit(X, V)
        e0 = ctx.energy(X, V, thr)
        run = (lambda: ctx.step(X, V, 100, thr=thr)) if name == "plain" else (lambda: ctx.step_hybrid(X, V, 100, thr=thr))
        Xw, Vw = X.clone(), V.clone()
        (ctx.step(Xw, Vw, 2, thr=thr) if name == "plain" else ctx.step_hybrid(Xw, Vw, 2, thr=thr))   # warm-up
        sec, stats = timed(run)
        e1 = ctx.energy(X, V, thr)
        out[name] = {"seconds": round(sec, 4), "ms_per_step": round(sec * 10, 4),
                     "E_rel_drift": float(abs(e1["E"] - e0["E"]) / abs(e0["E"])),
                     "Eprime_rel_drift": float(abs(e1["Eprime"] - e0["Eprime"]) / abs(e0["Eprime"]))}
        if name == "hybrid":
            out[name]["groups"] = stats
    # the same 100 hybrid steps with collisions as perfect mergers at f = 300 (radii from the
    # bodies' density): time per step and the number of mergers
    X = torch.tensor(xm, device="cuda:0")
    V = torch.tensor(v4, device="cuda:0")
    R = torch.tensor(d["radius"], device="cuda:0")
    thr = ctx.rcrit(X, V)
    sec, stats = timed(lambda: ctx.step_hybrid(X, V, 100, thr=thr, radius=R, f=300.0))
    out["hybrid_merge_f300"] = {"seconds": round(sec, 4), "ms_per_step": round(sec * 10, 4),
                                "mergers": stats["mergers"], "bodies_left": int((X[:, 3] > 0).sum().item())}
    return out


def variant_levels(nb, p):
    """The 32768-body disk, whose close pairs percolate into groups too large for the direct
    integrator: 10 steps plain, hybrid, and hybrid with one intermediate changeover level (s = 8)."""
    import torch

    import diskgen
    ctx = nb.Context(nb.Params(**p))
    d = diskgen.workload("disk32768")
    xm, v4 = diskgen.pack4(d["x"], d["v"], d["m"])
    big = {}
    for name, kw in (("plain", None), ("hybrid", {}), ("levels1_s8", {"levels": 1, "substeps": 8})):
        X = torch.tensor(xm, device="cuda:0")
        V = torch.tensor(v4, device="cuda:0")
        thr = ctx.rcrit(X, V)
        e0 = ctx.energy(X, V, thr)
        if kw is None:
            sec, st = timed(lambda: ctx.step(X, V, 10, thr=thr))
            st = None
        else:
            # the plain hybrid step has groups too large for the direct integrator here: the
            # binding's warning is expected, and the count is reported below
            with warnings.catch_warnings():
                warnings.simplefilter("ignore", nb.NBodyWarning)
                sec, st = timed(lambda: ctx.step_hybrid(X, V, 10, thr=thr, **kw))
        e1 = ctx.energy(X, V, thr)
        big[name] = {"ms_per_step": round(sec * 100, 4),
                     "E_rel_drift": float(abs(e1["E"] - e0["E"]) / abs(e0["E"]))}
        if st is not None:
            big[name]["groups"] = {k: st[k] for k in ("groups", "largest", "bodies", "too_large")}
    return {"workload": "disk32768", "steps": 10, **big}


def variant_small_n(nb, p):
    """Small systems: per-step launches (nbody_step) against the self-tuned switch (one persistent
    launch when that is faster) for disks of 32 ... 2048 bodies, 200 steps each."""
    import torch

    import diskgen
    ctx = nb.Context(nb.Params(**p))
    out = {"steps": 200, "sizes": {}}
    for n in (32, 64, 128, 256, 2048):
        d = diskgen.workload("disk2048", n=n)
        xm, v4 = diskgen.pack4(d["x"], d["v"], d["m"])
        X = torch.tensor(xm, device="cuda:0")
        V = torch.tensor(v4, device="cuda:0")
        path = ctx.autotune_step(X, V, ntrial=20)
        ctx.step(X.clone(), V.clone(), 5)
        t_plain, _ = timed(lambda: ctx.step(X, V, 200))
        t_auto, _ = timed(lambda: ctx.step_auto(X, V, 200))
        out["sizes"][str(n)] = {"path": path, "per_step_launches_us": round(t_plain / 200 * 1e6, 2),
                                "switch_us": round(t_auto / 200 * 1e6, 2)}
    return out


def host_cpu():
    """Model name and logical CPU counts of the host (the machine the oracle runs on)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "cpus_available": avail}


def cpu_baseline(budget_s=25.0, rows_1t=4096):
    """The oracle (plain C++, OpenMP) on the first steps of the same N = 32768 disk, with every
    thread it is given; then, on one thread, one force evaluation of a block of rows."""
    import numpy as np

    import diskgen
    import oracle
    p = diskgen.PARAMS
    d = diskgen.workload("disk32768")
    n = len(d["m"])
    thr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    x, v = d["x"], d["v"]
    threads = oracle.num_threads()
    steps = 0
    t0 = time.perf_counter()
    while steps < 10:
        x, v, _ = oracle.step(x, v, d["m"], p, 1, thr=thr)
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    evals = 2 * steps                # the oracle evaluates both half kicks of every step
    # one thread: the accelerations of the first rows_1t bodies (all n partners each)
    oracle.set_threads(1)
    try:
        rows = np.arange(rows_1t, dtype=np.int64)
        t1 = time.perf_counter()
        oracle.kick_acc_rows(d["x"], d["m"], thr, p, rows)
        el1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(threads)
    return {"value": evals * n * (n - 1) / el, "unit": "pair-interactions/s",
            "cores": threads, "kind": "oracle",
            "sample": f"first {steps} steps of the N={n} disk ({evals} force evaluations, "
                      f"{el:.1f} s), full step incl. drift and jumps",
            "host": host_cpu(),
            "one_thread": {"value": rows_1t * (n - 1) / el1, "unit": "pair-interactions/s", "cores": 1,
                           "sample": f"accelerations of {rows_1t} of the N={n} disk's bodies against all "
                                     f"{n - 1} partners ({el1:.2f} s)"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--settle", type=float, default=0.5,
                    help="seconds of pair-kernel launches before the timed region (clock ramp)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--only", choices=["split", "batched", "adjoint", "hybrid", "levels", "small_n"],
                    help="run only this variant and print its JSON (for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import diskgen
    import paper_2604_09184_amd as nb

    dev = torch.device("cuda:0")
    if args.only:
        p = diskgen.PARAMS
        fn = {"split": variant_split, "batched": variant_batched, "adjoint": variant_adjoint,
              "hybrid": variant_hybrid, "levels": variant_levels, "small_n": variant_small_n}[args.only]
        print(json.dumps({args.only: fn(nb, p)}), flush=True)
        return
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
    # the whole workspace of the timed call is sized here, and its list buffers are created here:
    # nothing is allocated (and nothing waits) between the two events
    ctx.reserve(n, nb.RESERVE_KICK | nb.RESERVE_LIST)
    thr = ctx.rcrit(X, V)
    cap = 1 << 22
    pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    print(f"[bench] N={n} warmup {args.warmup} steps (the timed call's own arguments)", file=sys.stderr, flush=True)
    if args.warmup:
        ctx.step(X, V, args.warmup, thr=thr, out=(pairs, count))
    torch.cuda.synchronize()
    # the clock ramps up over the first tenths of a second of binary64 load: settle it by time,
    # whatever the number of warm-up steps, with launches of the dominant kernel (no state change)
    t_set = time.perf_counter()
    settle_launches = 0
    while time.perf_counter() - t_set < args.settle:
        ctx.bench_pairs(X, thr, reps=25)
        settle_launches += 25
    settle_s = time.perf_counter() - t_set

    K = args.steps
    print(f"[bench] timing {K} steps (clock settled for {settle_s:.2f} s)", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    ctx.step(X, V, K, thr=thr, out=(pairs, count))
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    count = int(count.item())
    evals = K + 1
    value = evals * n * (n - 1) / (ms / 1e3)

    # the dominant kernel alone: mean launch time of the pair kernel (HIP events on the stream)
    kernel_ms = ctx.bench_pairs(X, thr, reps=20)
    achieved = FLOP_PER_PAIR * n * (n - 1) / (kernel_ms / 1e3) / 1e12
    traffic = traffic_bytes()
    hwf = hw_flop_per_pair()
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4),
                "traffic": traffic, "kernel": "k_pairs (binary64)",
                "kernel_ms": round(kernel_ms, 4),
                "pairs_per_s_kernel": n * (n - 1) / (kernel_ms / 1e3),
                # beside the algorithmic figure: the binary64 flop the hardware executes (counter
                # profile of this kernel source) and the HBM rate of the counted traffic
                "hw_fp64": None if hwf is None else {
                    "flop_per_pair": hwf,
                    "tflops": round(hwf * n * (n - 1) / (kernel_ms / 1e3) / 1e12, 3),
                    "frac": round(hwf * n * (n - 1) / (kernel_ms / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS, 4)},
                "hbm": None if traffic is None else {
                    "GBps": round(traffic / (kernel_ms / 1e3) / 1e9, 1), "peak_GBps": HBM_PEAK_GBPS,
                    "frac": round(traffic / (kernel_ms / 1e3) / 1e9 / HBM_PEAK_GBPS, 4)}}

    variants = {}
    if not args.no_variants:
        print("[bench] variant: split precision (ring131072)", file=sys.stderr, flush=True)
        variants["split_precision"] = variant_split(nb, p)
        print("[bench] variant: batched (ensemble4096)", file=sys.stderr, flush=True)
        variants["batched"] = variant_batched(nb, p)
        print("[bench] variant: adjoint (adjoint8192)", file=sys.stderr, flush=True)
        variants["adjoint"] = variant_adjoint(nb, p)
        print("[bench] variant: hybrid step (disk2048)", file=sys.stderr, flush=True)
        variants["hybrid"] = variant_hybrid(nb, p)
        print("[bench] variant: changeover levels (disk32768)", file=sys.stderr, flush=True)
        variants["levels"] = variant_levels(nb, p)
        print("[bench] variant: small-N switch", file=sys.stderr, flush=True)
        variants["small_n"] = variant_small_n(nb, p)

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
                   "encounter_pairs_final": count, "wall_s": round(wall, 3),
                   "clock_settle_s": round(settle_s, 3), "clock_settle_launches": settle_launches},
        "roofline": roofline,
        "variants": variants,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
