"""Benchmark: RLT2 dual-ascent iterations/s and assignment problems/s at N=25.

One step = one full iteration of the Algorithm 1 loop body (spread B->C->D,
six-way D transfer, N^2 (N-1)^2 concentrations D->C, C transfer, N^2
concentrations C->B, B->LB') on the clustered N=25 instance (seed 0), with the
whole state resident in HBM.  Timed with HIP events on the stream the library
launches on.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=25)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--kernel-iters", type=int, default=3,
                    help="extra step-by-step iterations used to time each kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the certified FP32 leg")
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="oracle iterations in the CPU baseline (0: pick ~15 s of work)")
    return ap.parse_args()


def cpu_baseline(F, D, iters):
    import oracle
    o = oracle.Rlt2Oracle(F, D)
    o.iteration0()
    o.iterate(1)                       # first touch of the dense state, not timed
    if iters <= 0:
        t = time.perf_counter()
        o.iterate(1)
        per = time.perf_counter() - t
        iters = max(1, min(30, int(15.0 / max(per, 1e-3))))
    t = time.perf_counter()
    o.iterate(iters)
    dt = time.perf_counter() - t
    return iters / dt, iters, oracle.threads()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import qapgen
    from paper_1510_02065_amd import Rlt2

    N = args.N
    F, D = qapgen.clustered(N, args.seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)
    n1, n2 = N - 1, N - 2
    nD = N * N * n1 * n1 * n2 * n2
    laps_per_iter = N * N * n1 * n1 + N * N + 1
    elem = 8

    g = Rlt2(F, D, trace_level=1, use_graph=True, device=0, stream=stream.cuda_stream)
    g.ascend(args.warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    bound = g.ascend(args.steps)
    stop.record(stream)
    stop.synchronize()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    ms_per_step = ms / args.steps
    it_s = 1000.0 / ms_per_step

    # Per-kernel durations, HIP events around each step on the same stream.
    names = {3: "sweep (steps 1-3)", 4: "concentrate D->C", 5: "transfer C", 6: "concentrate C->B",
             7: "concentrate B->LB"}
    dur = {s: 0.0 for s in names}
    for _ in range(args.kernel_iters):
        for s in names:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            g.step(s)
            b.record(stream)
            b.synchronize()
            dur[s] += a.elapsed_time(b)
    dur = {s: v / max(1, args.kernel_iters) for s, v in dur.items()}
    dom = max(dur, key=dur.get)
    alg_bytes = 2.0 * nD * elem            # read and write of D once
    achieved = alg_bytes / (dur[dom] * 1e-3) / 1e9
    iter_frac = alg_bytes * it_s / 1e9 / HBM_PEAK_GBS

    lb_trace, _ = g.trace()

    # Certified FP32 leg on the same instance and iteration count.
    f32 = None
    if not args.no_fp32:
        h = Rlt2(F, D, precision="fp32", trace_level=1, use_graph=True, device=0, stream=stream.cuda_stream)
        h.ascend(args.warmup)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        cert = h.ascend(args.steps)
        b.record(stream)
        b.synchronize()
        ms32 = a.elapsed_time(b) / args.steps
        ref = lb_trace[args.warmup + args.steps]
        f32 = {"iters_per_s": 1000.0 / ms32, "laps_per_s": laps_per_iter * 1000.0 / ms32,
               "ms_per_step": ms32, "certified_bound": cert,
               "rel_err_vs_fp64_gpu": abs(cert - ref) / abs(ref),
               "certified_below_fp64": bool(cert <= ref),
               "speedup_vs_fp64": ms_per_step / ms32,
               "iteration_hbm_fraction": 2.0 * nD * 4 * (1000.0 / ms32) / 1e9 / HBM_PEAK_GBS}
        h.close()
    rel_err = None
    gold = os.path.join(ROOT, "tests", "golden", f"clustered{N}_seed{args.seed}_oracle_lb.json")
    total_iters = args.warmup + args.steps
    if os.path.exists(gold):
        ref = json.load(open(gold))["lb"]
        if total_iters < len(ref):
            rel_err = abs(lb_trace[total_iters] - ref[total_iters]) / abs(ref[total_iters])
    g.close()

    out = {
        "metric": "RLT2 dual-ascent iters/s and LAPs/s at N=25; bound rel. error vs FP64",
        "value": it_s,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"clustered QAP N={N} seed {args.seed} (3-5 Gaussian clusters, "
                               f"70% sparse heavy-tailed flows), plain FP64 RLT2 dual ascent",
                   "N": N, "laps_per_iteration": laps_per_iter, "D_entries": nD,
                   "parallelism": "single GPU"},
        "laps_per_s": laps_per_iter * it_s,
        "bound": bound,
        "bound_rel_err_vs_oracle": rel_err,
        "bound_iteration": total_iters,
        "iteration_hbm_fraction": iter_frac,
        "kernel_ms": {names[s]: round(v, 4) for s, v in dur.items()},
        "fp32_certified": f32,
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
    }
    if not args.no_cpu_baseline:
        v, iters, cores = cpu_baseline(F, D, args.cpu_iters)
        out["cpu_baseline"] = {"value": v, "unit": "iters/s", "cores": cores, "kind": "oracle",
                               "sample": f"{iters} iterations (after iteration 0 and one untimed "
                                         f"iteration) of the same N={N} instance, FP64"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
