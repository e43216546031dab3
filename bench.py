"""Benchmark: RLT2 dual-ascent iterations/s and assignment problems/s at N=25.

One step = one full iteration of the Algorithm 1 loop body (spread B->C->D,
six-way D transfer, N^2 (N-1)^2 concentrations D->C, C transfer, N^2
concentrations C->B, B->LB') on the clustered N=25 instance (seed 0), with the
whole state resident in HBM.  The timed region launches the iterations step by
step with HIP events around every step on the stream the library launches on,
so the per-kernel durations behind the roofline figure come from the timed
iterations themselves; the same iterations launched as one HIP graph each are
timed after it as `graph_iters_per_s`.  Prints one JSON line.

`--calibrate-copy` instead runs the plain 1 GiB device copy whose FETCH_SIZE and
WRITE_SIZE counter readings scale the per-dispatch HBM traffic figures.
"""
import argparse
import json
import os
import sys
import hashlib
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per dispatch from `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE`
# runs of this script, each scaled by what the same counter reads for a plain
# 1 GiB copy (FETCH_SIZE reads 0.5 GiB there, WRITE_SIZE 1 GiB: factors 2.0 and
# 1.0).  Keyed by kernel step, N and precision, and valid only for the kernel
# sources whose digest is recorded: any change to them makes the figure null
# until the counters are taken again.
TRAFFIC = {
    # (step, N, dtype, complementary pairs once): (csrc digest, scaled FETCH bytes, scaled WRITE bytes)
    (4, 25, "f64", True): ("8c74117988d43250", 493808.9 * 1024 * 2.0, 782546.7 * 1024 * 1.0),
    (3, 25, "f64", True): ("8c74117988d43250", 397776.1 * 1024 * 2.0, 744000.8 * 1024 * 1.0),
}


def csrc_digest():
    d = os.path.join(ROOT, "paper_1510_02065_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".hpp", ".h")):
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=25)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--bound-iters", type=int, default=100,
                    help="iterations after which the bound is compared with the oracle's trace")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the 1 GiB copy used to scale the traffic counters")
    ap.add_argument("--all-blocks", action="store_true",
                    help="concentrate every D block instead of each complementary pair once")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the certified FP32 leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched branch-and-bound leg")
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


def batched_leg(stream, iters=20):
    """The batched workload: 256 branch-and-bound nodes cut from one clustered
    N=24 instance (seed 0) by fixing 2..14 assignments (N' = 10..22), all in
    one handle, FP64 and certified FP32; iterations launched as HIP graphs
    after one untimed iteration (which runs the tuner)."""
    import numpy as np
    import torch

    import qapgen
    from paper_1510_02065_amd import Rlt2, subproblem

    F, D, fixes = qapgen.nodes(count=256, parent_N=24, seed=0, m_lo=2, m_hi=14)
    nodes = [subproblem(F, D, fac, loc) for fac, loc in fixes]
    sizes = [n[0].shape[0] for n in nodes]
    laps = int(sum(n * n * (n - 1) * (n - 1) // 2 + n * n + 1 for n in sizes))
    args = ([n[0] for n in nodes], [n[1] for n in nodes], [n[2] for n in nodes], [n[3] for n in nodes])
    out = {"workload": f"256 branch-and-bound nodes of clustered N=24 seed 0 (N'={min(sizes)}..{max(sizes)})",
           "iterations": iters, "laps_per_iteration": laps}
    lb64 = None
    for prec in ("fp64", "fp32"):
        g = Rlt2.batch(*args, precision=prec, stream=stream.cuda_stream)
        g.ascend(1)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        g.ascend(iters)
        b.record(stream)
        b.synchronize()
        ms = a.elapsed_time(b) / iters
        leg = {"iters_per_s": 1000.0 / ms, "laps_per_s": laps * 1000.0 / ms, "ms_per_iteration": ms}
        if prec == "fp64":
            lb64 = g.bounds()
        else:
            _, cert = g.bounds(certified=True)
            leg["certified_rel_err_vs_fp64_max"] = float(np.max(np.abs(cert - lb64) / np.abs(lb64)))
            leg["certified_below_fp64"] = bool((cert <= lb64).all())
        out[prec] = leg
        g.close()
    out["speedup_fp32_vs_fp64"] = out["fp32"]["iters_per_s"] / out["fp64"]["iters_per_s"]
    return out


def calibrate_copy():
    import torch
    x = torch.empty(128 * 1024 * 1024, dtype=torch.float64, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(10):
        y.copy_(x)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / 10
    print(f"copy calibration: 1 GiB read + 1 GiB write per copy, {ms:.3f} ms, "
          f"{2.0 * x.numel() * 8 / (ms * 1e-3) / 1e9:.0f} GB/s of reads plus writes", flush=True)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
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
    nC = N * N * n1 * n1
    nD = nC * n2 * n2
    pair = not args.all_blocks
    d_laps = nC // 2 if pair else nC
    laps_per_iter = d_laps + N * N + 1
    elem = 8
    # Algorithmic HBM bytes of each step's kernels: every coefficient the step
    # must read and every one it must write, once.
    # With one block stored per complementary pair, D holds nD / 2 entries.
    nDs = nD // 2 if pair else nD
    step_bytes = {
        3: 2.0 * nDs * elem + 2.0 * nC * elem,   # stored D read and written, C read and cleared
        4: 2.0 * nDs * elem + 2.0 * nC * elem,   # stored blocks read and written, C read and written
        5: 2.0 * nC * elem,
        6: 2.0 * nC * elem + 2.0 * N * N * elem,
        7: 2.0 * N * N * elem,
    }

    names = {3: "sweep (steps 1-3)", 4: "concentrate D->C", 5: "transfer C", 6: "concentrate C->B",
             7: "concentrate B->LB"}
    g = Rlt2(F, D, trace_level=1, use_graph=True, device=0, stream=stream.cuda_stream, complementary=pair)
    g.ascend(args.warmup)
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in names]
          for _ in range(args.steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for t in range(args.steps):
        for (a, b), s in zip(ev[t], names):
            a.record(stream)
            g.step(s)
            b.record(stream)
    stop.record(stream)
    stop.synchronize()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    ms_per_step = ms / args.steps
    it_s = 1000.0 / ms_per_step
    dur = {s: sum(ev[t][q][0].elapsed_time(ev[t][q][1]) for t in range(args.steps)) / args.steps
           for q, s in enumerate(names)}
    dom = max(dur, key=dur.get)
    iter_frac = 2.0 * nDs * elem * it_s / 1e9 / HBM_PEAK_GBS   # against one read and write of D
    digest = csrc_digest()

    def roofline(step):
        rec = TRAFFIC.get((step, N, "f64", pair))
        ach = step_bytes[step] / (dur[step] * 1e-3) / 1e9
        return {"bound": "hbm", "kernel": names[step], "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS,
                "traffic": rec[1] + rec[2] if rec is not None and rec[0] == digest else None,
                "alg_bytes": step_bytes[step], "kernel_ms": dur[step]}

    # Further iterations as one HIP graph launch each (the library's ascend),
    # up to the iteration at which the bound is compared with the oracle.
    extra = max(args.steps, args.bound_iters - args.warmup - args.steps)
    total_iters = args.warmup + args.steps + extra
    ga = torch.cuda.Event(enable_timing=True)
    gb = torch.cuda.Event(enable_timing=True)
    ga.record(stream)
    g.ascend(extra)
    gb.record(stream)
    gb.synchronize()
    graph_it_s = 1000.0 * extra / ga.elapsed_time(gb)
    lb_trace, _ = g.trace()

    # Certified FP32 leg on the same instance: the same warm-up and timed
    # iterations, then on to the same final iteration for the bound.
    f32 = None
    if not args.no_fp32:
        h = Rlt2(F, D, precision="fp32", trace_level=1, use_graph=True, device=0, stream=stream.cuda_stream,
                 complementary=pair)
        h.ascend(args.warmup)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        h.ascend(args.steps)
        b.record(stream)
        b.synchronize()
        ms32 = a.elapsed_time(b) / args.steps
        cert = h.ascend(extra)
        ref = lb_trace[total_iters]
        f32 = {"iters_per_s": 1000.0 / ms32, "laps_per_s": laps_per_iter * 1000.0 / ms32,
               "ms_per_step": ms32, "certified_bound": cert, "bound_iteration": total_iters,
               "rel_err_vs_fp64_gpu": abs(cert - ref) / abs(ref),
               "certified_below_fp64": bool(cert <= ref),
               "speedup_vs_fp64": ms_per_step / ms32,
               "iteration_hbm_fraction": 2.0 * nDs * 4 * (1000.0 / ms32) / 1e9 / HBM_PEAK_GBS}
        h.close()
    rel_err = rel_err_max = None
    gold = os.path.join(ROOT, "tests", "golden", f"clustered{N}_seed{args.seed}_oracle_lb.json")
    if os.path.exists(gold):
        ref = json.load(open(gold))["lb"]
        m = min(len(ref), len(lb_trace))
        errs = [abs(lb_trace[t] - ref[t]) / abs(ref[t]) for t in range(m)]
        rel_err_max = max(errs)
        if total_iters < m:
            rel_err = errs[total_iters]
    bound = lb_trace[total_iters]
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
                   "D_blocks": "one stored and concentrated per complementary pair" if pair else "all stored and concentrated",
                   "parallelism": "single GPU"},
        "laps_per_s": laps_per_iter * it_s,
        "bound": bound,
        "bound_rel_err_vs_oracle": rel_err,
        "bound_rel_err_vs_oracle_max_over_iterations": rel_err_max,
        "bound_iteration": total_iters,
        "graph_iters_per_s": graph_it_s,
        "iteration_hbm_fraction": iter_frac,
        "kernel_ms": {names[s]: round(v, 4) for s, v in dur.items()},
        "fp32_certified": f32,
        "roofline": roofline(dom),
        # The cost sweep (steps 1-3) against the same peak: the step that
        # moves the whole cost array and is bound by HBM.
        "roofline_sweep": roofline(3),
    }
    if not args.no_batched:
        out["batched"] = batched_leg(stream)
    if not args.no_cpu_baseline:
        v, iters, cores = cpu_baseline(F, D, args.cpu_iters)
        out["cpu_baseline"] = {"value": v, "unit": "iters/s", "cores": cores, "kind": "oracle",
                               "sample": f"{iters} iterations (after iteration 0 and one untimed "
                                         f"iteration) of the same N={N} instance, FP64"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
