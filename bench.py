"""Benchmark: RLT2 dual-ascent iterations/s and assignment problems/s at N=25.

One step = one full iteration of the Algorithm 1 loop body (spread B->C->D,
six-way D transfer, N^2 (N-1)^2 concentrations D->C, C transfer, N^2
concentrations C->B, B->LB') on the clustered N=25 instance (seed 0), with the
whole state resident in HBM.  The timed region launches the iterations step by
step with HIP events around every step on the stream the library launches on,
so the per-kernel durations behind the roofline figure come from the timed
iterations themselves; the next iterations, launched as one HIP graph each
(the library's ascend), are timed after it as `graph_iters_per_s`.

Every other leg is timed the same two ways over the same iteration counts, so
rates compare like for like: certified FP32 and round-to-nearest FP32 on the
same instance, FP64 with every D block stored and solved, N=40 in FP64 and
certified FP32 (20 iterations), and the batched branch-and-bound nodes.  The
oracle is timed on the host single-threaded and on every core of the affinity
set.  Prints one JSON line (progress goes to stderr).

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
    # (step, N, precision, complementary pairs once): (csrc digest, scaled FETCH bytes, scaled WRITE bytes)
    (4, 25, "fp64", True): ("48ce863f5d0130d8", 373952.4 * 1024 * 2.0, 774286.3 * 1024 * 1.0),
    (3, 25, "fp64", True): ("48ce863f5d0130d8", 397714.9 * 1024 * 2.0, 743996.1 * 1024 * 1.0),
    (4, 25, "fp32", True): ("48ce863f5d0130d8", 187197.0 * 1024 * 2.0, 385420.4 * 1024 * 1.0),
    (3, 25, "fp32", True): ("48ce863f5d0130d8", 211227.3 * 1024 * 2.0, 390437.3 * 1024 * 1.0),
    (4, 25, "fp32n", True): ("48ce863f5d0130d8", 187172.3 * 1024 * 2.0, 386180.9 * 1024 * 1.0),
    (3, 25, "fp32n", True): ("48ce863f5d0130d8", 201844.8 * 1024 * 2.0, 372027.2 * 1024 * 1.0),
    (4, 40, "fp64", True): ("48ce863f5d0130d8", 6877959.3 * 1024 * 2.0, 14611774.7 * 1024 * 1.0),
    (3, 40, "fp64", True): ("48ce863f5d0130d8", 7947267.8 * 1024 * 2.0, 17150922.9 * 1024 * 1.0),
    (4, 40, "fp32", True): ("48ce863f5d0130d8", 3441542.8 * 1024 * 2.0, 7922078.5 * 1024 * 1.0),
    (3, 40, "fp32", True): ("48ce863f5d0130d8", 3716187.3 * 1024 * 2.0, 13650580.4 * 1024 * 1.0),
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
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 legs (certified and nearest)")
    ap.add_argument("--no-all-blocks", action="store_true", help="skip the every-block FP64 leg")
    ap.add_argument("--no-large", action="store_true", help="skip the N=40 legs")
    ap.add_argument("--no-solvers", action="store_true",
                    help="skip the canonical-vs-auction assignment solver comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched branch-and-bound leg")
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="oracle iterations in the CPU baseline (0: pick ~15 s of work)")
    return ap.parse_args()


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(F, D, iters, budget_s=12.0):
    """The oracle on the host: single-threaded, then on every core of the
    process's affinity set; each timed over a bounded number of iterations
    (about `budget_s` seconds) after iteration 0 and one untimed iteration."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    out = {}
    for label, threads in (("single_thread", 1), ("all_cores", cores)):
        oracle.set_threads(threads)
        o = oracle.Rlt2Oracle(F, D)
        o.iteration0()
        t = time.perf_counter()
        o.iterate(1)                   # first touch of the dense state, not counted
        per = time.perf_counter() - t
        n = iters if iters > 0 else max(1, min(30, int(budget_s / max(per, 1e-3))))
        t = time.perf_counter()
        o.iterate(n)
        dt = time.perf_counter() - t
        out[label] = {"iters_per_s": n / dt, "iterations": n, "threads": oracle.threads()}
        o.close()
    oracle.set_threads(cores)
    out["model"] = _cpu_model()
    out["affinity_cores"] = cores
    return out


def batched_leg(stream, iters=20):
    """The batched workload: 256 branch-and-bound nodes cut from one clustered
    N=24 instance (seed 0) by fixing 2..14 assignments (N' = 10..22), all in
    one handle, FP64 and certified FP32; iterations launched as HIP graphs
    after one untimed iteration (which runs the tuner).  Each size's D->C
    concentration overlaps the next size's sweep; FP64 is also timed with the
    steps one after the other."""
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
    for prec, key, overlap in (("fp64", "fp64", True), ("fp32", "fp32", True), ("fp64", "fp64_sequential", False)):
        g = Rlt2.batch(*args, precision=prec, stream=stream.cuda_stream, overlap=overlap)
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
        if key == "fp64":
            lb64 = g.bounds()
        elif key == "fp32":
            _, cert = g.bounds(certified=True)
            leg["certified_rel_err_vs_fp64_max"] = float(np.max(np.abs(cert - lb64) / np.abs(lb64)))
            leg["certified_below_fp64"] = bool((cert <= lb64).all())
        else:
            leg["bounds_equal_overlapped"] = bool((g.bounds() == lb64).all())
        out[key] = leg
        g.close()
    out["speedup_fp32_vs_fp64"] = out["fp32"]["iters_per_s"] / out["fp64"]["iters_per_s"]
    out["speedup_overlapped_vs_sequential_fp64"] = out["fp64"]["iters_per_s"] / out["fp64_sequential"]["iters_per_s"]
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


NAMES = {3: "sweep (steps 1-3)", 4: "concentrate D->C", 5: "transfer C", 6: "concentrate C->B",
         7: "concentrate B->LB"}


def sizes(N, pair):
    n1, n2 = N - 1, N - 2
    nC = N * N * n1 * n1
    nD = nC * n2 * n2
    return nC, nD, (nD // 2 if pair else nD)


def step_bytes(N, pair, elem):
    """Algorithmic HBM bytes of each step's kernels: every coefficient the
    step must read and every one it must write, once (with one block stored
    per complementary pair, D holds half the entries)."""
    nC, _, nDs = sizes(N, pair)
    return {
        3: 2.0 * nDs * elem + 2.0 * nC * elem,   # stored D read and written, C read and cleared
        4: 2.0 * nDs * elem + 2.0 * nC * elem,   # stored blocks read and written, C read and written
        5: 2.0 * nC * elem,
        6: 2.0 * nC * elem + 2.0 * N * N * elem,
        7: 2.0 * N * N * elem,
    }


def laps_per_iteration(N, pair):
    nC = N * N * (N - 1) * (N - 1)
    return (nC // 2 if pair else nC) + N * N + 1


def timed_leg(F, D, precision, pair, warmup, steps, graph_iters, stream, lap_solver="canonical"):
    """One handle on the stream: `warmup` untimed iterations (the first runs
    the tuner), `steps` iterations launched step by step with HIP events
    around every step, then `graph_iters` iterations launched as one HIP graph
    each (the library's ascend).  Both timed regions are bracketed by
    synchronisation."""
    import torch

    from paper_1510_02065_amd import Rlt2
    N = F.shape[0]
    elem = 8 if precision == "fp64" else 4
    g = Rlt2(F, D, precision=precision, trace_level=1, use_graph=True, device=0, stream=stream.cuda_stream,
             complementary=pair, lap_solver=lap_solver)
    if warmup:
        g.ascend(warmup)
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in NAMES]
          for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for t in range(steps):
        for (a, b), s in zip(ev[t], NAMES):
            a.record(stream)
            g.step(s)
            b.record(stream)
    stop.record(stream)
    stop.synchronize()
    torch.cuda.synchronize()
    ms_step = start.elapsed_time(stop) / steps
    dur = {s: sum(ev[t][q][0].elapsed_time(ev[t][q][1]) for t in range(steps)) / steps
           for q, s in enumerate(NAMES)}
    ms_graph = None
    if graph_iters > 0:
        g.bound()   # moves the step-launched iterations' trace entries to the host
        torch.cuda.synchronize()
        ga = torch.cuda.Event(enable_timing=True)
        gb = torch.cuda.Event(enable_timing=True)
        ga.record(stream)
        g.ascend(graph_iters)
        gb.record(stream)
        gb.synchronize()
        ms_graph = ga.elapsed_time(gb) / graph_iters
    lb_trace, _ = g.trace()
    cert = g.certify()
    g.close()
    bytes_ = step_bytes(N, pair, elem)
    dom = max(dur, key=dur.get)
    return {"N": N, "precision": precision, "pair": pair, "elem": elem, "ms_step": ms_step, "ms_graph": ms_graph,
            "dur": dur, "dom": dom, "bytes": bytes_, "lb_trace": lb_trace, "cert": cert,
            "iterations": warmup + steps + graph_iters}


def solver_leg(F, D, stream, state_iters=10, reps=3):
    """The two assignment solvers on the same live blocks: the stored D blocks
    (n = N-2) that step 4 of iteration `state_iters` + 1 concentrates at N=25,
    solved as one qap_lap_solve batch on device pointers with residuals
    written (the work of one D->C concentration), by the canonical dual and by
    the auction."""
    import numpy as np
    import torch

    from paper_1510_02065_amd import Rlt2, lap_solve_device
    N = F.shape[0]
    n = N - 2
    g = Rlt2(F, D, device=0, stream=stream.cuda_stream)
    g.ascend(state_iters)
    g.step(3)   # the next iteration's steps 1-3: D now holds the blocks step 4 concentrates
    _, _, _, Dst = g.read_state()
    g.close()
    nblk = N * N * (N - 1) * (N - 1)
    blocks = Dst.reshape(nblk, n * n)
    # one block of each complementary pair: (i, j, k, n) with i < k
    idx = []
    b = 0
    for i in range(N):
        for j in range(N):
            for k in range(N):
                if k == i:
                    continue
                for q in range(N):
                    if q == j:
                        continue
                    if i < k:
                        idx.append(b)
                    b += 1
    idx = np.array(idx)
    dev = torch.device("cuda:0")
    src = torch.tensor(blocks[idx].ravel(), dtype=torch.float64, device=dev)
    cnt = len(idx)
    nv = torch.full((cnt,), n, dtype=torch.int32, device=dev)
    mo = torch.arange(cnt, dtype=torch.int64, device=dev) * (n * n)
    value = torch.empty(cnt, dtype=torch.float64, device=dev)
    out = {"workload": f"{cnt} stored D blocks (n={n}) of clustered N={N} seed 0 as step 4 of iteration "
                       f"{state_iters + 1} receives them, one qap_lap_solve call on device pointers with "
                       f"residuals written",
           "problems": cnt}
    vals = {}
    for name, auction in (("canonical", False), ("auction", True)):
        times = []
        for _ in range(reps):
            cost = src.clone()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lap_solve_device(nv, mo, None, cost, value, residual=True, stream=stream, auction=auction)
            e.record(stream)
            e.synchronize()
            times.append(a.elapsed_time(e))
        ms = min(times)
        vals[name] = value.cpu().numpy()
        out[name] = {"ms": ms, "laps_per_s": cnt * 1000.0 / ms}
    # Gap of each auction value to the canonical one, relative to the mean
    # canonical value (many blocks have value 0).
    gap = (vals["canonical"] - vals["auction"]) / float(np.abs(vals["canonical"]).mean())
    out["auction"]["value_below_canonical_max"] = float(gap.max())
    out["auction"]["value_above_canonical_max"] = float((-gap).max())
    out["auction"]["value_gap_mean"] = float(gap.mean())
    out["auction_speed_vs_canonical"] = out["canonical"]["ms"] / out["auction"]["ms"]
    return out


def roofline(leg, step, digest):
    N, pair, elem, dur = leg["N"], leg["pair"], leg["elem"], leg["dur"]
    rec = TRAFFIC.get((step, N, leg["precision"], pair))
    ach = leg["bytes"][step] / (dur[step] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": NAMES[step], "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS,
            "traffic": rec[1] + rec[2] if rec is not None and rec[0] == digest else None,
            "alg_bytes": leg["bytes"][step], "kernel_ms": dur[step]}


def leg_summary(leg, digest, ref_leg=None, with_rooflines=True):
    N, pair = leg["N"], leg["pair"]
    laps = laps_per_iteration(N, pair)
    _, _, nDs = sizes(N, pair)
    it_s = 1000.0 / leg["ms_step"]
    out = {"iters_per_s": it_s, "laps_per_s": laps * it_s, "ms_per_step": leg["ms_step"],
           "iteration_hbm_fraction": 2.0 * nDs * leg["elem"] * it_s / 1e9 / HBM_PEAK_GBS,
           "kernel_ms": {NAMES[s]: round(v, 4) for s, v in leg["dur"].items()}}
    if leg["ms_graph"] is not None:
        out["graph_iters_per_s"] = 1000.0 / leg["ms_graph"]
        out["graph_laps_per_s"] = laps * 1000.0 / leg["ms_graph"]
    if with_rooflines:
        out["roofline"] = roofline(leg, leg["dom"], digest)
        out["roofline_sweep"] = roofline(leg, 3, digest)
    if ref_leg is not None:
        t = min(leg["iterations"], ref_leg["iterations"])
        ref = ref_leg["lb_trace"][t]
        out["bound"] = leg["lb_trace"][t]
        out["certified_bound"] = leg["cert"]
        out["bound_iteration"] = t
        out["rel_err_vs_fp64_gpu"] = abs(leg["lb_trace"][t] - ref) / abs(ref)
        errs = [abs(a - b) / abs(b) for a, b in zip(leg["lb_trace"][: t + 1], ref_leg["lb_trace"][: t + 1])]
        out["rel_err_vs_fp64_gpu_max_over_iterations"] = max(errs)
        out["certified_below_fp64"] = bool(leg["cert"] <= ref)
        out["speedup_vs_fp64_step_launched"] = ref_leg["ms_step"] / leg["ms_step"]
        if leg["ms_graph"] is not None and ref_leg["ms_graph"] is not None:
            out["speedup_vs_fp64_graph_launched"] = ref_leg["ms_graph"] / leg["ms_graph"]
    return out


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus must be 1)",
              file=sys.stderr, flush=True)
        print(json.dumps({"error": "one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)
    import torch

    import qapgen

    N = args.N
    F, D = qapgen.clustered(N, args.seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)
    pair = not args.all_blocks
    digest = csrc_digest()
    # Further iterations as one HIP graph launch each, up to the iteration at
    # which the bound is compared with the oracle.
    extra = max(args.steps, args.bound_iters - args.warmup - args.steps)
    total_iters = args.warmup + args.steps + extra

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    log(f"FP64 N={N}: {args.warmup} warm-up, {args.steps} step-launched, {extra} graph-launched iterations")
    main_leg = timed_leg(F, D, "fp64", pair, args.warmup, args.steps, extra, stream)
    it_s = 1000.0 / main_leg["ms_step"]
    lb_trace = main_leg["lb_trace"]

    legs = {}
    for prec, key, skip in (("fp32", "fp32_certified", args.no_fp32), ("fp32n", "fp32_nearest", args.no_fp32)):
        if skip:
            continue
        log(f"{prec} N={N}")
        leg = timed_leg(F, D, prec, pair, args.warmup, args.steps, extra, stream)
        legs[key] = leg_summary(leg, digest, ref_leg=main_leg)

    rel_err = rel_err_max = None
    gold = os.path.join(ROOT, "tests", "golden", f"clustered{N}_seed{args.seed}_oracle_lb.json")
    if os.path.exists(gold):
        ref = json.load(open(gold))["lb"]
        m = min(len(ref), len(lb_trace))
        errs = [abs(lb_trace[t] - ref[t]) / abs(ref[t]) for t in range(m)]
        rel_err_max = max(errs)
        if total_iters < m:
            rel_err = errs[total_iters]
            for key in ("fp32_certified", "fp32_nearest"):
                if key in legs:
                    legs[key]["rel_err_vs_oracle"] = abs(legs[key]["bound"] - ref[total_iters]) / abs(ref[total_iters])

    main_sum = leg_summary(main_leg, digest)
    out = {
        "metric": "RLT2 dual-ascent iters/s and LAPs/s at N=25; bound rel. error vs FP64",
        "value": it_s,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"clustered QAP N={N} seed {args.seed} (3-5 Gaussian clusters, "
                               f"70% sparse heavy-tailed flows), plain FP64 RLT2 dual ascent",
                   "N": N, "laps_per_iteration": laps_per_iteration(N, pair), "D_entries": sizes(N, pair)[1],
                   "D_blocks": "one stored and concentrated per complementary pair" if pair
                   else "all stored and concentrated",
                   "parallelism": "single GPU"},
        "laps_per_s": main_sum["laps_per_s"],
        "bound": lb_trace[total_iters],
        "bound_rel_err_vs_oracle": rel_err,
        "bound_rel_err_vs_oracle_max_over_iterations": rel_err_max,
        "bound_iteration": total_iters,
        "graph_iters_per_s": main_sum["graph_iters_per_s"],
        "graph_laps_per_s": main_sum["graph_laps_per_s"],
        "iteration_hbm_fraction": main_sum["iteration_hbm_fraction"],
        "kernel_ms": main_sum["kernel_ms"],
        "roofline": main_sum["roofline"],
        # The cost sweep (steps 1-3) against the same peak: the step that
        # moves the whole cost array and is bound by HBM.
        "roofline_sweep": main_sum["roofline_sweep"],
    }
    out.update(legs)
    if pair and not args.no_all_blocks:
        log(f"FP64 N={N}, every block stored and concentrated")
        leg = timed_leg(F, D, "fp64", False, args.warmup, args.steps, 0, stream)
        s = leg_summary(leg, digest, with_rooflines=False)
        s["laps_per_iteration"] = laps_per_iteration(N, False)
        s["bound_matches_pair_path"] = bool(leg["lb_trace"][args.warmup + args.steps] ==
                                            lb_trace[args.warmup + args.steps])
        out["all_blocks"] = s
    if not args.no_solvers:
        log(f"assignment solvers on the N={N} blocks; FP64 dual ascent with the auction solver")
        sl = solver_leg(F, D, stream)
        leg = timed_leg(F, D, "fp64", pair, args.warmup, args.steps, extra, stream, lap_solver="auction")
        sl["dual_ascent"] = leg_summary(leg, digest, ref_leg=main_leg, with_rooflines=False)
        if rel_err is not None:
            ref = json.load(open(gold))["lb"]
            sl["dual_ascent"]["bound_rel_to_oracle_canonical"] = leg["lb_trace"][total_iters] / ref[total_iters]
        out["lap_solvers"] = sl
    if not args.no_large:
        F40, D40 = qapgen.clustered(40, 0)
        large = {"workload": "clustered QAP N=40 seed 0, 20 iterations (1 warm-up, 19 step-launched)",
                 "laps_per_iteration": laps_per_iteration(40, True)}
        ref40 = None
        for prec, key in (("fp64", "fp64"), ("fp32", "fp32_certified")):
            log(f"{prec} N=40")
            leg = timed_leg(F40, D40, prec, True, 1, 19, 0, stream)
            large[key] = leg_summary(leg, digest, ref_leg=ref40)
            if prec == "fp64":
                ref40 = leg
                large[key]["bound"] = leg["lb_trace"][20]
        out["large_N40"] = large
    if not args.no_batched:
        log("batched branch-and-bound nodes")
        out["batched"] = batched_leg(stream)
    if not args.no_cpu_baseline:
        log("oracle on the host")
        cb = cpu_baseline(F, D, args.cpu_iters)
        out["cpu_baseline"] = {
            "value": cb["all_cores"]["iters_per_s"], "unit": "iters/s", "cores": cb["all_cores"]["threads"],
            "kind": "oracle",
            "sample": f"{cb['all_cores']['iterations']} iterations (after iteration 0 and one untimed iteration) "
                      f"of the same N={N} instance, FP64, on every core of the affinity set; single-threaded: "
                      f"{cb['single_thread']['iterations']} iterations",
            "single_thread_iters_per_s": cb["single_thread"]["iters_per_s"],
            "model": cb["model"], "affinity_cores": cb["affinity_cores"],
            "gpu_speedup_vs_all_cores": it_s / cb["all_cores"]["iters_per_s"],
            "gpu_speedup_vs_single_thread": it_s / cb["single_thread"]["iters_per_s"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
