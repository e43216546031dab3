"""Write oracle-only expected values used by the GPU tests and the benchmark.

Calls nothing but the CPU oracle (and the seeded generators).  Output:
clustered25_seed0_oracle_lb.json -- LB after iterations 0..100 and LB' of
each, for the clustered N=25 instance, seed 0 (FP64, Algorithm 1 of the
paper with the equal-split transfers and the canonical-dual residuals).

    python tests/golden/make_golden.py [--iters 100]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import qapgen  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--N", type=int, default=25)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args()
    F, D = qapgen.clustered(a.N, a.seed)
    o = oracle.Rlt2Oracle(F, D)
    t = time.time()
    o.iteration0()
    lb, lbp = [o.lb], [o.lbprime]
    for it in range(a.iters):
        o.iterate(1)
        lb.append(o.lb)
        lbp.append(o.lbprime)
        print(f"iteration {it + 1}: LB {o.lb!r} ({time.time() - t:.0f} s)", flush=True)
    out = {"workload": f"clustered N={a.N} seed {a.seed}", "generator": "qapgen.clustered",
           "source": "oracle (FP64 CPU)", "lb": lb, "lbprime": lbp}
    path = os.path.join(HERE, f"clustered{a.N}_seed{a.seed}_oracle_lb.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
