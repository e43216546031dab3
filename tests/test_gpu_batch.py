"""Many instances in one handle: branch-and-bound nodes of different sizes.

* a batch handle gives bit for bit the same trajectory and state as one handle
  per instance (the kernels treat each instance identically; an assignment
  wave that spans two nodes of different sizes runs the solver with per-lane
  sizes, a single instance's waves with a scalar size, so these tests also
  pin the two code paths to each other);
* every node's trajectory matches the FP64 oracle run on that node;
* node bound + node constant never exceeds the brute-force optimum of the
  completion problem;
* the 256-node workload cut from a clustered N=24 instance (N' = 10..22),
  in FP64 and certified FP32.
"""
import numpy as np
import pytest

import oracle
import qapgen
from oracle import brute
from paper_1510_02065_amd import Rlt2, subproblem
from tests import layout

pytestmark = pytest.mark.gpu


def _nodes(parent_N, count, seed, m_lo, m_hi):
    F, D, fixes = qapgen.nodes(count=count, parent_N=parent_N, seed=seed, m_lo=m_lo, m_hi=m_hi)
    return F, D, [subproblem(F, D, fac, loc) for fac, loc in fixes]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_individual_handles_bitwise(precision):
    # Nodes of N' = 6..10: steps 1-3 run one launch per node size.
    _, _, nodes = _nodes(12, 20, 3, 2, 6)
    print(f"batch of 20 nodes {precision}, N' =", sorted({n[0].shape[0] for n in nodes}), flush=True)
    g = Rlt2.batch([n[0] for n in nodes], [n[1] for n in nodes], [n[2] for n in nodes],
                   [n[3] for n in nodes], precision=precision, trace_level=2)
    g.ascend(4)
    lbs = g.bounds()
    for k, (Fs, Ds, Bs, c) in enumerate(nodes):
        h = Rlt2(Fs, Ds, B0=Bs, constant=c, precision=precision, trace_level=2)
        h.ascend(4)
        np.testing.assert_array_equal(h.trace()[0], g.trace_k(k)[0])
        assert h.bound()[0] == lbs[k]
        a = h.read_state()
        b = g.read_state_k(k)
        for x, y in zip(a[1:], b[1:]):
            np.testing.assert_array_equal(x, y)
        h.close()
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_of_large_nodes_equals_individual_handles_bitwise(precision):
    # Nodes of N' = 17..22, one steps 1-3 launch per node size.  In FP64 a CU
    # holds one 1024-thread triple workgroup, so N' >= 20 runs one persistent
    # workgroup per CU and smaller nodes 512-thread workgroups per triple; in
    # FP32 the larger nodes run two 1024-thread workgroups per CU.
    _, _, nodes = _nodes(24, 6, 7, 2, 7)
    print(f"batch of 6 nodes {precision}, N' =", sorted({n[0].shape[0] for n in nodes}), flush=True)
    g = Rlt2.batch([n[0] for n in nodes], [n[1] for n in nodes], [n[2] for n in nodes],
                   [n[3] for n in nodes], precision=precision, trace_level=2)
    g.ascend(2)
    for k, (Fs, Ds, Bs, c) in enumerate(nodes):
        h = Rlt2(Fs, Ds, B0=Bs, constant=c, precision=precision, trace_level=2)
        h.ascend(2)
        np.testing.assert_array_equal(h.trace()[0], g.trace_k(k)[0])
        for x, y in zip(h.lap_values(), g.lap_values_k(k)):
            np.testing.assert_array_equal(x, y)
        h.close()
    g.close()


def test_batch_nodes_match_oracle_and_stay_below_optimum():
    F, D, fixes = qapgen.nodes(count=12, parent_N=11, seed=5, m_lo=3, m_hi=5)
    nodes = [subproblem(F, D, fac, loc) for fac, loc in fixes]
    g = Rlt2.batch([n[0] for n in nodes], [n[1] for n in nodes], [n[2] for n in nodes],
                   [n[3] for n in nodes], trace_level=2)
    T = 4
    g.ascend(T)
    for k, (Fs, Ds, Bs, c) in enumerate(nodes):
        o = oracle.Rlt2Oracle(Fs, Ds, B0=Bs, constant=c)
        o.iteration0()
        o.iterate(T)
        lb, _ = g.trace_k(k)
        assert lb[-1] == pytest.approx(o.lb, rel=1e-9)
        sD, sC, _ = g.lap_values_k(k)
        ok, err = layout.close_family(sD, layout.compact_C(o.SD), 1e-9)
        assert ok, (k, err)
        opt, _ = brute.qap_brute(Fs, Ds, B0=Bs, constant=c)
        assert lb[-1] <= opt * (1 + 1e-12)
    g.close()


def test_c3_nodes_fp64_fp32_and_oracle_sample():
    # 256 nodes cut from one clustered N=24 instance by fixing 2..14
    # assignments: N' = 10..22, 20 iterations.
    _, _, nodes = _nodes(24, 256, 0, 2, 14)
    sizes = np.array([n[0].shape[0] for n in nodes])
    print(f"256 nodes, N' from {sizes.min()} to {sizes.max()}", flush=True)
    args = ([n[0] for n in nodes], [n[1] for n in nodes], [n[2] for n in nodes], [n[3] for n in nodes])
    g = Rlt2.batch(*args, precision="fp64")
    f = Rlt2.batch(*args, precision="fp32")
    T = 20
    g.ascend(T)
    f.ascend(T)
    lb64 = g.bounds()
    lb32, cert = f.bounds(certified=True)
    assert (np.abs(cert - lb64) <= 1e-5 * np.abs(lb64)).all()
    # Oracle on the smallest, a median and the largest node.
    order = np.argsort(sizes, kind="stable")
    for k in (order[0], order[len(order) // 2], order[-1]):
        Fs, Ds, Bs, c = nodes[k]
        print(f"oracle on node {k} (N'={Fs.shape[0]})", flush=True)
        o = oracle.Rlt2Oracle(Fs, Ds, B0=Bs, constant=c)
        o.iteration0()
        lbk, _ = g.trace_k(int(k))
        assert lbk[0] == pytest.approx(o.lb, rel=1e-9)
        for t in range(1, T + 1):
            o.iterate(1)
            assert lbk[t] == pytest.approx(o.lb, rel=1e-9), (k, t)
    # A node of size 10 is small enough for brute force.
    k10 = [k for k in range(len(nodes)) if sizes[k] == 10]
    if k10:
        Fs, Ds, Bs, c = nodes[k10[0]]
        opt, _ = brute.qap_brute(Fs, Ds, B0=Bs, constant=c)
        assert lb64[k10[0]] <= opt * (1 + 1e-12)
        assert cert[k10[0]] <= opt
    g.close()
    f.close()


@pytest.mark.parametrize("precision,use_graph", [("fp64", True), ("fp32", True), ("fp64", False)])
def test_overlapped_schedule_equals_sequential_bitwise(precision, use_graph):
    # Mixed sizes: with overlap each size's D->C concentration runs on a
    # second stream beside the next size's sweep; the state, the traces and
    # every per-LAP value must be those of the one-step-after-another run.
    _, _, nodes = _nodes(20, 24, 11, 2, 9)
    print(f"overlap vs sequential, {precision}, graph={use_graph}, N' =",
          sorted({n[0].shape[0] for n in nodes}), flush=True)
    args = ([n[0] for n in nodes], [n[1] for n in nodes], [n[2] for n in nodes], [n[3] for n in nodes])
    a = Rlt2.batch(*args, precision=precision, trace_level=2, use_graph=use_graph, overlap=True)
    b = Rlt2.batch(*args, precision=precision, trace_level=2, use_graph=use_graph, overlap=False)
    a.ascend(5)
    b.ascend(5)
    np.testing.assert_array_equal(a.bounds(), b.bounds())
    for k in range(len(nodes)):
        np.testing.assert_array_equal(a.trace_k(k)[0], b.trace_k(k)[0])
        for x, y in zip(a.lap_values_k(k), b.lap_values_k(k)):
            np.testing.assert_array_equal(x, y)
        for x, y in zip(a.read_state_k(k)[1:], b.read_state_k(k)[1:]):
            np.testing.assert_array_equal(x, y)
    a.close()
    b.close()
