"""GPU parity of the RLT2 dual ascent (qap_rlt2_*) against the FP64 oracle.

Every test runs the library and the oracle on the same seeded instance and
compares, per iteration, the bound LB, LB', every value moved by the D->C and
C->B concentrations, and the reduced-cost state.  FP64 tolerance: 1e-9
relative to max(|y|, mean |y| of the family).
"""
import numpy as np
import pytest

import oracle
import qapgen
from oracle import brute
from paper_1510_02065_amd import QapError, Rlt2
from tests import layout

pytestmark = pytest.mark.gpu
TOL = 1e-9


def _compare_iteration(g, o, it, tol=TOL, full_state=True, rng=None):
    N = o.N
    lb_g, _ = g.bound()
    assert lb_g == pytest.approx(o.lb, rel=tol), f"LB at iteration {it}"
    sD, sC, sB = g.lap_values()
    if it > 0:
        ok, err = layout.close_family(sD, layout.compact_C(o.SD), tol)
        assert ok, f"D->C values at iteration {it}: rel err {err}"
    ok, err = layout.close_family(sC, o.SC.ravel(), tol)
    assert ok, f"C->B values at iteration {it}: rel err {err}"
    assert sB == pytest.approx(o.lbprime, rel=tol, abs=tol * max(1.0, abs(o.lb)))
    _, B, C, D = g.read_state(want_D=True)
    assert B.min() >= 0 and C.min() >= 0 and D.min() >= 0
    ok, err = layout.close_family(B, o.B.ravel(), tol)
    assert ok, f"B at iteration {it}: {err}"
    ok, err = layout.close_family(C, layout.compact_C(o.C), tol)
    assert ok, f"C at iteration {it}: {err}"
    if full_state:
        ok, err = layout.close_family(D, layout.compact_D_full(o.D), tol)
    else:
        pos, vals = layout.compact_D_sample(o.D, rng, 20000)
        ok, err = layout.close_family(D[pos], vals, tol)
    assert ok, f"D at iteration {it}: {err}"


@pytest.mark.parametrize("seed", range(10))
def test_small_parity_every_iteration(seed):
    F, D = qapgen.small(8, seed)
    print(f"small N=8 seed={seed}", flush=True)
    g = Rlt2(F, D, trace_level=2)
    o = oracle.Rlt2Oracle(F, D)
    o.iteration0()
    _compare_iteration(g, o, 0)
    opt, _ = brute.qap_brute(F, D)
    for it in range(1, 6):
        g.ascend(1)
        o.iterate(1)
        _compare_iteration(g, o, it)
        assert g.bound()[0] <= opt * (1 + 1e-12)
    lb, lbp = g.trace()
    assert len(lb) == 6 and (np.diff(lb) >= 0).all()
    g.close()


def test_sweep_is_bitwise_equal_to_oracle_steps_1_to_3():
    # With integer data every dual of iteration 0 is an integer or half
    # integer, so both states agree bit for bit after iteration 0.  Steps 1-3
    # then perform the same IEEE operations in the same order on both sides.
    F, D = qapgen.small(8, 2)
    g = Rlt2(F, D, trace_level=2)
    o = oracle.Rlt2Oracle(F, D)
    o.iteration0()
    _, B, C, _ = g.read_state()
    np.testing.assert_array_equal(B, o.B.ravel())
    np.testing.assert_array_equal(C, layout.compact_C(o.C))
    g.step(3)
    for s in (1, 2, 3):
        o.step(s)
    _, B, C, Dg = g.read_state()
    np.testing.assert_array_equal(Dg, layout.compact_D_full(o.D))
    assert (B == 0).all() and (C == 0).all()


def test_uniform16_fifty_iterations():
    F, D = qapgen.uniform(16, 0)
    print("uniform N=16 seed=0 50 iterations", flush=True)
    g = Rlt2(F, D, trace_level=2)
    o = oracle.Rlt2Oracle(F, D)
    o.iteration0()
    _compare_iteration(g, o, 0, full_state=False, rng=np.random.default_rng(0))
    rng = np.random.default_rng(1)
    for it in range(1, 51):
        g.ascend(1)
        o.iterate(1)
        lb_g, _ = g.bound()
        assert lb_g == pytest.approx(o.lb, rel=TOL), f"LB at iteration {it}"
        sD, sC, sB = g.lap_values()
        ok, err = layout.close_family(sD, layout.compact_C(o.SD), TOL)
        assert ok, f"D->C values at iteration {it}: {err}"
        ok, err = layout.close_family(sC, o.SC.ravel(), TOL)
        assert ok, f"C->B values at iteration {it}: {err}"
        if it % 10 == 0:
            _compare_iteration(g, o, it, full_state=False, rng=rng)
    g.close()


def test_clustered25_bench_size_parity():
    # The benchmark's workload (N=25, clustered), in its launch configuration
    # (HIP-graph replay): full per-LAP parity for 3 iterations, sampled state.
    F, D = qapgen.clustered(25, 0)
    print("clustered N=25 seed=0", flush=True)
    g = Rlt2(F, D, trace_level=2, use_graph=True)
    o = oracle.Rlt2Oracle(F, D)
    o.iteration0()
    rng = np.random.default_rng(2)
    _compare_iteration(g, o, 0, full_state=False, rng=rng)
    for it in range(1, 4):
        g.ascend(1)
        o.iterate(1)
        _compare_iteration(g, o, it, full_state=False, rng=rng)
    g.close()


def test_three_facilities_exact():
    rng = np.random.default_rng(3)
    for _ in range(5):
        F = rng.integers(0, 10, (3, 3)).astype(float)
        Dm = rng.integers(0, 10, (3, 3)).astype(float)
        np.fill_diagonal(F, 0)
        np.fill_diagonal(Dm, 0)
        opt, _ = brute.qap_brute(F, Dm)
        g = Rlt2(F, Dm)
        assert g.ascend(1) == pytest.approx(opt, rel=1e-12, abs=1e-12)
        g.close()


def test_linear_costs_and_constant():
    rng = np.random.default_rng(5)
    N = 7
    F = rng.integers(0, 10, (N, N)).astype(float)
    Dm = rng.integers(0, 10, (N, N)).astype(float)
    B0 = rng.integers(0, 20, (N, N)).astype(float)
    g = Rlt2(F, Dm, B0=B0, constant=11.0, trace_level=2)
    o = oracle.Rlt2Oracle(F, Dm, B0=B0, constant=11.0)
    o.iteration0()
    _compare_iteration(g, o, 0)
    for it in range(1, 4):
        g.ascend(1)
        o.iterate(1)
        _compare_iteration(g, o, it)


def test_determinism_and_graph_equivalence():
    F, D = qapgen.uniform(16, 1)
    runs = []
    for use_graph in (True, True, False):
        g = Rlt2(F, D, use_graph=use_graph)
        g.ascend(5)
        runs.append((g.trace()[0], g.read_state()[3]))
        g.close()
    for lb, Dst in runs[1:]:
        np.testing.assert_array_equal(lb, runs[0][0])
        np.testing.assert_array_equal(Dst, runs[0][1])


def test_step_by_step_equals_ascend():
    F, D = qapgen.small(8, 7)
    a = Rlt2(F, D)
    a.ascend(2)
    b = Rlt2(F, D)
    for _ in range(2):
        for s in (3, 4, 5, 6, 7):
            b.step(s)
    assert a.bound() == b.bound()
    np.testing.assert_array_equal(a.read_state()[3], b.read_state()[3])


def test_errors():
    F, D = qapgen.small(8, 0)
    with pytest.raises(QapError):
        Rlt2(F[:2, :2], D[:2, :2])
    bad = F.copy()
    bad[0, 1] = np.nan
    with pytest.raises(QapError):
        Rlt2(bad, D)
    g = Rlt2(F, D)
    with pytest.raises(QapError):
        g.step(1)
    with pytest.raises(QapError):
        g.ascend(-1)
    with pytest.raises(QapError):
        g.lap_values()   # needs trace_level 2
    assert g.ascend(0) == g.bound()[0]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_slot_configurations_agree_bitwise(tmp_path, precision):
    # Every (lanes per problem, columns per lane) configuration makes the same
    # decisions and sums in the same order, so the autotuner's choice never
    # changes a bit of the state.  The tune cache forces each configuration
    # on the D and C families (n = 11 and 12 at N = 13).
    F, D = qapgen.clustered(13, 2)
    prec = {"fp64": 0, "fp32": 1}[precision]
    ref = None
    for seg, k in [(8, 2), (8, 3), (16, 1), (16, 2), (32, 1), (64, 1)]:
        cache = tmp_path / f"tune_{seg}_{k}.txt"
        cache.write_text(f"gfx950 prec={prec} fam=0 seg=16 nmax=11|{seg} {k}\n"
                         f"gfx950 prec={prec} fam=1 seg=16 nmax=12|{seg} {k}\n")
        print(f"configuration SEG={seg} K={k} {precision}", flush=True)
        h = Rlt2(F, D, precision=precision, trace_level=2, tune_cache=cache)
        h.ascend(4)
        got = (h.trace()[0], *h.read_state()[1:], *h.lap_values()[:2])
        h.close()
        if ref is None:
            ref = got
        else:
            for x, y in zip(got, ref):
                np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32n"])
def test_slot_configurations_agree_bitwise_n23(tmp_path, precision):
    # The benchmark's size: n = 23 (D family) and 24 (C family) in the
    # 32-lane bucket, forced to one column per lane on 32 lanes, two columns
    # per lane on 16 lanes (several problems' free rows in one loop) and three
    # columns per lane on 8 lanes (one free row at a time).
    F, D = qapgen.clustered(25, 0)
    prec = {"fp64": 0, "fp32": 1, "fp32n": 2}[precision]
    ref = None
    for seg, k in [(32, 1), (16, 2), (8, 3), (32, 2)]:
        cache = tmp_path / f"tune25_{seg}_{k}.txt"
        cache.write_text(f"gfx950 prec={prec} fam=0 seg=32 nmax=23|{seg} {k}\n"
                         f"gfx950 prec={prec} fam=1 seg=32 nmax=24|{seg} {k}\n")
        print(f"configuration SEG={seg} K={k} {precision} N=25", flush=True)
        h = Rlt2(F, D, precision=precision, trace_level=2, tune_cache=cache)
        h.ascend(3)
        got = (h.trace()[0], *h.read_state()[1:], *h.lap_values()[:2])
        h.close()
        if ref is None:
            ref = got
        else:
            for x, y in zip(got, ref):
                np.testing.assert_array_equal(x, y)


# ---- closed forms and symmetries on the GPU (no oracle involved) -------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32n"])
def test_closed_forms_flow_all_ones_and_zero(precision):
    # F = J - I: every permutation costs the sum of D's off-diagonal entries,
    # so LB_0 is the optimum and no iteration moves anything (LB' = 0).
    # F = 0: every bound is 0.
    N = 9
    _, Dm = qapgen.small(N, 4)
    F = np.ones((N, N)) - np.eye(N)
    total = Dm.sum()
    g = Rlt2(F, Dm, precision=precision)
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert g.bound()[0] == pytest.approx(total, rel=tol)
    g.ascend(4)
    lb, lbp = g.trace()
    assert np.abs(lb - total).max() <= tol * total
    assert np.abs(lbp[1:]).max() <= tol * total
    if precision == "fp32":
        assert (lb <= total).all()
    g.close()
    z = Rlt2(np.zeros((N, N)), Dm, precision=precision)
    z.ascend(3)
    assert (z.trace()[0] == 0.0).all()
    z.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32n"])
def test_relabel_and_flow_distance_swap_invariance(precision):
    # The canonical dual is equivariant under relabelling rows and columns and
    # transpose-symmetric, so relabelling facilities and locations, and
    # swapping F and D (the QAP of the inverse permutation), leave the whole
    # bound trajectory unchanged up to rounding.
    F, Dm = qapgen.uniform(12, 5)
    rng = np.random.default_rng(9)
    P = rng.permutation(12)
    Q = rng.permutation(12)
    runs = [(F, Dm), (F[np.ix_(P, P)], Dm[np.ix_(Q, Q)]), (Dm, F)]
    trajs = []
    for Fx, Dx in runs:
        g = Rlt2(Fx, Dx, precision=precision)
        g.ascend(8)
        trajs.append(g.trace()[0])
        g.close()
    tol = 1e-12 if precision == "fp64" else 1e-5
    for t in trajs[1:]:
        np.testing.assert_allclose(t, trajs[0], rtol=tol)
