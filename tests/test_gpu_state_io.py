"""State I/O on the GPU: qap_rlt2_load_state, the FP64 certification cascade
on states with negative entries, and snapshot/restore.

The cascade is checked against a host FP64 computation written here from its
definition (c~ = c + (N-2) min(0, min D_beta), b~ = b + (N-1) min(0, min
C~_ij), LB + N min(0, min b~)), and against brute force: the certified bound
never exceeds the smallest represented objective over all permutations.
"""
import numpy as np
import pytest

import qapgen
from oracle import brute
from paper_1510_02065_amd import QapError, Rlt2
from tests import layout

pytestmark = pytest.mark.gpu
PRECISIONS = ["fp64", "fp32", "fp32n"]


def _host_cascade(N, lb, B, C, D):
    n1, n2 = N - 1, N - 2
    md = np.minimum(0.0, D.reshape(-1, n2 * n2).min(axis=1))
    ct = C + n2 * md
    mc = np.minimum(0.0, ct.reshape(N * N, n1 * n1).min(axis=1))
    bt = B + n1 * mc
    return lb + N * min(0.0, bt.min())


@pytest.mark.parametrize("precision", PRECISIONS)
def test_load_state_round_trip(precision):
    F, D = qapgen.small(8, 3)
    g = Rlt2(F, D, precision=precision)
    g.ascend(2)
    lb, B, C, Dst = g.read_state()
    h = Rlt2(F, D, precision=precision)
    h.load_state(0, lb, B, C, Dst)
    lb2, B2, C2, D2 = h.read_state()
    assert lb2 == lb
    np.testing.assert_array_equal(B2, B)
    np.testing.assert_array_equal(C2, C)
    np.testing.assert_array_equal(D2, Dst)
    # Both continue identically from the same state.
    g.ascend(2)
    h.ascend(2)
    for x, y in zip(g.read_state(), h.read_state()):
        np.testing.assert_array_equal(x, y)
    g.close()
    h.close()


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("complementary", [True, False])
def test_certify_with_negative_entries(precision, complementary):
    F, D = qapgen.small(8, 5)
    N = 8
    print(f"cascade {precision} complementary={complementary}", flush=True)
    g = Rlt2(F, D, precision=precision, complementary=complementary)
    g.ascend(2)
    lb, B, C, Dst = g.read_state()
    rng = np.random.default_rng(11)
    n2 = N - 2
    nblk = N * N * (N - 1) ** 2
    # Plant negative entries: in D blocks (both blocks of a complementary
    # pair, which are stored once), in C and in B; magnitudes chosen so that
    # every level of the cascade contributes.
    Dn = Dst.reshape(nblk, n2 * n2).copy()
    I, J, K, Nn = layout.c_index_arrays(N)
    pos = {(int(I[x]), int(J[x]), int(K[x]), int(Nn[x])): x for x in range(nblk)}
    for beta in rng.choice(nblk, 40, replace=False):
        i, j, k, n = int(I[beta]), int(J[beta]), int(K[beta]), int(Nn[beta])
        twin = pos[(k, n, i, j)]
        e = rng.integers(0, n2 * n2)
        v = -float(rng.uniform(0.5, 20.0))
        Dn[beta, e] = v
        Dn[twin, e] = v
    Cn = C.copy()
    Cn[rng.choice(C.size, 30, replace=False)] -= rng.uniform(50.0, 400.0, 30)
    Bn = B.copy()
    Bn[rng.choice(B.size, 5, replace=False)] -= rng.uniform(100.0, 900.0, 5)
    g.load_state(0, lb, Bn, Cn, Dn.ravel())
    lb2, B2, C2, D2 = g.read_state()   # as stored (FP32 modes rounded once)
    cert = g.certify()
    ref = _host_cascade(N, lb2, B2, C2, D2)
    assert cert < lb2                     # the corrections ran
    assert cert <= ref + 1e-12 * abs(ref)  # directed rounding only lowers it
    assert cert == pytest.approx(ref, rel=1e-12, abs=1e-9)
    # Validity against brute force: every permutation's represented objective
    # is at least the certified bound.
    perms = brute.all_perms(N)
    rep = layout.represented(N, lb2, B2, C2, D2, perms)
    assert cert <= rep.min() + 1e-9 * abs(rep.min())
    g.close()


@pytest.mark.parametrize("complementary", [True, False])
def test_certified_sweep_rounds_down_with_negative_entries(complementary):
    """Steps 1-3 in certified FP32 on a loaded state holding negative entries
    (the six-way means then take the directed path for terms of either sign):
    every member of every six-way group must end at or below the exact mean
    of (member + spread share of its block), computed here in rational
    arithmetic from the stored floats, and within a few FP32 steps of it."""
    from fractions import Fraction
    F, D = qapgen.small(8, 5)
    N, n1, n2 = 8, 7, 6
    g = Rlt2(F, D, precision="fp32", complementary=complementary)
    g.ascend(2)
    lb, B, C, Dst = g.read_state()
    rng = np.random.default_rng(12)
    nblk = N * N * n1 * n1
    I, J, K, Nn = layout.c_index_arrays(N)
    pos = {(int(I[x]), int(J[x]), int(K[x]), int(Nn[x])): x for x in range(nblk)}
    Dn = Dst.reshape(nblk, n2 * n2).copy()
    for beta in rng.choice(nblk, 60, replace=False):
        i, j, k, n = int(I[beta]), int(J[beta]), int(K[beta]), int(Nn[beta])
        e = rng.integers(0, n2 * n2)
        v = -float(rng.uniform(0.5, 40.0))
        Dn[beta, e] = v
        Dn[pos[(k, n, i, j)], e] = v     # the complementary block's same entry
    Cn = C.copy()
    Cn[rng.choice(C.size, 40, replace=False)] -= rng.uniform(5.0, 200.0, 40)
    Bn = B.copy()
    Bn[rng.choice(B.size, 6, replace=False)] -= rng.uniform(50.0, 500.0, 6)
    g.load_state(0, lb, Bn, Cn, Dn.ravel())
    _, B2, C2, D2 = g.read_state()        # the stored floats
    g.step(3)
    _, B3, C3, D3 = g.read_state()
    g.close()
    assert not B3.any() and not C3.any()  # both spread onward and cleared
    D2 = D2.reshape(nblk, n2 * n2)
    D3 = D3.reshape(nblk, n2 * n2)
    assert (D2 < 0).any()

    def beta_of(a, la, b, lb_):
        return ((a * N + la) * n1 + (b - (b > a))) * n1 + (lb_ - (lb_ > la))

    def entry(a, la, b, lb_, c, lc):
        return (c - (c > a) - (c > b)) * n2 + (lc - (lc > la) - (lc > lb_))

    share = {}
    def share_of(bt):
        if bt not in share:
            i, j = int(I[bt]), int(J[bt])
            share[bt] = (Fraction(float(C2[bt])) + Fraction(float(B2[i * N + j])) / n1) / n2
        return share[bt]

    checked = signed = 0
    worst = 0.0
    for f0 in range(N):
        for f1 in range(f0 + 1, N):
            for f2 in range(f1 + 1, N):
                for l0 in range(N):
                    for l1 in range(N):
                        if l1 == l0:
                            continue
                        for l2 in range(N):
                            if l2 == l0 or l2 == l1:
                                continue
                            P = ((f0, l0), (f1, l1), (f2, l2))
                            members = []
                            for a, b, c in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
                                bt = beta_of(P[a][0], P[a][1], P[b][0], P[b][1])
                                e = entry(P[a][0], P[a][1], P[b][0], P[b][1], P[c][0], P[c][1])
                                members.append((bt, e))
                            terms = [Fraction(float(D2[bt, e])) + share_of(bt) for bt, e in members]
                            mean = sum(terms) / 6
                            got = {float(D3[bt, e]) for bt, e in members}
                            assert len(got) == 1, "members of one group differ"
                            v = got.pop()
                            assert Fraction(v) <= mean, (P, v, float(mean))
                            scale = max(abs(float(t)) for t in terms) + abs(float(mean))
                            gap = float(mean - Fraction(v))
                            assert gap <= 4 * 2.0 ** -23 * scale, (P, v, float(mean), gap)
                            worst = max(worst, gap / scale if scale else 0.0)
                            checked += 1
                            signed += any(float(D2[bt, e]) < 0 or share_of(bt) < 0 for bt, e in members)
    print(f"certified sweep: {checked} groups, {signed} with a negative term, worst gap {worst:.2e} of the scale",
          flush=True)
    assert signed > 0


def test_load_state_rejects_bad_input():
    F, D = qapgen.small(8, 0)
    g = Rlt2(F, D)
    lb, B, C, Dst = g.read_state()
    B[3] = np.nan
    with pytest.raises(QapError):
        g.load_state(0, lb, B, None, None)
    with pytest.raises(QapError):
        g.load_state(1, lb, None, None, None)   # one instance only
    g.close()


@pytest.mark.parametrize("precision", PRECISIONS)
def test_snapshot_restore_is_bitwise_continuation(precision):
    F, D = qapgen.uniform(12, 1)
    print(f"snapshot {precision}", flush=True)
    ref = Rlt2(F, D, precision=precision, trace_level=2)
    ref.ascend(7)
    a = Rlt2(F, D, precision=precision, trace_level=2)
    a.ascend(3)
    snap = a.snapshot()
    a.close()   # the run is "killed" after 3 iterations
    b = Rlt2(F, D, precision=precision, trace_level=2)
    b.restore(snap)
    assert b.bound()[1] == 3
    b.ascend(4)
    for x, y in zip(ref.read_state(), b.read_state()):
        np.testing.assert_array_equal(x, y)
    for x, y in zip(ref.trace(), b.trace()):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(ref.lap_values()[0], b.lap_values()[0])
    assert b.bound() == ref.bound()
    ref.close()
    b.close()


def test_snapshot_batch_and_mismatch():
    F, D, fixes = qapgen.nodes(count=6, parent_N=12, seed=3, m_lo=2, m_hi=5)
    from paper_1510_02065_amd import subproblem
    nodes = [subproblem(F, D, fac, loc) for fac, loc in fixes]
    args = ([n[0] for n in nodes], [n[1] for n in nodes], [n[2] for n in nodes], [n[3] for n in nodes])
    ref = Rlt2.batch(*args)
    ref.ascend(5)
    a = Rlt2.batch(*args)
    a.ascend(2)
    snap = a.snapshot()
    b = Rlt2.batch(*args)
    b.restore(snap)
    b.ascend(3)
    np.testing.assert_array_equal(ref.bounds(), b.bounds())
    for k in range(len(nodes)):
        for x, y in zip(ref.read_state_k(k), b.read_state_k(k)):
            np.testing.assert_array_equal(x, y)
    other = Rlt2(*qapgen.small(8, 0))
    with pytest.raises(QapError):
        other.restore(snap)   # different instances
    with pytest.raises(QapError):
        b.restore(snap[:-9])  # truncated
    for h in (ref, a, b, other):
        h.close()
