"""Pins of the oracle's RLT2 dual ascent (CPU only).

What fixes the answer here is mathematics, not another implementation:
* iteration 0 equals the Gilmore-Lawler bound computed by sorting;
* every step preserves the objective of every permutation (the dual state
  represents the same QAP; Sections 3-4 of the paper);
* reduced costs stay non-negative, LB is non-decreasing and never exceeds the
  brute-force optimum;
* the complementary structure (equations (10)-(11)) under the equal-split
  transfer makes complementary D blocks identical;
* special instances whose bound is known in closed form;
* relabelling and the flow/distance swap leave the trajectory unchanged.
"""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import oracle
import qapgen
from oracle import brute


def _scipy_lap(M):
    r, c = linear_sum_assignment(M)
    return float(M[r, c].sum())


def _trajectory(F, D, T):
    o = oracle.Rlt2Oracle(F, D)
    o.iteration0()
    lbs = [o.lb]
    for _ in range(T):
        o.iterate(1)
        lbs.append(o.lb)
    return np.array(lbs), o


@pytest.mark.parametrize("seed", range(10))
def test_iteration0_is_gilmore_lawler_small(seed):
    F, D = qapgen.small(8, seed)
    o = oracle.Rlt2Oracle(F, D)
    o.iteration0()
    assert o.lb == brute.gilmore_lawler(F, D)


@pytest.mark.parametrize("maker,N", [(qapgen.uniform, 16), (qapgen.clustered, 25)])
def test_iteration0_is_gilmore_lawler_large(maker, N):
    F, D = maker(N, 0)
    o = oracle.Rlt2Oracle(F, D)
    o.iteration0()
    assert o.lb == brute.gilmore_lawler(F, D, lap=_scipy_lap)


def test_iteration0_asymmetric_with_linear_costs():
    rng = np.random.default_rng(4)
    N = 7
    F = rng.integers(0, 10, (N, N)).astype(float)
    D = rng.integers(0, 10, (N, N)).astype(float)
    B0 = rng.integers(0, 20, (N, N)).astype(float)
    o = oracle.Rlt2Oracle(F, D, B0=B0, constant=3.0)
    o.iteration0()
    assert o.lb == 3.0 + brute.gilmore_lawler(F, D, B0=B0)


@pytest.mark.parametrize("seed", range(10))
def test_small_invariants_every_step(seed):
    F, D = qapgen.small(8, seed)
    opt, popt = brute.qap_brute(F, D)
    o = oracle.Rlt2Oracle(F, D)
    o.iteration0()
    rng = np.random.default_rng(100 + seed)
    perms = [rng.permutation(8) for _ in range(12)] + [popt]
    objs = [brute.qap_objective(F, D, p) for p in perms]

    def identity_error(in_transit):
        return max(abs(brute.represented_objective(o.lb + in_transit, o.B, o.C, o.D, p) - v)
                   for p, v in zip(perms, objs))

    assert identity_error(0.0) <= 1e-9 * opt
    prev = o.lb
    for t in range(5):
        for s in range(1, 9):
            o.step(s)
            assert identity_error(o.lbprime if s == 7 else 0.0) <= 1e-9 * opt, (t, s)
            assert o.B.min() >= 0 and o.C.min() >= 0 and o.D.min() >= 0, (t, s)
        assert o.lbprime >= -1e-12 * opt
        assert o.lb >= prev
        assert o.lb <= opt * (1 + 1e-12)
        prev = o.lb


def _group_members(N, i, j, k, n, p, q):
    P = [(i, j), (k, n), (p, q)]
    order = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    return [P[a] + P[b] + P[c] for a, b, c in order]


def test_complementary_structure():
    F, D = qapgen.small(8, 3)
    N = 8
    o = oracle.Rlt2Oracle(F, D)
    o.iteration0()
    o.iterate(1)
    for s in (1, 2, 3):
        o.step(s)
    Dd = o.D.copy()
    rng = np.random.default_rng(0)
    for _ in range(200):
        fac = rng.choice(N, 3, replace=False)
        loc = rng.choice(N, 3, replace=False)
        vals = [Dd[m] for m in _group_members(N, fac[0], loc[0], fac[1], loc[1], fac[2], loc[2])]
        assert len(set(vals)) == 1
    o.step(4)
    SD = o.SD.copy()
    # Complementary blocks D_ijkn and D_knij are identical after the transfer,
    # so they move identical values.
    np.testing.assert_array_equal(SD, SD.transpose(2, 3, 0, 1))
    C_before = o.C.copy()
    o.step(5)
    np.testing.assert_array_equal(o.C, C_before)


def test_three_facilities_reach_the_optimum():
    # N=3: D blocks are 1x1, so after one loop LB is the exact optimum.
    rng = np.random.default_rng(9)
    for _ in range(20):
        F = rng.integers(0, 10, (3, 3)).astype(float)
        D = rng.integers(0, 10, (3, 3)).astype(float)
        np.fill_diagonal(F, 0)
        np.fill_diagonal(D, 0)
        opt, _ = brute.qap_brute(F, D)
        lbs, _ = _trajectory(F, D, 1)
        assert lbs[1] == pytest.approx(opt, rel=1e-12, abs=1e-12)


def test_constant_flow_instance():
    # F = J - I: every permutation costs sum(D), so LB0 is the optimum and no
    # later iteration can add anything.
    F = np.ones((7, 7)) - np.eye(7)
    _, D = qapgen.small(7, 2)
    lbs, _ = _trajectory(F, D, 3)
    assert lbs[0] == D.sum()
    np.testing.assert_allclose(lbs, D.sum(), rtol=1e-12)


def test_zero_flow_instance():
    F = np.zeros((6, 6))
    _, D = qapgen.small(6, 1)
    lbs, o = _trajectory(F, D, 3)
    assert (lbs == 0).all()
    assert o.D.max() == 0 and o.C.max() == 0


@pytest.mark.parametrize("seed", [0, 4])
def test_relabel_invariance(seed):
    F, D = qapgen.small(8, seed)
    rng = np.random.default_rng(seed)
    P = rng.permutation(8)
    Q = rng.permutation(8)
    a, _ = _trajectory(F, D, 4)
    b, _ = _trajectory(F[np.ix_(P, P)], D[np.ix_(Q, Q)], 4)
    np.testing.assert_allclose(a, b, rtol=1e-12)


@pytest.mark.parametrize("seed", [1, 5])
def test_flow_distance_swap_invariance(seed):
    F, D = qapgen.small(8, seed)
    a, _ = _trajectory(F, D, 4)
    b, _ = _trajectory(D, F, 4)
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_uniform16_few_iterations_invariants():
    F, D = qapgen.uniform(16, 0)
    lbs, o = _trajectory(F, D, 3)
    assert (np.diff(lbs) >= 0).all()
    assert o.D.min() >= 0 and o.C.min() >= 0 and o.B.min() >= 0
    rng = np.random.default_rng(1)
    for _ in range(5):
        p = rng.permutation(16)
        rep = brute.represented_objective(o.lb, o.B, o.C, o.D, p)
        obj = brute.qap_objective(F, D, p)
        assert rep == pytest.approx(obj, rel=1e-9)
