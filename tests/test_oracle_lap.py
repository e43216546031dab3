"""Pins of the oracle's assignment solver and canonical dual (CPU only).

Cost concentration solves a linear assignment problem per block (Section 4.1
of the paper).  The optimal value is pinned by enumeration and by SciPy's
solver; the canonical dual (the reading that makes the residual unique) is
pinned by its defining properties and by an independent LP solve.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment, linprog

import oracle
import qapgen
from oracle import brute

KINDS = ["uniform", "ties", "int", "product", "zero"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_lap_value_matches_enumeration(n, kind):
    for seed in range(4):
        M = qapgen.random_matrix(n, seed, kind)
        val, r2c = oracle.lap_solve(M)
        assert sorted(r2c.tolist()) == list(range(n))
        assert val == pytest.approx(brute.lap_brute(M), rel=1e-12, abs=1e-12)
        assert val == pytest.approx(float(M[np.arange(n), r2c].sum()), rel=1e-15, abs=0)


@pytest.mark.parametrize("n", [8, 13, 23, 24, 25, 38, 40, 64])
def test_lap_value_matches_scipy(n):
    for seed, kind in itertools.product(range(3), ["uniform", "ties", "int"]):
        M = qapgen.random_matrix(n, seed, kind)
        val, _ = oracle.lap_solve(M)
        r, c = linear_sum_assignment(M)
        assert val == pytest.approx(float(M[r, c].sum()), rel=1e-12, abs=1e-9)


def test_lap_product_matrix_rearrangement():
    # M_rq = a_r b_q: the minimum pairs ascending a with descending b.
    rng = np.random.default_rng(7)
    for n in (5, 11, 23):
        a = rng.integers(0, 50, n).astype(float)
        b = rng.integers(0, 50, n).astype(float)
        closed = float(np.dot(np.sort(a), np.sort(b)[::-1]))
        val, _ = oracle.lap_solve(np.outer(a, b))
        assert val == closed


def _w_col(M, r2c):
    """Column-graph arc weights w(c, q) = M[s,q] - M[s,c], s = sigma^-1(c)."""
    n = M.shape[0]
    c2r = np.empty(n, dtype=int)
    c2r[r2c] = np.arange(n)
    return np.array([[M[c2r[c], q] - M[c2r[c], c] for q in range(n)] for c in range(n)])


def _check_canonical(M, uc, vc, ur, vr, S, tol):
    n = M.shape[0]
    for u, v in ((uc, vc), (ur, vr)):
        assert (u[:, None] + v[None, :] <= M + tol).all(), "dual infeasible"
        assert u.sum() + v.sum() == pytest.approx(S, rel=1e-12, abs=tol)
    assert vc.max() == 0.0
    assert ur.max() == 0.0
    # Maximality of vc: each vc_q is either 0 or held down by a tight
    # constraint u_r + v_q = M_rq with the row dual u_r at its largest.
    for q in range(n):
        if vc[q] < 0:
            assert np.min(M[:, q] - uc - vc[q]) <= tol
    for r in range(n):
        if ur[r] < 0:
            assert np.min(M[r, :] - vr - ur[r]) <= tol


@pytest.mark.parametrize("kind", ["uniform", "ties", "int", "product"])
@pytest.mark.parametrize("n", [2, 3, 5, 8, 23])
def test_canonical_dual_definition(n, kind):
    for seed in range(3):
        M = qapgen.random_matrix(n, seed, kind)
        S, r2c = oracle.lap_solve(M)
        uc, vc, ur, vr = oracle.lap_canonical_dual(M, r2c)
        _check_canonical(M, uc, vc, ur, vr, S, tol=1e-9 * max(1.0, abs(M).max()))


def _lp_greatest_v(M, S):
    """Greatest v <= 0 on the optimal dual face, by maximising sum(v) with an
    LP (HiGHS): variables [u, v], u_r + v_q <= M_rq, sum u + sum v = S."""
    n = M.shape[0]
    A = np.zeros((n * n, 2 * n))
    b = np.zeros(n * n)
    for r in range(n):
        for q in range(n):
            A[r * n + q, r] = 1.0
            A[r * n + q, n + q] = 1.0
            b[r * n + q] = M[r, q]
    cost = np.concatenate([np.zeros(n), -np.ones(n)])
    bounds = [(None, None)] * n + [(None, 0.0)] * n
    res = linprog(cost, A_ub=A, b_ub=b, A_eq=np.ones((1, 2 * n)), b_eq=[S],
                  bounds=bounds, method="highs")
    assert res.status == 0
    return res.x[n:]


@pytest.mark.parametrize("kind", ["uniform", "ties", "int"])
@pytest.mark.parametrize("n", [2, 3, 4, 6])
def test_canonical_dual_matches_lp(n, kind):
    for seed in range(3):
        M = qapgen.random_matrix(n, seed, kind)
        S, r2c = oracle.lap_solve(M)
        uc, vc, ur, vr = oracle.lap_canonical_dual(M, r2c)
        np.testing.assert_allclose(vc, _lp_greatest_v(M, S), atol=1e-7)
        # The row point is the column point of the transpose.
        np.testing.assert_allclose(ur, _lp_greatest_v(M.T.copy(), S), atol=1e-7)


def test_canonical_dual_independent_of_optimal_assignment():
    # Tie-heavy matrices have many optimal assignments; every one of them
    # must give the same canonical dual.
    rng = np.random.default_rng(3)
    checked = 0
    for trial in range(40):
        n = 5
        M = rng.integers(0, 3, size=(n, n)).astype(float)
        best = brute.lap_brute(M)
        opts = [np.array(p) for p in itertools.permutations(range(n))
                if M[np.arange(n), list(p)].sum() == best]
        if len(opts) < 2:
            continue
        ref = oracle.lap_canonical_dual(M, opts[0].astype(np.int32))
        for p in opts[1:]:
            got = oracle.lap_canonical_dual(M, p.astype(np.int32))
            for a, b in zip(ref, got):
                np.testing.assert_array_equal(a, b)
        checked += 1
    assert checked >= 10


@pytest.mark.parametrize("kind", ["uniform", "ties", "int", "product"])
@pytest.mark.parametrize("n", [1, 3, 6, 14, 23])
def test_concentrate_properties(n, kind):
    rng = np.random.default_rng(11)
    for seed in range(3):
        M = qapgen.random_matrix(n, seed, kind)
        S, R, duals, r2c = oracle.lap_concentrate(M)
        opt, _ = oracle.lap_solve(M)
        scale = max(1.0, abs(M).max()) * n
        assert S == pytest.approx(opt, rel=1e-12, abs=1e-12 * scale)
        assert (R >= 0).all()
        # Conservation: for every assignment tau, sum M_tau = S + sum R_tau.
        for _ in range(10):
            tau = rng.permutation(n)
            lhs = float(M[np.arange(n), tau].sum())
            rhs = S + float(R[np.arange(n), tau].sum())
            assert rhs == pytest.approx(lhs, rel=1e-12, abs=1e-12 * scale)
        # The optimal assignment is fully reduced.
        assert float(R[np.arange(n), r2c].sum()) <= 1e-12 * scale


@pytest.mark.parametrize("n", [4, 7, 23])
def test_concentrate_transpose_and_relabel(n):
    rng = np.random.default_rng(5)
    for kind in ("uniform", "ties", "int"):
        M = qapgen.random_matrix(n, 2, kind)
        S, R, _, _ = oracle.lap_concentrate(M)
        St, Rt, _, _ = oracle.lap_concentrate(M.T.copy())
        assert St == pytest.approx(S, rel=1e-13, abs=1e-12)
        np.testing.assert_allclose(Rt, R.T, rtol=1e-12, atol=1e-12 * abs(M).max())
        P = rng.permutation(n)
        Q = rng.permutation(n)
        Sp, Rp, _, _ = oracle.lap_concentrate(M[np.ix_(P, Q)])
        assert Sp == pytest.approx(S, rel=1e-13, abs=1e-12)
        np.testing.assert_allclose(Rp, R[np.ix_(P, Q)], rtol=1e-12,
                                   atol=1e-12 * abs(M).max())


def test_concentrate_continuity_at_ties():
    # A tiny perturbation that breaks a tie moves the residual only a little.
    M = qapgen.random_matrix(6, 1, "ties")
    _, R0, _, _ = oracle.lap_concentrate(M)
    rng = np.random.default_rng(0)
    for _ in range(5):
        E = rng.uniform(-1e-7, 1e-7, size=M.shape)
        _, R1, _, _ = oracle.lap_concentrate(M + E)
        assert np.abs(R1 - R0).max() < 1e-5
