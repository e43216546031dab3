"""The auction-algorithm concentration (the paper's GPU solver, Section 6) on
the GPU.  Its dual comes from the final prices, so it is not the canonical
point the oracle computes: what is checked is what makes it a valid cost
concentration and a valid bound.

* qap_lap_solve with QAP_LAP_AUCTION: the value is a lower bound on the
  optimum (oracle LAP) within n * 2^-38 max|M| of it; the residual is >= 0
  and conserves every permutation's cost (S + sum R_tau = sum M_tau); the
  assignment is a permutation within that gap of optimal.  In FP32 certified
  mode the conservation holds as an inequality, checked exactly.
* The dual ascent with lap_solver="auction": the bound stays below the
  brute-force optimum and never falls (up to the auction's gap), and the state
  represents every permutation's objective (objective identity), exactly
  below it in certified FP32.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import qapgen
from oracle import brute
from paper_1510_02065_amd import Rlt2, lap_solve
from paper_1510_02065_amd import _binding as B
from tests import layout

pytestmark = pytest.mark.gpu

KINDS = ["uniform", "ties", "int", "product", "zero"]
GAP64 = 2.0 ** -38


def _mats(sizes, seed):
    return [qapgen.random_matrix(int(n), seed * 100 + i, KINDS[i % len(KINDS)]) for i, n in enumerate(sizes)]


@pytest.mark.parametrize("sizes", [[1, 2, 3, 6, 7, 8], [9, 14, 16, 17, 23, 24], [25, 31, 32, 33, 38, 40, 63, 64]])
def test_auction_lap_values_residuals_assignment(sizes):
    mats = _mats(sizes * 3, len(sizes))
    print(f"auction lap_solve sizes {sizes}", flush=True)
    out = lap_solve(mats, residual=True, auction=True)
    rng = np.random.default_rng(3)
    for b, M in enumerate(mats):
        n = M.shape[0]
        S_opt = oracle.lap_solve(M)[0] if n else 0.0
        big = float(np.abs(M).max()) if n else 0.0
        gap = 2 * n * GAP64 * big + 1e-12 * max(big, 1.0) * max(n, 1)
        S = out["value"][b]
        assert S <= S_opt + 1e-12 * max(big, 1.0) * max(n, 1), (b, n, S, S_opt)
        assert S >= S_opt - gap, (b, n, S, S_opt)
        R = out["residual"][b]
        assert (R >= 0).all()
        sig = out["assign"][b]
        assert sorted(sig.tolist()) == list(range(n))
        assert M[np.arange(n), sig].sum() <= S_opt + gap
        for _ in range(4):
            tau = rng.permutation(n)
            lhs = M[np.arange(n), tau].sum()
            assert abs(S + R[np.arange(n), tau].sum() - lhs) <= 1e-12 * max(big, 1.0) * max(n, 1) * 4


def test_auction_lap_fp32_certified_conservation_is_exact_inequality():
    rng = np.random.default_rng(5)
    mats = [qapgen.random_matrix(int(n), i, KINDS[i % 4]).astype(np.float32)
            for i, n in enumerate(rng.integers(1, 40, size=40))]
    batch = len(mats)
    n = np.array([m.shape[0] for m in mats], np.int32)
    mo = np.zeros(batch, np.int64)
    mo[1:] = np.cumsum(n.astype(np.int64) ** 2)[:-1]
    cost = np.concatenate([m.ravel() for m in mats]).astype(np.float32)
    value = np.empty(batch)
    st = B.lib().qap_lap_solve(batch, n.ctypes.data, mo.ctypes.data, None, cost.ctypes.data,
                               B.QAP_FP32_CERTIFIED, value.ctypes.data, None, None,
                               B.QAP_LAP_RESIDUAL | B.QAP_LAP_AUCTION, None)
    assert st == 0
    for b, M in enumerate(mats):
        nb = M.shape[0]
        R = cost[mo[b]: mo[b] + nb * nb].reshape(nb, nb)
        assert (R >= 0).all()
        S_opt = oracle.lap_solve(M.astype(np.float64))[0]
        assert value[b] <= S_opt
        assert value[b] >= S_opt - 2 * nb * 2.0 ** -20 * float(np.abs(M).max()) - 1e-6 * nb
        for _ in range(5):
            tau = rng.permutation(nb)
            lhs = sum(Fraction(float(M[r, tau[r]])) for r in range(nb))
            rhs = Fraction(value[b]) + sum(Fraction(float(R[r, tau[r]])) for r in range(nb))
            assert rhs <= lhs


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_auction_dual_ascent_valid_bound_and_objective_identity(precision, seed):
    F, D = qapgen.small(8, seed)
    print(f"auction dual ascent {precision} N=8 seed {seed}", flush=True)
    opt, _ = brute.qap_brute(F, D)
    g = Rlt2(F, D, precision=precision, lap_solver="auction")
    h = Rlt2(F, D, precision=precision)
    # Iteration 0: both are the Gilmore-Lawler bound, to the auction's gap
    # (n eps per problem: 2^-38 of the entries in FP64, 2^-20 in FP32).
    assert g.bound()[0] == pytest.approx(h.bound()[0], rel=1e-9 if precision == "fp64" else 1e-4)
    if precision == "fp64":
        assert g.bound()[0] <= h.bound()[0] * (1 + 1e-12)   # each auction value <= the LAP optimum
    perms = brute.all_perms(8)[::97]
    slack = 8 * 4 * 2.0 ** (-38 if precision == "fp64" else -20) * float(np.abs(F).max() * np.abs(D).max()) * 64
    for it in range(1, 8):
        lb = g.ascend(1)
        assert lb <= opt + slack, (it, lb, opt)
        lbs, lbp = g.trace()
        assert (np.diff(lbs) >= -slack).all()
        L, Bst, Cst, Dst = g.read_state()
        assert Bst.min() >= 0 and Cst.min() >= 0 and Dst.min() >= 0
        rep = layout.represented(8, L, Bst, Cst, Dst, perms)
        true = np.array([brute.qap_objective(F, D, p) for p in perms])
        if precision == "fp64":
            np.testing.assert_allclose(rep, true, rtol=1e-11)
        else:
            assert (rep <= true * (1 + 1e-12)).all()
    lb_c = h.ascend(7)
    print(f"after 7 iterations: auction LB {lb!r}, canonical LB {lb_c!r}, optimum {opt}", flush=True)
    assert g.certify() <= opt + slack
    g.close()
    h.close()


def test_auction_dual_ascent_clustered16_runs_and_tracks():
    # The auction's trajectory is its own; at N=16 it must stay valid and come
    # within a few per cent of the canonical trajectory's bound.
    F, D = qapgen.uniform(16, 1)
    g = Rlt2(F, D, lap_solver="auction")
    h = Rlt2(F, D)
    a = g.ascend(20)
    c = h.ascend(20)
    print(f"N=16, 20 iterations: auction LB {a!r}, canonical LB {c!r}", flush=True)
    lbs, _ = g.trace()
    assert (np.diff(lbs) >= -1e-9 * lbs[-1]).all()
    assert 0.9 * c <= a <= 1.1 * c
    g.close()
    h.close()
