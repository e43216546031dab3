"""Certified FP32 mode (QAP_FP32_CERTIFIED) on the GPU.

Two kinds of check:
* accuracy: the FP32 trajectory (LB and every per-LAP value) stays within
  1e-5 relative of the FP64 oracle (the long trajectories are in
  test_gpu_trajectory.py);
* certificate: with every FP32 rounding directed toward -inf, the stored state
  never represents more than the true objective.  Checked exactly (rational
  arithmetic) on sampled permutations, and the certified bound is checked
  against brute-force optima.  In the round-to-nearest mode the represented
  objective is checked to stay within 1e-5 of the true one.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import oracle
import qapgen
from oracle import brute
from paper_1510_02065_amd import Rlt2, lap_solve
from paper_1510_02065_amd import _binding as B
from tests import layout

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


def _represented_exact(N, lb, Bst, Cst, Dst, perm):
    """Exact rational value of LB + sum b + sum c + sum d on perm, from the
    compact state arrays."""
    I, J, K, Nn = layout.c_index_arrays(N)
    cpos = {(int(I[x]), int(J[x]), int(K[x]), int(Nn[x])): x for x in range(len(I))}
    n2 = N - 2
    tot = Fraction(lb)
    for i in range(N):
        tot += Fraction(float(Bst[i * N + perm[i]]))
    for i in range(N):
        for k in range(N):
            if k == i:
                continue
            b = cpos[(i, perm[i], k, perm[k])]
            tot += Fraction(float(Cst[b]))
            rows = [p for p in range(N) if p != i and p != k]
            cols = [q for q in range(N) if q != perm[i] and q != perm[k]]
            for r, p in enumerate(rows):
                c = cols.index(perm[p])
                tot += Fraction(float(Dst[b * n2 * n2 + r * n2 + c]))
    return tot


@pytest.mark.parametrize("precision", ["fp32", "fp32n"])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_fp32_small_certificate_and_accuracy(seed, precision):
    # Certified mode: the stored state never represents more than the true
    # objective (checked exactly).  Nearest mode: it differs from the true
    # objective only by accumulated FP32 roundings, far below 1e-5.
    F, D = qapgen.small(8, seed)
    print(f"{precision} small N=8 seed={seed}", flush=True)
    opt, _ = brute.qap_brute(F, D)
    g = Rlt2(F, D, precision=precision, trace_level=2)
    o = oracle.Rlt2Oracle(F, D)
    o.iteration0()
    rng = np.random.default_rng(seed)
    perms = [rng.permutation(8) for _ in range(6)]
    for it in range(1, 6):
        cert = g.ascend(1)
        o.iterate(1)
        # Only the directed-rounding mode is a proof; the nearest mode's
        # bound may exceed a tight optimum by its rounding drift (<= 1e-5).
        assert cert <= (opt if precision == "fp32" else opt * (1 + TOL32)), (it, cert, opt)
        assert abs(cert - o.lb) <= TOL32 * o.lb, (it, cert, o.lb)
        sD, sC, sB = g.lap_values()
        ok, err = layout.close_family(sD, layout.compact_C(o.SD), TOL32)
        assert ok, (it, err)
        lb, Bst, Cst, Dst = g.read_state()
        assert Bst.min() >= 0 and Cst.min() >= 0 and Dst.min() >= 0
        for p in perms:
            rep = _represented_exact(8, lb, Bst, Cst, Dst, p)
            true = Fraction(brute.qap_objective(F, D, p))
            if precision == "fp32":
                assert rep <= true, (it, p)
            else:
                assert abs(rep - true) <= Fraction(TOL32) * true, (it, p, float(rep - true))
    g.close()


@pytest.mark.parametrize("precision", ["fp32", "fp32n"])
def test_fp32_certify_equals_lb_when_state_nonnegative(precision):
    F, D = qapgen.uniform(16, 2)
    g = Rlt2(F, D, precision=precision)
    g.ascend(3)
    lb, _ = g.bound()
    assert g.certify() == lb     # every stored reduced cost is >= 0
    g.close()


def test_fp32_lap_solve_certified_residuals():
    rng = np.random.default_rng(8)
    mats = [qapgen.random_matrix(int(n), i, ["uniform", "ties", "int"][i % 3]).astype(np.float32)
            for i, n in enumerate(rng.integers(1, 40, size=48))]
    batch = len(mats)
    n = np.array([m.shape[0] for m in mats], np.int32)
    mo = np.zeros(batch, np.int64)
    vo = np.zeros(batch, np.int64)
    mo[1:] = np.cumsum(n.astype(np.int64) ** 2)[:-1]
    vo[1:] = np.cumsum(n.astype(np.int64))[:-1]
    cost = np.concatenate([m.ravel() for m in mats]).astype(np.float32)
    value = np.empty(batch)
    st = B.lib().qap_lap_solve(batch, n.ctypes.data, mo.ctypes.data, vo.ctypes.data, cost.ctypes.data,
                               B.QAP_FP32_CERTIFIED, value.ctypes.data, None, None, B.QAP_LAP_RESIDUAL, None)
    assert st == 0
    for b, M in enumerate(mats):
        nb = M.shape[0]
        R = cost[mo[b]: mo[b] + nb * nb].reshape(nb, nb)
        assert (R >= 0).all()
        S_ref, _, _, _ = oracle.lap_concentrate(M.astype(np.float64))
        assert abs(value[b] - S_ref) <= TOL32 * max(1.0, abs(S_ref)) + 1e-6 * nb
        # S + sum of R over a permutation never exceeds the sum of M over it:
        # for random permutations and for the one that minimises sum(M - R)
        # (the hardest case; M - R is exact in FP64), summed exactly.
        _, tight = linear_sum_assignment(M.astype(np.float64) - R.astype(np.float64))
        for tau in [tight] + [rng.permutation(nb) for _ in range(5)]:
            lhs = sum(Fraction(float(M[r, tau[r]])) for r in range(nb))
            rhs = Fraction(value[b]) + sum(Fraction(float(R[r, tau[r]])) for r in range(nb))
            assert rhs <= lhs


@pytest.mark.parametrize("precision", ["fp32", "fp32n"])
def test_fp32_clustered25_vs_fp64_gpu(precision):
    F, D = qapgen.clustered(25, 0)
    print(f"{precision} vs fp64 clustered N=25", flush=True)
    a = Rlt2(F, D, precision="fp64")
    b = Rlt2(F, D, precision=precision)
    for it in range(1, 11):
        la = a.ascend(1)
        lb_ = b.ascend(1)
        assert abs(lb_ - la) <= TOL32 * la, (it, la, lb_)
    a.close()
    b.close()
