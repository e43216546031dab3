"""Brute-force and closed-form references used to pin the oracle.

TEST INFRASTRUCTURE ONLY.  Everything here is an independent definition:
enumeration over permutations, the Gilmore-Lawler bound by sorting, and the
objective identity that every step of the dual ascent must preserve.
"""
import itertools

import numpy as np


def lap_brute(M):
    """min over permutations sigma of sum_r M[r, sigma(r)] (n <= 8)."""
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[0]
    if n == 0:
        return 0.0
    rows = np.arange(n)
    best = np.inf
    for perm in itertools.permutations(range(n)):
        best = min(best, float(M[rows, list(perm)].sum()))
    return best


def all_perms(N):
    return np.array(list(itertools.permutations(range(N))), dtype=np.int64)


def qap_objective(F, D, perm, B0=None, constant=0.0):
    """Koopmans-Beckmann cost of placing facility i at location perm[i]:
    sum_{i,k} f_ik d_{perm(i) perm(k)} (diagonal included, it is the
    linear part b_ij = f_ii d_jj), plus optional linear costs and constant."""
    F = np.asarray(F, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    perm = np.asarray(perm)
    val = float((F * D[np.ix_(perm, perm)]).sum()) + constant
    if B0 is not None:
        val += float(np.asarray(B0)[np.arange(len(perm)), perm].sum())
    return val


def qap_brute(F, D, B0=None, constant=0.0):
    """Exact QAP optimum by enumeration (N <= 10); returns (value, perm)."""
    F = np.asarray(F, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    N = F.shape[0]
    best, best_p = np.inf, None
    idx = np.arange(N)
    B0a = None if B0 is None else np.asarray(B0, dtype=np.float64)
    chunk = []
    for perm in itertools.permutations(range(N)):
        chunk.append(perm)
        if len(chunk) == 20000:
            best, best_p = _qap_chunk(F, D, B0a, idx, chunk, best, best_p)
            chunk = []
    if chunk:
        best, best_p = _qap_chunk(F, D, B0a, idx, chunk, best, best_p)
    return best + constant, best_p


def _qap_chunk(F, D, B0a, idx, chunk, best, best_p):
    P = np.array(chunk, dtype=np.int64)                # (m, N)
    Dp = D[P[:, :, None], P[:, None, :]]               # (m, N, N)
    vals = (Dp * F[None]).sum(axis=(1, 2))
    if B0a is not None:
        vals = vals + B0a[idx[None, :], P].sum(axis=1)
    a = int(np.argmin(vals))
    if vals[a] < best:
        return float(vals[a]), P[a].copy()
    return best, best_p


def gilmore_lawler(F, D, B0=None, lap=None):
    """Gilmore-Lawler bound: LAP over l_ij = f_ii d_jj (+B0_ij) + minimal
    scalar product of row i of F (off-diagonal) and row j of D (off-diagonal),
    which by the rearrangement inequality pairs the ascending sort of one with
    the descending sort of the other.  `lap` solves the final assignment
    (default: brute force)."""
    F = np.asarray(F, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    N = F.shape[0]
    L = np.empty((N, N))
    for i in range(N):
        fi = np.sort(np.delete(F[i], i))
        for j in range(N):
            dj = np.sort(np.delete(D[j], j))[::-1]
            L[i, j] = F[i, i] * D[j, j] + float(np.dot(fi, dj))
    if B0 is not None:
        L = L + np.asarray(B0, dtype=np.float64)
    solver = lap or lap_brute
    return solver(L)


def represented_objective(lb, B, C, Dd, perm):
    """Objective of permutation perm as represented by a dual state:
    LB + sum_i b_{i,perm(i)} + sum_{i != k} c_{i perm(i) k perm(k)}
       + sum_{distinct i,k,p} d_{i perm(i) k perm(k) p perm(p)}
    with dense C[i,j,k,n] and D[i,j,k,n,p,q]."""
    perm = np.asarray(perm)
    N = len(perm)
    idx = np.arange(N)
    total = float(lb) + float(B[idx, perm].sum())
    I, K = np.meshgrid(idx, idx, indexing="ij")
    mask2 = I != K
    total += float(C[I, perm[I], K, perm[K]][mask2].sum())
    I3, K3, P3 = np.meshgrid(idx, idx, idx, indexing="ij")
    mask3 = (I3 != K3) & (I3 != P3) & (K3 != P3)
    total += float(Dd[I3, perm[I3], K3, perm[K3], P3, perm[P3]][mask3].sum())
    return total


def node_instance(F, D, fac, loc):
    """Branch-and-bound node of a QAP with facility fac[t] fixed at location
    loc[t]: returns (F', D', B0', constant) over the free facilities and
    locations in ascending order, written from the objective
    sum_{i,k} f_ik d_{pi(i) pi(k)} split into free-free, free-fixed (both
    directions, a linear cost) and fixed-fixed (a constant) terms."""
    F = np.asarray(F, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    N = F.shape[0]
    fac = list(int(a) for a in fac)
    loc = list(int(b) for b in loc)
    free_f = [i for i in range(N) if i not in fac]
    free_l = [j for j in range(N) if j not in loc]
    Fp = F[np.ix_(free_f, free_f)]
    Dp = D[np.ix_(free_l, free_l)]
    B0 = (F[np.ix_(free_f, fac)] @ D[np.ix_(free_l, loc)].T
          + F[np.ix_(fac, free_f)].T @ D[np.ix_(loc, free_l)])
    const = float((F[np.ix_(fac, fac)] * D[np.ix_(loc, loc)]).sum())
    return Fp, Dp, B0, const
