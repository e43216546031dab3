"""Test-side map between the library's compact state layout and the oracle's
dense [i][j][k][n] / [i][j][k][n][p][q] indexing.

Written from the layout the C header documents, independently of the kernels:
block C_ij holds rows k != i and columns n != j in ascending order; block
D_ijkn (the beta(ijkn)-th block) holds rows p not in {i,k} and columns q not
in {j,n} in ascending order.
"""
import functools

import numpy as np


@functools.lru_cache(maxsize=8)
def c_index_arrays(N):
    """(I, J, K, Nn) dense indices for every compact C position, in order."""
    I, J, K, Nn = [], [], [], []
    for i in range(N):
        for j in range(N):
            for k in range(N):
                if k == i:
                    continue
                for n in range(N):
                    if n == j:
                        continue
                    I.append(i); J.append(j); K.append(k); Nn.append(n)
    return tuple(np.array(a, dtype=np.int64) for a in (I, J, K, Nn))


def compact_C(Cdense):
    N = Cdense.shape[0]
    I, J, K, Nn = c_index_arrays(N)
    return Cdense[I, J, K, Nn]


def d_block_rows(N, i, k):
    return [p for p in range(N) if p != i and p != k]


def compact_D_sample(Ddense, rng, count):
    """Random sample of compact D positions: returns (positions, dense values)."""
    N = Ddense.shape[0]
    n1, n2 = N - 1, N - 2
    nblk = N * N * n1 * n1
    I, J, K, Nn = c_index_arrays(N)
    beta = rng.integers(0, nblk, size=count)
    e = rng.integers(0, n2 * n2, size=count)
    pp, qq = e // n2, e % n2
    vals = np.empty(count)
    for x in range(count):
        i, j, k, n = I[beta[x]], J[beta[x]], K[beta[x]], Nn[beta[x]]
        p = d_block_rows(N, i, k)[pp[x]]
        q = [c for c in range(N) if c != j and c != n][qq[x]]
        vals[x] = Ddense[i, j, k, n, p, q]
    return beta * (n2 * n2) + e, vals


def compact_D_full(Ddense):
    """Whole compact D from the dense oracle array (small N only)."""
    N = Ddense.shape[0]
    I, J, K, Nn = c_index_arrays(N)
    n2 = N - 2
    out = np.empty((len(I), n2 * n2))
    for b in range(len(I)):
        i, j, k, n = I[b], J[b], K[b], Nn[b]
        rows = d_block_rows(N, i, k)
        cols = [c for c in range(N) if c != j and c != n]
        out[b] = Ddense[i, j, k, n][np.ix_(rows, cols)].ravel()
    return out.ravel()


def close_family(x, y, tol):
    """|x - y| <= tol * max(|y|, mean |y| of the family) elementwise."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    scale = np.maximum(np.abs(y), np.abs(y).mean() if y.size else 0.0)
    bad = np.abs(x - y) > tol * scale
    return (not bad.any()), (np.abs(x - y) / np.maximum(scale, 1e-300)).max() if y.size else 0.0


def represented(N, lb, B, C, D, perms):
    """LB + sum_i b_{i p(i)} + sum_{i!=k} c_{i p(i) k p(k)} + sum over ordered
    distinct triples of d_{i p(i) k p(k) r p(r)}, for every row p of `perms`
    (compact state arrays, FP64).  D may be None (level-1 state)."""
    P = np.asarray(perms, dtype=np.int64)
    if P.ndim == 1:
        P = P[None, :]
    n1, n2 = N - 1, N - 2
    B = np.asarray(B).reshape(N, N)
    tot = np.full(P.shape[0], float(lb))
    for i in range(N):
        tot += B[i, P[:, i]]
    for i in range(N):
        for k in range(N):
            if k == i:
                continue
            pi, pk = P[:, i], P[:, k]
            beta = (i * N + pi) * n1 * n1 + (k - (k > i)) * n1 + (pk - (pk > pi))
            tot += C[beta]
            if D is None:
                continue
            lo, hi = min(i, k), max(i, k)
            plo, phi = np.minimum(pi, pk), np.maximum(pi, pk)
            for r in range(N):
                if r == i or r == k:
                    continue
                pr = P[:, r]
                row = r - (r > lo) - (r > hi)
                col = pr - (pr > plo) - (pr > phi)
                tot += D[beta * n2 * n2 + row * n2 + col]
    return tot
