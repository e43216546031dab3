"""Seeded synthetic QAP instances.

This module only draws random numbers and shapes them into flow (F) and
distance (D) matrices; it contains none of the dual-ascent arithmetic.  Both
the GPU library's tests/benchmark and the CPU oracle are fed from here.

The paper evaluates on QAPLIB instances (nug, tai-a/b, kra, tho), which are
not available here; these generators stand in for them with the same sizes and
the two structures that matter for the bound: Euclidean (grid-like or
clustered) distances and sparse, possibly heavy-tailed flows.

Recipes (numpy PCG64 via ``default_rng(seed)``; all matrices symmetric with
zero diagonal, float64 holding integers):

* ``small``      N=8:  F, D off-diagonal uniform integers in [0, 9].
* ``uniform``    N=16: D = rounded Euclidean distances of N points uniform in
  [0,100]^2; F: each i<k is 0 with probability 0.5, else uniform in [1, 99].
* ``clustered``  N=25 (also N=24, N=40): 3-5 cluster centres uniform in
  [0,100]^2, each point joins a uniform cluster and is displaced by N(0, 5^2)
  per coordinate, clipped to the square; D = rounded Euclidean distance; F:
  each i<k is 0 with probability 0.7, else round(10^U(0,3)) in [1, 1000].
* ``nodes``      branch-and-bound nodes of one clustered N=24 parent: each node
  fixes m ~ U{2..14} facilities (uniform m-subset) to distinct locations
  (uniform injection).

Rounding is half away from zero (all values are non-negative).
"""
import numpy as np


def _round_half_up(x):
    return np.floor(np.asarray(x, dtype=np.float64) + 0.5)


def _symmetric_from_upper(N, upper_values):
    M = np.zeros((N, N))
    iu = np.triu_indices(N, 1)
    M[iu] = upper_values
    return M + M.T


def _euclid(points):
    diff = points[:, None, :] - points[None, :, :]
    Dm = _round_half_up(np.sqrt((diff ** 2).sum(-1)))
    np.fill_diagonal(Dm, 0.0)
    return Dm


def small(N=8, seed=0):
    """Uniform integer instance (N=8 workload)."""
    rng = np.random.default_rng(seed)
    m = N * (N - 1) // 2
    F = _symmetric_from_upper(N, rng.integers(0, 10, size=m).astype(np.float64))
    D = _symmetric_from_upper(N, rng.integers(0, 10, size=m).astype(np.float64))
    return F, D


def uniform(N=16, seed=0):
    """Uniform Euclidean distances, 50 % sparse flows (N=16 workload)."""
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 100.0, size=(N, 2))
    D = _euclid(pts)
    m = N * (N - 1) // 2
    zero = rng.random(m) < 0.5
    vals = rng.integers(1, 100, size=m).astype(np.float64)
    F = _symmetric_from_upper(N, np.where(zero, 0.0, vals))
    return F, D


def clustered(N=25, seed=0):
    """Clustered Euclidean distances, 70 % sparse heavy-tailed flows
    (N=25 headline workload; also used at N=24 and N=40)."""
    rng = np.random.default_rng(seed)
    K = int(rng.integers(3, 6))
    centres = rng.uniform(0.0, 100.0, size=(K, 2))
    which = rng.integers(0, K, size=N)
    pts = centres[which] + rng.normal(0.0, 5.0, size=(N, 2))
    pts = np.clip(pts, 0.0, 100.0)
    D = _euclid(pts)
    m = N * (N - 1) // 2
    zero = rng.random(m) < 0.7
    vals = _round_half_up(10.0 ** rng.uniform(0.0, 3.0, size=m))
    F = _symmetric_from_upper(N, np.where(zero, 0.0, vals))
    return F, D


def nodes(count=256, parent_N=24, seed=0, m_lo=2, m_hi=14):
    """Branch-and-bound nodes of one clustered parent instance.

    Returns (F, D, fixes) where fixes is a list of (facilities, locations)
    integer arrays: facility facilities[t] is fixed at location locations[t].
    """
    F, D = clustered(parent_N, seed)
    rng = np.random.default_rng(seed + 1_000_003)
    fixes = []
    for _ in range(count):
        m = int(rng.integers(m_lo, m_hi + 1))
        fac = np.sort(rng.choice(parent_N, size=m, replace=False))
        loc = rng.choice(parent_N, size=m, replace=False)
        fixes.append((fac.astype(np.int32), loc.astype(np.int32)))
    return F, D, fixes


def random_matrix(n, seed=0, kind="uniform"):
    """Test matrices for the assignment solver: 'uniform' reals, 'ties'
    (integers in [0,3]), 'product' (rank one), 'int' (integers in [0,99])."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.uniform(0.0, 100.0, size=(n, n))
    if kind == "ties":
        return rng.integers(0, 4, size=(n, n)).astype(np.float64)
    if kind == "int":
        return rng.integers(0, 100, size=(n, n)).astype(np.float64)
    if kind == "product":
        a = rng.integers(0, 20, size=n).astype(np.float64)
        b = rng.integers(0, 20, size=n).astype(np.float64)
        return np.outer(a, b)
    if kind == "zero":
        return np.zeros((n, n))
    raise ValueError(kind)


WORKLOADS = {
    "small": dict(fn=small, N=8, iters=5),
    "uniform": dict(fn=uniform, N=16, iters=50),
    "clustered": dict(fn=clustered, N=25, iters=100),
    "large": dict(fn=clustered, N=40, iters=20),
}
