"""Branch-and-bound node construction (qap_subproblem) on the host.

Pinned two ways: against an independent numpy construction (the oracle's
node_instance) and by the defining identity: for every completion of the
fixed assignments, the parent's objective equals the node's constant plus the
node's objective with its linear costs (checked exhaustively on small nodes)."""
import itertools

import numpy as np
import pytest

import qapgen
from oracle import brute
from paper_1510_02065_amd import QapError, subproblem


@pytest.fixture(scope="module", autouse=True)
def _built():
    from paper_1510_02065_amd import build
    if build.needs_build():
        build.build()


@pytest.mark.parametrize("seed", range(6))
def test_matches_independent_construction(seed):
    rng = np.random.default_rng(seed)
    N = 12
    F = rng.integers(0, 20, (N, N)).astype(float)
    D = rng.integers(0, 20, (N, N)).astype(float)
    m = int(rng.integers(0, 8))
    fac = rng.choice(N, m, replace=False)
    loc = rng.choice(N, m, replace=False)
    got = subproblem(F, D, fac, loc)
    ref = brute.node_instance(F, D, fac, loc)
    for a, b in zip(got[:3], ref[:3]):
        np.testing.assert_array_equal(a, b)
    assert got[3] == ref[3]


@pytest.mark.parametrize("seed", range(4))
def test_objective_identity_exhaustive(seed):
    rng = np.random.default_rng(100 + seed)
    N = 7
    F = rng.integers(0, 10, (N, N)).astype(float)
    D = rng.integers(0, 10, (N, N)).astype(float)
    m = 3
    fac = rng.choice(N, m, replace=False)
    loc = rng.choice(N, m, replace=False)
    Fs, Ds, Bs, c = subproblem(F, D, fac, loc)
    free_f = [i for i in range(N) if i not in fac]
    free_l = [j for j in range(N) if j not in loc]
    for p in itertools.permutations(range(N - m)):
        perm = np.empty(N, dtype=int)
        perm[list(fac)] = loc
        perm[free_f] = [free_l[x] for x in p]
        parent = brute.qap_objective(F, D, perm)
        node = brute.qap_objective(Fs, Ds, np.array(p), B0=Bs, constant=c)
        assert parent == node


def test_nodes_workload_shapes():
    F, D, fixes = qapgen.nodes(count=16, parent_N=24, seed=0)
    for fac, loc in fixes:
        Fs, Ds, Bs, c = subproblem(F, D, fac, loc)
        assert Fs.shape == (24 - len(fac),) * 2
        assert c >= 0 and (Bs >= 0).all()


def test_errors():
    F = np.zeros((5, 5))
    with pytest.raises(QapError):
        subproblem(F, F, [0, 0], [1, 2])
    with pytest.raises(QapError):
        subproblem(F, F, [0], [7])
