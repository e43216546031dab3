"""Host-side pieces of the library that need no GPU: the QAP objective and
the pairwise-exchange upper-bound heuristic (Algorithm 1's UB), against the
independent numpy objective and brute force."""
import itertools

import numpy as np
import pytest

import qapgen
from oracle import brute
from paper_1510_02065_amd import QapError, local_search, objective


@pytest.fixture(scope="module", autouse=True)
def _built():
    from paper_1510_02065_amd import build
    if build.needs_build():
        build.build()


def test_objective_matches_numpy_with_linear_costs():
    rng = np.random.default_rng(0)
    F = rng.integers(0, 20, (9, 9)).astype(float)   # asymmetric, nonzero diagonal
    D = rng.integers(0, 20, (9, 9)).astype(float)
    B0 = rng.uniform(0, 5, (9, 9))
    for _ in range(20):
        p = rng.permutation(9)
        assert objective(F, D, p, B0, 3.5) == pytest.approx(brute.qap_objective(F, D, p, B0, 3.5), rel=1e-15)


def test_objective_rejects_non_permutation():
    F, D = qapgen.small(6, 0)
    with pytest.raises(QapError):
        objective(F, D, [0, 1, 2, 3, 4, 4])


@pytest.mark.parametrize("seed", range(4))
def test_local_search_reaches_an_exchange_local_optimum(seed):
    rng = np.random.default_rng(seed)
    F = rng.integers(0, 30, (10, 10)).astype(float)
    D = rng.integers(0, 30, (10, 10)).astype(float)
    B0 = rng.integers(0, 10, (10, 10)).astype(float) if seed % 2 else None
    start = rng.permutation(10)
    p, v = local_search(F, D, start, B0, 1.0)
    assert sorted(p) == list(range(10))
    assert v == pytest.approx(brute.qap_objective(F, D, p, B0, 1.0), rel=1e-14)
    assert v <= brute.qap_objective(F, D, start, B0, 1.0)
    # No exchange of two facilities' locations improves it (brute force).
    for r, s in itertools.combinations(range(10), 2):
        q = p.copy()
        q[r], q[s] = q[s], q[r]
        assert brute.qap_objective(F, D, q, B0, 1.0) >= v - 1e-9 * abs(v)


def test_local_search_from_optimum_stays():
    F, D = qapgen.small(7, 3)
    opt, perm = brute.qap_brute(F, D)
    p, v = local_search(F, D, perm)
    assert v == opt
