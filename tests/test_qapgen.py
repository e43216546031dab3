"""The seeded instance generators are deterministic and have the stated shape."""
import numpy as np
import pytest

import qapgen


@pytest.mark.parametrize("fn,N", [(qapgen.small, 8), (qapgen.uniform, 16),
                                  (qapgen.clustered, 25), (qapgen.clustered, 40)])
def test_generators(fn, N):
    F1, D1 = fn(N, 3)
    F2, D2 = fn(N, 3)
    np.testing.assert_array_equal(F1, F2)
    np.testing.assert_array_equal(D1, D2)
    for M in (F1, D1):
        assert M.shape == (N, N)
        np.testing.assert_array_equal(M, M.T)
        assert (np.diag(M) == 0).all()
        assert (M >= 0).all()
        np.testing.assert_array_equal(M, np.round(M))
    F3, _ = fn(N, 4)
    assert not np.array_equal(F1, F3)


def test_clustered_flow_sparsity_and_range():
    F, D = qapgen.clustered(40, 0)
    off = F[np.triu_indices(40, 1)]
    assert 0.6 < (off == 0).mean() < 0.8
    assert off.max() <= 1000 and off[off > 0].min() >= 1
    assert D.max() <= 142


def test_nodes():
    F, D, fixes = qapgen.nodes(count=32, parent_N=24, seed=0)
    assert F.shape == (24, 24)
    for fac, loc in fixes:
        assert 2 <= len(fac) <= 14
        assert len(set(fac.tolist())) == len(fac) and len(set(loc.tolist())) == len(loc)
