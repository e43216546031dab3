"""The test helper `layout.represented` against the objective identity on
the oracle's state (no GPU): after every step the represented objective of a
permutation equals its QAP objective."""
import numpy as np

import oracle
import qapgen
from oracle import brute
from tests import layout


def test_represented_matches_objective_on_oracle_state():
    F, D = qapgen.small(7, 4)
    o = oracle.Rlt2Oracle(F, D)
    o.iteration0()
    o.iterate(2)
    N = 7
    perms = np.random.default_rng(0).permuted(np.tile(np.arange(N), (50, 1)), axis=1)
    rep = layout.represented(N, o.lb, o.B.ravel(), layout.compact_C(o.C), layout.compact_D_full(o.D), perms)
    obj = np.array([brute.qap_objective(F, D, p) for p in perms])
    np.testing.assert_allclose(rep, obj, rtol=1e-12)
