"""The size limits of one handle on one MI355X.

* N = 64, the largest size (one wave64 lane per column of the C->B and
  B->LB problems), in FP32 round-to-nearest: 125 GB of stored D.  The oracle's
  dense state would need 550 GB, so this size is checked by what holds at any
  size: iteration 0 is the Gilmore-Lawler bound (computed here with the
  oracle's assignment solver), the bound does not fall, stays below the
  objective of the B-level assignment improved by pairwise exchanges, and the
  reduced costs stay >= 0.
* A state that cannot fit in HBM (N = 64 in FP64 with every block stored:
  500 GB) is refused with QAP_ENOMEM before anything is allocated.
"""
import numpy as np
import pytest

import oracle
import qapgen
from oracle import brute
from paper_1510_02065_amd import QapError, Rlt2, local_search
from paper_1510_02065_amd import _binding as B

pytestmark = pytest.mark.gpu


def test_state_larger_than_hbm_is_refused():
    F, D = qapgen.clustered(64, 0)
    with pytest.raises(QapError) as e:
        Rlt2(F, D, precision="fp64", complementary=False)
    assert e.value.status == B.QAP_ENOMEM


def test_maximum_size_n64_fp32_nearest():
    F, D = qapgen.clustered(64, 0)
    print("N=64 FP32 nearest: create", flush=True)
    g = Rlt2(F, D, precision="fp32n")
    glb = brute.gilmore_lawler(F, D, lap=lambda L: oracle.lap_solve(L)[0])
    lb0 = g.bound()[0]
    assert lb0 == pytest.approx(glb, rel=1e-5)
    print("N=64 FP32 nearest: one iteration", flush=True)
    lb1 = g.ascend(1)
    assert lb1 >= lb0 * (1 - 1e-6)
    perm, ub = local_search(F, D, g.assignment(0))
    assert sorted(perm.tolist()) == list(range(64))
    assert lb1 <= ub * (1 + 1e-5)
    _, Bst, Cst, _ = g.read_state(want_D=False)
    assert Bst.min() >= 0 and Cst.min() >= 0
    print(f"N=64: GLB {glb:.6g}, LB_0 {lb0:.6g}, LB_1 {lb1:.6g}, UB {ub:.6g}", flush=True)
    g.close()
