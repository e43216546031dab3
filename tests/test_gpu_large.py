"""The large single instance: clustered N=40, a 3.5e9-entry reduced-cost
array (28 GB in FP64, 14 GB in certified FP32) on one GPU.

The oracle's dense state would not fit, so this size is checked through
properties that hold at any size: iteration 0 equals the Gilmore-Lawler bound
(computed independently, exact for integer data), the bound never decreases,
certification finds no negative reduced cost, and certified FP32 tracks FP64
within 1e-5."""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import qapgen
from oracle import brute
from paper_1510_02065_amd import Rlt2

pytestmark = pytest.mark.gpu


def _lap(M):
    r, c = linear_sum_assignment(M)
    return float(M[r, c].sum())


def test_clustered40_fp64_and_fp32():
    F, D = qapgen.clustered(40, 0)
    glb = brute.gilmore_lawler(F, D, lap=_lap)
    print("clustered N=40 FP64", flush=True)
    g = Rlt2(F, D, precision="fp64")
    assert g.bound()[0] == glb
    T = 4
    g.ascend(T)
    lb64, lbp = g.trace()
    assert len(lb64) == T + 1
    assert (np.diff(lb64) >= 0).all() and (lbp[1:] >= 0).all()
    assert g.certify() == lb64[-1]
    g.close()
    print("clustered N=40 FP32 certified", flush=True)
    f = Rlt2(F, D, precision="fp32")
    assert f.bound()[0] == pytest.approx(glb, rel=1e-6)
    cert = f.ascend(T)
    lb32, _ = f.trace()
    assert abs(cert - lb64[-1]) <= 1e-5 * lb64[-1]
    np.testing.assert_allclose(lb32, lb64, rtol=1e-5)
    f.close()
