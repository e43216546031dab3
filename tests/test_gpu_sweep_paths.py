"""The steps 1-3 kernels for one stored block per complementary pair (one
workgroup per facility triple when the triple fits in LDS, location cubes
otherwise) against the every-block comparison path, at the sizes where the
choice changes: bit for bit after two iterations, on the trace and on every
concentration's value."""
import numpy as np
import pytest

import qapgen
from paper_1510_02065_amd import Rlt2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,precision", [(25, "fp64"), (26, "fp64"), (32, "fp32"), (33, "fp32")])
def test_stored_half_matches_every_block(N, precision):
    F, D = qapgen.clustered(N, 3)
    print(f"sweep paths N={N} {precision}", flush=True)
    a = Rlt2(F, D, precision=precision, trace_level=2, complementary=True)
    a.ascend(2)
    ta, va = a.trace()[0], a.lap_values()
    a.close()
    b = Rlt2(F, D, precision=precision, trace_level=2, complementary=False)
    b.ascend(2)
    tb, vb = b.trace()[0], b.lap_values()
    b.close()
    np.testing.assert_array_equal(ta, tb)
    for x, y in zip(va, vb):
        np.testing.assert_array_equal(x, y)
