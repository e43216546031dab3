"""Complementary D blocks (Section 6): storing one block of each pair
D_ijkn, D_knij and concentrating it once (S to both parents) gives bit for
bit the state of storing and concentrating every block, in FP64 and
certified FP32, for a single instance and for a batch of branch-and-bound
nodes of different sizes, after every step and after whole iterations; with
every block stored, the two blocks of each pair are equal."""
import numpy as np
import pytest

import qapgen
from paper_1510_02065_amd import Rlt2, subproblem
from tests import layout

pytestmark = pytest.mark.gpu


def _pairs_equal(Dc, N):
    """Compact D: block (i,j,k,n) equals block (k,n,i,j) entry by entry (the
    two blocks share their row and column index sets and order)."""
    I, J, K, Nn = layout.c_index_arrays(N)
    pos = {(int(i), int(j), int(k), int(n)): b for b, (i, j, k, n) in enumerate(zip(I, J, K, Nn))}
    blocks = Dc.reshape(len(I), (N - 2) ** 2)
    twin = np.array([pos[(int(k), int(n), int(i), int(j))] for i, j, k, n in zip(I, J, K, Nn)])
    np.testing.assert_array_equal(blocks, blocks[twin])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("N,gen", [(8, "small"), (13, "clustered")])
def test_complementary_equals_all_blocks(precision, N, gen):
    F, D = qapgen.small(N, 0) if gen == "small" else qapgen.clustered(N, 1)
    print(f"complementary vs all blocks: N={F.shape[0]} {gen} {precision}", flush=True)
    a = Rlt2(F, D, precision=precision, trace_level=2, complementary=True)
    b = Rlt2(F, D, precision=precision, trace_level=2, complementary=False)
    for t in range(4):
        for s in (3, 4, 5, 6, 7):
            a.step(s)
            b.step(s)
        for x, y in zip(a.read_state(), b.read_state()):
            np.testing.assert_array_equal(x, y)
        for x, y in zip(a.lap_values(), b.lap_values()):
            np.testing.assert_array_equal(x, y)
    a.ascend(6)
    b.ascend(6)
    np.testing.assert_array_equal(a.trace()[0], b.trace()[0])
    if precision == "fp32":
        assert a.certify() == b.certify()
    _pairs_equal(b.read_state()[3], F.shape[0])
    a.close()
    b.close()


def test_complementary_batch_of_nodes():
    F, D, fixes = qapgen.nodes(count=24, parent_N=14, seed=2, m_lo=2, m_hi=8)
    nodes = [subproblem(F, D, fac, loc) for fac, loc in fixes]
    args = ([n[0] for n in nodes], [n[1] for n in nodes], [n[2] for n in nodes], [n[3] for n in nodes])
    print("batch of 24 nodes, N' =", sorted({n[0].shape[0] for n in nodes}), flush=True)
    a = Rlt2.batch(*args, complementary=True)
    b = Rlt2.batch(*args, complementary=False)
    a.ascend(5)
    b.ascend(5)
    np.testing.assert_array_equal(a.bounds(), b.bounds())
    for k in range(len(nodes)):
        for x, y in zip(a.read_state_k(k), b.read_state_k(k)):
            np.testing.assert_array_equal(x, y)
    a.close()
    b.close()
