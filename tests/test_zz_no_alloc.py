"""qap_lap_solve_noalloc (the batched assignment solve that allocates nothing)
against qap_lap_solve with device pointers: the same problems must give the
same bits (values, residuals, canonical duals, assignments) on two calls in a
row, the second with a smaller batch, through the C ABI."""
import ctypes

import numpy as np
import pytest

import qapgen
from paper_1510_02065_amd import _binding as B

pytestmark = pytest.mark.gpu

KINDS = ["uniform", "ties", "int", "product"]


def _problems(count, seed, npdt):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(0, 65, size=count).astype(np.int32)
    mats = [qapgen.random_matrix(int(n), seed * 1000 + i, KINDS[i % 4]).astype(npdt) for i, n in enumerate(sizes)]
    mo = np.zeros(count, np.int64)
    vo = np.zeros(count, np.int64)
    mo[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    vo[1:] = np.cumsum(sizes.astype(np.int64))[:-1]
    cost = np.concatenate([m.ravel() for m in mats]).astype(npdt)
    return sizes, mo, vo, cost


def _solve(fn, torch, sizes, mo, vo, cost, code, tdt, stream):
    dev = torch.device("cuda:0")
    nv = int(sizes.sum())
    n = torch.tensor(sizes, device=dev)
    mod = torch.tensor(mo, device=dev)
    vod = torch.tensor(vo, device=dev)
    c = torch.tensor(cost, dtype=tdt, device=dev)
    value = torch.full((len(sizes),), -1.0, dtype=torch.float64, device=dev)
    duals = torch.zeros(max(4 * nv, 1), dtype=tdt, device=dev)
    assign = torch.full((max(nv, 1),), -1, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    st = fn(len(sizes), n.data_ptr(), mod.data_ptr(), vod.data_ptr(), c.data_ptr(), code, value.data_ptr(),
            duals.data_ptr(), assign.data_ptr(), B.QAP_LAP_DEVICE | B.QAP_LAP_RESIDUAL, stream.cuda_stream)
    assert st == 0, B.lib().qap_last_error()
    stream.synchronize()
    return value.cpu().numpy(), c.cpu().numpy(), duals.cpu().numpy(), assign.cpu().numpy()


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_noalloc_matches_allocating_entry_point(dtype):
    torch = pytest.importorskip("torch")
    L = B.lib()
    npdt = np.float64 if dtype == "fp64" else np.float32
    tdt = torch.float64 if dtype == "fp64" else torch.float32
    code = B.QAP_FP64 if dtype == "fp64" else B.QAP_FP32_CERTIFIED
    stream = torch.cuda.Stream()
    # Two calls in a row, the second smaller: the shared scratch keeps the
    # first call's lists and counters, which the second must not use.
    for count, seed in ((700, 1), (90, 2)):
        print(f"noalloc {dtype}: batch {count}, seed {seed}", flush=True)
        prob = _problems(count, seed, npdt)
        ref = _solve(L.qap_lap_solve, torch, *prob, code, tdt, stream)
        got = _solve(L.qap_lap_solve_noalloc, torch, *prob, code, tdt, stream)
        for r, g, what in zip(ref, got, ("value", "residual", "duals", "assign")):
            np.testing.assert_array_equal(g, r, err_msg=what)
        assert np.isfinite(got[0]).all()


def test_noalloc_rejects_what_it_cannot_do():
    L = B.lib()
    n = np.array([3], np.int32)
    mo = np.zeros(1, np.int64)
    cost = np.zeros(9)
    val = np.zeros(1)
    # host pointers would need staging buffers
    st = L.qap_lap_solve_noalloc(1, n.ctypes.data, mo.ctypes.data, None, cost.ctypes.data, B.QAP_FP64,
                                 val.ctypes.data, None, None, 0, None)
    assert st == B.QAP_EINVAL
    assert b"QAP_LAP_DEVICE" in L.qap_last_error()
    # more problems than the static workspace holds (rejected before any
    # pointer is read)
    big = 1048576 + 1
    st = L.qap_lap_solve_noalloc(big, n.ctypes.data, mo.ctypes.data, None, cost.ctypes.data, B.QAP_FP64,
                                 val.ctypes.data, None, None, B.QAP_LAP_DEVICE, None)
    assert st == B.QAP_EINVAL
    assert b"QAP_LAP_NOALLOC_MAX_BATCH" in L.qap_last_error()
    assert L.qap_lap_solve_noalloc(0, None, None, None, None, B.QAP_FP64, None, None, None, B.QAP_LAP_DEVICE,
                                   None) == 0
