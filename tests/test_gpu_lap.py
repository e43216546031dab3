"""GPU parity of the batched assignment solver (qap_lap_solve) against the
oracle: values, canonical duals and residuals, element by element."""
import numpy as np
import pytest

import oracle
import qapgen
from paper_1510_02065_amd import QapError, lap_solve

pytestmark = pytest.mark.gpu

KINDS = ["uniform", "ties", "int", "product", "zero"]


def _check(mats, out, tol=1e-12):
    for b, M in enumerate(mats):
        n = M.shape[0]
        S, R, duals, _ = oracle.lap_concentrate(M)
        scale = max(1.0, float(np.abs(M).max())) if M.size else 1.0
        assert abs(out["value"][b] - S) <= tol * scale * max(n, 1), (b, n)
        np.testing.assert_allclose(out["duals"][b], duals, rtol=0, atol=tol * scale * 4, err_msg=f"duals b={b} n={n}")
        if "residual" in out:
            Rg = out["residual"][b]
            assert (Rg >= 0).all()
            np.testing.assert_allclose(Rg, R, rtol=0, atol=tol * scale * 4, err_msg=f"residual b={b} n={n}")
        sig = out["assign"][b]
        assert sorted(sig.tolist()) == list(range(n))
        assert abs(float(M[np.arange(n), sig].sum()) - S) <= 1e-9 * scale * max(n, 1)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 7, 8, 9, 14, 16, 17, 23, 24, 25, 31, 32, 33, 38, 39, 40, 63, 64])
def test_lap_sizes_and_kinds(n):
    mats = [qapgen.random_matrix(n, seed, kind) for kind in KINDS for seed in range(3)]
    out = lap_solve(mats, residual=True)
    _check(mats, out)


def test_lap_mixed_sizes_one_batch():
    rng = np.random.default_rng(0)
    sizes = rng.integers(0, 65, size=300)
    mats = [qapgen.random_matrix(int(n), i, KINDS[i % 4]) for i, n in enumerate(sizes)]
    out = lap_solve(mats, residual=True)
    _check(mats, out)


def test_lap_adversarial_ties_and_scales():
    mats = []
    for n in (6, 23, 38):
        mats.append(np.ones((n, n)))                         # all ties
        mats.append(np.eye(n) * 5.0)                          # zero diagonal optimum avoided
        mats.append(np.arange(n * n, dtype=float).reshape(n, n) % 3)
        mats.append(qapgen.random_matrix(n, 1, "uniform") * 1e6)
        mats.append(qapgen.random_matrix(n, 2, "uniform") * 1e-6)
        M = qapgen.random_matrix(n, 3, "int")
        mats.append(M - 50.0)                                 # negative entries
    out = lap_solve(mats, residual=True)
    _check(mats, out)


def test_lap_empty_batch_and_errors():
    out = lap_solve([])
    assert out["value"].shape == (0,)
    with pytest.raises(QapError):
        lap_solve([np.zeros((65, 65))])


def test_lap_device_pointers():
    torch = pytest.importorskip("torch")
    from paper_1510_02065_amd import lap_solve_device
    rng = np.random.default_rng(4)
    sizes = rng.integers(1, 40, size=64).astype(np.int32)
    mats = [qapgen.random_matrix(int(n), i, "int") for i, n in enumerate(sizes)]
    mo = np.zeros(len(sizes), np.int64)
    vo = np.zeros(len(sizes), np.int64)
    mo[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    vo[1:] = np.cumsum(sizes.astype(np.int64))[:-1]
    dev = torch.device("cuda:0")
    cost = torch.tensor(np.concatenate([m.ravel() for m in mats]), dtype=torch.float64, device=dev)
    value = torch.empty(len(sizes), dtype=torch.float64, device=dev)
    duals = torch.empty(4 * int(sizes.sum()), dtype=torch.float64, device=dev)
    assign = torch.empty(int(sizes.sum()), dtype=torch.int32, device=dev)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        lap_solve_device(torch.tensor(sizes, device=dev), torch.tensor(mo, device=dev),
                         torch.tensor(vo, device=dev), cost, value, duals, assign, residual=True,
                         stream=stream)
    stream.synchronize()
    c = cost.cpu().numpy()
    d = duals.cpu().numpy()
    a = assign.cpu().numpy()
    out = {"value": value.cpu().numpy(),
           "duals": [d[4 * vo[b]: 4 * vo[b] + 4 * sizes[b]].reshape(4, sizes[b]) for b in range(len(sizes))],
           "assign": [a[vo[b]: vo[b] + sizes[b]] for b in range(len(sizes))],
           "residual": [c[mo[b]: mo[b] + sizes[b] ** 2].reshape(sizes[b], sizes[b]) for b in range(len(sizes))]}
    _check(mats, out)


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "fp32n"])
def test_lap_device_buckets_match_host_bitwise(dtype):
    """The device-pointer path sorts problems by size on the device; each
    problem must come out bit for bit as from the host path (same segment
    width per size), and sizes outside [0, 64] must come out unsolved (NaN)."""
    torch = pytest.importorskip("torch")
    from paper_1510_02065_amd import _binding as B
    rng = np.random.default_rng(11)
    sizes = rng.integers(0, 65, size=257).astype(np.int32)
    sizes[:6] = [0, 1, 8, 9, 64, 33]
    npdt = np.float64 if dtype == "fp64" else np.float32
    tdt = torch.float64 if dtype == "fp64" else torch.float32
    code = {"fp64": B.QAP_FP64, "fp32": B.QAP_FP32_CERTIFIED, "fp32n": B.QAP_FP32_NEAREST}[dtype]
    mats = [qapgen.random_matrix(int(n), i, KINDS[i % 4]).astype(npdt) for i, n in enumerate(sizes)]
    mo = np.zeros(len(sizes), np.int64)
    vo = np.zeros(len(sizes), np.int64)
    mo[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    vo[1:] = np.cumsum(sizes.astype(np.int64))[:-1]
    cost_h = np.concatenate([m.ravel() for m in mats]).astype(npdt)
    nv = int(sizes.sum())
    val_h = np.empty(len(sizes))
    dual_h = np.empty(4 * nv, npdt)
    asg_h = np.empty(nv, np.int32)
    st = B.lib().qap_lap_solve(len(sizes), sizes.ctypes.data, mo.ctypes.data, vo.ctypes.data, cost_h.ctypes.data,
                               code, val_h.ctypes.data, dual_h.ctypes.data, asg_h.ctypes.data, B.QAP_LAP_RESIDUAL,
                               None)
    assert st == 0
    dev = torch.device("cuda:0")
    bad = np.array([65, -3, 70], np.int32)          # never solved: value NaN, nothing written
    nd = torch.tensor(np.concatenate([sizes, bad]), device=dev)
    mod = torch.tensor(np.concatenate([mo, np.zeros(3, np.int64)]), device=dev)
    vod = torch.tensor(np.concatenate([vo, np.zeros(3, np.int64)]), device=dev)
    cost = torch.tensor(np.concatenate([m.ravel() for m in mats]).astype(npdt), dtype=tdt, device=dev)
    value = torch.empty(len(sizes) + 3, dtype=torch.float64, device=dev)
    duals = torch.empty(4 * nv, dtype=tdt, device=dev)
    assign = torch.empty(nv, dtype=torch.int32, device=dev)
    stream = torch.cuda.Stream()
    st = B.lib().qap_lap_solve(int(nd.numel()), nd.data_ptr(), mod.data_ptr(), vod.data_ptr(), cost.data_ptr(),
                               code, value.data_ptr(), duals.data_ptr(), assign.data_ptr(),
                               B.QAP_LAP_DEVICE | B.QAP_LAP_RESIDUAL, stream.cuda_stream)
    assert st == 0
    stream.synchronize()
    v = value.cpu().numpy()
    np.testing.assert_array_equal(v[: len(sizes)], val_h)
    assert np.isnan(v[len(sizes):]).all()
    np.testing.assert_array_equal(cost.cpu().numpy(), cost_h)
    np.testing.assert_array_equal(duals.cpu().numpy(), dual_h)
    np.testing.assert_array_equal(assign.cpu().numpy(), asg_h)
