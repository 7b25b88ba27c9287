"""Host-side argument checks of the torch helpers (no GPU needed).

The library reads every array through its device pointer, so the helpers in
``paper_2202_12817_amd.ops`` must refuse host tensors, strided views, wrong
dtypes and malformed offsets before any library call: a host address handed
to a kernel would fault the GPU, a strided view would give wrong results.
"""
import pytest
import torch

from paper_2202_12817_amd import ops


def _x(n=64, dtype=torch.float32):
    return torch.ones(n, dtype=dtype)


def test_sum_1d_refuses_host_tensor():
    with pytest.raises(ValueError, match="device"):
        ops.sum_1d(_x(), 4, "greedy")


def test_sum_1d_refuses_bad_dtype():
    # a float64 tensor is refused before its device is looked at
    x = torch.ones(8, dtype=torch.float64)
    with pytest.raises((ValueError, TypeError)):
        ops.sum_1d(x, 4, "greedy")


def test_sum_batched_refuses_host_tensors():
    off = torch.tensor([0, 32, 64], dtype=torch.int64)
    with pytest.raises(ValueError, match="device"):
        ops.sum_batched(_x(), off, 4, "greedy")


def test_offsets_checks_without_gpu():
    # _check_offsets refuses host, non-int64 and too short offsets (checked on
    # host tensors standing in for device ones: the first test fails on is_cuda)
    x = _x()
    for off in (torch.tensor([0, 64]), torch.tensor([0.0, 64.0]), torch.tensor([0])):
        with pytest.raises(ValueError):
            ops._check_offsets(off, x)


def test_powers_check_rejects_strided_view(monkeypatch):
    # pretend the tensor is on a device: the contiguity check must still refuse a strided view
    x = torch.ones(128)[::2]
    monkeypatch.setattr(torch.Tensor, "is_cuda", property(lambda self: True))
    with pytest.raises(ValueError, match="contiguous"):
        ops._check_powers(x)
    with pytest.raises((ValueError, TypeError)):
        ops._check_powers(torch.ones(8, dtype=torch.float64))
    ops._check_powers(torch.ones(8, dtype=torch.float16))


def test_norm_table_shape_checked():
    with pytest.raises(ValueError):
        ops._norm_tensor([1.0, 2.0, 3.0], 1, "cpu", H=2, table=True)
    t = ops._norm_tensor([0.0, 0.0, 1.0, 1.0], 1, "cpu", H=2, table=True)
    assert t.dtype == torch.float64 and t.numel() == 4
    with pytest.raises(ValueError):
        ops._norm_tensor([1.0, 2.0, 3.0], 1, "cpu")


def test_other_helpers_refuse_host_tensors():
    with pytest.raises(ValueError):
        ops.power_spectrum(torch.ones(8, dtype=torch.complex64))
    with pytest.raises(ValueError):
        ops.quantize_f16(_x(), 1.0)
    with pytest.raises(ValueError):
        ops.interleave(torch.ones(4, 8))
    with pytest.raises(ValueError):
        ops.sum_2d(torch.ones(3, 8), -1, 1, 4)
    with pytest.raises(ValueError):
        ops.cluster_peaks(torch.ones(8), torch.ones(8, dtype=torch.uint8), None, 1.0, 1)
