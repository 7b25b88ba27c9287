"""The allocation-free batched sum (hs_sum_batched_static, workspace in the
library's static device scratch) against hs_sum_batched with a plan: the
same kernels, so dense outputs and candidate records must be identical, bit
for bit, on two calls in a row (the second with fewer, shorter spectra: the
scratch keeps the first call's contents and must not leak them)."""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_12817_amd import hs
    hs.load()
    return torch.device("cuda:0")


def _run(hs, dev, x, off, H, mode, dtype, static, thr=4.0):
    n = int(x.numel())
    B = int(off.numel()) - 1
    snr = torch.full((n,), -7.0, dtype=torch.float32, device=dev)
    harm = torch.full((n,), 99, dtype=torch.uint8, device=dev)
    drift = torch.full((n,), 99, dtype=torch.uint8, device=dev)
    cap = n
    cand = torch.zeros((cap, 4), dtype=torch.int32, device=dev)
    count = torch.full((1,), 12345, dtype=torch.int64, device=dev)
    desc = hs.hs_plan_desc_init(harmonics=H, mode=mode, dtype=dtype, threshold=thr, max_spectra=max(B, 1))
    if static:
        hs.hs_sum_batched_static(desc, x, off, B, None, snr, harm, drift, cand, cap, count)
    else:
        plan = hs.Plan(harmonics=H, mode=mode, dtype=dtype, threshold=thr, max_spectra=max(B, 1))
        hs.hs_sum_batched(plan.handle, x, off, B, None, snr, harm, drift, cand, cap, count)
        torch.cuda.synchronize()
        plan.close()
    torch.cuda.synchronize()
    k = int(count.item())
    recs = cand[:k].cpu().numpy().view(np.uint32).reshape(k, 4)
    order = np.lexsort((recs[:, 1], recs[:, 0]))
    return snr.cpu().numpy(), harm.cpu().numpy(), drift.cpu().numpy(), k, recs[order]


@pytest.mark.parametrize("mode,dtype", [(1, 0), (0, 0), (1, 1)])
def test_static_equals_planned_two_calls(dev, mode, dtype):
    from paper_2202_12817_amd import hs
    for call, (B, lo, hi, seed) in enumerate([(40, 30000, 90000, 61), (7, 2000, 20011, 62)]):
        x, off = synthetic.config3(n_spectra=B, lo=lo, hi=hi, seed=seed)
        print("static vs planned: call", call, "B", B, "mode", mode, "dtype", dtype, flush=True)
        xt = torch.from_numpy(x).to(dev)
        if dtype == 1:
            q = torch.empty(x.size, dtype=torch.int16, device=dev)
            for s in range(B):
                sc = float(np.float32(x[off[s]:off[s + 1]].mean(dtype=np.float64)))
                hs.hs_quantize_f16(xt.data_ptr() + 4 * int(off[s]), int(off[s + 1] - off[s]), sc,
                                   q.data_ptr() + 2 * int(off[s]))
            xt = q
        ot = torch.from_numpy(off).to(dev)
        a = _run(hs, dev, xt, ot, 32, mode, dtype, static=True)
        b = _run(hs, dev, xt, ot, 32, mode, dtype, static=False)
        assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32)), "snr differs"
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]), "harm/drift differ"
        assert a[3] == b[3] and a[3] > 0, "candidate counts %d vs %d" % (a[3], b[3])
        assert np.array_equal(a[4], b[4]), "candidate records differ"


def test_static_rejects_too_many_spectra(dev):
    from paper_2202_12817_amd import hs
    x = torch.zeros(1025 * 4, dtype=torch.float32, device=dev)
    off = torch.arange(0, 1026 * 4, 4, dtype=torch.int64, device=dev)
    snr = torch.zeros(x.numel(), dtype=torch.float32, device=dev)
    harm = torch.zeros(x.numel(), dtype=torch.uint8, device=dev)
    desc = hs.hs_plan_desc_init()
    with pytest.raises(hs.HsError) as e:
        hs.hs_sum_batched_static(desc, x, off, 1025, None, snr, harm, None, None, 0, None)
    assert e.value.status == hs.HS_ERR_ARG and "1024" in str(e.value)
