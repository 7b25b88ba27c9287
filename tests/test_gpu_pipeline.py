"""GPU parity of the pipeline neighbours: power spectrum with inter-binning
and peak clustering, against the oracle, alone and chained with the sum.

Bars: powers bitwise (the same float operations in the same order); kept
peaks equal as sorted record sets, SNR bit for bit.
"""
import numpy as np
import pytest

import oracle
import synthetic
from gpu_checks import _np, _same_records

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_12817_amd import hs
    hs.load()
    return torch.device("cuda:0")


def _ops():
    from paper_2202_12817_amd import ops
    return ops


def _recs(out):
    recs, n = _ops().candidates_numpy(out)
    return np.sort(recs, order=["spectrum", "bin"]), n


@pytest.mark.parametrize("n", [1, 2, 3, 255, 256, 257, 100003])
@pytest.mark.parametrize("interbin", [False, True])
@pytest.mark.parametrize("scale", [1.0, 1.0 / 3.0, 2.0 ** -20])
def test_power_spectrum_bitwise(dev, n, interbin, scale):
    g = np.random.default_rng(n)
    F = (g.normal(size=n) + 1j * g.normal(size=n)).astype(np.complex64) * np.float32(100.0)
    got = _np(_ops().power_spectrum(torch.from_numpy(F).to(dev), interbin, scale))
    want = oracle.power_spectrum(F, interbin, scale)
    assert got.shape == want.shape
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_power_spectrum_unaligned_output(dev):
    # an output 4 but not 8 bytes aligned takes the single-float stores
    F = (np.random.default_rng(99).normal(size=4097) + 1j).astype(np.complex64)
    buf = torch.zeros(2 * F.size + 2, dtype=torch.float32, device=dev)
    from paper_2202_12817_amd import hs
    hs.hs_power_spectrum(torch.from_numpy(F).to(dev), F.size, 1, 0.5, buf.data_ptr() + 4)
    got = _np(buf)[1:1 + 2 * F.size - 1]
    assert np.array_equal(got.view(np.uint32), oracle.power_spectrum(F, True, 0.5).view(np.uint32))
    assert _np(buf)[0] == 0 and _np(buf)[-1] == 0


@pytest.mark.parametrize("radius", [0, 1, 5, 64, 1024, 1025, 3000])
@pytest.mark.parametrize("thr", [2.0, 4.0])
def test_cluster_peaks_batched(dev, radius, thr):
    x, off = synthetic.config3(n_spectra=23, lo=2, hi=60000, seed=95)
    xt, ot = torch.from_numpy(x).to(dev), torch.from_numpy(off).to(dev)
    d = _ops().sum_batched(xt, ot, 16, "greedy", thr, dense=True, candidates=False)
    got = _ops().cluster_peaks(d["snr"], d["harm"], d["drift"], thr, radius, offsets=ot, capacity=x.size)
    recs, n = _recs(got)
    want = oracle.cluster_peaks(_np(d["snr"]), _np(d["harm"]), _np(d["drift"]), thr, radius, offsets=off)
    assert n == want.size
    assert _same_records(recs, want)


def test_cluster_peaks_one_spectrum_without_drift(dev):
    x, _ = synthetic.config2(n=300007, seed=96, n_trains=20)
    d = _ops().sum_1d(torch.from_numpy(x).to(dev), 32, "greedy")
    got = _ops().cluster_peaks(d["snr"], d["harm"], None, 6.0, 16)
    recs, n = _recs(got)
    want = oracle.cluster_peaks(_np(d["snr"]), _np(d["harm"]), np.zeros(x.size, np.uint8), 6.0, 16)
    assert n == want.size and _same_records(recs, want)
    # capacity 0 still counts
    got = _ops().cluster_peaks(d["snr"], d["harm"], None, 6.0, 16, capacity=0)
    assert int(got["count"].item()) == want.size


def test_pipeline_chain_equals_oracle_chain(dev):
    """Time series -> FFT (numpy) -> inter-binned power spectrum -> greedy sum
    -> peak clustering, every step after the FFT on the GPU, against the same
    chain on the oracle."""
    N = 1 << 20
    ts = synthetic.von_mises_series(37.31, T=N * 64e-6, ts=64e-6, duty=0.05, amp=0.01)
    ts = ts + np.random.default_rng(97).normal(0.0, 1.0, size=N)
    F = np.fft.rfft(ts).astype(np.complex64)
    P_gpu = _ops().power_spectrum(torch.from_numpy(F).to(dev), True, 1.0 / N)
    P = oracle.power_spectrum(F, True, 1.0 / N)
    assert np.array_equal(_np(P_gpu).view(np.uint32), P.view(np.uint32))
    d = _ops().sum_1d(P_gpu, 32, "greedy")
    w = oracle.hs_1d(P, 32, oracle.GREEDY)
    assert np.array_equal(_np(d["harm"]), w["harm"]) and np.array_equal(_np(d["drift"]), w["drift"])
    assert np.array_equal(_np(d["snr"]).view(np.uint32), w["snr"].view(np.uint32))
    got = _ops().cluster_peaks(d["snr"], d["harm"], d["drift"], 8.0, 32)
    recs, n = _recs(got)
    want = oracle.cluster_peaks(w["snr"], w["harm"], w["drift"], 8.0, 32)
    assert n == want.size and _same_records(recs, want)
    assert n >= 1        # the injected pulsar is found
