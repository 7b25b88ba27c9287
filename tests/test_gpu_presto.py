"""GPU parity of the PRESTO-style sums (Sec. 3.2, Eq. (4), Algorithm 1) against the oracle.

Bars as for the other sums: harmonic orders (harm) bit-exact against the
oracle's float mirror, drift zero, SNR bitwise equal to the mirror and within
1e-5 * max(1, |snr|) of the float64 oracle; candidates equal as sorted sets.
"""
import numpy as np
import pytest

import oracle
import synthetic
from gpu_checks import _cands, _np, _same_records, check_dense, check_norm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MODES = {"presto": oracle.PRESTO, "presto_all": oracle.PRESTO_ALL, "presto_plus": oracle.PRESTO_PLUS}


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


@pytest.mark.parametrize("n", [2, 3, 5, 257, 4099, 65537, 300001])
@pytest.mark.parametrize("mode", sorted(MODES))
def test_presto_sizes_and_ragged_tails(dev, n, mode):
    x = synthetic.exp_noise(n, 200 + n)
    for H in (1, 3, 8, 17, 32):
        print("presto 1d", mode, n, H, flush=True)
        got = _ops().sum_1d(torch.from_numpy(x).to(dev), H, mode, with_norm=n > 2)
        check_dense(got, oracle.hs_1d(x, H, MODES[mode]), oracle.hs_1d(x, H, MODES[mode], precision="f64"),
                    "n=%d H=%d %s" % (n, H, mode))


@pytest.mark.parametrize("mode", sorted(MODES))
def test_presto_options(dev, mode):
    x, _ = synthetic.config2(n=200003, seed=71, n_trains=10)
    xt = torch.from_numpy(x).to(dev)
    cases = [dict(first_bin=7), dict(first_bin=1000), dict(fundamental_end=5000),
             dict(first_bin=3, fundamental_end=150000), dict(harmonic_mask=sum(1 << (k - 1) for k in (2, 8, 32))),
             dict(harmonic_mask=1 << 31), dict(harmonic_mask=0b1010), dict(harmonic_mask=0b100)]
    for c in cases:
        print("presto options", mode, c, flush=True)
        got = _ops().sum_1d(xt, 32, mode, with_norm=True, **c)
        check_dense(got, oracle.hs_1d(x, 32, MODES[mode], **c),
                    oracle.hs_1d(x, 32, MODES[mode], precision="f64", **c), "%s %s" % (mode, c))
        check_norm(got, x, c.get("first_bin", 1), 32, str(c))


def test_presto_h1_and_caller_normalisation(dev):
    x = synthetic.exp_noise(70001, 73)
    xt = torch.from_numpy(x).to(dev)
    got = _ops().sum_1d(xt, 1, "presto_plus", norm=(0.0, 1.0))
    assert np.array_equal(_np(got["snr"])[1:], x[1:]) and _np(got["snr"])[0] == 0
    assert np.all(_np(got["harm"])[1:] == 1)
    for mode in ("presto", "presto_all"):
        got = _ops().sum_1d(xt, 1, mode)
        assert not _np(got["snr"]).any() and not _np(got["harm"]).any()
    for mode in sorted(MODES):
        for norm in ((1.25, 0.75), (0.0, 0.0), (float("nan"), 1.0)):
            got = _ops().sum_1d(xt, 16, mode, norm=norm)
            check_dense(got, oracle.hs_1d(x, 16, MODES[mode], norm=norm), None, "%s norm %r" % (mode, norm))


@pytest.mark.parametrize("mode", sorted(MODES))
def test_presto_fp16_storage(dev, mode):
    x, _ = synthetic.config2(n=(1 << 19) + 13, seed=74)
    mu1, _ = oracle.stats(x)
    q = oracle.quantize_f16(x, np.float32(mu1))
    dec = q.astype(np.float32)
    got = _ops().sum_1d(torch.from_numpy(q.view(np.int16)).to(dev).view(torch.float16), 32, mode, with_norm=True)
    check_dense(got, oracle.hs_1d(dec, 32, MODES[mode]), oracle.hs_1d(dec, 32, MODES[mode], precision="f64"),
                "fp16 " + mode)
    check_norm(got, dec, 1, 32, "fp16 " + mode)


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("f16", [False, True])
@pytest.mark.parametrize("H", [13, 32])
def test_presto_batched_small(dev, mode, f16, H):
    B = 37
    x, off = synthetic.config3(n_spectra=B, lo=2, hi=90000, seed=75)
    thr = 4.0
    if f16:
        x = oracle.quantize_f16(x, np.float32(1.0)).astype(np.float32)
        xt = torch.from_numpy(x.astype(np.float16).view(np.int16)).to(dev).view(torch.float16)
    else:
        xt = torch.from_numpy(x).to(dev)
    ot = torch.from_numpy(off).to(dev)
    print("presto batched", mode, f16, H, flush=True)
    got = _ops().sum_batched(xt, ot, H, mode, thr, dense=True, candidates=True, capacity=x.size, with_norm=True)
    w = oracle.hs_batched(x, off, H, MODES[mode], thr, dense=True)
    for s in range(B):
        sl = slice(off[s], off[s + 1])
        w64 = oracle.hs_1d(x[sl], H, MODES[mode], precision="f64")
        check_dense({k: got[k][sl] for k in ("snr", "harm", "drift")}, w["spectra"][s], w64, "spectrum %d" % s)
    recs, n = _cands(got)
    assert n == w["candidates"].size
    assert _same_records(recs, w["candidates"])


def test_presto_batched_equals_1d(dev):
    x, off = synthetic.config3(n_spectra=5, lo=50000, hi=120000, seed=76)
    xt, ot = torch.from_numpy(x).to(dev), torch.from_numpy(off).to(dev)
    for mode in sorted(MODES):
        got = _ops().sum_batched(xt, ot, 32, mode, 6.0, dense=True, candidates=False)
        for s in range(5):
            one = _ops().sum_1d(xt[off[s]:off[s + 1]].clone(), 32, mode)
            for k in ("snr", "harm", "drift"):
                assert torch.equal(got[k][off[s]:off[s + 1]], one[k]), (mode, s, k)


def test_presto_unsupported_calls(dev):
    from paper_2202_12817_amd import hs
    plan = _ops().make_plan(8, "presto_plus")
    try:
        x = torch.ones((3, 100), dtype=torch.float32, device=dev)
        snr = torch.empty((3, 100), dtype=torch.float32, device=dev)
        harm = torch.empty((3, 100), dtype=torch.uint8, device=dev)
        with pytest.raises(hs.HsError) as e:
            hs.hs_sum_2d(plan.handle, x, 100, 100, -1, 1, None, snr, harm, None, None, 0, None, None)
        assert e.value.status == hs.HS_ERR_UNSUPPORTED
        with pytest.raises(hs.HsError) as e:
            hs.hs_plan_set_launch(plan.handle, 2, 1)
        assert e.value.status == hs.HS_ERR_UNSUPPORTED
    finally:
        plan.close()


@pytest.mark.parametrize("mode", sorted(MODES))
def test_table2_workload_sampled(dev, mode):
    """The paper's performance shape (1024 spectra of 2^17 bins, H = 32), in the
    launch the benchmark times: dense outputs and SNR > 6 candidates, checked on
    sampled spectra against the oracle."""
    x, off = synthetic.table2()
    xt, ot = torch.from_numpy(x).to(dev), torch.from_numpy(off).to(dev)
    print("table2", mode, flush=True)
    got = _ops().sum_batched(xt, ot, 32, mode, 6.0, dense=True, candidates=True, capacity=1 << 22,
                             with_norm=True)
    recs, n = _cands(got)
    assert n == recs.size
    for s in (0, 1, 511, 1000, 1023):
        sl = slice(off[s], off[s + 1])
        w32 = oracle.hs_1d(x[sl], 32, MODES[mode])
        check_dense({k: got[k][sl] for k in ("snr", "harm", "drift")}, w32, None, "%s spectrum %d" % (mode, s))
        wc = oracle.candidates(w32["snr"], w32["harm"], w32["drift"], 6.0, spectrum=s)
        assert _same_records(recs[recs["spectrum"] == s], wc), s
    del xt, got


@pytest.mark.slow
def test_presto_plus_max_length(dev):
    """PRESTO+ (and PRESTO) on the longest spectrum a call accepts, 2^30 - 1
    FP32 bins, H = 32: every bin offset of every chain stays in 32 bits;
    sampled last bins (both ends, random) against the oracle."""
    n = (1 << 30) - 1
    x = synthetic.exp_noise(n, 94)
    mu1, sigma1 = oracle.norm_from_data(x, 1)
    xt = torch.from_numpy(x).to(dev)
    g = np.random.default_rng(94)
    idx = np.unique(np.concatenate([np.arange(0, 2000), np.arange(n - 2000, n), g.integers(0, n, 20000)]))
    it = torch.from_numpy(idx).to(dev)
    for mode in ("presto_plus", "presto"):
        print("presto max length", mode, flush=True)
        w = oracle.hs_1d(x, 32, MODES[mode], norm=(mu1, sigma1), idx=idx)
        got = _ops().sum_1d(xt, 32, mode, with_norm=True)
        ms = _np(got["mu_sigma"])[0]
        assert (ms[0], ms[1]) == (mu1, sigma1)
        check_dense({k: got[k][it] for k in ("snr", "harm", "drift")}, w, None, "max length " + mode)
        del got
