"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars (written out per check below):
* harmonic counts, drifts, candidate bins: bit-exact against the oracle's
  float mirror (precision "f32"), which takes the argmax in the same precision
  as the kernels;
* SNR: bitwise equal to the float mirror as well, and within
  1e-5 * max(1, |snr|) of the float64 oracle (the stated tolerance; the
  floor of 1 covers the cancellation S_k - mu_k near zero SNR);
* statistics (mu1, sigma1) and the float tables: bitwise equal to the
  oracle's exactly rounded values.
"""
import numpy as np
import pytest

import oracle
import synthetic
from gpu_checks import TOL, _cands, _np, _same_records, check_dense, check_norm  # noqa: F401

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MODES = {"standard": oracle.STANDARD, "greedy": oracle.GREEDY}


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


# ---------------------------------------------------------------------------
# 1D
# ---------------------------------------------------------------------------

def test_config1_standard_and_greedy_with_partials(dev):
    x, noise = synthetic.config1()
    xt = torch.from_numpy(x).to(dev)
    for mode in ("standard", "greedy"):
        print("config1", mode, flush=True)
        got = _ops().sum_1d(xt, 8, mode, report=(1, 2, 4, 8), with_norm=True)
        w32 = oracle.hs_1d(x, 8, MODES[mode], report=(1, 2, 4, 8))
        w64 = oracle.hs_1d(x, 8, MODES[mode], precision="f64")
        check_dense(got, w32, w64, "config1 " + mode)
        check_norm(got, x, 1, 8, "config1")
        assert np.array_equal(_np(got["partial"]).view(np.uint32), w32["partial"].view(np.uint32))
    # the injected train at bin 1234: K-harmonic excess 8 H_K (simple sum)
    got = _ops().sum_1d(xt, 8, "standard", report=(1, 2, 4, 8))
    P = _np(got["partial"])[:, 1234].astype(np.float64)
    for row, K in enumerate((1, 2, 4, 8)):
        excess = P[row] - sum(float(noise[1234 * k]) for k in range(1, K + 1))
        assert abs(excess - 8.0 * sum(1.0 / k for k in range(1, K + 1))) < 1e-4


SIZES = [2, 3, 5, 255, 256, 257, 1000, 4099, 65537, 300001]


@pytest.mark.parametrize("kernel", ["persistent", "plain"])
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_1d_sizes_and_ragged_tails(dev, n, mode, kernel):
    x = synthetic.exp_noise(n, 100 + n)
    for H in (1, 3, 8, 17, 32):
        print("1d", kernel, n, mode, H, flush=True)
        got = _ops().sum_1d(torch.from_numpy(x).to(dev), H, mode, with_norm=n > 2, kernel=kernel)
        check_dense(got, oracle.hs_1d(x, H, MODES[mode]), oracle.hs_1d(x, H, MODES[mode], precision="f64"),
                    "n=%d H=%d %s %s" % (n, H, mode, kernel))


@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_1d_options(dev, mode):
    x, _ = synthetic.config2(n=200003, seed=31, n_trains=10)
    xt = torch.from_numpy(x).to(dev)
    cases = [dict(first_bin=7), dict(fundamental_end=5000), dict(first_bin=3, fundamental_end=150000),
             dict(harmonic_mask=sum(1 << (k - 1) for k in (1, 2, 4, 8, 16, 32))),
             dict(harmonic_mask=1 << 31), dict(harmonic_mask=0b1010)]
    for c in cases:
        print("options", mode, c, flush=True)
        got = _ops().sum_1d(xt, 32, mode, with_norm=True, **c)
        check_dense(got, oracle.hs_1d(x, 32, MODES[mode], **c), oracle.hs_1d(x, 32, MODES[mode], precision="f64", **c),
                    "%s %s" % (mode, c))
        check_norm(got, x, c.get("first_bin", 1), 32, str(c))


@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_1d_caller_normalisation(dev, mode):
    x = synthetic.exp_noise(70001, 41)
    xt = torch.from_numpy(x).to(dev)
    # H = 1 with mu1 = 0, sigma1 = 1 returns the input (simple) / the larger neighbour (greedy)
    got = _ops().sum_1d(xt, 1, mode, norm=(0.0, 1.0))
    snr = _np(got["snr"])
    if mode == "standard":
        assert np.array_equal(snr[1:], x[1:]) and snr[0] == 0
    else:
        want = np.where(x[2:] > x[1:-1], x[2:], x[1:-1])
        assert np.array_equal(snr[1:-1], want) and snr[-1] == 0
        assert np.array_equal(_np(got["drift"])[1:-1], (x[2:] > x[1:-1]).astype(np.uint8))
    for norm in ((1.25, 0.75), (0.0, 0.0), (float("nan"), 1.0)):
        got = _ops().sum_1d(xt, 16, mode, norm=norm)
        check_dense(got, oracle.hs_1d(x, 16, MODES[mode], norm=norm), None, "norm %r" % (norm,))


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_1d_unaligned_start(dev, shift):
    x = synthetic.exp_noise(100003, 43)
    buf = torch.zeros(x.size + 8, dtype=torch.float32, device=dev)
    buf[shift:shift + x.size] = torch.from_numpy(x).to(dev)
    got = _ops().sum_1d(buf[shift:shift + x.size], 32, "greedy", with_norm=True)
    check_dense(got, oracle.hs_1d(x, 32, oracle.GREEDY), None, "shift %d" % shift)
    check_norm(got, x, 1, 32, "shift %d" % shift)


def test_1d_degenerate_spectrum_gives_zeros(dev):
    x = np.full(5000, 2.5, dtype=np.float32)
    for mode in ("standard", "greedy"):
        got = _ops().sum_1d(torch.from_numpy(x).to(dev), 8, mode, with_norm=True)
        assert not _np(got["snr"]).any() and not _np(got["harm"]).any() and not _np(got["drift"]).any()
        assert int(_np(got["valid"])[0]) == 0


@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_config2_full_size(dev, mode):
    x, _ = synthetic.config2()
    print("config2", mode, flush=True)
    xt = torch.from_numpy(x).to(dev)
    got = _ops().sum_1d(xt, 32, mode, with_norm=True)
    check_dense(got, oracle.hs_1d(x, 32, MODES[mode]), oracle.hs_1d(x, 32, MODES[mode], precision="f64"),
                "config2 " + mode)
    check_norm(got, x, 1, 32, "config2")
    plain = _ops().sum_1d(xt, 32, mode, kernel="plain")
    for k in ("snr", "harm", "drift"):
        assert torch.equal(plain[k], got[k]), k


def test_1d_deterministic(dev):
    x, _ = synthetic.config2(n=1 << 20, seed=8)
    xt = torch.from_numpy(x).to(dev)
    a = _ops().sum_1d(xt, 32, "greedy")
    b = _ops().sum_1d(xt, 32, "greedy")
    for k in ("snr", "harm", "drift"):
        assert torch.equal(a[k], b[k])


# ---------------------------------------------------------------------------
# FP16 storage
# ---------------------------------------------------------------------------

def test_quantize_f16_bitwise(dev):
    x, _ = synthetic.config2(n=300007, seed=51)
    x[:3] = [0.0, 1e9, 7e4]
    scale = np.float32(0.87)
    got = _ops().quantize_f16(torch.from_numpy(x).to(dev), float(scale))
    want = oracle.quantize_f16(x, scale)
    assert np.array_equal(_np(got).view(np.uint16), want.view(np.uint16))


@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_fp16_storage_sums(dev, mode):
    x, _ = synthetic.config2(n=(1 << 20) + 13, seed=52)
    mu1, _ = oracle.stats(x)
    q = oracle.quantize_f16(x, np.float32(mu1))
    dec = q.astype(np.float32)
    got = _ops().sum_1d(torch.from_numpy(q.view(np.int16)).to(dev).view(torch.float16), 32, mode, with_norm=True)
    check_dense(got, oracle.hs_1d(dec, 32, MODES[mode]), oracle.hs_1d(dec, 32, MODES[mode], precision="f64"),
                "fp16 " + mode)
    check_norm(got, dec, 1, 32, "fp16")


# ---------------------------------------------------------------------------
# batched
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["persistent", "plain"])
@pytest.mark.parametrize("mode", ["standard", "greedy"])
@pytest.mark.parametrize("f16", [False, True])
@pytest.mark.parametrize("H", [13, 32])
def test_batched_small(dev, mode, f16, kernel, H):
    B = 37
    x, off = synthetic.config3(n_spectra=B, lo=2, hi=90000, seed=61)
    thr = 4.0
    if f16:
        x = oracle.quantize_f16(x, np.float32(1.0)).astype(np.float32)
        xt = torch.from_numpy(x.astype(np.float16).view(np.int16)).to(dev).view(torch.float16)
    else:
        xt = torch.from_numpy(x).to(dev)
    ot = torch.from_numpy(off).to(dev)
    print("batched", mode, f16, kernel, H, flush=True)
    got = _ops().sum_batched(xt, ot, H, mode, thr, dense=True, candidates=True, capacity=x.size,
                             with_norm=True, kernel=kernel)
    w = oracle.hs_batched(x, off, H, MODES[mode], thr, dense=True)
    ms = _np(got["mu_sigma"])
    for s in range(B):
        sl = slice(off[s], off[s + 1])
        w32 = w["spectra"][s]
        w64 = oracle.hs_1d(x[sl], H, MODES[mode], precision="f64")
        check_dense({k: got[k][sl] for k in ("snr", "harm", "drift")}, w32, w64, "spectrum %d" % s)
        if off[s + 1] - off[s] > 1:
            assert (ms[s, 0], ms[s, 1]) == (w32["mu1"], w32["sigma1"]) or not np.isfinite(w32["sigma1"])
    recs, n = _cands(got)
    assert n == w["candidates"].size
    assert _same_records(recs, w["candidates"])


def test_batched_candidate_overflow(dev):
    x, off = synthetic.config3(n_spectra=8, lo=20000, hi=40000, seed=62)
    w = oracle.hs_batched(x, off, 16, oracle.GREEDY, 2.0)["candidates"]
    assert w.size > 100
    cap = w.size // 3
    got = _ops().sum_batched(torch.from_numpy(x).to(dev), torch.from_numpy(off).to(dev), 16, "greedy", 2.0,
                             capacity=cap)
    recs, n = _ops().candidates_numpy(got)
    assert n == w.size and recs.size == cap
    # every written record is a true candidate, no duplicates
    key = lambda r: (int(r["spectrum"]), int(r["bin"]))  # noqa: E731
    truth = {key(r): r for r in w}
    seen = set()
    for r in recs:
        k = key(r)
        assert k in truth and k not in seen
        seen.add(k)
        t = truth[k]
        assert (r["harm"], r["drift"], r["snr"]) == (t["harm"], t["drift"], t["snr"])
    # zero capacity still counts
    got = _ops().sum_batched(torch.from_numpy(x).to(dev), torch.from_numpy(off).to(dev), 16, "greedy", 2.0,
                             capacity=0)
    assert int(got["count"].item()) == w.size


def test_batched_equals_1d(dev):
    x, off = synthetic.config3(n_spectra=5, lo=50000, hi=120000, seed=63)
    xt, ot = torch.from_numpy(x).to(dev), torch.from_numpy(off).to(dev)
    got = _ops().sum_batched(xt, ot, 32, "greedy", 6.0, dense=True, candidates=False)
    for s in range(5):
        one = _ops().sum_1d(xt[off[s]:off[s + 1]].clone(), 32, "greedy")
        for k in ("snr", "harm", "drift"):
            assert torch.equal(got[k][off[s]:off[s + 1]], one[k])


@pytest.mark.slow
def test_config3_full_size_sampled(dev):
    """The batched workload at full size (512 spectra, 2^20..2^22 bins, H = 32, greedy,
    SNR > 6 candidates), checked on a sample of spectra against the oracle."""
    x, off = synthetic.config3()
    xt, ot = torch.from_numpy(x).to(dev), torch.from_numpy(off).to(dev)
    print("config3 full size: %d bins" % x.size, flush=True)
    got = _ops().sum_batched(xt, ot, 32, "greedy", 6.0, capacity=1 << 23, with_norm=True)
    recs, n = _cands(got)
    assert n == recs.size
    ms = _np(got["mu_sigma"])
    for s in (0, 1, 100, 255, 256, 400, 511):
        sl = slice(off[s], off[s + 1])
        w = oracle.hs_1d(x[sl], 32, oracle.GREEDY)
        assert (ms[s, 0], ms[s, 1]) == (w["mu1"], w["sigma1"]), s
        wc = oracle.candidates(w["snr"], w["harm"], w["drift"], 6.0, spectrum=s)
        assert _same_records(recs[recs["spectrum"] == s], wc), s
    del xt


def test_batched_max_spectra(dev):
    """The most spectra one call accepts (65535), lengths 2..40 (length 2: no
    fundamental sums a harmonic beyond the fundamental step), greedy H = 32:
    sampled spectra checked against the oracle, dense and candidates."""
    B = 65535
    g = np.random.default_rng(92)
    lengths = g.integers(2, 41, size=B)
    off = np.zeros(B + 1, dtype=np.int64)
    off[1:] = np.cumsum(lengths)
    x = synthetic.exp_noise(int(off[-1]), 92)
    xt, ot = torch.from_numpy(x).to(dev), torch.from_numpy(off).to(dev)
    got = _ops().sum_batched(xt, ot, 32, "greedy", 3.0, dense=True, candidates=True, capacity=x.size,
                             with_norm=True)
    sample = np.unique(np.concatenate([np.arange(50), np.arange(B - 50, B), g.choice(B, 1500, replace=False)]))
    w = oracle.hs_batched(x, off, 32, oracle.GREEDY, 3.0, dense=True, spectra=sample)
    ms = _np(got["mu_sigma"])
    for s in sample:
        sl = slice(off[s], off[s + 1])
        w32 = w["spectra"][s]
        check_dense({k: got[k][sl] for k in ("snr", "harm", "drift")}, w32, None, "spectrum %d" % s)
        assert (ms[s, 0], ms[s, 1]) == (w32["mu1"], w32["sigma1"]) or not np.isfinite(w32["sigma1"])
    recs, n = _cands(got)
    keep = np.isin(recs["spectrum"], sample)
    assert _same_records(recs[keep], w["candidates"])


@pytest.mark.slow
def test_1d_max_length(dev):
    """The longest spectrum a call accepts, 2^30 - 1 FP32 bins (4 GiB), greedy
    H = 32, both kernels: exact statistics, and sampled fundamentals (both
    ends, every harmonic-count boundary, random bins)."""
    n = (1 << 30) - 1
    x = synthetic.exp_noise(n, 93)
    print("1d max length: statistics", flush=True)
    mu1, sigma1 = oracle.norm_from_data(x, 1)
    xt = torch.from_numpy(x).to(dev)
    g = np.random.default_rng(93)
    edges = [(n - 1) // (k + 1) - 1 for k in range(1, 33)]   # greedy K changes after these bins
    idx = np.unique(np.concatenate([np.arange(0, 3000), np.arange(n - 3000, n), g.integers(0, n, 20000),
                                    np.array([e + dlt for e in edges for dlt in (-2, -1, 0, 1, 2)])]))
    idx = idx[(idx >= 0) & (idx < n)]
    w = oracle.hs_1d(x, 32, oracle.GREEDY, norm=(mu1, sigma1), idx=idx)
    it = torch.from_numpy(idx).to(dev)
    for kernel in ("plain", "persistent"):
        got = _ops().sum_1d(xt, 32, "greedy", with_norm=True, kernel=kernel)
        ms = _np(got["mu_sigma"])[0]
        assert (ms[0], ms[1]) == (mu1, sigma1)
        check_dense({k: got[k][it] for k in ("snr", "harm", "drift")}, w, None, "1d max length " + kernel)
        del got


# ---------------------------------------------------------------------------
# 2D
# ---------------------------------------------------------------------------

def _plane(n_z, n_r, seed):
    g = np.random.default_rng(seed)
    return g.standard_exponential((n_z, n_r)).astype(np.float32)


@pytest.mark.parametrize("mode", ["standard", "greedy"])
@pytest.mark.parametrize("shape", [(-3, 4, 1000), (0, 0, 5000), (-7, -2, 777), (2, 9, 3001), (-20, 20, 20011)])
def test_2d_dense(dev, mode, shape):
    z_min, z_max, n_r = shape
    p = _plane(z_max - z_min + 1, n_r, n_r)
    for H in (4, 16):
        print("2d", mode, shape, H, flush=True)
        got = _ops().sum_2d(torch.from_numpy(p).to(dev), z_min, z_max, H, mode, with_norm=True)
        check_dense(got, oracle.hs_2d(p, z_min, z_max, H, MODES[mode]),
                    oracle.hs_2d(p, z_min, z_max, H, MODES[mode], precision="f64"), "2d %s %s" % (mode, shape))
        check_norm(got, p, 1, H, "2d")


@pytest.mark.parametrize("mode", ["standard", "greedy"])
@pytest.mark.parametrize("shape", [(-20, 20, 20011), (-100, 100, 3001), (3, 11, 9000), (-13, -1, 7001),
                                   (-2, 30, 12007), (-126, 126, 700), (-130, 130, 300), (-1, 1, 65537)])
@pytest.mark.parametrize("opts", [{}, {"first_bin": 5, "fundamental_end": 1700, "harmonic_mask": 0b1010101010}])
@pytest.mark.parametrize("H", [5, 16, 32])
def test_2d_ray_tiles_equal_plain_kernel(dev, mode, shape, opts, H):
    """The ray-tiled plane kernel against the one-thread-per-fundamental kernel,
    bit for bit, and against the oracle; z ranges of one side, both sides, beyond the
    tile budget (the default falls back to the plain kernel) and a ragged last tile."""
    z_min, z_max, n_r = shape
    p = _plane(z_max - z_min + 1, n_r, n_r + 3)
    pt = torch.from_numpy(p).to(dev)
    print("2d ray", mode, shape, opts, H, flush=True)
    got = _ops().sum_2d(pt, z_min, z_max, H, mode, candidates=True, threshold=3.5, capacity=p.size,
                        kernel="persistent", **opts)
    ref = _ops().sum_2d(pt, z_min, z_max, H, mode, candidates=True, threshold=3.5, capacity=p.size,
                        kernel="plain", **opts)
    for k in ("harm", "drift"):
        assert torch.equal(got[k], ref[k]), k
    assert torch.equal(got["snr"].view(torch.int32), ref["snr"].view(torch.int32))
    ra, na = _cands(got)
    rb, nb = _cands(ref)
    assert na == nb and _same_records(ra, rb)
    if p.size <= 2_000_000 and H != 5:
        w = oracle.hs_2d(p, z_min, z_max, H, MODES[mode], **opts)
        check_dense(got, w, None, "2d ray %s %s" % (mode, shape))


@pytest.mark.parametrize("kernel", ["auto", "persistent"])
@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_2d_fp16_storage(dev, mode, kernel):
    z_min, z_max, n_r = -9, 9, 30011
    p = _plane(z_max - z_min + 1, n_r, 77)
    q = oracle.quantize_f16(p.reshape(-1), np.float32(1.0)).reshape(p.shape)
    dec = q.astype(np.float32)
    pt = torch.from_numpy(q.view(np.int16)).to(dev).view(torch.float16)
    got = _ops().sum_2d(pt, z_min, z_max, 16, mode, with_norm=True, kernel=kernel)
    check_dense(got, oracle.hs_2d(dec, z_min, z_max, 16, MODES[mode]),
                oracle.hs_2d(dec, z_min, z_max, 16, MODES[mode], precision="f64"), "2d fp16 " + mode)
    check_norm(got, dec, 1, 16, "2d fp16")


def test_2d_strided_rows_and_candidates(dev):
    z_min, z_max, n_r, stride = -5, 5, 4000, 4100
    full = _plane(z_max - z_min + 1, stride, 9)
    pt = torch.from_numpy(full).to(dev)[:, :n_r]
    p = full[:, :n_r].copy()
    got = _ops().sum_2d(pt, z_min, z_max, 16, "greedy", candidates=True, threshold=3.0, capacity=p.size)
    w = oracle.hs_2d(p, z_min, z_max, 16, oracle.GREEDY)
    check_dense(got, w, None, "strided")
    recs, n = _cands(got)
    wc = oracle.candidates(w["snr"].reshape(-1), w["harm"].reshape(-1), w["drift"].reshape(-1), 3.0)
    assert n == wc.size and _same_records(recs, wc)


def test_2d_max_rows(dev):
    """The most rows a plane may have (65535, z = -32767..32767), 48 columns,
    greedy H = 16: every row's harmonic rows k z stay inside the plane only
    for small |z|, the truncation rule is exercised on every row."""
    z_min, z_max, n_r = -32767, 32767, 48
    p = _plane(z_max - z_min + 1, n_r, 94)
    got = _ops().sum_2d(torch.from_numpy(p).to(dev), z_min, z_max, 16, "greedy", with_norm=True)
    check_dense(got, oracle.hs_2d(p, z_min, z_max, 16, oracle.GREEDY), None, "2d max rows")
    check_norm(got, p, 1, 16, "2d max rows")


@pytest.mark.slow
@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_config4_full_size_sampled_rows(dev, mode):
    plane, _ = synthetic.config4()
    z_min, z_max = -100, 100
    print("config4 full size", mode, flush=True)
    got = _ops().sum_2d(torch.from_numpy(plane).to(dev), z_min, z_max, 16, mode, with_norm=True)
    mu1, sigma1 = oracle.norm_from_data(plane, 1)
    ms = _np(got["mu_sigma"])[0]
    assert (ms[0], ms[1]) == (mu1, sigma1)
    n_r = plane.shape[1]
    rows = [0, 50, 94, 99, 100, 101, 106, 150, 200]
    idx = np.concatenate([np.arange(i * n_r, (i + 1) * n_r) for i in rows])
    w = oracle.hs_2d(plane, z_min, z_max, 16, MODES[mode], norm=(mu1, sigma1), idx=idx)
    sub = {k: got[k].reshape(-1)[torch.from_numpy(idx).to(dev)] for k in ("snr", "harm", "drift")}
    check_dense(sub, w, None, "config4 rows")
