"""GPU parity at the edges of the boundary: up to 64 harmonics, caller per-k
normalisation tables, candidates exactly at the threshold, and non-finite
SNRs from a caller normalisation.

Bars as in test_gpu_parity: harmonic counts, drifts and candidate bins
bit-exact against the oracle's float mirror, SNR bitwise equal to it and
within 1e-5 * max(1, |snr|) of the float64 oracle.
"""
import math

import numpy as np
import pytest

import oracle
import synthetic
from golden_io import read_candidates
from gpu_checks import _cands, _np, _same_records, check_dense

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
# H up to 64
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["persistent", "plain"])
@pytest.mark.parametrize("mode", ["standard", "greedy"])
@pytest.mark.parametrize("n", [3, 257, 4099, 65537, 300001])
def test_1d_up_to_64_harmonics(dev, n, mode, kernel):
    x = synthetic.exp_noise(n, 500 + n)
    xt = torch.from_numpy(x).to(dev)
    for H in (33, 48, 64):
        print("1d H", H, n, mode, kernel, flush=True)
        got = _ops().sum_1d(xt, H, mode, kernel=kernel)
        check_dense(got, oracle.hs_1d(x, H, MODES[mode]), oracle.hs_1d(x, H, MODES[mode], precision="f64"),
                    "n=%d H=%d %s %s" % (n, H, mode, kernel))


def test_1d_64_harmonics_masks_and_partials(dev):
    x, _ = synthetic.config2(n=70001, seed=33, n_trains=6, max_harm=64)
    xt = torch.from_numpy(x).to(dev)
    for c in (dict(harmonic_mask=1 << 63), dict(harmonic_mask=(1 << 40) | (1 << 47) | 1),
              dict(report=(1, 33, 64))):
        print("1d H=64", c, flush=True)
        got = _ops().sum_1d(xt, 64, "greedy", **c)
        w = oracle.hs_1d(x, 64, oracle.GREEDY, **c)
        check_dense(got, w, None, "H=64 %s" % c)
        if "report" in c:
            assert np.array_equal(_np(got["partial"]).view(np.uint32), w["partial"].view(np.uint32))


@pytest.mark.parametrize("kernel", ["persistent", "plain"])
@pytest.mark.parametrize("f16", [False, True])
@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_batched_64_harmonics(dev, mode, f16, kernel):
    B, H, thr = 21, 64, 4.0
    x, off = synthetic.config3(n_spectra=B, lo=2, hi=120000, seed=71)
    if f16:
        x = oracle.quantize_f16(x, np.float32(1.0)).astype(np.float32)
        xt = torch.from_numpy(x.astype(np.float16).view(np.int16)).to(dev).view(torch.float16)
    else:
        xt = torch.from_numpy(x).to(dev)
    print("batched H=64", mode, f16, kernel, flush=True)
    got = _ops().sum_batched(xt, torch.from_numpy(off).to(dev), H, mode, thr, dense=True, capacity=x.size,
                             kernel=kernel)
    w = oracle.hs_batched(x, off, H, MODES[mode], thr, dense=True)
    for s in range(B):
        sl = slice(off[s], off[s + 1])
        check_dense({k: got[k][sl] for k in ("snr", "harm", "drift")}, w["spectra"][s], None, "spectrum %d" % s)
    recs, n = _cands(got)
    assert n == w["candidates"].size and _same_records(recs, w["candidates"])


@pytest.mark.parametrize("kernel", ["auto", "persistent"])
@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_2d_48_harmonics(dev, mode, kernel):
    z_min, z_max, n_r = -3, 5, 40001
    g = np.random.default_rng(72)
    p = g.standard_exponential((z_max - z_min + 1, n_r)).astype(np.float32)
    print("2d H=48", mode, kernel, flush=True)
    got = _ops().sum_2d(torch.from_numpy(p).to(dev), z_min, z_max, 48, mode, kernel=kernel)
    check_dense(got, oracle.hs_2d(p, z_min, z_max, 48, MODES[mode]),
                oracle.hs_2d(p, z_min, z_max, 48, MODES[mode], precision="f64"), "2d H=48 " + mode)


@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_interleaved_64_harmonics(dev, mode):
    B, N, H = 70, 20011, 64
    g = np.random.default_rng(73)
    x = g.standard_exponential((B, N)).astype(np.float32)
    xi = torch.from_numpy(np.ascontiguousarray(x.T)).to(dev)
    print("interleaved H=64", mode, flush=True)
    got = _ops().sum_interleaved(xi, H, mode)
    for s in (0, 33, 69):
        w = oracle.hs_1d(x[s], H, MODES[mode])
        check_dense({k: got[k][:, s] for k in ("snr", "harm", "drift")}, w, None, "column %d" % s)


# ---------------------------------------------------------------------------
# caller per-k tables (Eq. (2): mean and deviation of a k-element sum)
# ---------------------------------------------------------------------------

def _table(H, seed):
    g = np.random.default_rng(seed)
    mu = np.cumsum(g.uniform(0.8, 1.6, H))
    sig = np.sqrt(np.cumsum(g.uniform(0.7, 1.4, H)))
    return mu, sig


@pytest.mark.parametrize("kernel", ["persistent", "plain"])
@pytest.mark.parametrize("mode", ["standard", "greedy"])
@pytest.mark.parametrize("H", [7, 32, 64])
def test_1d_table_normalisation(dev, mode, kernel, H):
    x = synthetic.exp_noise(90001, 74)
    mu, sig = _table(H, H)
    print("1d table", mode, kernel, H, flush=True)
    got = _ops().sum_1d(torch.from_numpy(x).to(dev), H, mode, norm_table=np.stack([mu, sig]), with_norm=True,
                        kernel=kernel)
    check_dense(got, oracle.hs_1d(x, H, MODES[mode], norm_table=(mu, sig)),
                oracle.hs_1d(x, H, MODES[mode], norm_table=(mu, sig), precision="f64"), "table H=%d" % H)
    _, _, rs, nm, ok = oracle.caller_tables(mu, sig)
    tab = _np(got["tables"])[0]
    assert ok and np.array_equal(tab[0], rs) and np.array_equal(tab[1], nm)
    assert tuple(_np(got["mu_sigma"])[0]) == (mu[0], sig[0]) and int(_np(got["valid"])[0]) == 1


@pytest.mark.parametrize("kernel", ["persistent", "plain"])
def test_batched_table_normalisation(dev, kernel):
    B, H = 9, 32
    x, off = synthetic.config3(n_spectra=B, lo=1000, hi=60000, seed=75)
    tabs = [_table(H, 100 + s) for s in range(B)]
    tabs[4] = (tabs[4][0], np.where(np.arange(H) == 20, 0.0, tabs[4][1]))   # sigma_21 = 0: spectrum 4 unusable
    arr = np.stack([np.stack(t) for t in tabs])                              # [B][2][H]
    print("batched table", kernel, flush=True)
    got = _ops().sum_batched(torch.from_numpy(x).to(dev), torch.from_numpy(off).to(dev), H, "greedy", 3.0,
                             dense=True, capacity=x.size, norm_table=arr, kernel=kernel, with_norm=True)
    w = oracle.hs_batched(x, off, H, oracle.GREEDY, 3.0, dense=True, norm_tables=tabs)
    for s in range(B):
        sl = slice(off[s], off[s + 1])
        check_dense({k: got[k][sl] for k in ("snr", "harm", "drift")}, w["spectra"][s], None, "spectrum %d" % s)
    assert int(_np(got["valid"])[4]) == 0 and not _np(got["harm"][off[4]:off[5]]).any()
    recs, n = _cands(got)
    assert n == w["candidates"].size and _same_records(recs, w["candidates"])


@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_2d_and_interleaved_table_normalisation(dev, mode):
    H = 16
    mu, sig = _table(H, 76)
    z_min, z_max, n_r = -4, 4, 9001
    g = np.random.default_rng(77)
    p = g.standard_exponential((z_max - z_min + 1, n_r)).astype(np.float32)
    got = _ops().sum_2d(torch.from_numpy(p).to(dev), z_min, z_max, H, mode, norm_table=np.stack([mu, sig]))
    check_dense(got, oracle.hs_2d(p, z_min, z_max, H, MODES[mode], norm_table=(mu, sig)), None, "2d table")
    from paper_2202_12817_amd import hs
    B, N = 5, 3001
    x = g.standard_exponential((B, N)).astype(np.float32)
    tabs = [_table(H, 200 + s) for s in range(B)]
    xi = torch.from_numpy(np.ascontiguousarray(x.T)).to(dev)
    plan = _ops().make_plan(H, mode, max_spectra=B, norm_table=True)
    nt = torch.from_numpy(np.stack([np.stack(t) for t in tabs]).reshape(-1)).to(dev)
    snr = torch.empty((N, B), dtype=torch.float32, device=dev)
    harm = torch.empty((N, B), dtype=torch.uint8, device=dev)
    drift = torch.empty((N, B), dtype=torch.uint8, device=dev)
    hs.hs_sum_interleaved(plan.handle, xi, N, B, nt, snr, harm, drift)
    torch.cuda.synchronize()
    plan.close()
    for s in range(B):
        w = oracle.hs_1d(x[s], H, MODES[mode], norm_table=tabs[s])
        check_dense({"snr": snr[:, s], "harm": harm[:, s], "drift": drift[:, s]}, w, None, "interleaved %d" % s)


def test_table_mode_needs_the_table(dev):
    from paper_2202_12817_amd import hs
    x = torch.ones(1000, dtype=torch.float32, device=dev)
    out = [torch.empty(1000, dtype=t, device=dev) for t in (torch.float32, torch.uint8, torch.uint8)]
    with hs.Plan(harmonics=8, norm_kind=hs.HS_NORM_TABLE) as plan:
        with pytest.raises(hs.HsError) as e:
            hs.hs_sum_1d(plan.handle, x, 1000, None, *out)
        assert e.value.status == hs.HS_ERR_ARG


# ---------------------------------------------------------------------------
# candidates exactly at the threshold (reading: strict snr > threshold)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["persistent", "plain"])
def test_hand_candidates_at_threshold(dev, kernel):
    values, offsets, cases = read_candidates()
    xt, ot = torch.from_numpy(values).to(dev), torch.from_numpy(offsets).to(dev)
    for c in cases:
        mode = c["mode"]
        got = _ops().sum_batched(xt, ot, c["H"], mode, c["thr"], harmonic_mask=c["mask"], capacity=64,
                                 kernel=kernel)
        recs, n = _cands(got)
        have = sorted((int(r["spectrum"]), int(r["bin"]), float(r["snr"]), int(r["harm"]), int(r["drift"]))
                      for r in recs)
        assert have == sorted(c["cands"]), (kernel, c)


@pytest.mark.parametrize("kernel", ["persistent", "plain"])
@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_threshold_set_to_an_oracle_snr(dev, mode, kernel):
    x, off = synthetic.config3(n_spectra=12, lo=20000, hi=80000, seed=78)
    w = oracle.hs_batched(x, off, 32, MODES[mode], 0.0)["candidates"]
    snrs = np.sort(w["snr"])[::-1]
    for thr in (snrs[7], snrs[len(snrs) // 2], snrs[-1]):
        thr = float(thr)
        want = oracle.hs_batched(x, off, 32, MODES[mode], thr)["candidates"]
        at = int(np.sum(w["snr"] == np.float32(thr)))
        assert at >= 1 and want.size == int(np.sum(w["snr"] > np.float32(thr)))
        got = _ops().sum_batched(torch.from_numpy(x).to(dev), torch.from_numpy(off).to(dev), 32, mode, thr,
                                 capacity=x.size, kernel=kernel)
        recs, n = _cands(got)
        assert n == want.size and _same_records(recs, want), (mode, kernel, thr)
        assert not np.any(recs["snr"] == np.float32(thr))


# ---------------------------------------------------------------------------
# non-finite SNR from a caller normalisation: the first eligible k is taken
# whatever its SNR (Algorithm 2 starts from the fundamental's SNR), then only
# a strictly larger SNR replaces it
# ---------------------------------------------------------------------------

def _same_nan_aware(got, want, label):
    for k in ("harm", "drift"):
        assert np.array_equal(_np(got[k]).reshape(-1), want[k].reshape(-1)), (label, k)
    a, b = _np(got["snr"]).reshape(-1), want["snr"].reshape(-1)
    na, nb = np.isnan(a), np.isnan(b)
    assert np.array_equal(na, nb), label
    assert np.array_equal(a[~na].view(np.uint32), b[~nb].view(np.uint32)), label


@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_non_finite_snr_same_on_every_kernel(dev, mode):
    x = synthetic.exp_noise(20011, 79)
    norm = (1.0, 1e-45)           # 1 / sigma_k overflows in float: SNRs are NaN or infinite
    w = oracle.hs_1d(x, 16, MODES[mode], norm=norm)
    assert np.isnan(w["snr"]).any() and (w["harm"] == 1).any()
    for kernel in ("persistent", "plain"):
        got = _ops().sum_1d(torch.from_numpy(x).to(dev), 16, mode, norm=norm, kernel=kernel)
        _same_nan_aware(got, w, "1d " + kernel)
    off = np.array([0, 9000, 20011], dtype=np.int64)
    for kernel in ("persistent", "plain"):
        got = _ops().sum_batched(torch.from_numpy(x).to(dev), torch.from_numpy(off).to(dev), 16, mode, 3.0,
                                 dense=True, candidates=False, norm=[1.0, 1e-45, 1.0, 1e-45], kernel=kernel)
        for s in range(2):
            ws = oracle.hs_1d(x[off[s]:off[s + 1]], 16, MODES[mode], norm=norm)
            _same_nan_aware({k: got[k][off[s]:off[s + 1]] for k in ("snr", "harm", "drift")}, ws,
                            "batched %s %d" % (kernel, s))
    p = np.stack([x[:2001 * 9].reshape(9, 2001)])[0]
    wp = oracle.hs_2d(p, -4, 4, 16, MODES[mode], norm=norm)
    for kernel in ("auto", "persistent"):
        got = _ops().sum_2d(torch.from_numpy(p).to(dev), -4, 4, 16, mode, norm=norm, kernel=kernel)
        _same_nan_aware(got, wp, "2d " + kernel)
