"""Exact invariants and reductions of the oracle (P6-P8).

* P6: multiplying every power by 2^j scales the sums, statistics and
  normalisation exactly, so SNR, harmonic count and drift are bit-identical.
* P7: a plane whose only row is z = 0 is the 1D sum of that row; a plane of
  identical rows with a fixed normalisation gives, in row z, the 1D sum with
  H limited to the harmonics whose row k z stays inside the plane; a batch is
  its spectra summed one by one; FP16 storage is the float sum of the decoded
  values.
* P8: the number of harmonics summed is min(H, (N-1) // n) (simple) and
  min(H, (N-1) // (n+1)) (greedy) at every band boundary.
"""
import numpy as np
import pytest

import oracle
import synthetic


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("snr", "harm", "drift"))


@pytest.mark.parametrize("j", [-12, 5])
@pytest.mark.parametrize("mode", [oracle.STANDARD, oracle.GREEDY])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_power_of_two_scaling(j, mode, prec):
    x, _ = synthetic.config2(n=1 << 15, seed=5, n_trains=5)
    y = np.ldexp(x, j).astype(np.float32)
    assert _same(oracle.hs_1d(x, 32, mode, precision=prec), oracle.hs_1d(y, 32, mode, precision=prec))


@pytest.mark.parametrize("mode", [oracle.STANDARD, oracle.GREEDY])
def test_2d_single_row_is_1d(mode):
    x, _ = synthetic.config2(n=3000, seed=6, n_trains=3)
    a = oracle.hs_2d(x[None, :], 0, 0, 16, mode)
    b = oracle.hs_1d(x, 16, mode)
    for k in ("snr", "harm", "drift"):
        assert np.array_equal(a[k][0], b[k])


@pytest.mark.parametrize("mode", [oracle.STANDARD, oracle.GREEDY])
def test_2d_identical_rows(mode):
    z_min, z_max, H = -7, 5, 8
    row = synthetic.exp_noise(2000, 8)
    plane = np.repeat(row[None, :], z_max - z_min + 1, axis=0)
    a = oracle.hs_2d(plane, z_min, z_max, H, mode, norm=(1.0, 1.0))
    for i, z in enumerate(range(z_min, z_max + 1)):
        kz = H if z == 0 else (z_max // z if z > 0 else z_min // z)
        b = oracle.hs_1d(row, min(H, kz), mode, norm=(1.0, 1.0))
        for k in ("snr", "harm", "drift"):
            assert np.array_equal(a[k][i], b[k]), (z, k)


def test_batched_is_per_spectrum():
    x, off = synthetic.config3(n_spectra=4, lo=1000, hi=5000, seed=9)
    r = oracle.hs_batched(x, off, 16, oracle.GREEDY, 3.0, dense=True)
    for s in range(4):
        one = oracle.hs_1d(x[off[s]:off[s + 1]], 16, oracle.GREEDY)
        assert _same(r["spectra"][s], one)
        c = r["candidates"][r["candidates"]["spectrum"] == s]
        sel = one["snr"] > np.float32(3.0)
        assert np.array_equal(c["bin"], np.flatnonzero(sel))
        assert np.array_equal(c["snr"], one["snr"][sel])


def test_fp16_storage_is_sum_of_decoded_values():
    x, _ = synthetic.config2(n=1 << 14, seed=10, n_trains=4)
    mu1, _ = oracle.stats(x)
    q = oracle.quantize_f16(x, np.float32(mu1))
    dec = q.astype(np.float32)
    a = oracle.hs_1d(dec, 32, oracle.GREEDY)
    # the SNR does not depend on the storage scale: decoding at any power of two scale is the same
    b = oracle.hs_1d(np.ldexp(dec, 3).astype(np.float32), 32, oracle.GREEDY)
    assert _same(a, b)


@pytest.mark.parametrize("mode", [oracle.STANDARD, oracle.GREEDY])
def test_truncation_at_band_boundaries(mode):
    N, H = 997, 12
    x = np.random.default_rng(3).uniform(1.0, 2.0, N).astype(np.float32)
    P = oracle.hs_1d(x, H, mode, precision="f64", norm=(0.0, 1.0), report=range(1, H + 1))["partial"]
    summed = np.count_nonzero(P > 0, axis=0)
    for n in range(N):
        reach = n + 1 if mode == oracle.GREEDY else n
        want = 0 if n == 0 else min(H, (N - 1) // reach)
        assert summed[n] == want, n


def test_first_bin_and_fundamental_end():
    x = synthetic.exp_noise(5000, 12)
    r = oracle.hs_1d(x, 8, oracle.GREEDY, first_bin=10, fundamental_end=3000)
    assert not r["harm"][:10].any() and not r["harm"][3000:].any()
    assert r["harm"][10:3000].all()
    # the statistics still cover every bin from first_bin on
    assert (r["mu1"], r["sigma1"]) == oracle.norm_from_data(x, 10)


def test_harmonic_mask_power_of_two_only():
    x = synthetic.exp_noise(1 << 12, 13)
    mask = sum(1 << (k - 1) for k in (1, 2, 4, 8, 16))
    r = oracle.hs_1d(x, 16, oracle.STANDARD, harmonic_mask=mask)
    assert set(np.unique(r["harm"])) <= {0, 1, 2, 4, 8, 16}
