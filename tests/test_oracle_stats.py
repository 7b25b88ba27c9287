"""Pins for the oracle's normalisation statistics and tables.

The statistics are the population mean and variance of the stored powers
(the mean and standard deviation used to normalise partial sums, Sec. 2
Eq. (2); computed once and shared by every algorithm, Sec. 4), each rounded
once to float64.  They are pinned against closed forms, a brute-force
Fraction evaluation, numpy's float64 routines and exact scaling.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synthetic


def _brute(v):
    fr = [Fraction(float(a)) for a in np.asarray(v, dtype=np.float32)]
    s1 = sum(fr, Fraction(0))
    s2 = sum((a * a for a in fr), Fraction(0))
    return len(fr), s1, s2


@pytest.mark.parametrize("seed", range(6))
def test_exact_sums_match_fraction_bruteforce(seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(1, 400))
    # wide exponent spread, both signs, subnormals and zeros
    v = (g.standard_normal(n) * np.exp2(g.integers(-140, 120, size=n))).astype(np.float32)
    v[g.integers(0, n, size=max(1, n // 20))] = 0.0
    v[0] = np.float32(1e-45)
    assert oracle.exact_sums(v) == _brute(v)


def test_exact_sums_chunked():
    v = synthetic.exp_noise(10007, 5)
    assert oracle.exact_sums(v, chunk=1000) == oracle.exact_sums(v) == _brute(v)


@pytest.mark.parametrize("M", [1, 2, 3, 10, 1000, 65535])
def test_stats_closed_form_ramp(M):
    # values 1..M: mean (M+1)/2, population variance (M^2-1)/12
    x = np.concatenate([[np.float32(123.0)], np.arange(1, M + 1, dtype=np.float32)])
    mu, var = oracle.stats(x, first_bin=1)
    assert mu == float(Fraction(M + 1, 2))
    assert var == float(Fraction(M * M - 1, 12))


def test_stats_constant_is_degenerate():
    x = np.full(100, 3.25, dtype=np.float32)
    mu, var = oracle.stats(x)
    assert mu == 3.25 and var == 0.0
    mu1, s1 = oracle.norm_from_data(x)
    assert oracle.is_degenerate(mu1, s1)
    r = oracle.hs_1d(x, 4, oracle.GREEDY)
    assert not r["snr"].any() and not r["harm"].any() and not r["drift"].any()


def test_stats_first_bin_excludes_dc():
    x = synthetic.exp_noise(4096, 7)
    y = x.copy()
    y[0] = 1e6
    assert oracle.stats(x, 1) == oracle.stats(y, 1)
    assert oracle.stats(x, 3) == oracle.stats(x[3:], 0)


@pytest.mark.parametrize("seed", range(4))
def test_stats_close_to_numpy(seed):
    x = synthetic.exp_noise(1 << 16, 10 + seed)
    mu, var = oracle.stats(x)
    v = x[1:].astype(np.float64)
    assert abs(mu - v.mean()) <= 1e-13 * mu
    assert abs(var - v.var()) <= 1e-12 * var


@pytest.mark.parametrize("j", [-20, -3, 1, 7, 30])
def test_stats_power_of_two_scaling_is_exact(j):
    x = synthetic.exp_noise(5000, 3)
    mu, var = oracle.stats(x)
    mu2, var2 = oracle.stats(np.ldexp(x, j).astype(np.float32))
    assert mu2 == math.ldexp(mu, j) and var2 == math.ldexp(var, 2 * j)


def test_stats_2d_covers_all_rows():
    g = np.random.default_rng(1)
    p = g.standard_exponential((5, 300)).astype(np.float32)
    assert oracle.stats(p, 2) == oracle.stats(p[:, 2:].reshape(-1), 0)


def test_tables_relations():
    mu1, s1 = 1.0009, 1.0073
    mu, sig, rs, nm = oracle.tables(mu1, s1, 32)
    k = np.arange(1, 33)
    assert np.all(mu == k * mu1)
    assert np.all(sig == np.sqrt(k.astype(np.float64)) * s1)
    assert np.all(rs == (1.0 / sig).astype(np.float32))
    assert np.all(nm == (-(mu / sig)).astype(np.float32))
    # the fused float SNR of the mean partial sum is ~0 and of mean + sigma ~1
    for i in range(32):
        s = np.float32(mu[i])
        assert abs(float(s) * float(rs[i]) + float(nm[i])) < 1e-6 * k[i]


def test_unit_normalisation_tables():
    # mu1 = 0, sigma1 = 1: sigma_k = sqrt(k); k = 1, 4, 16 give exact powers of two
    mu, sig, rs, nm = oracle.tables(0.0, 1.0, 16)
    assert (rs[0], rs[3], rs[15]) == (1.0, 0.5, 0.25)
    assert np.all(nm == 0.0)


def test_quantize_f16_matches_struct_rounding():
    import struct
    g = np.random.default_rng(2)
    x = np.concatenate([g.standard_exponential(2000) * 3, [0.0, 1e-9, 70000.0, 65519.0, 65520.0]])
    x = x.astype(np.float32)
    scale = np.float32(1.37)
    q = oracle.quantize_f16(x, scale)
    for a, b in zip(x, q):
        y = np.float32(a) / scale
        y = min(max(float(y), -65504.0), 65504.0)
        want = struct.unpack("<e", struct.pack("<e", y))[0]
        assert float(b) == want
