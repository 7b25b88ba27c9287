"""Pins of the oracle's PRESTO-style sums (Sec. 3.2, Eq. (4), Algorithm 1).

The output index n is the last bin of the harmonic series; stage K sums the
bins nearest to h n / K.  What fixes the oracle here, independently of its code:

* hand-worked stages of a tiny spectrum and the paper's own last-bin example
  (bin 800 ends the series of fundamental 100 at order 8 and of fundamental
  200 at order 4), in tests/golden/hand_presto.txt;
* brute force: the bin each harmonic reads is found by searching every bin for
  the one closest to h n / K (ties to the upper bin), the read multiset of
  every stage is recovered from the oracle by linearity (unit impulses), and
  the best stage is chosen with exact rational comparisons;
* reductions: at n = K f the stage-K series is the simple sum of fundamental
  f (Eq. (3)), so it must equal the simple-sum oracle bit for bit (PRESTO:
  the simple sum with the odd harmonics above 1 removed, normalised as a sum
  of 1 + K/2 elements); with H = 1 PRESTO+ is the input itself;
* the noise null: a stage of m distinct Exp(1) bins has mean m and variance
  m, so its SNR has mean 0 and variance 1 (pins the element count m);
* a noise-free harmonic train at an integer fundamental f0 gives, at the last
  bin K f0, the closed-form SNR sum(a_h) / sqrt(m);
* PRESTO+ forms every PRESTO_all stage with the same sums, so its best SNR is
  never lower; exact scaling by 2^j leaves every output bit-identical.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from golden_io import read_presto

SPECTRA, CASES, LASTBINS = read_presto()
MODE = {"presto": oracle.PRESTO, "presto_all": oracle.PRESTO_ALL, "presto_plus": oracle.PRESTO_PLUS}
MODES = (oracle.PRESTO, oracle.PRESTO_ALL, oracle.PRESTO_PLUS)


# ---------------------------------------------------------------------------
# the hand-worked cases and the paper's example
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-H%d-m%d-f%d-n%d" % (
    c["mode"], c["H"], c["mask"], c["first"], c["n"]))
def test_hand_presto(case, prec):
    x = SPECTRA[case["spectrum"]]
    mode, H, n = MODE[case["mode"]], case["H"], case["n"]
    r = oracle.hs_1d(x, H, mode, harmonic_mask=case["mask"], first_bin=case["first"], precision=prec,
                     norm=(0.0, 1.0), idx=[n])
    kb = case["harm"]
    assert int(r["harm"][0]) == kb
    assert int(r["drift"][0]) == 0
    if kb == 0:
        assert float(r["snr"][0]) == 0.0
    else:
        _, S, m = next(s for s in case["stages"] if s[0] == kb)
        want = S / math.sqrt(m)
        tol = 1e-6 * max(1.0, abs(want)) if prec == "f32" else 1e-14 * max(1.0, abs(want))
        assert abs(float(r["snr"][0]) - want) <= tol
    # every listed stage, one at a time through the mask: its SNR is S / sqrt(m)
    formed = {K for K, _, _ in case["stages"]}
    for K in range(1, H + 1):
        r1 = oracle.hs_1d(x, H, mode, harmonic_mask=1 << (K - 1), first_bin=case["first"], precision=prec,
                          norm=(0.0, 1.0), idx=[n])
        if K not in formed:
            assert int(r1["harm"][0]) == 0
            continue
        _, S, m = next(s for s in case["stages"] if s[0] == K)
        assert int(r1["harm"][0]) == K
        assert abs(float(r1["snr"][0]) - S / math.sqrt(m)) <= 1e-6 * max(1.0, S / math.sqrt(m))


def _read_multiset(N, n, K, mode, first_bin=1):
    """Bins stage K of last bin n reads, with multiplicity, recovered by linearity:
    with mu1 = 0, sigma1 = 1 and a unit impulse at bin b, the stage's sum counts
    how often b is read."""
    counts = {}
    m = None
    for b in range(N):
        x = np.zeros(N, dtype=np.float32)
        x[b] = 1.0
        r = oracle.hs_1d(x, K, mode, harmonic_mask=1 << (K - 1), first_bin=first_bin, precision="f64",
                         norm=(0.0, 1.0), idx=[n])
        if int(r["harm"][0]) != K:
            return None                      # stage not formed
        if m is None:
            # the SNR of the all-ones spectrum gives m / sqrt(m)
            ones = oracle.hs_1d(np.ones(N, dtype=np.float32), K, mode, harmonic_mask=1 << (K - 1),
                                first_bin=first_bin, precision="f64", norm=(0.0, 1.0), idx=[n])
            m = int(round(float(ones["snr"][0]) ** 2))
        c = int(round(float(r["snr"][0]) * math.sqrt(m)))
        if c:
            counts[b] = c
    return counts


@pytest.mark.parametrize("ex", LASTBINS, ids=lambda e: "n%d-K%d" % (e["n"], e["K"]))
@pytest.mark.parametrize("mode", MODES)
def test_paper_last_bin_example(ex, mode):
    # Sec. 3.2: the series ending at bin n at order K starts at the fundamental
    # the paper names and ends at n.  Probing all N bins is slow, so probe the
    # few bins around the two ends and the total count.
    n, K, f = ex["n"], ex["K"], ex["fundamental"]
    N = n + 8
    for b, want in ((f - 1, 0), (f, 1), (f + 1, 0), (n - 1, 0), (n, 1)):
        x = np.zeros(N, dtype=np.float32)
        x[b] = 1.0
        r = oracle.hs_1d(x, K, mode, harmonic_mask=1 << (K - 1), precision="f64", norm=(0.0, 1.0), idx=[n])
        m = K if mode != oracle.PRESTO else 1 + K // 2
        assert int(r["harm"][0]) == K
        assert round(float(r["snr"][0]) * math.sqrt(m)) == want, (b, want)
    # nothing below the fundamental is read
    x = np.zeros(N, dtype=np.float32)
    x[:f] = 1.0
    r = oracle.hs_1d(x, K, mode, harmonic_mask=1 << (K - 1), precision="f64", norm=(0.0, 1.0), idx=[n])
    assert float(r["snr"][0]) == 0.0


# ---------------------------------------------------------------------------
# brute force on tiny spectra
# ---------------------------------------------------------------------------

def _closest_bin(h, n, K):
    """Search every bin 0..n for the one closest to h n / K; a tie goes up."""
    best, bd = None, None
    for b in range(n + 1):
        d = abs(Fraction(b) - Fraction(h * n, K))
        if best is None or d < bd or (d == bd and b > best):
            best, bd = b, d
    return best


def _stage_plan(mode, H):
    """(K, harmonics) of every stage, written from Sec. 3.2's description."""
    out = []
    for K in range(1, H + 1):
        pow2 = K >= 2 and (K & (K - 1)) == 0
        if mode == oracle.PRESTO_PLUS:
            out.append((K, list(range(1, K + 1))))
        elif pow2 and mode == oracle.PRESTO_ALL:
            out.append((K, list(range(1, K + 1))))
        elif pow2 and mode == oracle.PRESTO:
            out.append((K, [1] + list(range(2, K + 1, 2))))
    return out


def _gt(a, p, b, q):
    """a/sqrt(p) > b/sqrt(q) exactly, for rationals a, b and positive ints p, q."""
    if a >= 0 and b <= 0:
        return not (a == 0 and b == 0)
    if a <= 0 and b >= 0:
        return False
    lhs, rhs = a * a * q, b * b * p
    return lhs > rhs if a > 0 else lhs < rhs


@settings(max_examples=120, deadline=None)
@given(vals=st.lists(st.integers(min_value=0, max_value=6), min_size=2, max_size=40),
       H=st.integers(1, 8), first_bin=st.integers(1, 3), mode=st.sampled_from(MODES),
       mask=st.integers(0, 255))
def test_presto_bruteforce(vals, H, first_bin, mode, mask):
    x = np.array(vals, dtype=np.float32)
    N = x.size
    mu, sigma = 1.5, 1.25
    r64 = oracle.hs_1d(x, H, mode, precision="f64", norm=(mu, sigma), first_bin=first_bin, harmonic_mask=mask)
    r32 = oracle.hs_1d(x, H, mode, precision="f32", norm=(mu, sigma), first_bin=first_bin, harmonic_mask=mask)
    eligible = (1 << H) - 1 if mask == 0 else mask & ((1 << H) - 1)    # 0 = every stage
    for n in range(N):
        best = None
        exact = {}                         # stage -> exact SNR (as a float of the exact value)
        for K, hs in _stage_plan(mode, H):
            bins = [_closest_bin(h, n, K) for h in hs]
            if n < first_bin or min(bins) < first_bin:
                continue
            assert max(bins) == n <= N - 1
            if not (eligible >> (K - 1)) & 1:
                continue
            m = len(bins)
            num = sum(Fraction(float(x[b])) for b in bins) - m * Fraction(mu)
            exact[K] = float(num) / (math.sqrt(m) * sigma)
            if best is None or _gt(num, m, best[1], best[2]):
                best = (K, num, m)
        kb = best[0] if best else 0
        assert r64["drift"][n] == 0 and r32["drift"][n] == 0
        if kb == 0:
            assert r64["harm"][n] == 0 and r32["harm"][n] == 0
            assert r64["snr"][n] == 0 and r32["snr"][n] == 0
            continue
        want = exact[kb]
        # the exact argmax, except where another stage's exact SNR ties it within
        # the precision's rounding (stages of different element counts have
        # separately rounded tables, so an exact tie can break either way)
        for r, tol in ((r64, 1e-12), (r32, 2e-6)):
            got = int(r["harm"][n])
            assert got in exact, (n, got)
            if got != kb:
                assert abs(exact[got] - want) <= tol * max(1, abs(want)), (n, kb, got)
            assert abs(float(r["snr"][n]) - want) <= tol * max(1, abs(want))


@pytest.mark.parametrize("mode", MODES)
def test_read_multisets_by_impulses(mode):
    # the multiset each stage reads, recovered from the oracle's outputs alone
    N = 30
    for n in (1, 2, 5, 7, 12, 23, 29):
        for K, hs in _stage_plan(mode, 6):
            want = {}
            for h in hs:
                b = _closest_bin(h, n, K)
                want[b] = want.get(b, 0) + 1
            got = _read_multiset(N, n, K, mode)
            if min(want) < 1:
                assert got is None
            else:
                assert got == want, (n, K)


# ---------------------------------------------------------------------------
# reductions to the simple sum
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("K", [1, 2, 3, 4, 6, 8, 16, 32])
def test_exact_multiple_is_simple_sum(K):
    # at n = K f every h n / K = h f is an integer: the stage-K series of last
    # bin K f is the simple sum of fundamental f (same bins, same order)
    rng = np.random.default_rng(11 + K)
    N = 1 << 12
    x = rng.standard_exponential(N).astype(np.float32)
    fs = np.arange(1, (N - 1) // K + 1, 7)
    norm = oracle.norm_from_data(x)
    for prec in ("f32", "f64"):
        std = oracle.hs_1d(x, K, oracle.STANDARD, harmonic_mask=1 << (K - 1), precision=prec, norm=norm, idx=fs)
        plus = oracle.hs_1d(x, K, oracle.PRESTO_PLUS, harmonic_mask=1 << (K - 1), precision=prec, norm=norm,
                            idx=fs * K)
        assert np.array_equal(plus["harm"], std["harm"])
        assert np.array_equal(plus["snr"].view(np.uint8), std["snr"].view(np.uint8))
        if K >= 2 and K & (K - 1) == 0:
            pall = oracle.hs_1d(x, K, oracle.PRESTO_ALL, harmonic_mask=1 << (K - 1), precision=prec, norm=norm,
                                idx=fs * K)
            assert np.array_equal(pall["snr"].view(np.uint8), std["snr"].view(np.uint8))


@pytest.mark.parametrize("K", [2, 4, 8, 16, 32])
def test_presto_exact_multiple_is_even_simple_sum(K):
    # PRESTO at n = K f: the simple sum of f with the odd harmonics 3, 5, ...
    # zeroed (adding an exact zero leaves a float sum unchanged), normalised as
    # a sum of m = 1 + K/2 elements
    rng = np.random.default_rng(31 + K)
    N = 1 << 12
    x = rng.standard_exponential(N).astype(np.float32)
    mu1, s1 = oracle.norm_from_data(x)
    mu, sig, rs, nm = oracle.tables(mu1, s1, K)
    m = 1 + K // 2
    for f in range(3, (N - 1) // K + 1, 13):
        xz = x.copy()
        xz[[h * f for h in range(3, K + 1, 2)]] = 0.0
        s64 = oracle.hs_1d(xz, K, oracle.STANDARD, precision="f64", norm=(mu1, s1), idx=[f], report=[K])
        p64 = oracle.hs_1d(x, K, oracle.PRESTO, harmonic_mask=1 << (K - 1), precision="f64", norm=(mu1, s1),
                           idx=[K * f])
        S = float(s64["partial"][0, 0])
        assert float(p64["snr"][0]) == (S - mu[m - 1]) / sig[m - 1]
        s32 = oracle.hs_1d(xz, K, oracle.STANDARD, precision="f32", norm=(mu1, s1), idx=[f], report=[K])
        p32 = oracle.hs_1d(x, K, oracle.PRESTO, harmonic_mask=1 << (K - 1), precision="f32", norm=(mu1, s1),
                           idx=[K * f])
        S32 = float(s32["partial"][0, 0])
        # fused float SNR of the float sum: exact product and sum in rationals, rounded once
        exact = Fraction(S32) * Fraction(float(rs[m - 1])) + Fraction(float(nm[m - 1]))
        assert abs(Fraction(float(p32["snr"][0])) - exact) <= Fraction(abs(float(np.spacing(np.float32(float(exact)))))) / 2


def test_h1():
    x = np.random.default_rng(5).standard_exponential(5000).astype(np.float32)
    std = oracle.hs_1d(x, 1, oracle.STANDARD)
    plus = oracle.hs_1d(x, 1, oracle.PRESTO_PLUS)
    assert np.array_equal(plus["harm"], std["harm"])
    assert np.array_equal(plus["snr"].view(np.uint8), std["snr"].view(np.uint8))
    for mode in (oracle.PRESTO, oracle.PRESTO_ALL):
        r = oracle.hs_1d(x, 1, mode)
        assert not r["harm"].any() and not r["snr"].any()


# ---------------------------------------------------------------------------
# statistics and signals
# ---------------------------------------------------------------------------

def _disjoint_outputs(N, K, hs, rng, tries=60000):
    """Last bins whose stage-K read sets are disjoint from each other and hold
    distinct bins (so their sums are independent), picked at random.  Uses the
    nearest-bin rule of Sec. 3.2 only to choose samples, not to check them."""
    used = np.zeros(N, dtype=bool)
    out = []
    for n in rng.integers(2 * K, N, size=tries):
        bins = [(2 * h * int(n) + K) // (2 * K) for h in hs]
        if len(set(bins)) != len(bins) or used[bins].any():
            continue
        used[bins] = True
        out.append(int(n))
    return np.array(sorted(out), dtype=np.int64)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noise_null(mode, prec):
    # a stage of m distinct Exp(1) bins sums to mean m and variance m, so with
    # mu1 = sigma1 = 1 its SNR has mean 0 and variance 1; a wrong element count
    # (say K for a PRESTO stage of 1 + K/2 bins) shifts the mean by many errors
    rng = np.random.default_rng(21)
    N = 1 << 19
    x = rng.standard_exponential(N).astype(np.float32)
    for K, hs in _stage_plan(mode, 32):
        if K not in (1, 2, 3, 4, 8, 12, 16, 32):
            continue
        idx = _disjoint_outputs(N, K, hs, rng)
        cnt, m = idx.size, len(hs)
        assert cnt > 1000
        r = oracle.hs_1d(x, K, mode, harmonic_mask=1 << (K - 1), norm=(1.0, 1.0), precision=prec, idx=idx)
        assert np.all(r["harm"] == K)
        s = r["snr"].astype(np.float64)
        assert abs(s.mean()) < 5.0 / math.sqrt(cnt), (K, cnt, s.mean())
        # variance of the sample variance: (2 + excess kurtosis 6/m) / count
        assert abs(s.var() - 1.0) < 5.0 * math.sqrt((2.0 + 6.0 / m) / cnt), (K, cnt, s.var())


@pytest.mark.parametrize("mode", MODES)
def test_noise_free_train(mode):
    # harmonic h of an integer fundamental f0 carries a_h; at the last bin K f0
    # stage K collects exactly its harmonics
    N = 1 << 13
    f0 = 97
    a = 1.0 + 0.25 * np.arange(1, 33)
    x = np.zeros(N, dtype=np.float32)
    for h in range(1, 33):
        x[h * f0] = a[h - 1]
    for K, hs in _stage_plan(mode, 32):
        r = oracle.hs_1d(x, K, mode, harmonic_mask=1 << (K - 1), norm=(0.0, 1.0), precision="f64",
                         idx=[K * f0])
        want = sum(a[h - 1] for h in hs) / math.sqrt(len(hs))
        assert int(r["harm"][0]) == K
        assert abs(float(r["snr"][0]) - want) <= 1e-12 * want


def test_plus_dominates_all():
    x = np.random.default_rng(8).standard_exponential(1 << 14).astype(np.float32)
    for prec in ("f32", "f64"):
        plus = oracle.hs_1d(x, 16, oracle.PRESTO_PLUS, precision=prec)
        pall = oracle.hs_1d(x, 16, oracle.PRESTO_ALL, precision=prec)
        assert np.all(plus["snr"] >= pall["snr"])
        same = plus["harm"] == pall["harm"]
        assert np.array_equal(plus["snr"][same], pall["snr"][same])


@pytest.mark.parametrize("mode", MODES)
def test_exact_scaling(mode):
    x = np.random.default_rng(9).standard_exponential(1 << 13).astype(np.float32)
    a = oracle.hs_1d(x, 16, mode)
    b = oracle.hs_1d(x * np.float32(8.0), 16, mode)
    assert np.array_equal(a["harm"], b["harm"])
    assert np.array_equal(a["snr"].view(np.uint8), b["snr"].view(np.uint8))
