"""Brute force on tiny spectra (P2).

* Simple sum (Sec. 3.1, Eq. (3)): the partial sums over explicit index sets
  {k n : k <= K}, the SNR of Eq. (2) compared exactly (rationals and square
  roots squared), the best one chosen with ties to the smaller K.
* Greedy sum (Sec. 3.3, Eq. (5), Algorithm 2): every monotone drift path of the
  drift tree (Sec. 2.2, Fig. 4: at each harmonic the drift stays or grows by
  one) is enumerated; the greedy path is the unique one whose every step took
  the larger of its two candidate bins (ties to the lower bin).  Its partial
  sums and drift must be the oracle's.
* The best path over the whole tree bounds both the greedy and the simple SNR
  from above (the simple sum is the all-zero-drift path).
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle


def _gt(a, p, b, q):
    """a/sqrt(p) > b/sqrt(q) exactly, for rationals a, b and positive ints p, q."""
    if a >= 0 and b <= 0:
        return not (a == 0 and b == 0)
    if a <= 0 and b >= 0:
        return False
    lhs, rhs = a * a * q, b * b * p          # same strict sign: compare squares
    return lhs > rhs if a > 0 else lhs < rhs


def _best(sums, mu, sig2):
    """Index (1-based) of the best SNR (S_k - k mu)/sqrt(k sig2); ties to the smaller k."""
    best = 0
    for k, s in enumerate(sums, start=1):
        num = Fraction(s) - k * Fraction(mu)
        if best == 0:
            best, bnum = k, num
            continue
        # compare num/sqrt(k sig2) > bnum/sqrt(best sig2)  <=>  num/sqrt(k) > bnum/sqrt(best)
        if _gt(num, k, bnum, best):
            best, bnum = k, num
    return best


def _check_choice(r, n, sums, mu, sigma, kb, tol):
    """The chosen harmonic count is the exact argmax kb, or one whose exact SNR
    ties kb's within the precision's rounding (the float tables of different
    counts are rounded separately, so an exact tie can break either way)."""
    got = int(r["harm"][n])
    snr = lambda k: (float(sums[k - 1]) - k * mu) / (math.sqrt(k) * sigma)   # noqa: E731
    assert 1 <= got <= len(sums), (n, got)
    if got != kb:
        assert abs(snr(got) - snr(kb)) <= tol * max(1, abs(snr(kb))), (n, kb, got)
    return got


def _keff(n, N, H, greedy):
    if n < 1:
        return 0
    return min(H, (N - 1) // (n + 1 if greedy else n))


def _tree_paths(x, n, K):
    """All 2^K drift paths: list of (bits, chosen bins)."""
    out = []
    for bits in itertools.product((0, 1), repeat=K):
        d, bins = 0, []
        for k, b in enumerate(bits, start=1):
            d += b
            bins.append(k * n + d)
        out.append((bits, bins))
    return out


def _greedy_by_tree(x, n, K):
    """The unique path whose every step took the larger bin (ties: lower bin)."""
    found = []
    for bits, bins in _tree_paths(x, n, K):
        ok, d = True, 0
        for k, b in enumerate(bits, start=1):
            lo, hi = x[k * n + d], x[k * n + d + 1]
            if b != (1 if hi > lo else 0):
                ok = False
                break
            d += b
        if ok:
            found.append((bits, bins))
    assert len(found) == 1
    return found[0]


values = st.lists(st.integers(min_value=0, max_value=6), min_size=4, max_size=48)


@settings(max_examples=150, deadline=None)
@given(vals=values, H=st.integers(1, 6), seed=st.integers(0, 10))
def test_standard_bruteforce(vals, H, seed):
    x = np.array(vals, dtype=np.float32)
    N = x.size
    mu, sigma = 1.5, 1.25   # given normalisation: exact in binary
    r64 = oracle.hs_1d(x, H, oracle.STANDARD, precision="f64", norm=(mu, sigma),
                       report=range(1, H + 1))
    r32 = oracle.hs_1d(x, H, oracle.STANDARD, precision="f32", norm=(mu, sigma))
    for n in range(N):
        K = _keff(n, N, H, False)
        sums = list(itertools.accumulate(Fraction(float(x[k * n])) for k in range(1, K + 1)))
        for k in range(H):
            assert r64["partial"][k, n] == (float(sums[k]) if k < K else 0.0)
        kb = _best(sums, mu, sigma * sigma) if K else 0
        if kb:
            _check_choice(r64, n, sums, mu, sigma, kb, 1e-12)
            _check_choice(r32, n, sums, mu, sigma, kb, 2e-6)
        else:
            assert r64["harm"][n] == 0 and r32["harm"][n] == 0
        assert r64["drift"][n] == 0 and r32["drift"][n] == 0
        if kb:
            want = (float(sums[kb - 1]) - kb * mu) / (math.sqrt(kb) * sigma)
            assert abs(r64["snr"][n] - want) <= 1e-12 * max(1, abs(want))
            assert abs(float(r32["snr"][n]) - want) <= 2e-6 * max(1, abs(want))


@settings(max_examples=150, deadline=None)
@given(vals=values, H=st.integers(1, 6))
def test_greedy_bruteforce_tree(vals, H):
    x = np.array(vals, dtype=np.float32)
    N = x.size
    mu, sigma = 1.5, 1.25
    r64 = oracle.hs_1d(x, H, oracle.GREEDY, precision="f64", norm=(mu, sigma),
                       report=range(1, H + 1))
    r32 = oracle.hs_1d(x, H, oracle.GREEDY, precision="f32", norm=(mu, sigma))
    for n in range(N):
        K = _keff(n, N, H, True)
        if K == 0:
            assert r64["harm"][n] == 0 and r32["harm"][n] == 0 and r64["snr"][n] == 0
            continue
        bits, bins = _greedy_by_tree(x, n, K)
        sums = list(itertools.accumulate(Fraction(float(x[m])) for m in bins))
        for k in range(K):
            assert r64["partial"][k, n] == float(sums[k])
        kb = _best(sums, mu, sigma * sigma)
        g64 = _check_choice(r64, n, sums, mu, sigma, kb, 1e-12)
        g32 = _check_choice(r32, n, sums, mu, sigma, kb, 2e-6)
        assert r64["drift"][n] == sum(bits[:g64]) and r32["drift"][n] == sum(bits[:g32])
        # both bins read at every step stay inside the spectrum
        assert all(k * n + sum(bits[:k - 1]) + 1 <= N - 1 for k in range(1, K + 1))


@settings(max_examples=60, deadline=None)
@given(vals=st.lists(st.floats(0, 10, width=32), min_size=8, max_size=40), H=st.integers(1, 5))
def test_tree_best_bounds_greedy_and_standard(vals, H):
    x = np.array(vals, dtype=np.float32)
    N = x.size
    mu, sigma = 1.0, 1.0
    g = oracle.hs_1d(x, H, oracle.GREEDY, precision="f64", norm=(mu, sigma))
    s = oracle.hs_1d(x, H, oracle.STANDARD, precision="f64", norm=(mu, sigma))
    for n in range(1, N):
        K = _keff(n, N, H, True)
        if K == 0:
            continue
        best_tree = -math.inf
        for _, bins in _tree_paths(x, n, K):
            acc = 0.0
            for k, m in enumerate(bins, start=1):
                acc += float(x[m])
                best_tree = max(best_tree, (acc - k * mu) / math.sqrt(k))
        assert g["snr"][n] <= best_tree + 1e-9
        # the simple sum over the same K harmonics is the all-zero path
        acc, best_std = 0.0, -math.inf
        for k in range(1, K + 1):
            acc += float(x[k * n])
            best_std = max(best_std, (acc - k * mu) / math.sqrt(k))
        assert best_std <= best_tree + 1e-9
        if _keff(n, N, H, False) == K:
            assert abs(s["snr"][n] - best_std) <= 1e-9 * max(1, abs(best_std))


def test_f32_and_f64_agree_on_noise():
    # away from float near-ties the float argmax equals the float64 one
    x = np.random.default_rng(0).standard_exponential(1 << 14).astype(np.float32)
    for mode in (oracle.STANDARD, oracle.GREEDY):
        a = oracle.hs_1d(x, 16, mode, precision="f32")
        b = oracle.hs_1d(x, 16, mode, precision="f64")
        flips = np.count_nonzero(a["harm"] != b["harm"])
        assert flips <= 3
        ok = a["harm"] == b["harm"]
        assert np.array_equal(a["drift"][ok], b["drift"][ok])
        err = np.abs(a["snr"].astype(np.float64) - b["snr"])
        assert np.all(err <= 1e-5 * np.maximum(1.0, np.abs(b["snr"])))
