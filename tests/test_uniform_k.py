"""Host checks of the harmonic-count identity behind the wave-uniform walk.

The kernels sum K(n) = min(cap, (N - 1) // (n + g)) harmonics for
fundamental n (g = 1 for the greedy pair, 0 for the simple sum; Sec. 3.3
Algorithm 2 with the truncation that keeps every read inside the spectrum).
Each lane j of a wave holds T(j + 1) = (N - 1) // (j + 1) - g, and the count
of a position n is the number of k <= cap with T(k) >= n (one ballot).  A
wave of fundamentals [wf, wl] is walked without per-lane bounds when the
counts of wf and wl agree, which must mean every fundamental in between
has that count.  Brute force over small and boundary cases.
"""
import numpy as np
import pytest


def k_direct(N, n, cap, g):
    return min(cap, (N - 1) // (n + g))


def thresholds(N, cap, g):
    return [(N - 1) // k - g for k in range(1, cap + 1)]


def k_ballot(T, n):
    return sum(1 for t in T if t >= n)


@pytest.mark.parametrize("g", [0, 1])
def test_ballot_count_equals_direct_count(g):
    rng = np.random.default_rng(5)
    cases = [(N, cap) for N in (2, 3, 17, 64, 65, 1000, 19204, 19297, 19396) for cap in (1, 4, 17, 32, 64)]
    cases += [(int(rng.integers(2, 1 << 20)), int(rng.integers(1, 65))) for _ in range(40)]
    for N, cap in cases:
        T = thresholds(N, cap, g)
        ns = list(range(1, min(N + 3, 300)))          # fundamentals start at 1 (first_bin >= 1)
        ns += [int(v) for v in rng.integers(1, N + 1, 200)]
        for n in ns:
            assert k_ballot(T, n) == k_direct(N, n, cap, g), (N, cap, g, n)


@pytest.mark.parametrize("g", [0, 1])
def test_equal_end_counts_mean_a_uniform_wave(g):
    rng = np.random.default_rng(6)
    for _ in range(300):
        N = int(rng.integers(70, 1 << 18))
        cap = int(rng.integers(1, 65))
        T = thresholds(N, cap, g)
        wf = int(rng.integers(1, N - 64))
        wl = wf + 63
        kf, kl = k_ballot(T, wf), k_ballot(T, wl)
        counts = {k_direct(N, n, cap, g) for n in range(wf, wl + 1)}
        assert (kf == kl) == (len(counts) == 1), (N, cap, g, wf)
        if kf == kl:
            assert counts == {kf}


def test_thresholds_on_chosen_lanes():
    """The spectrum lengths of the GPU test put a threshold on lanes 0, 31, 63."""
    for g in (0, 1):
        for k, m in ((2, 150), (3, 100), (17, 20), (32, 9)):
            for s in (0, 31, 63):
                t = 64 * m + s
                N = k * (t + g) + 1
                assert (N - 1) // k - g == t
                assert k_direct(N, t, 64, g) >= k and k_direct(N, t + 1, 64, g) < k
