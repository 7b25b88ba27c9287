"""Pins of the oracle's pipeline neighbours: the power spectrum with
inter-binning (before the sum) and peak clustering (after it).

Power spectrum: closed forms of pure tones (an integer-bin tone has power
(A N / 2)^2 in its bin and (pi/4)^2 of that in the neighbouring half bins; a
tone half-way between bins is recovered by its inter-bin), the noise means
(1 per integer bin, pi^2 / 8 per half bin for unit-normalised white noise),
and the plain powers are the inter-binned output's even entries bit for bit.
Clustering: a hand-worked fixture (ties, harmonic-less bins, spectrum
borders, thresholds), the reduction radius 0 = the plain candidate list, and
properties of the kept peaks (each the strict winner of its window, kept
peaks more than `radius` apart, every spectrum's maximum above the threshold
kept).
"""
import math

import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
from golden_io import read_peaks


def _tone(N, f, A=2.0):
    t = np.arange(N)
    return np.fft.rfft(A * np.cos(2 * np.pi * f * t / N)).astype(np.complex64)


def test_integer_bin_tone():
    N, k, A = 1 << 12, 100, 2.0
    p = oracle.power_spectrum(_tone(N, k, A), interbin=True)
    peak = (A * N / 2) ** 2
    assert abs(p[2 * k] / peak - 1) < 1e-6
    assert abs(p[2 * k - 1] / peak - math.pi ** 2 / 16) < 1e-5
    assert abs(p[2 * k + 1] / peak - math.pi ** 2 / 16) < 1e-5
    others = np.delete(p[0::2], k)
    assert others.max() < 1e-6 * peak


def test_half_bin_tone_recovered_by_interbinning():
    N, k, A = 1 << 12, 100, 2.0
    p = oracle.power_spectrum(_tone(N, k + 0.5, A), interbin=True)
    peak = (A * N / 2) ** 2
    assert abs(p[2 * k + 1] / peak - 1) < 1e-3          # the scalloped power comes back
    assert abs(p[2 * k] / peak - 4 / math.pi ** 2) < 0.01   # the integer neighbours see (2/pi)^2
    assert p.argmax() == 2 * k + 1


def test_noise_means_and_scale():
    N = 1 << 18
    x = np.random.default_rng(3).normal(0.0, 1.0, size=N)
    F = np.fft.rfft(x).astype(np.complex64)[1:-1]        # drop DC and Nyquist
    p = oracle.power_spectrum(F, interbin=True, scale=1.0 / N)
    ints, halves = p[0::2].astype(np.float64), p[1::2].astype(np.float64)
    assert abs(ints.mean() - 1.0) < 5 * 1.0 / math.sqrt(ints.size)
    # F_m - F_{m+1} has twice the variance: half-bin mean 2 (pi/4)^2 = pi^2 / 8
    assert abs(halves.mean() - math.pi ** 2 / 8) < 5 * (math.pi ** 2 / 8) / math.sqrt(halves.size)


def test_plain_powers_are_the_even_entries():
    F = (np.random.default_rng(4).normal(size=5001) + 1j * np.random.default_rng(5).normal(size=5001)).astype(
        np.complex64)
    a = oracle.power_spectrum(F, interbin=False, scale=0.37)
    b = oracle.power_spectrum(F, interbin=True, scale=0.37)
    assert b.size == 2 * F.size - 1
    assert np.array_equal(a.view(np.uint32), b[0::2].view(np.uint32))


OFF, SNR, HARM, CASES = read_peaks()


def test_hand_peaks():
    drift = np.zeros_like(HARM)
    for c in CASES:
        got = oracle.cluster_peaks(SNR, HARM, drift, c["threshold"], c["radius"], offsets=OFF)
        assert [(int(r["spectrum"]), int(r["bin"])) for r in got] == c["keep"], c
        for r in got:
            assert r["snr"] == SNR[OFF[r["spectrum"]] + r["bin"]]


def test_radius_zero_is_the_candidate_list():
    g = np.random.default_rng(6)
    snr = g.normal(size=3000).astype(np.float32) * 3
    harm = g.integers(0, 4, size=3000).astype(np.uint8)
    drift = g.integers(0, 3, size=3000).astype(np.uint8)
    a = oracle.cluster_peaks(snr, harm, drift, 2.0, 0)
    b = oracle.candidates(snr, harm, drift, 2.0)
    assert np.array_equal(a, b)


@settings(max_examples=80, deadline=None)
@given(vals=st.lists(st.integers(0, 9), min_size=1, max_size=60), radius=st.integers(0, 5),
       cut=st.integers(0, 60), thr=st.integers(0, 8))
def test_peak_properties(vals, radius, cut, thr):
    snr = np.array(vals, dtype=np.float32)
    harm = np.ones(snr.size, dtype=np.uint8)
    cut = min(cut, snr.size)
    off = np.array([0, cut, snr.size], dtype=np.int64)
    got = oracle.cluster_peaks(snr, harm, harm, thr, radius, offsets=off)
    for s in (0, 1):
        lo, hi = off[s], off[s + 1]
        kept = sorted(int(r["bin"]) + lo for r in got if r["spectrum"] == s)
        for a, b in zip(kept, kept[1:]):
            assert b - a > radius
        for n in kept:
            w = snr[max(lo, n - radius):min(hi, n + radius + 1)]
            assert snr[n] == w.max() and snr[n] > thr
            assert n == max(lo, n - radius) + int(np.argmax(w))       # first maximum of its window
        if hi > lo and snr[lo:hi].max() > thr:
            assert lo + int(np.argmax(snr[lo:hi])) in kept
