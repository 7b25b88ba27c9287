"""Seeded synthetic inputs for the harmonic-sum tests and benchmarks.

This module only draws noise and injects pulse trains; it holds none of the
harmonic-sum arithmetic, so both the CPU oracle and the GPU library can be fed
from it without sharing any of the method's code.

Recipe (all draws from numpy PCG64 streams keyed by ``(seed, stream ids)``):

* noise: i.i.d. Exp(1) powers, the distribution of a whitened power spectrum
  of Gaussian noise (two degrees of freedom, unit mean);
* pulse train: fundamental ``f0 = n0 + delta`` (bins), Gaussian pulse of duty
  cycle ``D`` (FWHM as a fraction of the period), whose harmonic k carries the
  power weight ``w_k = exp(-pi^2 k^2 D^2 / (2 ln 2))``; the amplitude ``A`` is
  set so that the ideal best partial sum reaches the requested SNR,
  ``A = snr / max_K (sum_{k<=K} w_k / sqrt(K))`` for unit-variance noise;
  harmonic k adds ``A w_k`` to bin ``k n0`` (``delta = 0``) or spreads it as
  ``sinc^2(m - k f0)`` over the bins within 4 of ``k f0`` (fractional ``f0``);
* 2D: an accelerated track adds ``A w_k`` at row ``k z0`` and column ``k r0``
  of an f-fdot plane.

Power is added to the noise (a stated simplification: the power of signal plus
noise is non-central chi-square in reality).
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "rng", "exp_noise", "gaussian_weights", "train_amplitude", "inject_train",
    "random_trains", "config1", "config2", "config3_lengths", "config3_spectrum",
    "config3", "config4", "inject_track", "random_tracks", "table2",
    "von_mises_kappa", "von_mises_series", "power_spectrum",
]


def rng(seed: int, *stream: int) -> np.random.Generator:
    """Independent PCG64 stream for ``(seed, *stream)``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), *map(int, stream)])))


def exp_noise(n: int, seed: int, *stream: int) -> np.ndarray:
    """``n`` i.i.d. Exp(1) powers as float32."""
    return rng(seed, *stream).standard_exponential(int(n), dtype=np.float32)


def gaussian_weights(duty: float, n_harm: int) -> np.ndarray:
    """Power weight of harmonics 1..n_harm of a Gaussian pulse of duty ``duty``."""
    k = np.arange(1, n_harm + 1, dtype=np.float64)
    return np.exp(-(math.pi ** 2) * k * k * duty * duty / (2.0 * math.log(2.0)))


def train_amplitude(weights: np.ndarray, snr: float) -> float:
    """Amplitude that makes the best ideal partial sum reach ``snr`` (unit noise)."""
    c = np.cumsum(weights) / np.sqrt(np.arange(1, len(weights) + 1))
    return float(snr / c.max())


def inject_train(x: np.ndarray, f0: float, weights: np.ndarray, amp: float,
                 spread: bool = False) -> None:
    """Add a pulse train in place (float64 arithmetic, stored back as float32).

    Harmonic k (1-based, ``k <= len(weights)``) is injected only where ``k f0``
    lies inside the array.
    """
    n = len(x)
    for k, w in enumerate(weights, start=1):
        centre = k * f0
        if centre >= n - 1:
            break
        p = amp * float(w)
        if not spread:
            m = int(round(centre))
            x[m] = np.float32(float(x[m]) + p)
            continue
        lo = max(0, int(math.floor(centre)) - 4)
        hi = min(n - 1, int(math.floor(centre)) + 5)
        for m in range(lo, hi + 1):
            u = m - centre
            s = 1.0 if u == 0.0 else math.sin(math.pi * u) / (math.pi * u)
            x[m] = np.float32(float(x[m]) + p * s * s)


def random_trains(g: np.random.Generator, count: int, n0_lo: int, n0_hi: int,
                  fractional: bool = False):
    """Draw ``count`` pulse trains: (f0, duty, snr), n0 uniform in [n0_lo, n0_hi)."""
    out = []
    for _ in range(count):
        n0 = int(g.integers(n0_lo, n0_hi))
        delta = float(g.random()) if fractional else 0.0
        duty = float(g.uniform(0.01, 0.2))
        snr = float(g.uniform(3.0, 15.0))
        out.append((n0 + delta, duty, snr))
    return out


def config1(n: int = 65536, seed: int = 1, n0: int = 1234, n_harm: int = 16,
            power: float = 8.0):
    """One spectrum of Exp(1) noise plus a train at bin ``n0`` with ``power/h`` at harmonic h."""
    noise = exp_noise(n, seed)
    x = noise.copy()
    for h in range(1, n_harm + 1):
        m = n0 * h
        x[m] = np.float32(float(noise[m]) + power / h)
    return x, noise


def config2(n: int = 1 << 22, seed: int = 2, n_trains: int = 50, max_harm: int = 32,
            fractional: bool = False):
    """Exp(1) spectrum with ``n_trains`` trains, fundamentals in [100, n/32)."""
    x = exp_noise(n, seed)
    g = rng(seed, 1)
    trains = random_trains(g, n_trains, 100, max(101, n // 32), fractional)
    for f0, duty, snr in trains:
        w = gaussian_weights(duty, 4 * max_harm)
        inject_train(x, f0, w, train_amplitude(w[:max_harm], snr), spread=fractional)
    return x, trains


def config3_lengths(n_spectra: int = 512, lo: int = 1 << 20, hi: int = 1 << 22,
                    seed: int = 3) -> np.ndarray:
    """Spectrum lengths drawn uniformly from [lo, hi]."""
    return rng(seed, 0).integers(lo, hi + 1, size=n_spectra).astype(np.int64)


def config3_spectrum(i: int, length: int, seed: int = 3, n_trains: int = 5,
                     max_harm: int = 32) -> np.ndarray:
    """Spectrum ``i`` of the batched workload: Exp(1) noise plus ``n_trains`` trains."""
    x = exp_noise(length, seed, 1, i)
    g = rng(seed, 2, i)
    for f0, duty, snr in random_trains(g, n_trains, 100, max(101, length // 32)):
        w = gaussian_weights(duty, 4 * max_harm)
        inject_train(x, f0, w, train_amplitude(w[:max_harm], snr))
    return x


def config3(n_spectra: int = 512, lo: int = 1 << 20, hi: int = 1 << 22, seed: int = 3,
            n_trains: int = 5, max_harm: int = 32, threads: int = 8):
    """Concatenated batch: (x float32 [sum N_s], offsets int64 [B+1])."""
    lengths = config3_lengths(n_spectra, lo, hi, seed)
    offsets = np.zeros(n_spectra + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    x = np.empty(int(offsets[-1]), dtype=np.float32)

    def fill(i: int) -> None:
        x[offsets[i]:offsets[i + 1]] = config3_spectrum(i, int(lengths[i]), seed, n_trains, max_harm)

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(fill, range(n_spectra)))
    return x, offsets


def inject_track(plane: np.ndarray, z_min: int, r0: int, z0: int, weights: np.ndarray,
                 amp: float) -> None:
    """Add an accelerated-pulsar track: harmonic k at (row k z0 - z_min, column k r0)."""
    n_z, n_r = plane.shape
    for k, w in enumerate(weights, start=1):
        r, i = k * r0, k * z0 - z_min
        if r >= n_r or i < 0 or i >= n_z:
            break
        plane[i, r] = np.float32(float(plane[i, r]) + amp * float(w))


def random_tracks(g: np.random.Generator, n_r: int, n_small: int = 15, n_large: int = 5,
                  small_z: int = 6, large_z=(7, 50)):
    """Tracks (r0, z0, duty, snr): ``n_small`` with |z0| <= small_z, ``n_large`` with |z0| in large_z."""
    out = []
    for j in range(n_small + n_large):
        r0 = int(g.integers(100, max(101, n_r // 16)))
        if j < n_small:
            z0 = int(g.integers(-small_z, small_z + 1))
        else:
            z0 = int(g.integers(large_z[0], large_z[1] + 1)) * (1 if g.random() < 0.5 else -1)
        out.append((r0, z0, float(g.uniform(0.01, 0.2)), float(g.uniform(3.0, 15.0))))
    return out


def config4(n_r: int = 1 << 21, z_min: int = -100, z_max: int = 100, seed: int = 4,
            max_harm: int = 16, threads: int = 8):
    """f-fdot plane [z_max - z_min + 1][n_r] of Exp(1) powers plus 20 tracks."""
    n_z = z_max - z_min + 1
    plane = np.empty((n_z, n_r), dtype=np.float32)

    def fill(i: int) -> None:
        plane[i] = exp_noise(n_r, seed, 1, i)

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(fill, range(n_z)))
    tracks = random_tracks(rng(seed, 2), n_r)
    for r0, z0, duty, snr in tracks:
        w = gaussian_weights(duty, 4 * max_harm)
        inject_track(plane, z_min, r0, z0, w, train_amplitude(w[:max_harm], snr))
    return plane, tracks


def table2(n_spectra: int = 1024, length: int = 131072, seed: int = 5, threads: int = 8):
    """The shape of the paper's performance comparison (Sec. 4.3: 1024 power
    spectra of 2^17 bins each): noise and trains drawn as for the batched
    workload, every spectrum ``length`` bins.  Returns (x, offsets)."""
    return config3(n_spectra=n_spectra, lo=length, hi=length, seed=seed, threads=threads)


def von_mises_kappa(duty: float) -> float:
    """Shape parameter of the modified von Mises pulse whose full width at half
    maximum is ``duty`` of the period: the half-maximum phase theta solves
    exp(kappa (cos theta - 1)) = 1/2 with theta = pi duty."""
    return math.log(2.0) / (1.0 - math.cos(math.pi * duty))


def von_mises_series(f_r: float, T: float = 20.0, ts: float = 64e-6, duty: float = 0.04, amp: float = 1.0,
                     phase: float = 0.0) -> np.ndarray:
    """Noise-free pulsar time series from the modified von Mises profile of
    Sec. 4.1 (float64): amp (exp(kappa cos(2 pi f_r t + phase)) - exp(-kappa))
    / (I0(kappa) - exp(-kappa)) at t = 0, ts, ..., the profile's mean removed
    is not done here (the DC bin is excluded from the sums anyway)."""
    kappa = von_mises_kappa(duty)
    n = int(round(T / ts))
    t = np.arange(n, dtype=np.float64) * ts
    # exp(kappa cos x) / I0(kappa) evaluated as exp(kappa (cos x - 1)) / (I0(kappa) e^-kappa) for large kappa
    i0e = float(np.i0(kappa)) * math.exp(-kappa) if kappa < 700 else 1.0 / math.sqrt(2.0 * math.pi * kappa)
    num = np.exp(kappa * (np.cos(2.0 * np.pi * f_r * t + phase) - 1.0)) - math.exp(-2.0 * kappa)
    return amp * num / (i0e - math.exp(-2.0 * kappa))


def power_spectrum(series: np.ndarray, noise_sigma: float = 1.0, seed: int | None = None) -> np.ndarray:
    """Power spectrum |FFT|^2 / (N sigma^2) of a real series, float32 (bins
    0..N/2), normalised so that white noise of standard deviation ``noise_sigma``
    per sample has unit mean power; with ``seed`` that noise is added to the
    series first."""
    x = np.asarray(series, dtype=np.float64)
    if seed is not None:
        x = x + rng(seed, 7).normal(0.0, noise_sigma, size=x.size)
    X = np.fft.rfft(x)
    return ((X.real ** 2 + X.imag ** 2) / (x.size * noise_sigma ** 2)).astype(np.float32)
