"""CPU oracle of the incoherent harmonic sum -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library (package
``paper_2202_12817_amd``) never imports it, and the two share no code: the
oracle is written from the paper (Adamek, Roy & Armour, "A Novel Greedy
Approach To Harmonic Summing Using GPUs", arXiv:2202.12817) and checked
against what the paper and the mathematics fix (see ``tests/test_oracle_*``).

What it computes, in the paper's order:

1. Normalisation statistics (Sec. 2, Eq. (2); the mean and standard deviation
   of a partial sum, obtained by ``GetMeanStdev`` in Algorithms 1-2 and shared
   by all algorithms, Sec. 4).  Reading: per spectrum (per plane in 2D) the
   population mean ``mu1`` and variance ``var1`` of the stored powers over bins
   ``[first_bin, N)``, each the exact rational value rounded once to float64;
   ``sigma1 = sqrt(var1)`` rounded once.  The k-element partial sum is
   normalised with ``mu_k = k mu1`` and ``sigma_k = sqrt(k) sigma1`` (exact for
   independent bins of the simple sum).  :func:`stats` computes the sums
   exactly with integer arithmetic, so no summation order is involved.
2. Float tables for the float SNR: ``rs_k = float(1 / sigma_k)`` and
   ``nm_k = float(-(mu_k / sigma_k))``, each rounded once from float64.
3. The per-fundamental sums and the best SNR (``hs_oracle.c``): simple sum,
   Sec. 3.1 Eq. (3); greedy sum, Sec. 3.3 Eq. (5) and Algorithm 2; running
   maximum of the partial-sum SNRs, Eq. (2).  The PRESTO-style comparators of
   Sec. 3.2 (Eq. (4), Algorithm 1: PRESTO, PRESTO_all, PRESTO+) are indexed by
   the last bin of the series: stage K sums the bins nearest to ``h n / K``.
4. Candidates: every bin whose best SNR is strictly above a threshold.
5. The pipeline's neighbours: the power spectrum of complex FFT bins with
   optional inter-binning (the step before the sum, Sec. 2), and peak
   clustering of the candidates (the step after it).

Precision ``"f32"`` mirrors the precision of the GPU's decisions (float sums
in harmonic order, fused float SNR) for bit-exact comparison of harmonic
counts and drifts; ``"f64"`` is the float64 accuracy reference.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from fractions import Fraction

import numpy as np

__all__ = [
    "build", "exact_sums", "stats", "norm_from_data", "tables", "caller_tables", "is_degenerate",
    "hs_1d", "hs_2d", "hs_batched", "candidates", "quantize_f16",
    "GREEDY", "STANDARD", "PRESTO", "PRESTO_ALL", "PRESTO_PLUS",
    "power_spectrum", "cluster_peaks", "INTERBIN_FACTOR",
]

STANDARD = 0
GREEDY = 1
PRESTO = 2        # Sec. 3.2: power-of-two stages, fundamental + even harmonics
PRESTO_ALL = 3    # Sec. 3.2 / Sec. 5: power-of-two stages, every harmonic
PRESTO_PLUS = 4   # Sec. 3.2 / Sec. 5: every stage 1..H, every harmonic
MAX_H = 64

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_hs_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``hs_oracle.c`` into ``_hs_oracle.so`` with gcc."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
                        "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("HS_ORACLE_LIB")    # a deliberately broken build, for the pin audit
        if not path:
            path = build(force=False)
        lib = ctypes.CDLL(path)
        p = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        lib.hso_1d_f32.argtypes = [p, i64, i32, i32, i64, i64, u64, p, p, p, i64, p, p, p, i32, p, p]
        lib.hso_1d_f64.argtypes = [p, i64, i32, i32, i64, i64, u64, p, p, p, i64, p, p, p, i32, p, p]
        lib.hso_2d_f32.argtypes = [p, i64, i64, i32, i32, i32, i32, i64, i64, u64, p, p, p, i64, p, p, p]
        lib.hso_2d_f64.argtypes = [p, i64, i64, i32, i32, i32, i32, i64, i64, u64, p, p, p, i64, p, p, p]
        lib.hso_presto_f32.argtypes = [p, i64, i32, i32, i64, i64, u64, p, p, p, i64, p, p]
        lib.hso_presto_f64.argtypes = [p, i64, i32, i32, i64, i64, u64, p, p, p, i64, p, p]
        for f in (lib.hso_1d_f32, lib.hso_1d_f64, lib.hso_2d_f32, lib.hso_2d_f64,
                  lib.hso_presto_f32, lib.hso_presto_f64):
            f.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# 1. statistics, exactly
# ---------------------------------------------------------------------------

def exact_sums(values: np.ndarray, chunk: int = 1 << 24):
    """Exact ``(count, sum x, sum x^2)`` of float32 values, as Python Fractions.

    Every float32 is ``m 2^(e-24)`` with an integer significand ``|m| < 2^24``
    (``frexp``), so grouping by exponent and adding the integer significands
    (and their squares, split in 12-bit halves to stay inside int64) is exact.
    """
    v = np.asarray(values, dtype=np.float32).reshape(-1)
    if not np.all(np.isfinite(v)):
        raise ValueError("non-finite input")
    s1, s2 = Fraction(0), Fraction(0)
    for lo in range(0, v.size, chunk):
        m, e = np.frexp(v[lo:lo + chunk].astype(np.float64))
        mi = np.ldexp(m, 24).astype(np.int64)          # exact significand, |mi| < 2^24
        ai = np.abs(mi)
        order = np.argsort(e, kind="stable")
        es = e[order]
        starts = np.flatnonzero(np.r_[True, es[1:] != es[:-1]])
        exps = es[starts].astype(np.int64)
        hi, lw = ai >> 12, ai & 0xFFF                   # ai = hi 2^12 + lw
        sm = np.add.reduceat(mi[order], starts)
        shh = np.add.reduceat((hi * hi)[order], starts)
        shl = np.add.reduceat((hi * lw)[order], starts)
        sll = np.add.reduceat((lw * lw)[order], starts)
        for j, ev in enumerate(exps.tolist()):
            sq = (int(shh[j]) << 24) + (int(shl[j]) << 13) + int(sll[j])   # sum of ai^2
            s1 += Fraction(int(sm[j])) * (Fraction(2) ** (ev - 24))
            s2 += Fraction(sq) * (Fraction(2) ** (2 * ev - 48))
    return v.size, s1, s2


def stats(x: np.ndarray, first_bin: int = 1):
    """``(mu1, var1)``: population mean and variance of ``x[..., first_bin:]``.

    Both are the exact rational values rounded once to float64.  For a 2D plane
    the statistics cover every row (columns ``>= first_bin``).
    """
    a = np.asarray(x, dtype=np.float32)
    sel = a[..., first_bin:]
    count, s1, s2 = exact_sums(sel)
    if count == 0:
        return float("nan"), float("nan")
    mean = s1 / count
    var = (s2 - s1 * s1 / count) / count
    return float(mean), float(var)


def norm_from_data(x: np.ndarray, first_bin: int = 1):
    """``(mu1, sigma1)`` with ``sigma1 = sqrt(var1)`` rounded once."""
    mu1, var1 = stats(x, first_bin)
    return mu1, (math.sqrt(var1) if var1 >= 0 and math.isfinite(var1) else float("nan"))


def is_degenerate(mu1: float, sigma1: float) -> bool:
    """No usable normalisation: every output is zero."""
    return not (math.isfinite(mu1) and math.isfinite(sigma1) and sigma1 > 0.0)


# ---------------------------------------------------------------------------
# 2. tables
# ---------------------------------------------------------------------------

def tables(mu1: float, sigma1: float, H: int):
    """Per-k normalisation for k = 1..H.

    Returns ``(mu, sig, rs, nm)``: float64 ``mu_k = k mu1``,
    ``sig_k = sqrt(k) sigma1`` and the float32 ``rs_k = 1/sig_k``,
    ``nm_k = -(mu_k/sig_k)``, each operation rounded once in float64 and the
    float32 values rounded once from those.
    """
    mu = np.empty(H, dtype=np.float64)
    sig = np.empty(H, dtype=np.float64)
    rs = np.empty(H, dtype=np.float32)
    nm = np.empty(H, dtype=np.float32)
    for k in range(1, H + 1):
        m = float(k) * mu1
        s = math.sqrt(float(k)) * sigma1
        mu[k - 1], sig[k - 1] = m, s
        rs[k - 1] = np.float32(1.0 / s)
        nm[k - 1] = np.float32(-(m / s))
    return mu, sig, rs, nm


def caller_tables(mu_k, sigma_k):
    """Per-k normalisation supplied by the caller (Eq. (2): the k-element sum
    is normalised by the mean and deviation of a k-element sum, here given
    for each k instead of derived from the one-bin statistics).

    Returns ``(mu, sig, rs, nm, usable)``: the float64 tables as given, the
    float32 ``rs_k = 1/sigma_k`` and ``nm_k = -(mu_k/sigma_k)`` (each operation
    rounded once in float64, then once to float32), and whether every entry
    is finite with every ``sigma_k > 0`` (otherwise every output is zero).
    """
    mu = np.array(mu_k, dtype=np.float64).reshape(-1)
    sig = np.array(sigma_k, dtype=np.float64).reshape(-1)
    if mu.size != sig.size or mu.size < 1:
        raise ValueError("mu_k and sigma_k need one entry per k")
    usable = bool(np.all(np.isfinite(mu)) and np.all(np.isfinite(sig)) and np.all(sig > 0.0))
    rs = np.zeros(mu.size, dtype=np.float32)
    nm = np.zeros(mu.size, dtype=np.float32)
    if usable:
        for i in range(mu.size):
            rs[i] = np.float32(1.0 / float(sig[i]))
            nm[i] = np.float32(-(float(mu[i]) / float(sig[i])))
    return mu, sig, rs, nm, usable


# ---------------------------------------------------------------------------
# 3. the sums
# ---------------------------------------------------------------------------

def _kmask(mask: int, H: int) -> int:
    return ((1 << H) - 1) if not mask else (mask & ((1 << H) - 1))


def _check(H, mode, modes=(STANDARD, GREEDY, PRESTO, PRESTO_ALL, PRESTO_PLUS)):
    if not (1 <= H <= MAX_H):
        raise ValueError("H out of range")
    if mode not in modes:
        raise ValueError("bad mode")


def hs_1d(x, H, mode, *, first_bin=1, fundamental_end=0, harmonic_mask=0,
          precision="f32", norm=None, norm_table=None, idx=None, report=()):
    """Harmonic sum of one spectrum.

    ``norm``: ``(mu1, sigma1)`` to use instead of the statistics of ``x``;
    ``norm_table``: ``(mu_k, sigma_k)``, two sequences of H values, used as
    given for the k-element sums (see :func:`caller_tables`).
    ``idx``: fundamentals to evaluate (default: every bin, output index = bin).
    ``report``: harmonic counts K whose partial sums are returned (zero where a
    fundamental sums fewer than K harmonics; simple and greedy sums only).
    PRESTO modes: the output index is the last bin of the series, ``harm`` the
    order K of the best stage and ``drift`` zero; ``fundamental_end`` bounds
    the last bin.
    Returns a dict with ``snr``, ``harm``, ``drift``, ``partial``, ``mu1``, ``sigma1``.
    """
    _check(H, mode)
    presto = mode in (PRESTO, PRESTO_ALL, PRESTO_PLUS)
    if presto and len(list(report)):
        raise ValueError("partial sums are reported for the simple and greedy sums only")
    x = np.ascontiguousarray(x, dtype=np.float32)
    N = x.size
    tab = None
    if norm_table is not None:
        tab = caller_tables(norm_table[0], norm_table[1])
        if tab[0].size != H:
            raise ValueError("norm_table needs H entries")
        mu1, sigma1 = float(tab[0][0]), float(tab[1][0])
    elif norm is None:
        mu1, sigma1 = norm_from_data(x, first_bin)
    else:
        mu1, sigma1 = float(norm[0]), float(norm[1])
    idx_a = None if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    n_out = N if idx_a is None else idx_a.size
    f64 = precision == "f64"
    snr = np.zeros(n_out, dtype=np.float64 if f64 else np.float32)
    harm = np.zeros(n_out, dtype=np.uint8)
    drift = np.zeros(n_out, dtype=np.uint8)
    rep = np.ascontiguousarray(list(report), dtype=np.int32)
    partial = np.zeros((len(rep), n_out), dtype=snr.dtype) if len(rep) else None
    out = dict(snr=snr, harm=harm, drift=drift, partial=partial, mu1=mu1, sigma1=sigma1)
    if (not tab[4] if tab is not None else is_degenerate(mu1, sigma1)) or n_out == 0:
        return out
    mu, sig, rs, nm = tab[:4] if tab is not None else tables(mu1, sigma1, H)
    n_end = N if not fundamental_end else min(N, int(fundamental_end))
    lib = _load()
    t1, t2 = (mu, sig) if f64 else (rs, nm)
    if presto:
        fn = lib.hso_presto_f64 if f64 else lib.hso_presto_f32
        fn(_ptr(x), N, H, mode, int(first_bin), n_end, _kmask(harmonic_mask, H), _ptr(t1), _ptr(t2),
           _ptr(idx_a), n_out, _ptr(snr), _ptr(harm))
        return out
    fn = lib.hso_1d_f64 if f64 else lib.hso_1d_f32
    fn(_ptr(x), N, H, mode, int(first_bin), n_end, _kmask(harmonic_mask, H), _ptr(t1), _ptr(t2),
       _ptr(idx_a), n_out, _ptr(snr), _ptr(harm), _ptr(drift), len(rep),
       _ptr(rep) if len(rep) else None, _ptr(partial))
    return out


def hs_2d(plane, z_min, z_max, H, mode, *, first_bin=1, fundamental_end=0,
          harmonic_mask=0, precision="f32", norm=None, norm_table=None, idx=None):
    """Harmonic sum of an f-fdot plane (rows ``z_min..z_max``, row-major).

    Harmonic k of fundamental (r, z) reads row ``k z`` at column ``k r`` (plus
    the drift along r); the sum stops before the first row outside the plane.
    Statistics cover the whole plane (columns ``>= first_bin``).
    ``idx``: flat fundamentals ``i n_r + r`` (default: all).
    """
    _check(H, mode, (STANDARD, GREEDY))
    p = np.ascontiguousarray(plane, dtype=np.float32)
    n_z, n_r = p.shape
    if n_z != z_max - z_min + 1:
        raise ValueError("plane rows do not match z range")
    tab = None
    if norm_table is not None:
        tab = caller_tables(norm_table[0], norm_table[1])
        if tab[0].size != H:
            raise ValueError("norm_table needs H entries")
        mu1, sigma1 = float(tab[0][0]), float(tab[1][0])
    elif norm is None:
        mu1, sigma1 = norm_from_data(p, first_bin)
    else:
        mu1, sigma1 = float(norm[0]), float(norm[1])
    idx_a = None if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    n_out = n_z * n_r if idx_a is None else idx_a.size
    f64 = precision == "f64"
    snr = np.zeros(n_out, dtype=np.float64 if f64 else np.float32)
    harm = np.zeros(n_out, dtype=np.uint8)
    drift = np.zeros(n_out, dtype=np.uint8)
    out = dict(snr=snr, harm=harm, drift=drift, mu1=mu1, sigma1=sigma1)
    if (not tab[4] if tab is not None else is_degenerate(mu1, sigma1)) or n_out == 0:
        return out
    mu, sig, rs, nm = tab[:4] if tab is not None else tables(mu1, sigma1, H)
    n_end = n_r if not fundamental_end else min(n_r, int(fundamental_end))
    lib = _load()
    fn = lib.hso_2d_f64 if f64 else lib.hso_2d_f32
    t1, t2 = (mu, sig) if f64 else (rs, nm)
    fn(_ptr(p), n_r, n_r, int(z_min), int(z_max), H, mode, int(first_bin), n_end,
       _kmask(harmonic_mask, H), _ptr(t1), _ptr(t2), _ptr(idx_a), n_out,
       _ptr(snr), _ptr(harm), _ptr(drift))
    if idx_a is None:
        for k in ("snr", "harm", "drift"):
            out[k] = out[k].reshape(n_z, n_r)
    return out


# ---------------------------------------------------------------------------
# 4. batches and candidates
# ---------------------------------------------------------------------------

CANDIDATE_DTYPE = np.dtype([("spectrum", "<u4"), ("bin", "<u4"), ("snr", "<f4"),
                            ("harm", "<u2"), ("drift", "<u2")])


def candidates(snr, harm, drift, threshold, spectrum=0, bins=None):
    """Records ``(spectrum, bin, snr, harm, drift)`` with ``snr > threshold``
    (float32 comparison) and at least one harmonic summed, sorted by bin."""
    snr32 = np.asarray(snr, dtype=np.float32)
    sel = (snr32 > np.float32(threshold)) & (np.asarray(harm) > 0)
    b = np.flatnonzero(sel) if bins is None else np.asarray(bins)[sel]
    out = np.zeros(b.size, dtype=CANDIDATE_DTYPE)
    out["spectrum"] = spectrum
    out["bin"] = b
    out["snr"] = snr32[sel]
    out["harm"] = np.asarray(harm)[sel]
    out["drift"] = np.asarray(drift)[sel]
    return out


def hs_batched(x, offsets, H, mode, threshold, *, first_bin=1, fundamental_end=0,
               harmonic_mask=0, precision="f32", spectra=None, dense=False, norm_tables=None):
    """Independent spectra ``x[offsets[s]:offsets[s+1]]``, each with its own statistics.

    Returns ``candidates`` (sorted by spectrum then bin) and, with ``dense``,
    the per-spectrum outputs.  ``spectra`` restricts the work to a subset.
    ``norm_tables``: ``[n_spectra][2][H]`` caller tables (mu_k, then sigma_k)
    instead of the statistics.
    """
    offsets = np.asarray(offsets, dtype=np.int64)
    which = range(len(offsets) - 1) if spectra is None else spectra
    cands, per = [], {}
    for s in which:
        r = hs_1d(x[offsets[s]:offsets[s + 1]], H, mode, first_bin=first_bin,
                  fundamental_end=fundamental_end, harmonic_mask=harmonic_mask,
                  precision=precision,
                  norm_table=None if norm_tables is None else (norm_tables[s][0], norm_tables[s][1]))
        cands.append(candidates(r["snr"], r["harm"], r["drift"], threshold, spectrum=s))
        if dense:
            per[s] = r
    c = np.concatenate(cands) if cands else np.zeros(0, dtype=CANDIDATE_DTYPE)
    return dict(candidates=c, spectra=per)


def quantize_f16(x, scale):
    """FP16 storage of powers: ``fp16_rne(clamp(float32(x) / float32(scale), +-65504))``.

    The division is one correctly rounded float32 operation; the conversion to
    half rounds to nearest even.  Decoding (``astype(float32)``) is exact.
    """
    q = np.asarray(x, dtype=np.float32) / np.float32(scale)
    return np.clip(q, np.float32(-65504.0), np.float32(65504.0)).astype(np.float16)


# ---------------------------------------------------------------------------
# 5. pipeline neighbours: power spectrum with inter-binning, peak clustering
# ---------------------------------------------------------------------------

INTERBIN_FACTOR = np.float32((math.pi * math.pi) / 16.0)    # (pi/4)^2, rounded once to float


def power_spectrum(fft, interbin=False, scale=1.0):
    """Powers of complex FFT bins ``fft`` (complex64, N bins), float32.

    The harmonic sum runs on a power spectrum, possibly inter-binned (Sec. 2;
    the paper cites Ransom et al. 2002 for the step).  Integer bin m:
    ``scale * (re^2 + im^2)``; with ``interbin`` the N - 1 half bins between m
    and m + 1 are added, interleaved (output 2N - 1 values, bin 2m = bin m,
    bin 2m + 1 = half bin m + 1/2): the half-bin amplitude of a
    rectangular-window DFT is estimated as (pi/4)(F_m - F_{m+1}), so its power
    is ``(scale (pi/4)^2) |F_m - F_{m+1}|^2``.  Every operation is one float32
    rounding in the order written: ``p = re*re + im*im`` (two products, one
    sum), then one product with the float factor.
    """
    F = np.ascontiguousarray(fft, dtype=np.complex64)
    re, im = F.real.astype(np.float32), F.imag.astype(np.float32)
    sc = np.float32(scale)
    p = (re * re + im * im) * sc
    if not interbin:
        return p
    dr = re[:-1] - re[1:]
    di = im[:-1] - im[1:]
    fh = np.float32(float(scale) * float(INTERBIN_FACTOR))      # scale (pi/4)^2, one rounding from float64
    h = (dr * dr + di * di) * fh
    out = np.empty(2 * F.size - 1, dtype=np.float32)
    out[0::2] = p
    out[1::2] = h
    return out


def cluster_peaks(snr, harm, drift, threshold, radius, offsets=None):
    """Candidates that are peaks: ``snr > threshold`` (float32, strict), at
    least one harmonic summed, and no bin of the same spectrum within
    ``radius`` bins beats it (a larger SNR, or an equal SNR at a lower bin).
    Returns CANDIDATE_DTYPE records sorted by (spectrum, bin); ``offsets``
    (CSR) splits the dense arrays into spectra (None: one spectrum)."""
    snr = np.asarray(snr, dtype=np.float32)
    harm = np.asarray(harm)
    drift = np.asarray(drift)
    off = np.array([0, snr.size], dtype=np.int64) if offsets is None else np.asarray(offsets, dtype=np.int64)
    recs = []
    for s in range(off.size - 1):
        lo, hi = int(off[s]), int(off[s + 1])
        for n in range(lo, hi):
            v = snr[n]
            if not (v > np.float32(threshold)) or harm[n] == 0:
                continue
            keep = True
            for j in range(max(lo, n - radius), min(hi, n + radius + 1)):
                if j != n and (snr[j] > v or (snr[j] == v and j < n)):
                    keep = False
                    break
            if keep:
                recs.append((s, n - lo, v, int(harm[n]), int(drift[n])))
    out = np.zeros(len(recs), dtype=CANDIDATE_DTYPE)
    for i, r in enumerate(recs):
        out[i] = r
    return out
