"""Sensitivity and recovered-SNR experiments of Sec. 4.1 on noise-free pulsars.

A pulsar time series from the modified von Mises profile (Sec. 4.1, Eq. (10))
is turned into a power spectrum (``synthetic``) and every harmonic-sum
algorithm's recovered SNR (RSNR) is read off it:

* sensitivity loss (Eq. (11)): the pulsar frequency steps from the centre of
  bin n0 to the centre of bin n0 + 1 (50 steps in the paper) and
  ``l(f) = RSNR(f) / RSNR(centre)``;
* RSNR against the sub-bin frequency at H = 32 (the paper's Fig. 9);
* the average RSNR over the sub-bin steps for several fundamental
  frequencies, maximum harmonic orders H and sampling times (Fig. 10).

Readings (the paper does not fix them):

* normalisation: the spectrum is scaled so that white noise of unit
  standard deviation per sample has unit mean power, and the sums are
  normalised with mu1 = sigma1 = 1 (the unit-noise reference), so that the
  RSNR of a noise-free pulsar does not depend on statistics of the signal
  itself and is comparable between algorithms;
* RSNR of an algorithm = the largest SNR it reports at the bins where it
  reports this pulsar: the fundamental bin n0 - 1 .. n0 + 2 for the simple
  and greedy sums (fundamental-indexed outputs), and the last bins
  K n0 - 1 .. K n0 + K + 1 of every stage K for the PRESTO-style sums
  (last-bin-indexed outputs);
* "duty cycle" = full width at half maximum of the pulse over its period.

The sums run on the GPU through the library by default; ``backend`` lets a
caller substitute another implementation of the same call (the tests pass
the CPU oracle there to check the experiments' claims, and compare the two
backends bit for bit).
"""
from __future__ import annotations

import json
import sys

import numpy as np

MODES = {"standard": 0, "greedy": 1, "presto": 2, "presto_all": 3, "presto_plus": 4}
LAST_BIN_MODES = (2, 3, 4)


def detection_bins(n0: int, H: int, mode: int, n_bins: int) -> np.ndarray:
    """Output bins at which ``mode`` reports a pulsar of fundamental bin n0..n0+1."""
    if mode in LAST_BIN_MODES:
        out = set()
        for K in range(1, H + 1):
            for b in range(K * n0 - 1, K * (n0 + 1) + 2):
                if 0 < b < n_bins:
                    out.add(b)
        return np.array(sorted(out), dtype=np.int64)
    return np.arange(max(1, n0 - 1), min(n_bins, n0 + 3), dtype=np.int64)


def gpu_backend(P: np.ndarray, H: int, mode: int, norm, idx: np.ndarray) -> np.ndarray:
    """SNR at the bins ``idx`` of spectrum ``P`` from the library (dense call on cuda:0)."""
    import torch

    from . import ops
    dev = torch.device("cuda:0")
    got = ops.sum_1d(torch.from_numpy(np.ascontiguousarray(P, dtype=np.float32)).to(dev), H, mode, norm=norm)
    return got["snr"][torch.from_numpy(idx).to(dev)].cpu().numpy()


def rsnr(P: np.ndarray, n0: int, H: int, mode: int, backend=None) -> float:
    """Recovered SNR of ``mode`` for a pulsar of fundamental bin n0 (see the readings above)."""
    backend = backend or gpu_backend
    idx = detection_bins(n0, H, mode, P.size)
    return float(np.max(backend(P, H, mode, (1.0, 1.0), idx)))


def sensitivity_sweep(n0: int = 200, steps: int = 50, H: int = 32, modes=tuple(MODES), T: float = 20.0,
                      ts: float = 64e-6, duty: float = 0.04, amp: float = 0.02, backend=None):
    """RSNR and sensitivity loss l(f) of each mode as the pulsar frequency steps
    from the centre of bin n0 to the centre of bin n0 + 1 (steps + 1 points)."""
    import synthetic
    wf = 1.0 / T
    freqs = [(n0 + j / steps) * wf for j in range(steps + 1)]
    out = {"frequency_hz": freqs, "bin_width_hz": wf, "H": H, "n0": n0}
    spectra = [synthetic.power_spectrum(synthetic.von_mises_series(f, T, ts, duty, amp)) for f in freqs]
    for name in modes:
        m = MODES[name]
        r = np.array([rsnr(P, n0, H, m, backend) for P in spectra])
        out[name] = {"rsnr": r.tolist(), "loss": (r / r[0]).tolist()}
    return out


def average_rsnr(freqs_hz=(10.0, 100.0, 200.0, 400.0, 800.0, 1600.0), Hs=(4, 8, 16, 32), ts_list=(64e-6, 32e-6),
                 mode: str = "greedy", steps: int = 10, T: float = 20.0, duty: float = 0.04, amp: float = 0.02,
                 backend=None):
    """Mean RSNR over ``steps`` sub-bin positions of a pulsar near each
    fundamental frequency, for each H and sampling time."""
    import synthetic
    wf = 1.0 / T
    out = {"frequency_hz": list(freqs_hz), "H": list(Hs), "ts": list(ts_list), "mode": mode, "avg_rsnr": {}}
    for ts in ts_list:
        rows = []
        for fc in freqs_hz:
            n0 = int(round(fc / wf))
            spectra = [synthetic.power_spectrum(synthetic.von_mises_series((n0 + j / steps) * wf, T, ts, duty, amp))
                       for j in range(steps)]
            rows.append([float(np.mean([rsnr(P, n0, H, MODES[mode], backend) for P in spectra])) for H in Hs])
        out["avg_rsnr"]["%g" % ts] = rows
    return out


def main(argv=None) -> None:
    """Print both experiments as one JSON object (sums on the GPU)."""
    argv = sys.argv[1:] if argv is None else argv
    steps = int(argv[0]) if argv else 50
    res = {"sensitivity": sensitivity_sweep(steps=steps), "average": average_rsnr()}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
