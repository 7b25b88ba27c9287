"""The sensitivity experiments of Sec. 4.1 on noise-free von Mises pulsars.

CPU: the experiments run on the oracle and must show what the paper states
about them (Sec. 4.1 and Sec. 5; no values are printed, so the checks are the
stated relations):
* PRESTO+ has the same sensitivity loss as the greedy sum, and on data without
  noise the two recover the same SNR;
* the greedy loss is symmetric about the border between the two bins
  (correct drift tracking);
* the simple sum suffers the largest loss;
* PRESTO recovers less than the greedy sum (it sums fewer harmonics), and
  PRESTO_all has almost the same loss as PRESTO;
* the average RSNR falls at high fundamental frequencies for coarse sampling,
  and the fall starts at a higher frequency with twice the sampling rate;
  more harmonics never lower the RSNR.
GPU: the same experiments with the sums on the GPU give the oracle's numbers
bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2202_12817_amd import sensitivity


def oracle_backend(P, H, mode, norm, idx):
    return oracle.hs_1d(P, H, mode, norm=norm, idx=idx)["snr"]


@pytest.fixture(scope="module")
def sweep():
    return sensitivity.sensitivity_sweep(steps=20, backend=oracle_backend)


def test_presto_plus_matches_greedy(sweep):
    # "the same" of a plot: within 5 % at every step and 1 % on average (50 steps:
    # at most 3.2 %, 0.4 % on average)
    g, p = np.array(sweep["greedy"]["rsnr"]), np.array(sweep["presto_plus"]["rsnr"])
    dev = np.abs(p / g - 1.0)
    assert np.all(dev < 0.05) and dev.mean() < 0.01
    dl = np.abs(np.array(sweep["presto_plus"]["loss"]) - np.array(sweep["greedy"]["loss"]))
    assert np.all(dl < 0.05) and dl.mean() < 0.01


def test_greedy_loss_symmetric_about_the_bin_border(sweep):
    loss = np.array(sweep["greedy"]["loss"])
    assert np.all(np.abs(loss - loss[::-1]) < 0.03)
    assert loss.min() < 0.9             # there is a loss between the centres


def test_simple_sum_loses_most(sweep):
    simple = np.array(sweep["standard"]["loss"])
    for other in ("greedy", "presto", "presto_all", "presto_plus"):
        assert simple.min() < np.array(sweep[other]["loss"]).min() - 0.3, other
    assert np.argmin(simple) == len(simple) // 2         # worst at the border between the bins


def test_presto_recovers_less_and_presto_all_loses_alike(sweep):
    assert np.all(np.array(sweep["presto"]["rsnr"]) < np.array(sweep["greedy"]["rsnr"]))
    assert np.all(np.abs(np.array(sweep["presto_all"]["loss"]) - np.array(sweep["presto"]["loss"])) < 0.06)


def test_average_rsnr_against_frequency_h_and_sampling():
    r = sensitivity.average_rsnr(freqs_hz=(100.0, 1600.0), Hs=(4, 16, 32), steps=5, backend=oracle_backend)
    a64, a32 = np.array(r["avg_rsnr"]["6.4e-05"]), np.array(r["avg_rsnr"]["3.2e-05"])
    assert np.all(np.diff(a64, axis=1) >= 0) and np.all(np.diff(a32, axis=1) >= 0)   # H never hurts
    fall64 = a64[1, -1] / a64[0, -1]
    fall32 = a32[1, -1] / a32[0, -1]
    assert fall64 < 0.9                  # coarse sampling: the high fundamental loses
    assert fall32 > fall64               # finer sampling keeps more


def test_detection_bins():
    assert list(sensitivity.detection_bins(200, 4, 1, 10 ** 6)) == [199, 200, 201, 202]
    b = sensitivity.detection_bins(10, 3, 4, 10 ** 6)
    for K in (1, 2, 3):
        assert {K * 10 - 1, K * 11 + 1} <= set(b)


@pytest.mark.gpu
def test_gpu_sweep_equals_oracle_sweep():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    a = sensitivity.sensitivity_sweep(steps=10, backend=oracle_backend)
    b = sensitivity.sensitivity_sweep(steps=10)
    for m in sensitivity.MODES:
        assert a[m]["rsnr"] == b[m]["rsnr"], m
    c = sensitivity.average_rsnr(freqs_hz=(100.0, 1600.0), Hs=(8, 32), steps=3, backend=oracle_backend)
    d = sensitivity.average_rsnr(freqs_hz=(100.0, 1600.0), Hs=(8, 32), steps=3)
    assert c["avg_rsnr"] == d["avg_rsnr"]
