"""Oracle vs hand-worked examples of Eq. (3), Eq. (5)/Algorithm 2 and Eq. (2).

The fixtures in tests/golden/ were worked out by hand from the paper's
definitions; they pin the bin choices, drift updates, tie rules, truncation
and the SNR argmax independently of the oracle's code.
"""
import math

import numpy as np
import pytest

import oracle
from golden_io import read_1d, read_2d

SPECTRA, CASES_1D = read_1d()
PLANE, Z_MIN, Z_MAX, CASES_2D = read_2d()
MODE = {"standard": oracle.STANDARD, "greedy": oracle.GREEDY}


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES_1D, ids=lambda c: "%s-%s-H%d-m%d-n%d" % (
    c["spectrum"], c["mode"], c["H"], c["mask"], c["n"]))
def test_hand_1d(case, prec):
    x = SPECTRA[case["spectrum"]]
    H = case["H"]
    r = oracle.hs_1d(x, H, MODE[case["mode"]], harmonic_mask=case["mask"], precision=prec,
                     norm=(0.0, 1.0), idx=[case["n"]], report=range(1, H + 1))
    S = case["S"]
    got = [float(r["partial"][k, 0]) for k in range(H)]
    want = S + [0.0] * (H - len(S))
    assert got == want
    assert int(r["harm"][0]) == case["harm"]
    assert int(r["drift"][0]) == case["drift"]
    kb = case["harm"]
    want_snr = 0.0 if kb == 0 else S[kb - 1] / math.sqrt(kb)
    tol = 1e-6 * max(1.0, abs(want_snr)) if prec == "f32" else 1e-14 * max(1.0, abs(want_snr))
    assert abs(float(r["snr"][0]) - want_snr) <= tol


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES_2D, ids=lambda c: "%s-r%d-z%d" % (c["mode"], c["r"], c["z"]))
def test_hand_2d(case, prec):
    n_r = PLANE.shape[1]
    flat = (case["z"] - Z_MIN) * n_r + case["r"]
    r = oracle.hs_2d(PLANE, Z_MIN, Z_MAX, case["H"], MODE[case["mode"]], precision=prec,
                     norm=(0.0, 1.0), idx=[flat])
    assert int(r["harm"][0]) == case["harm"]
    assert int(r["drift"][0]) == case["drift"]
    kb = case["harm"]
    want_snr = 0.0 if kb == 0 else case["S"][kb - 1] / math.sqrt(kb)
    assert abs(float(r["snr"][0]) - want_snr) <= 1e-6 * max(1.0, abs(want_snr))


def test_golden_files_cover_both_modes():
    modes = {c["mode"] for c in CASES_1D} | {c["mode"] for c in CASES_2D}
    assert modes == {"standard", "greedy"}
    assert any(c["mask"] for c in CASES_1D)
