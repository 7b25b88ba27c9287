"""Oracle candidate lists vs hand-worked cases at the threshold.

A candidate is a bin whose best SNR (Eq. (2)) is strictly above the threshold
(reading R14: strict float compare, at least one harmonic summed).  The
fixture's spectra have dyadic statistics, so every SNR is exact in float and
several bins sit exactly on the threshold: a non-strict compare would list
them.  Both the batched path (statistics from the data) and the per-spectrum
path with the hand normalisation are checked, in both precisions.
"""
import numpy as np
import pytest

import oracle
from golden_io import read_candidates

VALUES, OFFSETS, CASES = read_candidates()
MODE = {"standard": oracle.STANDARD, "greedy": oracle.GREEDY}
HAND_NORM = [(2.0, 1.0), (3.0, 2.0)]     # (mu1, sigma1) of the two spectra, worked by hand


def _recs(c):
    return sorted((int(r["spectrum"]), int(r["bin"]), float(r["snr"]), int(r["harm"]), int(r["drift"])) for r in c)


def test_fixture_statistics_are_the_hand_values():
    for s, (mu1, sigma1) in enumerate(HAND_NORM):
        x = VALUES[OFFSETS[s]:OFFSETS[s + 1]]
        assert oracle.stats(x) == (mu1, sigma1 * sigma1)
        assert oracle.norm_from_data(x) == (mu1, sigma1)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-H%d-m%d-thr%g" % (c["mode"], c["H"], c["mask"], c["thr"]))
def test_batched_candidates(case, prec):
    r = oracle.hs_batched(VALUES, OFFSETS, case["H"], MODE[case["mode"]], case["thr"],
                          harmonic_mask=case["mask"], precision=prec)
    assert _recs(r["candidates"]) == sorted(case["cands"])


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-H%d-m%d-thr%g" % (c["mode"], c["H"], c["mask"], c["thr"]))
def test_candidates_of_hand_normalised_sums(case):
    got = []
    for s, norm in enumerate(HAND_NORM):
        x = VALUES[OFFSETS[s]:OFFSETS[s + 1]]
        r = oracle.hs_1d(x, case["H"], MODE[case["mode"]], harmonic_mask=case["mask"], norm=norm)
        got += _recs(oracle.candidates(r["snr"], r["harm"], r["drift"], case["thr"], spectrum=s))
    assert sorted(got) == sorted(case["cands"])


def test_fixture_has_ties_at_the_threshold():
    # at least one case whose listed candidates exclude a bin with an SNR equal to the threshold
    ties = 0
    for case in CASES:
        r = oracle.hs_batched(VALUES, OFFSETS, case["H"], MODE[case["mode"]], case["thr"] - 1.0,
                              harmonic_mask=case["mask"])
        ties += int(np.sum(r["candidates"]["snr"] == np.float32(case["thr"])))
    assert ties >= 6
