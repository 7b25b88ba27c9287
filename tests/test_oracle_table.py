"""Oracle with a caller-supplied per-k normalisation table (Eq. (2)).

Eq. (2) normalises the k-element partial sum by the mean and standard
deviation of a k-element sum.  With a table the caller gives (mu_k, sigma_k)
for every k directly; the SNR of the k-th partial sum is then
(S_k - mu_k) / sigma_k with the table's k-th entries.  The hand cases reuse
the hand-worked greedy sums of spectrum ``a`` in tests/golden/hand_1d.txt
(fundamental 1, H = 3: S = 4, 11, 16) and pick tables whose SNRs are exact,
so a table entry used for the wrong k changes the winner.
"""
import math

import numpy as np
import pytest

import oracle
from golden_io import read_1d

SPECTRA, _ = read_1d()
X = SPECTRA["a"]

# (mu_k, sigma_k), expected (harm, snr) of greedy fundamental 1 with H = 3
HAND = [
    (((0, 0, 0), (1, 1, 1)), (3, 16.0)),        # snr 4, 11, 16
    (((0, 0, 0), (1, 1, 4)), (2, 11.0)),        # snr 4, 11, 4
    (((0, 7, 12), (1, 1, 1)), (1, 4.0)),        # snr 4, 4, 4: ties go to the smaller k
    (((0, 7, 8), (1, 1, 2)), (1, 4.0)),         # snr 4, 4, 4
    (((4, 0, 0), (1, 1, 1)), (3, 16.0)),        # snr 0, 11, 16
    (((0, 0, 16), (2, 0.5, 1)), (2, 22.0)),     # snr 2, 22, 0
]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("table,want", HAND)
def test_hand_tables(table, want, prec):
    r = oracle.hs_1d(X, 3, oracle.GREEDY, norm_table=table, idx=[1], precision=prec)
    assert (int(r["harm"][0]), float(r["snr"][0])) == want
    assert int(r["drift"][0]) == {1: 1, 2: 2, 3: 3}[want[0]]    # drifts after steps 1, 2, 3 (hand_1d.txt)


@pytest.mark.parametrize("bad", [(0, 1, 1), (1, -1, 1), (1, 1, math.inf), (1, 1, math.nan)])
def test_unusable_sigma_gives_zeros(bad):
    r = oracle.hs_1d(X, 3, oracle.GREEDY, norm_table=((0, 0, 0), bad))
    assert not r["harm"].any() and not r["snr"].any()


def test_unusable_mean_gives_zeros():
    r = oracle.hs_1d(X, 3, oracle.STANDARD, norm_table=((0, math.inf, 0), (1, 1, 1)))
    assert not r["harm"].any() and not r["snr"].any()


def test_float_tables_rounded_once():
    mu, sig, rs, nm, ok = oracle.caller_tables([0.1, 0.3], [3.0, 7.0])
    assert ok and rs.dtype == np.float32
    assert rs[1] == np.float32(1.0 / 7.0) and nm[1] == np.float32(-(0.3 / 7.0))


@pytest.mark.parametrize("mode", [oracle.STANDARD, oracle.GREEDY])
def test_affine_table_equals_one_bin_statistics(mode):
    # the table mu_k = k mu1, sigma_k = sqrt(k) sigma1 is what the one-bin statistics imply
    g = np.random.default_rng(11)
    x = g.standard_exponential(5000).astype(np.float32)
    H = 17
    mu1, sigma1 = oracle.norm_from_data(x)
    table = ([k * mu1 for k in range(1, H + 1)], [math.sqrt(k) * sigma1 for k in range(1, H + 1)])
    for prec in ("f32", "f64"):
        a = oracle.hs_1d(x, H, mode, precision=prec)
        b = oracle.hs_1d(x, H, mode, precision=prec, norm_table=table)
        for k in ("snr", "harm", "drift"):
            assert np.array_equal(a[k], b[k]), (prec, k)


def test_batched_tables_are_per_spectrum():
    g = np.random.default_rng(12)
    off = np.array([0, 300, 700, 701 + 400], dtype=np.int64)
    x = g.standard_exponential(int(off[-1])).astype(np.float32)
    H = 4
    tabs = [((0.0,) * H, (1.0,) * H), ((1.0, 2.0, 3.0, 4.0), (1.0, 1.5, 2.0, 2.5)), ((0.5,) * H, (2.0,) * H)]
    r = oracle.hs_batched(x, off, H, oracle.GREEDY, 1.0, norm_tables=tabs, dense=True)
    for s in range(3):
        one = oracle.hs_1d(x[off[s]:off[s + 1]], H, oracle.GREEDY, norm_table=tabs[s])
        assert np.array_equal(r["spectra"][s]["snr"], one["snr"])
