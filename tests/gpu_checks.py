"""Comparison helpers of the GPU tests (bars stated in test_gpu_parity)."""
import numpy as np

import oracle

TOL = 1e-5


def _np(t):
    return t.cpu().numpy()


def check_dense(got, want32, want64, label=""):
    harm, drift, snr = _np(got["harm"]).reshape(-1), _np(got["drift"]).reshape(-1), _np(got["snr"]).reshape(-1)
    wh, wd, ws = want32["harm"].reshape(-1), want32["drift"].reshape(-1), want32["snr"].reshape(-1)
    bad = np.flatnonzero((harm != wh) | (drift != wd))
    assert bad.size == 0, "%s: %d index mismatches, first at %s: gpu (%d,%d) oracle (%d,%d)" % (
        label, bad.size, bad[:5], harm[bad[0]], drift[bad[0]], wh[bad[0]], wd[bad[0]])
    sb = np.flatnonzero(snr.view(np.uint32) != ws.view(np.uint32))
    assert sb.size == 0, "%s: %d SNR values differ from the float mirror, first %s: %r vs %r" % (
        label, sb.size, sb[:5], snr[sb[0]], ws[sb[0]])
    if want64 is not None:
        s64 = want64["snr"].reshape(-1)
        err = np.abs(snr.astype(np.float64) - s64) / np.maximum(1.0, np.abs(s64))
        assert float(err.max(initial=0.0)) <= TOL, "%s: SNR error %.3g" % (label, float(err.max()))


def check_norm(got, x, first_bin, H, label=""):
    mu1, sigma1 = oracle.norm_from_data(x, first_bin)
    ms = _np(got["mu_sigma"])[0]
    assert ms[0] == mu1 and ms[1] == sigma1, "%s: stats (%r, %r) vs oracle (%r, %r)" % (
        label, ms[0], ms[1], mu1, sigma1)
    _, _, rs, nm = oracle.tables(mu1, sigma1, H)
    tab = _np(got["tables"])[0]
    assert np.array_equal(tab[0], rs) and np.array_equal(tab[1], nm), label


def _cands(out):
    recs, n = _candidates_numpy(out)
    recs = np.sort(recs, order=["spectrum", "bin"])
    return recs, n


def _same_records(a, b):
    if a.size != b.size:
        return False
    return all(np.array_equal(a[f], b[f]) for f in ("spectrum", "bin", "harm", "drift")) and \
        np.array_equal(a["snr"].view(np.uint32), b["snr"].view(np.uint32))


def _candidates_numpy(out):
    from paper_2202_12817_amd import ops
    return ops.candidates_numpy(out)
