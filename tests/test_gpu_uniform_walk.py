"""GPU: the wave-uniform walk against the walk with a bound per lane.

The harmonic-sum kernels walk a wave without per-lane bounds when all 64 of
its fundamentals sum the same number of harmonics K(n) = min(H, (N-1)/(n +
greedy)), lie inside [first_bin, fundamental_end) and have every harmonic
eligible; any other wave takes the walk with a bound per lane.  These cases
put the meeting points where they are easiest to get wrong: spectrum
lengths whose harmonic-count thresholds (N-1)/k - greedy fall on the first,
a middle and the last lane of a wave, first_bin and fundamental_end inside a
wave, on its first lane and just past it, and partial eligibility masks.
The persistent kernel at every fundamentals-per-lane shape and the plain
kernel, batched and single-spectrum, FP32 and FP16 storage, are held to the
oracle's float mirror bit for bit (Sec. 3.3 Algorithm 2, Eq. (2)).
"""
import numpy as np
import pytest

import oracle
from gpu_checks import _cands, _same_records, check_dense

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MODES = {"standard": oracle.STANDARD, "greedy": oracle.GREEDY}
THR = 4.0
OPTIONS = [{}, {"first_bin": 37}, {"first_bin": 64}, {"first_bin": 65}, {"fundamental_end": 4097},
           {"fundamental_end": 9613}, {"harmonic_mask": 0b1011},
           {"first_bin": 37, "fundamental_end": 9613, "harmonic_mask": (1 << 17) - 1}]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_12817_amd import hs
    hs.load()
    return torch.device("cuda:0")


def _lengths(greedy):
    """Lengths N with (N - 1) // k - greedy = 64 m + s for lanes s = 0, 31, 63."""
    g = 1 if greedy else 0
    out = []
    for k, m in ((2, 150), (3, 100), (17, 20), (32, 9)):
        for s in (0, 31, 63):
            t = 64 * m + s
            n = k * (t + g) + 1
            assert (n - 1) // k - g == t
            out.append(n)
    return out


def _input(mode, f16, seed):
    lens = _lengths(mode == "greedy")
    rng = np.random.default_rng(seed)
    x = rng.exponential(1.0, sum(lens)).astype(np.float32)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    if f16:
        x = oracle.quantize_f16(x, np.float32(1.0)).astype(np.float32)
    return x, off


def _device(x, f16, dev):
    if f16:
        return torch.from_numpy(x.astype(np.float16).view(np.int16)).to(dev).view(torch.float16)
    return torch.from_numpy(x).to(dev)


@pytest.mark.parametrize("H", [17, 32])
@pytest.mark.parametrize("f16", [False, True])
@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_batched_walks_meet(dev, mode, f16, H):
    from paper_2202_12817_amd import hs, ops
    x, off = _input(mode, f16, 900 + H + (7 if f16 else 0))
    xt, ot = _device(x, f16, dev), torch.from_numpy(off).to(dev)
    for opts in OPTIONS:
        w = oracle.hs_batched(x, off, H, MODES[mode], THR, dense=True, **opts)
        for shape in ((1, 1), (2, 1), (4, 1), (4, 3), (0, 0)):
            print("batched", mode, "f16" if f16 else "f32", H, opts, shape, flush=True)
            plan = ops.make_plan(H, mode, hs.HS_F16 if f16 else hs.HS_F32, max_spectra=off.size - 1, threshold=THR,
                                 **opts)
            try:
                hs.hs_plan_set_launch(plan.handle, *shape)
                got = ops.sum_batched(xt, ot, H, mode, THR, dense=True, candidates=True, capacity=x.size,
                                      plan=plan)
                torch.cuda.synchronize()
            finally:
                plan.close()
            label = "%s %s H=%d %s shape %s" % (mode, f16, H, opts, shape)
            for s in range(off.size - 1):
                sl = slice(off[s], off[s + 1])
                check_dense({k: got[k][sl] for k in ("snr", "harm", "drift")}, w["spectra"][s], None,
                            "%s spectrum %d" % (label, s))
            recs, n = _cands(got)
            assert n == w["candidates"].size, label
            assert _same_records(recs, w["candidates"]), label


@pytest.mark.parametrize("f16", [False, True])
@pytest.mark.parametrize("mode", ["standard", "greedy"])
def test_single_spectrum_walks_meet(dev, mode, f16):
    from paper_2202_12817_amd import ops
    x, off = _input(mode, f16, 950 + (3 if f16 else 0))
    for s in (1, 7, 11):   # thresholds of k = 2, 17 and 32 on lanes 31, 31 and 63
        xs = np.ascontiguousarray(x[off[s]:off[s + 1]])
        xt = _device(xs, f16, dev)
        for opts in OPTIONS:
            w = oracle.hs_1d(xs, 32, MODES[mode], **opts)
            for kernel in ("plain", "persistent"):
                print("1d", mode, "f16" if f16 else "f32", xs.size, opts, kernel, flush=True)
                got = ops.sum_1d(xt, 32, mode, kernel=kernel, **opts)
                check_dense(got, w, None, "1d %s %s n=%d %s %s" % (mode, f16, xs.size, opts, kernel))
