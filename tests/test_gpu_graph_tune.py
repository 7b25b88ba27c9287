"""GPU: graph replay, caller-side stream capture, launch shapes and the tuner.

Every replayed or re-shaped call is held to the parity bar of
test_gpu_parity against the oracle's float mirror: indices and SNR bit for
bit, candidate sets equal.  Between graph replays the test runs its own eager
work (a fresh input written in place) and synchronises, and every replay is
checked.
"""
import numpy as np
import pytest

import oracle
import synthetic
from gpu_checks import _cands, _np, _same_records, check_dense

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

H, THR = 32, 4.0


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_12817_amd import hs
    hs.load()
    return torch.device("cuda:0")


def _hs():
    from paper_2202_12817_amd import hs
    return hs


def _batch(seed, B=9):
    return synthetic.config3(n_spectra=B, lo=2000, hi=70000, seed=seed)


def _shuffled(x, seed):
    """Another input of the same size: the bins of x in a seeded random order."""
    return np.ascontiguousarray(x[np.random.default_rng(seed).permutation(x.size)])


class Buffers:
    """Static device buffers of one batched call (inputs written in place)."""

    def __init__(self, dev, x, off):
        self.n = x.size
        self.B = off.size - 1
        self.x = torch.from_numpy(x).to(dev)
        self.off = torch.from_numpy(off).to(dev)
        self.snr = torch.empty(self.n, dtype=torch.float32, device=dev)
        self.harm = torch.empty(self.n, dtype=torch.uint8, device=dev)
        self.drift = torch.empty(self.n, dtype=torch.uint8, device=dev)
        self.cap = self.n
        self.cand = torch.empty((self.cap, 4), dtype=torch.int32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int64, device=dev)

    def call(self, plan, stream=None):
        _hs().hs_sum_batched(plan.handle, self.x, self.off, self.B, None, self.snr, self.harm, self.drift,
                             self.cand, self.cap, self.count, stream)

    def out(self):
        return dict(snr=self.snr, harm=self.harm, drift=self.drift, cand_raw=self.cand, count=self.count)


def check_batch(got, x, off, mode, label):
    w = oracle.hs_batched(x, off, H, mode, THR, dense=True)
    for s in range(off.size - 1):
        sl = slice(off[s], off[s + 1])
        check_dense({k: got[k][sl] for k in ("snr", "harm", "drift")}, w["spectra"][s], None,
                    "%s spectrum %d" % (label, s))
    recs, n = _cands(got)
    assert n == w["candidates"].size, label
    assert _same_records(recs, w["candidates"]), label


@pytest.mark.parametrize("mode", [oracle.STANDARD, oracle.GREEDY])
def test_library_graph_replays(dev, mode):
    hs = _hs()
    x, off = _batch(71)
    buf = Buffers(dev, x, off)
    with hs.Plan(harmonics=H, mode=mode, threshold=THR, max_spectra=buf.B) as plan:
        hs.hs_plan_set_graph(plan.handle, True)
        xs = [x] + [_shuffled(x, 72 + i) for i in range(3)]
        for i, xi in enumerate(xs):
            # eager work between replays: a new input written in place
            buf.x.copy_(torch.from_numpy(xi))
            torch.cuda.synchronize()
            print("graph replay", mode, i, flush=True)
            buf.call(plan)
            torch.cuda.synchronize()
            check_batch(buf.out(), xi, off, mode, "replay %d" % i)
        assert hs.hs_plan_graph_info(plan.handle) == (1, 3)
        # a different argument set is recorded separately; the first stays cached
        other = Buffers(dev, x, off)
        other.call(plan)
        buf.call(plan)
        torch.cuda.synchronize()
        assert hs.hs_plan_graph_info(plan.handle) == (2, 4)
        check_batch(other.out(), x, off, mode, "second argument set")
        check_batch(buf.out(), xs[-1], off, mode, "first set after the second")
        hs.hs_plan_set_graph(plan.handle, False)


def test_library_graph_1d_and_2d(dev):
    hs = _hs()
    x, _ = synthetic.config2(n=(1 << 18) + 5, seed=74)
    p = np.random.default_rng(75).standard_exponential((11, 20011)).astype(np.float32)
    xt, pt = torch.from_numpy(x).to(dev), torch.from_numpy(p).to(dev)
    snr = torch.empty(x.size, dtype=torch.float32, device=dev)
    harm = torch.empty(x.size, dtype=torch.uint8, device=dev)
    drift = torch.empty(x.size, dtype=torch.uint8, device=dev)
    snr2 = torch.empty(p.shape, dtype=torch.float32, device=dev)
    harm2 = torch.empty(p.shape, dtype=torch.uint8, device=dev)
    drift2 = torch.empty(p.shape, dtype=torch.uint8, device=dev)
    w1 = oracle.hs_1d(x, H, oracle.GREEDY)
    w2 = oracle.hs_2d(p, -5, 5, 16, oracle.GREEDY)
    with hs.Plan(harmonics=H) as p1, hs.Plan(harmonics=16) as p2:
        hs.hs_plan_set_graph(p1.handle, True)
        hs.hs_plan_set_graph(p2.handle, True)
        for i in range(3):
            snr.zero_()
            snr2.zero_()
            torch.cuda.synchronize()
            hs.hs_sum_1d(p1.handle, xt, x.size, None, snr, harm, drift, None)
            hs.hs_sum_2d(p2.handle, pt, p.shape[1], p.shape[1], -5, 5, None, snr2, harm2, drift2)
            torch.cuda.synchronize()
            check_dense(dict(snr=snr, harm=harm, drift=drift), w1, None, "1d replay %d" % i)
            check_dense(dict(snr=snr2, harm=harm2, drift=drift2), w2, None, "2d replay %d" % i)
        assert hs.hs_plan_graph_info(p1.handle) == (1, 2)
        assert hs.hs_plan_graph_info(p2.handle) == (1, 2)


def test_caller_stream_capture(dev):
    """The batched call recorded into the caller's own graph (torch.cuda.graph)."""
    hs = _hs()
    x, off = _batch(76)
    buf = Buffers(dev, x, off)
    with hs.Plan(harmonics=H, threshold=THR, max_spectra=buf.B) as plan:
        buf.call(plan)   # eager warm-up outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            buf.call(plan)   # torch's capture stream is the current stream
        assert hs.hs_plan_graph_info(plan.handle) == (0, 0)
        for i in range(3):
            xi = _shuffled(x, 77 + i)
            buf.x.copy_(torch.from_numpy(xi))
            buf.snr.zero_()
            buf.count.fill_(12345)
            torch.cuda.synchronize()
            print("caller graph replay", i, flush=True)
            g.replay()
            torch.cuda.synchronize()
            check_batch(buf.out(), xi, off, oracle.GREEDY, "caller replay %d" % i)


def test_launch_shapes_identical(dev):
    hs = _hs()
    x, off = _batch(80, B=13)
    buf = Buffers(dev, x, off)
    ref = None
    with hs.Plan(harmonics=H, threshold=THR, max_spectra=buf.B) as plan:
        f0, w0 = hs.hs_plan_get_launch(plan.handle)
        assert f0 in (1, 2, 4) and 1 <= w0 <= 8
        for F in (0, 1, 2, 4):
            for Wg in ((0,) if F == 0 else (1, 2, 3, 4, 5, 6, 7, 8)):
                try:
                    hs.hs_plan_set_launch(plan.handle, F, Wg)
                except hs.HsError:
                    assert Wg > 1, "one workgroup per CU (and the plain kernel) must always be accepted"
                    continue
                assert hs.hs_plan_get_launch(plan.handle) == (F, Wg)
                buf.call(plan)
                torch.cuda.synchronize()
                got = {k: _np(v).copy() for k, v in buf.out().items() if k != "cand_raw"}
                recs, n = _cands(buf.out())
                if ref is None:
                    ref = (got, recs, n)
                    check_batch(buf.out(), x, off, oracle.GREEDY, "shape %d/%d" % (F, Wg))
                else:
                    for k in ("harm", "drift"):
                        assert np.array_equal(got[k], ref[0][k]), (F, Wg, k)
                    assert np.array_equal(got["snr"].view(np.uint32), ref[0]["snr"].view(np.uint32)), (F, Wg)
                    assert n == ref[2] and _same_records(recs, ref[1]), (F, Wg)
        for bad in ((3, 1), (4, 0), (4, 9), (1, 9), (8, 1)):
            with pytest.raises(hs.HsError):
                hs.hs_plan_set_launch(plan.handle, *bad)


def test_tuner_and_cache(dev, tmp_path):
    hs = _hs()
    x, off = _batch(81, B=17)
    buf = Buffers(dev, x, off)
    cache = tmp_path / "hs_tune.jsonl"
    with hs.Plan(harmonics=H, threshold=THR, max_spectra=buf.B) as plan:
        hs.hs_plan_tune_batched(plan.handle, buf.x, buf.off, buf.B, None, buf.snr, buf.harm, buf.drift, buf.cand,
                                buf.cap, buf.count, str(cache))
        torch.cuda.synchronize()
        shape = hs.hs_plan_get_launch(plan.handle)
        check_batch(buf.out(), x, off, oracle.GREEDY, "after tuning")
        lines = cache.read_text().splitlines()
        assert len(lines) == 1 and '"fundamentals_per_lane": %d' % shape[0] in lines[0]
        assert '"workgroups_per_cu": %d' % shape[1] in lines[0]
    with hs.Plan(harmonics=H, threshold=THR, max_spectra=buf.B) as plan:
        other = (2, 1) if shape != (2, 1) else (4, 1)
        hs.hs_plan_set_launch(plan.handle, *other)
        hs.hs_plan_tune_batched(plan.handle, buf.x, buf.off, buf.B, None, buf.snr, buf.harm, buf.drift, buf.cand,
                                buf.cap, buf.count, str(cache))
        torch.cuda.synchronize()
        assert hs.hs_plan_get_launch(plan.handle) == shape   # taken from the cache, not re-timed
        assert len(cache.read_text().splitlines()) == 1
        check_batch(buf.out(), x, off, oracle.GREEDY, "cached shape")
        hs.hs_plan_set_timing(plan.handle, True)
        with pytest.raises(hs.HsError):
            hs.hs_plan_tune_batched(plan.handle, buf.x, buf.off, buf.B, None, buf.snr, buf.harm, buf.drift)
        hs.hs_plan_set_timing(plan.handle, False)
    with hs.Plan(harmonics=H, threshold=THR, max_spectra=buf.B, kernel=hs.HS_KERNEL_PLAIN) as plan:
        with pytest.raises(hs.HsError):
            hs.hs_plan_tune_batched(plan.handle, buf.x, buf.off, buf.B, None, buf.snr, buf.harm, buf.drift)


def test_caller_workspace(dev):
    """A plan in a caller-owned workspace gives the same bits as a plan that
    allocates its own; the buffer is the caller's again after destroy."""
    hs = _hs()
    x, off = _batch(95, B=11)
    buf = Buffers(dev, x, off)
    desc = dict(harmonics=H, threshold=THR, max_spectra=buf.B)
    need = hs.hs_plan_workspace_bytes(hs.hs_plan_desc_init(**desc))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    assert ws.data_ptr() % 256 == 0
    with hs.Plan(workspace=ws, **desc) as plan:
        buf.call(plan)
        torch.cuda.synchronize()
        check_batch(buf.out(), x, off, oracle.GREEDY, "caller workspace")
    ref = Buffers(dev, x, off)
    with hs.Plan(**desc) as plan:
        ref.call(plan)
        torch.cuda.synchronize()
    for k in ("snr", "harm", "drift"):
        assert torch.equal(getattr(buf, k), getattr(ref, k)), k
    ws.fill_(7)   # the workspace is the caller's again
    torch.cuda.synchronize()
    with pytest.raises(hs.HsError):
        hs.Plan(workspace=ws[:need - 256], **desc)
