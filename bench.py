"""Benchmark of the harmonic-sum hot path on one MI355X.

One step = one ``hs_sum_batched`` call over the batched workload (512
DM-trial spectra of 2^20..2^22 FP32 bins, Exp(1) noise + 5 pulse trains each,
H = 32, greedy, SNR > 6 candidate compaction): the per-spectrum FP64
statistics, the float tables, the harmonic walk and the compaction.  Inputs
are resident in HBM before the timed region.  Prints one JSON line.

Also timed (extra keys): the plain per-spectrum FP32 path (one
``hs_sum_1d`` per spectrum, dense outputs) and the FP16-storage batched path,
plus the CPU oracle on a bounded sample of the same workload.
"""
import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
H = 32
THRESHOLD = 6.0
SUM_KERNEL = "k_sum_xcd<32, true, false, %d>"         # dominant kernel (FP32 greedy; fundamentals per lane)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_sum_xcd_batched_512x_h32_greedy_f32.txt")
CALIB_BYTES = 1 << 30


def _code_tokens(text):
    """C/C++ source without comments and whitespace (comment edits do not change the kernel)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return "".join(text.split())


def source_hash(kernel_file="hs_sum_xcd.hip"):
    """Hash of what a kernel is compiled from (its source and the headers it
    includes, comments stripped, and the build script with its flags): a
    counter figure is valid only for the kernel it was taken from."""
    import hashlib
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2202_12817_amd")
    for f in (os.path.join(pkg, "csrc", kernel_file), os.path.join(pkg, "csrc", "hs_device.h"),
              os.path.join(pkg, "csrc", "hs_internal.h"), os.path.join(ROOT, "include", "hs.h")):
        h.update(os.path.basename(f).encode())
        h.update(_code_tokens(open(f).read()).encode())
    h.update(open(os.path.join(pkg, "build.py"), "rb").read())
    return h.hexdigest()[:16]


TABLE2_FILE = os.path.join(ROOT, "profiles", "table2_1024x131072_greedy_presto.txt")
VALU_PEAK = 256 * 2.4e9      # wave instructions per second: 256 CUs, one VALU wave instruction per clock


def table2_counters():
    """Per-kernel counters (VALU instructions, HBM-side bytes per dispatch) of the
    Table 2 workload from the committed rocprofv3 summary, for the kernels whose
    sources still match."""
    out = {}
    try:
        for line in open(TABLE2_FILE):
            if line.startswith("json: "):
                rec = json.loads(line[6:])
                if rec.get("source") == source_hash(rec.get("file", "")):
                    out[(rec["algorithm"], rec["H"])] = rec
    except (OSError, KeyError, ValueError):
        pass
    return out


def read_traffic(kernel):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 summary, or None."""
    try:
        for line in open(TRAFFIC_FILE):
            if line.startswith("json: "):
                rec = json.loads(line[6:])
                if rec.get("source") == source_hash() and rec.get("kernel") == kernel:
                    return rec["fetch_bytes"] + rec["write_bytes"]
    except (OSError, KeyError, ValueError):
        pass
    return None


def pmc_summary(dirs):
    """Summarise rocprofv3 --pmc CSV output (FETCH_SIZE, WRITE_SIZE runs) into per-dispatch bytes.

    Each counter is scaled by what it reads for the calibration kernel (an
    elementwise negation that reads and writes CALIB_BYTES, run in the same
    process).  One ``json:`` line per batched FP32 greedy harmonic-sum kernel
    found (one per launch shape profiled)."""
    import csv
    import glob
    out = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            per = {}
            for r in csv.DictReader(open(f)):
                key = (r["Kernel_Name"], r["Counter_Name"])
                per.setdefault(key, []).append(float(r["Counter_Value"]))
            for (kname, cname), vals in per.items():
                out.setdefault(cname, {}).setdefault(kname, []).extend(vals)
    lines = []
    recs = {}
    for cname, key in (("FETCH_SIZE", "fetch_bytes"), ("WRITE_SIZE", "write_bytes")):
        kern = out.get(cname, {})
        copy = [v for k, vs in kern.items() if "neg" in k for v in vs]
        calib = max(copy) if copy else None
        scale = CALIB_BYTES / (calib * 1024.0) if calib else None
        lines.append("%s: calibration copy of %d bytes reads %s KiB -> scale %s" % (
            cname, CALIB_BYTES, "%.1f" % calib if calib else "n/a", "%.4f" % scale if scale else "n/a"))
        for k, vs in sorted(kern.items()):
            if "hs::" not in k:
                continue
            avg = sum(vs) / len(vs)
            lines.append("  %-70s dispatches %3d  avg %12.1f KiB  scaled %14.0f bytes" % (
                k[:70], len(vs), avg, avg * 1024.0 * (scale or 1.0)))
            m = re.search(r"k_sum_xcd<32, true, false, (\d)>", k)
            if m:
                name = SUM_KERNEL % int(m.group(1))
                recs.setdefault(name, {"kernel": name, "source": source_hash()})[key] = avg * 1024.0 * (scale or 1.0)
    for rec in recs.values():
        lines.append("json: " + json.dumps(rec))
    return "\n".join(lines)


def keff_sum(lengths, H, greedy, first_bin=1):
    """Sum over fundamentals of the harmonics summed (exact, per the truncation rule)."""
    total = 0
    for N in lengths:
        N = int(N)
        for k in range(1, H + 1):
            # fundamentals n >= first_bin with k (n + greedy) <= N - 1
            hi = (N - 1) // k - (1 if greedy else 0)
            if hi >= first_bin:
                total += min(hi, N - 1) - first_bin + 1
    return total


def line_bytes_sum(lengths, H, greedy, elem, first_bin=1):
    """Bytes moved from L2 to the CUs at cache-line granularity (128 B lines,
    waves of 64 consecutive fundamentals): a fundamental-step at harmonic k
    moves about min(k elem, 128) bytes, summed over every step."""
    total = 0
    for N in lengths:
        N = int(N)
        for k in range(1, H + 1):
            hi = (N - 1) // k - (1 if greedy else 0)
            if hi >= first_bin:
                total += (min(hi, N - 1) - first_bin + 1) * min(k * elem, 128)
    return total


def keff_sum_2d(n_r, z_min, z_max, H, greedy, first_bin=1):
    """Sum of K_eff over the f-fdot plane (row z truncates at the first harmonic row outside the plane)."""
    total = 0
    for z in range(z_min, z_max + 1):
        kz = H if z == 0 else (z_max // z if z > 0 else z_min // z)
        for k in range(1, min(H, kz) + 1):
            hi = (n_r - 1) // k - (1 if greedy else 0)
            if hi >= first_bin:
                total += min(hi, n_r - 1) - first_bin + 1
    return total


def plane_2d_leg(hs, torch, dev, steps, warmup):
    """The f-fdot plane (2^21 columns x 201 rows, z = -100..100, H = 16, dense outputs)."""
    import synthetic
    plane, _ = synthetic.config4(threads=16)
    n_z, n_r = plane.shape
    z_min, z_max, h2 = -100, 100, 16
    p32 = torch.from_numpy(plane).to(dev)
    p16 = torch.empty(plane.shape, dtype=torch.int16, device=dev)
    scale = float(np.float32(plane.mean(dtype=np.float64)))
    hs.hs_quantize_f16(p32, plane.size, scale, p16)
    del plane
    snr = torch.empty((n_z, n_r), dtype=torch.float32, device=dev)
    harm = torch.empty((n_z, n_r), dtype=torch.uint8, device=dev)
    drift = torch.empty((n_z, n_r), dtype=torch.uint8, device=dev)
    out = {"workload": "f-fdot plane %d x %d (z = %d..%d), H=%d, dense snr/harm/drift" % (n_r, n_z, z_min, z_max, h2)}
    for dname, dt, pin, eb in (("f32", hs.HS_F32, p32, 4), ("f16", hs.HS_F16, p16, 2)):
        for mname, mode in (("standard", hs.HS_STANDARD), ("greedy", hs.HS_GREEDY)):
            plan = hs.Plan(harmonics=h2, mode=mode, dtype=dt)
            for _ in range(warmup):
                hs.hs_sum_2d(plan.handle, pin, n_r, n_r, z_min, z_max, None, snr, harm, drift)
            torch.cuda.synchronize()
            hs.hs_plan_set_timing(plan.handle, True)
            t0 = time.perf_counter()
            for _ in range(steps):
                hs.hs_sum_2d(plan.handle, pin, n_r, n_r, z_min, z_max, None, snr, harm, drift)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / steps
            c, nm, sm = hs.hs_plan_get_timing(plan.handle)
            plan.close()
            work = keff_sum_2d(n_r, z_min, z_max, h2, mode == hs.HS_GREEDY)
            comp = n_z * n_r * (eb + 6)
            sum_ms = sm / max(1, c)
            out["%s_%s" % (dname, mname)] = {
                "value": work / el, "unit": "bin·harmonics/s", "ms_per_step": 1e3 * el,
                "stage_ms": {"normalisation": nm / max(1, c), "harmonic_sum": sum_ms},
                "sum_kernel_gbs_compulsory": comp / (sum_ms * 1e-3) / 1e9,
                "sum_kernel_frac_compulsory": comp / (sum_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


# Table 2 of the paper (V100, sum kernels only, 1024 spectra of 2^17 bins):
# fundamental bins per second, in Gbin/s.  Context, not a target.
PAPER_TABLE2_GBINS = {"greedy": {32: 8.64, 16: 14.70, 8: 26.10, 4: 39.9},
                      "presto": {32: 9.64, 16: 15.24, 8: 23.38, 4: 37.49},
                      "presto_plus": {32: 1.16, 16: 3.79, 8: 11.03, 4: 26.80}}


def table2_leg(hs, torch, dev, steps, warmup):
    """The paper's performance comparison (Sec. 4.3, Table 2): 1024 spectra of
    2^17 FP32 bins, dense snr/harm outputs, greedy vs PRESTO vs PRESTO+ (and
    PRESTO_all) at H = 4, 8, 16, 32; bins per second of the harmonic-sum kernel
    (the statistics stage, shared by all algorithms, reported beside it)."""
    import synthetic
    x, off = synthetic.table2(threads=16)
    B, n_bins = off.size - 1, int(x.size)
    xt, ot = torch.from_numpy(x).to(dev), torch.from_numpy(off).to(dev)
    del x
    snr = torch.empty(n_bins, dtype=torch.float32, device=dev)
    harm = torch.empty(n_bins, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    out = {"workload": "%d spectra of %d FP32 bins (Exp(1) noise + 5 pulse trains each), dense snr/harm"
                       % (B, n_bins // B),
           "unit": "Gbin/s (all bins / harmonic-sum kernel time)", "paper_v100_gbin_s": PAPER_TABLE2_GBINS}
    counters = table2_counters()
    modes = (("greedy", hs.HS_GREEDY), ("presto", hs.HS_PRESTO), ("presto_all", hs.HS_PRESTO_ALL),
             ("presto_plus", hs.HS_PRESTO_PLUS))
    for mname, mode in modes:
        res = {}
        for h in (4, 8, 16, 32):
            plan = hs.Plan(harmonics=h, mode=mode, dtype=hs.HS_F32, max_spectra=B)
            if mode == hs.HS_GREEDY:
                hs.hs_plan_tune_batched(plan.handle, xt, ot, B, None, snr, harm, None, None, 0, None, None, stream)
            for _ in range(warmup):
                hs.hs_sum_batched(plan.handle, xt, ot, B, None, snr, harm, None, None, 0, None, stream)
            torch.cuda.synchronize()
            hs.hs_plan_set_timing(plan.handle, True)
            t0 = time.perf_counter()
            for _ in range(steps):
                hs.hs_sum_batched(plan.handle, xt, ot, B, None, snr, harm, None, None, 0, None, stream)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / steps
            c, nm, sm = hs.hs_plan_get_timing(plan.handle)
            plan.close()
            sum_ms = sm / max(1, c)
            comp = n_bins * 9      # 4 B read, 4 + 1 B written per bin
            r = {"gbin_s": n_bins / (sum_ms * 1e-3) / 1e9, "sum_ms": sum_ms,
                 "normalisation_ms": nm / max(1, c), "call_ms": 1e3 * el,
                 "gbin_s_whole_call": n_bins / el / 1e9,
                 "sum_kernel_gbs_compulsory": comp / (sum_ms * 1e-3) / 1e9}
            rec = counters.get((mname, h))
            hbm_frac = comp / (sum_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
            if rec:
                valu_rate = rec["valu"] / (sum_ms * 1e-3)
                alu = valu_rate / VALU_PEAK > hbm_frac
                r["roofline"] = {"bound": "alu" if alu else "hbm", "kernel": rec["kernel"],
                                 "achieved": valu_rate / 1e9 if alu else comp / (sum_ms * 1e-3) / 1e9,
                                 "peak": VALU_PEAK / 1e9 if alu else HBM_PEAK_GBS,
                                 "unit": "G VALU wave-instructions/s" if alu else "GB/s",
                                 "frac": valu_rate / VALU_PEAK if alu else hbm_frac,
                                 "valu_frac": valu_rate / VALU_PEAK, "hbm_frac_compulsory": hbm_frac,
                                 "traffic": rec["fetch_bytes"] + rec["write_bytes"]}
            paper = PAPER_TABLE2_GBINS.get(mname, {}).get(h)
            if paper:
                r["ratio_to_paper_v100"] = r["gbin_s"] / paper
            res["H%d" % h] = r
        out[mname] = res
    out["interleaved"] = interleaved_leg(hs, torch, xt, ot, B, n_bins // B, snr, harm, steps, warmup, stream)
    out["pipeline"] = pipeline_leg(hs, torch, xt, ot, B, n_bins, snr, harm, steps, stream)
    del xt, snr, harm
    return out


def _event_ms(torch, stream, call, steps):
    call()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        call()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def pipeline_leg(hs, torch, xt, ot, B, n_bins, snr, harm, steps, stream):
    """The sum's neighbours at the same size: the inter-binned power spectrum of
    n_bins complex FFT bins (8 B read, 8 B written per bin) and peak clustering
    of the greedy H = 32 dense outputs (5 B read per bin + the window reads of
    the candidates), HIP events on the launch stream."""
    fft = torch.empty(n_bins, dtype=torch.complex64, device=xt.device)
    fft.real.copy_(xt)
    fft.imag.copy_(xt.flip(0))
    pw = torch.empty(2 * n_bins - 1, dtype=torch.float32, device=xt.device)
    ms_p = _event_ms(torch, stream, lambda: hs.hs_power_spectrum(fft, n_bins, 1, 1.0, pw, stream), steps)
    del fft, pw
    plan = hs.Plan(harmonics=32, mode=hs.HS_GREEDY, dtype=hs.HS_F32, max_spectra=B)
    hs.hs_sum_batched(plan.handle, xt, ot, B, None, snr, harm, None, None, 0, None, stream)
    torch.cuda.synchronize()
    plan.close()
    cap = 1 << 22
    cand = torch.empty((cap, 4), dtype=torch.int32, device=xt.device)
    count = torch.zeros(1, dtype=torch.int64, device=xt.device)
    ms_c = _event_ms(torch, stream, lambda: hs.hs_cluster_peaks(snr, harm, None, ot, n_bins, B, 16, 6.0, cand, cap,
                                                               count, stream), steps)
    peaks = int(count.item())
    bp, bc = 16.0 * n_bins, 5.0 * n_bins
    return {"power_spectrum_interbinned": {"ms": ms_p, "gbs": bp / (ms_p * 1e-3) / 1e9,
                                           "frac": bp / (ms_p * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "cluster_peaks_r16_snr6": {"ms": ms_c, "gbs": bc / (ms_c * 1e-3) / 1e9,
                                       "frac": bc / (ms_c * 1e-3) / 1e9 / HBM_PEAK_GBS, "peaks": peaks}}


def _timed_sum(hs, torch, plan, call, steps, warmup):
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    hs.hs_plan_set_timing(plan.handle, True)
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    c, nm, sm = hs.hs_plan_get_timing(plan.handle)
    hs.hs_plan_set_timing(plan.handle, False)
    return sm / max(1, c), nm / max(1, c)


def interleaved_leg(hs, torch, xt, ot, B, N, snr, harm, steps, warmup, stream):
    """The same spectra in the interleaved layout of Sec. 3.1.1 (bin-major, one
    lane per spectrum) against the natural layout, simple and greedy sums, dense
    snr/harm: harmonic-sum kernel time of each, and the transpose that builds
    the layout (HIP events)."""
    xi = torch.empty((N, B), dtype=torch.float32, device=xt.device)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    hs.hs_interleave(xt, N, B, 4, xi, stream)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(steps):
        hs.hs_interleave(xt, N, B, 4, xi, stream)
    t1.record(stream)
    torch.cuda.synchronize()
    res = {"transpose_ms": t0.elapsed_time(t1) / steps,
           "note": "sum-kernel ms per call; natural = hs_sum_batched (tuned launch), interleaved = hs_sum_interleaved"}
    for mname, mode in (("standard", hs.HS_STANDARD), ("greedy", hs.HS_GREEDY)):
        r = {}
        for h in (4, 8, 16, 32):
            plan = hs.Plan(harmonics=h, mode=mode, dtype=hs.HS_F32, max_spectra=B)
            hs.hs_plan_tune_batched(plan.handle, xt, ot, B, None, snr, harm, None, None, 0, None, None, stream)
            nat, _ = _timed_sum(hs, torch, plan, lambda: hs.hs_sum_batched(
                plan.handle, xt, ot, B, None, snr, harm, None, None, 0, None, stream), steps, warmup)
            il, il_norm = _timed_sum(hs, torch, plan, lambda: hs.hs_sum_interleaved(
                plan.handle, xi, N, B, None, snr, harm, None, None, 0, None, stream), steps, warmup)
            plan.close()
            r["H%d" % h] = {"natural_sum_ms": nat, "interleaved_sum_ms": il, "interleaved_norm_ms": il_norm,
                            "gbin_s_interleaved": N * B / (il * 1e-3) / 1e9, "speedup": nat / il}
        res[mname] = r
    del xi
    return res


def small_1d_leg(hs, torch, dev):
    """Call latency of a small spectrum (65536 FP32 bins, H = 8, greedy, dense
    outputs): six launches per call, replayed as one captured graph or not."""
    import synthetic
    x, _ = synthetic.config1()
    xt = torch.from_numpy(x).to(dev)
    snr = torch.empty(x.size, dtype=torch.float32, device=dev)
    harm = torch.empty(x.size, dtype=torch.uint8, device=dev)
    drift = torch.empty(x.size, dtype=torch.uint8, device=dev)
    out = {"workload": "one spectrum of 65536 FP32 bins, H=8, greedy, dense outputs"}
    reps = 2000
    for name, graph, kern in (("eager_us", False, hs.HS_KERNEL_AUTO), ("graph_us", True, hs.HS_KERNEL_AUTO),
                              ("plain_eager_us", False, hs.HS_KERNEL_PLAIN), ("plain_graph_us", True, hs.HS_KERNEL_PLAIN)):
        plan = hs.Plan(harmonics=8, kernel=kern)
        hs.hs_plan_set_graph(plan.handle, graph)
        for _ in range(20):
            hs.hs_sum_1d(plan.handle, xt, x.size, None, snr, harm, drift)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            hs.hs_sum_1d(plan.handle, xt, x.size, None, snr, harm, drift)
        torch.cuda.synchronize()
        out[name] = 1e6 * (time.perf_counter() - t0) / reps
        plan.close()
    return out


def calibration_copy(torch, dev):
    """An elementwise negation that reads and writes CALIB_BYTES once; its
    kernel name ("neg") identifies it in the counter output."""
    src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--spectra", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the plain and FP16 legs")
    ap.add_argument("--cpu-sample", type=int, default=72, help="spectra in the CPU oracle sample (about 10-15 s of one core)")
    ap.add_argument("--tune-cache", default=None, help="launch-shape cache file of the tuner (default: tune afresh)")
    ap.add_argument("--launch", default=None, metavar="F,W",
                    help="fixed launch shape (fundamentals per lane, workgroups per CU) instead of tuning")
    ap.add_argument("--plane-2d", action="store_true", help="also time the f-fdot plane (2^21 x 201, H=16)")
    ap.add_argument("--leg", choices=["table2", "plane_2d"], default=None,
                    help="run only this leg and print its JSON object (profiling aid)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="also run a 1 GiB read + 1 GiB write elementwise kernel (reference for rocprofv3 byte counters)")
    ap.add_argument("--pmc-summary", nargs="+", metavar="DIR",
                    help="summarise rocprofv3 --pmc CSV directories and exit (no GPU work)")
    args = ap.parse_args()
    if args.pmc_summary:
        print(pmc_summary(args.pmc_summary))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the harmonic-sum library runs on a single device "
              "(independent spectra shard across GPUs by the caller); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import synthetic
    from paper_2202_12817_amd import hs

    dev = torch.device("cuda:0")
    if args.leg:
        if args.calibration_copy:
            calibration_copy(torch, dev)
        legs = {"table2": lambda: table2_leg(hs, torch, dev, min(args.steps, 10), args.warmup),
                "plane_2d": lambda: plane_2d_leg(hs, torch, dev, args.steps, args.warmup)}
        print(json.dumps({args.leg: legs[args.leg]()}))
        return
    x, off = synthetic.config3(n_spectra=args.spectra, threads=16)
    lengths = np.diff(off)
    n_bins = int(x.size)
    xt = torch.from_numpy(x).to(dev)
    ot = torch.from_numpy(off).to(dev)
    B = args.spectra
    work = keff_sum(lengths, H, True)

    plan = hs.Plan(harmonics=H, mode=hs.HS_GREEDY, dtype=hs.HS_F32, max_spectra=B, threshold=THRESHOLD)
    cap = 1 << 24
    cand = torch.empty((cap, 4), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(p, xin):
        hs.hs_sum_batched(p.handle, xin, ot, B, None, None, None, None, cand, cap, count, stream)

    # launch shape of the persistent kernel: tuned on this batch (the tuner
    # times every shape; results do not depend on it)
    if args.launch:
        hs.hs_plan_set_launch(plan.handle, *[int(v) for v in args.launch.split(",")])
    else:
        hs.hs_plan_tune_batched(plan.handle, xt, ot, B, None, None, None, None, cand, cap, count, args.tune_cache,
                                stream)
    shape = hs.hs_plan_get_launch(plan.handle)
    for _ in range(args.warmup):
        step(plan, xt)
    torch.cuda.synchronize()
    hs.hs_plan_set_timing(plan.handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(plan, xt)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    calls, norm_ms, sum_ms = hs.hs_plan_get_timing(plan.handle)
    hs.hs_plan_set_timing(plan.handle, False)
    n_cand = int(count.item())
    # the same step replayed as one captured hipGraph per call
    hs.hs_plan_set_graph(plan.handle, True)
    step(plan, xt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(plan, xt)
    torch.cuda.synchronize()
    graph_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    graph_info = hs.hs_plan_graph_info(plan.handle)
    hs.hs_plan_set_graph(plan.handle, False)
    ms_step = 1e3 * elapsed / args.steps
    value = work * args.steps / elapsed

    in_bytes = 4 * n_bins
    lines = line_bytes_sum(lengths, H, True, 4)
    sum_kernel = SUM_KERNEL % shape[0] if shape[0] else "k_sum_1d<32, true, false>"
    cand_bytes = 16 * min(n_cand, cap)
    sum_avg_ms = sum_ms / max(1, calls)
    norm_avg_ms = norm_ms / max(1, calls)
    achieved = (in_bytes + cand_bytes) / (sum_avg_ms * 1e-3) / 1e9

    result = {
        "metric": "spectral bins·harmonics/sec and achieved HBM GB/s (% of peak), plain vs batched/FP16",
        "value": value,
        "unit": "bin·harmonics/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched 1D greedy harmonic sum: %d spectra of 2^20..2^22 FP32 bins "
                               "(Exp(1) noise + 5 pulse trains each), H=%d, SNR>%g candidate compaction"
                               % (B, H, THRESHOLD),
                   "spectra": B, "bins": n_bins, "H": H, "mode": "greedy", "threshold": THRESHOLD,
                   "bin_harmonics": work, "candidates": n_cand},
        "bins_per_s": n_bins * args.steps / elapsed,
        "hbm_gbs_compulsory": (in_bytes + cand_bytes) / (ms_step * 1e-3) / 1e9,
        "hbm_frac_compulsory": (in_bytes + cand_bytes) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "stage_ms": {"normalisation": norm_avg_ms, "harmonic_sum": sum_avg_ms},
        "launch": {"fundamentals_per_lane": shape[0], "workgroups_per_cu": shape[1], "tuned": not args.launch},
        "graph_replay": {"ms_per_step": graph_ms, "value": work / (graph_ms * 1e-3),
                         "graphs_recorded": graph_info[0], "replays": graph_info[1]},
        "gather": {"touched_bytes": 8 * work, "touched_gbs": 8 * work / (sum_avg_ms * 1e-3) / 1e9,
                   "l2_to_cu_bytes": lines, "l2_to_cu_tbs": lines / (sum_avg_ms * 1e-3) / 1e12,
                   "note": "harmonic-sum kernel: 8 B touched per greedy step (the compared pair); "
                           "min(4 k, 128) B per step at cache-line granularity"},
        "roofline": {"bound": "hbm", "kernel": sum_kernel, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": read_traffic(sum_kernel)},
    }

    if args.calibration_copy:
        calibration_copy(torch, dev)

    if not args.no_extra:
        # plain: one hs_sum_1d per spectrum, dense outputs, no graph
        pplan = hs.Plan(harmonics=H, mode=hs.HS_GREEDY, dtype=hs.HS_F32, threshold=THRESHOLD,
                        kernel=hs.HS_KERNEL_PLAIN)
        nmax = int(lengths.max())
        snr = torch.empty(nmax, dtype=torch.float32, device=dev)
        harm = torch.empty(nmax, dtype=torch.uint8, device=dev)
        drift = torch.empty(nmax, dtype=torch.uint8, device=dev)
        base = xt.data_ptr()

        def plain_step():
            for s in range(B):
                hs.hs_sum_1d(pplan.handle, base + 4 * int(off[s]), int(lengths[s]), None, snr, harm, drift, None,
                             stream)
        plain_step()
        torch.cuda.synchronize()
        reps = 2
        t0 = time.perf_counter()
        for _ in range(reps):
            plain_step()
        torch.cuda.synchronize()
        plain_s = (time.perf_counter() - t0) / reps
        pplan.close()
        result["plain_fp32"] = {"value": work / plain_s, "ms_per_step": 1e3 * plain_s,
                                "speedup_batched": plain_s / (ms_step * 1e-3)}
        # FP16 storage with a per-spectrum scale
        x16 = torch.empty(n_bins, dtype=torch.int16, device=dev)
        for s in range(B):
            scale = float(np.float32(x[off[s]:off[s + 1]].mean(dtype=np.float64)))
            hs.hs_quantize_f16(base + 4 * int(off[s]), int(lengths[s]), scale, x16.data_ptr() + 2 * int(off[s]),
                               stream)
        plan16 = hs.Plan(harmonics=H, mode=hs.HS_GREEDY, dtype=hs.HS_F16, max_spectra=B, threshold=THRESHOLD)
        if not args.launch:
            hs.hs_plan_tune_batched(plan16.handle, x16, ot, B, None, None, None, None, cand, cap, count,
                                    args.tune_cache, stream)
        shape16 = hs.hs_plan_get_launch(plan16.handle)
        for _ in range(args.warmup):
            step(plan16, x16)
        torch.cuda.synchronize()
        hs.hs_plan_set_timing(plan16.handle, True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(plan16, x16)
        torch.cuda.synchronize()
        e16 = (time.perf_counter() - t0) / args.steps
        c16, n16, s16 = hs.hs_plan_get_timing(plan16.handle)
        n_cand16 = int(count.item())
        plan16.close()
        result["batched_fp16"] = {"value": work / e16, "ms_per_step": 1e3 * e16,
                                  "speedup_vs_plain_fp32": plain_s / e16,
                                  "hbm_gbs_compulsory": (2 * n_bins + 16 * n_cand16) / e16 / 1e9,
                                  "stage_ms": {"normalisation": n16 / max(1, c16), "harmonic_sum": s16 / max(1, c16)},
                                  "launch": {"fundamentals_per_lane": shape16[0], "workgroups_per_cu": shape16[1]},
                                  "candidates": n_cand16}
        del x16

    if args.plane_2d:
        result["plane_2d"] = plane_2d_leg(hs, torch, dev, args.steps, args.warmup)
    if not args.no_extra:
        result["small_1d"] = small_1d_leg(hs, torch, dev)
        result["table2"] = table2_leg(hs, torch, dev, min(args.steps, 10), args.warmup)

    if not args.no_cpu_baseline:
        import oracle
        sample = list(range(min(args.cpu_sample, B)))
        t0 = time.perf_counter()
        for s in sample:
            r = oracle.hs_1d(x[off[s]:off[s + 1]], H, oracle.GREEDY)
            oracle.candidates(r["snr"], r["harm"], r["drift"], THRESHOLD, spectrum=s)
        cpu_s = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": keff_sum(lengths[sample], H, True) / cpu_s, "unit": "bin·harmonics/s",
                                  "cores": 1, "kind": "oracle",
                                  "sample": "first %d spectra of the same batch (%d bins), float mirror, "
                                            "exact statistics + per-fundamental C loops, one thread"
                                            % (len(sample), int(lengths[sample].sum()))}
    plan.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
