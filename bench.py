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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batched_512x_h32_greedy_k_sum_xcd.txt")
CALIB_BYTES = 1 << 30


def _code_tokens(text):
    """C/C++ source without comments and whitespace (comment edits do not change the kernel)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return "".join(text.split())


CSRC = os.path.join(ROOT, "paper_2202_12817_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")


def _local_includes(path, seen):
    """``path`` and every header it includes with quotes, recursively (found in csrc/ or include/)."""
    if path in seen or not os.path.exists(path):
        return
    seen.append(path)
    for name in re.findall(r'#include\s+"([^"]+)"', open(path).read()):
        for d in (CSRC, INCLUDE):
            if os.path.exists(os.path.join(d, name)):
                _local_includes(os.path.join(d, name), seen)
                break


def source_hash(kernel_file="hs_sum_xcd.hip"):
    """Hash of what a kernel is compiled from (its source and the headers it
    includes, comments stripped, and the build script with its flags): a
    counter figure is valid only for the kernel it was taken from."""
    import hashlib
    h = hashlib.sha256()
    files = []
    _local_includes(os.path.join(CSRC, kernel_file), files)
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(_code_tokens(open(f).read()).encode())
    h.update(open(os.path.join(ROOT, "paper_2202_12817_amd", "build.py"), "rb").read())
    return h.hexdigest()[:16]


def kernel_files():
    """Kernel name (``k_...``) -> the csrc file that defines it."""
    out = {}
    for f in sorted(os.listdir(CSRC)):
        if f.endswith(".hip"):
            for name in re.findall(r"__global__[^;{]*?\b(k_\w+)\s*\(", open(os.path.join(CSRC, f)).read()):
                out.setdefault(name, f)
    return out


def short_kernel_name(full):
    """``void hs::(anonymous namespace)::k_sum_xcd<32, true, false, 2>(hs::XcdArgs)`` -> ``k_sum_xcd<32, true, false, 2>``."""
    m = re.search(r"\b(k_\w+)(<[^()]*>)?", full)
    return (m.group(1) + (m.group(2) or "")) if m else None


TABLE2_FILE = os.path.join(ROOT, "profiles", "table2_1024x131072_greedy_presto.txt")
VALU_PEAK = 256 * 2.4e9      # wave instructions per second: 256 CUs, one VALU wave instruction per clock


def profile_records(path=None):
    """``json:`` records of the committed counter summaries (``profiles/*.txt``)
    whose kernel sources still hash to the recorded value, keyed by
    (summary file name, kernel)."""
    import glob
    out = {}
    files = [path] if path else sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt")))
    for f in files:
        try:
            for line in open(f):
                if not line.startswith("json: "):
                    continue
                rec = json.loads(line[6:])
                kf = rec.get("file") or kernel_files().get((rec.get("kernel") or "").split("<")[0])
                if kf and rec.get("source") == source_hash(kf):
                    out[(os.path.basename(f), rec["kernel"])] = rec
        except (OSError, KeyError, ValueError):
            continue
    return out


def read_counters(kernel, summary=None):
    """The newest valid counter record of ``kernel`` (from ``summary`` if given), or None."""
    recs = profile_records(summary)
    for (_, k), rec in sorted(recs.items()):
        if k == kernel:
            return rec
    return None


def read_traffic(kernel):
    """HBM bytes per launch of a kernel from the committed rocprofv3 summary, or None."""
    rec = read_counters(kernel, TRAFFIC_FILE)
    if rec and "fetch_bytes" in rec and "write_bytes" in rec:
        return rec["fetch_bytes"] + rec["write_bytes"]
    return None


PMC_KEYS = {"FETCH_SIZE": "fetch_bytes", "WRITE_SIZE": "write_bytes", "TCC_HIT_sum": "l2_hit",
            "TCC_MISS_sum": "l2_miss", "TCC_REQ_sum": "l2_req", "SQ_INSTS_VALU": "valu",
            "SQ_INSTS_VMEM_RD": "vmem_rd", "SQ_INSTS_SALU": "salu", "SQ_INSTS_LDS": "lds",
            "SQ_WAVES": "waves", "SQ_BUSY_CYCLES": "busy_cycles", "SQ_WAVE_CYCLES": "wave_cycles"}


def pmc_summary(dirs):
    """Summarise rocprofv3 output directories (``--kernel-trace --stats`` runs
    and ``--pmc`` runs, CSV) into per-dispatch figures of every harmonic-sum
    library kernel: average duration, HBM bytes (FETCH_SIZE and WRITE_SIZE,
    each scaled by what the counter reads for the calibration kernel -- an
    elementwise negation that reads and writes CALIB_BYTES in the same
    process), L2 hits and misses, and instruction counts.  Ends with one
    ``json:`` line per kernel carrying the hash of the sources it was compiled
    from (``source``)."""
    import csv
    import glob
    per = {}
    dur = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                per.setdefault((r["Kernel_Name"], r["Counter_Name"]), []).append(float(r["Counter_Value"]))
        for f in glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                name = r.get("Name") or r.get("KERNEL_NAME") or ""
                calls, total = int(r.get("Calls", 0) or 0), float(r.get("TotalDurationNs", 0) or 0)
                c0, t0 = dur.get(name, (0, 0.0))
                dur[name] = (c0 + calls, t0 + total)
    lines, recs = [], {}
    scales = {}
    for cname in ("FETCH_SIZE", "WRITE_SIZE"):
        copy = [v for (k, c), vs in per.items() if c == cname and "neg" in k for v in vs]
        calib = max(copy) if copy else None
        scales[cname] = CALIB_BYTES / (calib * 1024.0) if calib else None
        if cname in {c for (_, c) in per}:
            lines.append("%s: calibration copy of %d bytes reads %s KiB -> scale %s" % (
                cname, CALIB_BYTES, "%.1f" % calib if calib else "n/a",
                "%.4f" % scales[cname] if scales[cname] else "n/a"))
    files = kernel_files()

    def rec_of(full):
        short = short_kernel_name(full)
        if not short or short.split("<")[0] not in files:
            return None
        f = files[short.split("<")[0]]
        return recs.setdefault(short, {"kernel": short, "file": f, "source": source_hash(f)})

    for (kname, cname), vs in sorted(per.items()):
        r = rec_of(kname)
        if r is None or cname not in PMC_KEYS:
            continue
        avg = sum(vs) / len(vs)
        if cname in ("FETCH_SIZE", "WRITE_SIZE"):
            avg = avg * 1024.0 * (scales[cname] or 1.0)
        r[PMC_KEYS[cname]] = avg
        r.setdefault("dispatches", {})[cname] = len(vs)
    for kname, (calls, total) in dur.items():
        r = rec_of(kname)
        if r is not None and calls:
            r["avg_ns"] = total / calls
            r["calls"] = calls
    lines.append("%-36s %6s %11s %12s %12s %8s %12s" % ("kernel", "calls", "avg_us", "fetch_MB", "write_MB",
                                                       "L2_hit", "VALU"))
    for k in sorted(recs):
        r = recs[k]
        hit = r.get("l2_hit")
        miss = r.get("l2_miss")
        lines.append("%-36s %6s %11s %12s %12s %8s %12s" % (
            k[:36], r.get("calls", "-"), "%.1f" % (r["avg_ns"] / 1e3) if "avg_ns" in r else "-",
            "%.1f" % (r["fetch_bytes"] / 1e6) if "fetch_bytes" in r else "-",
            "%.1f" % (r["write_bytes"] / 1e6) if "write_bytes" in r else "-",
            "%.1f%%" % (100.0 * hit / (hit + miss)) if hit is not None and miss is not None and hit + miss > 0 else "-",
            "%.4g" % r["valu"] if "valu" in r else "-"))
    for k in sorted(recs):
        r = dict(recs[k])
        r.pop("dispatches", None)
        lines.append("json: " + json.dumps(r))
    return "\n".join(lines)


def keff_sum(lengths, H, greedy, first_bin=1, fundamental_end=0):
    """Sum over fundamentals of the harmonics summed (exact, per the truncation rule)."""
    total = 0
    for N in lengths:
        N = int(N)
        top = N - 1 if not fundamental_end else min(N, int(fundamental_end)) - 1
        for k in range(1, H + 1):
            # fundamentals first_bin <= n <= top with k (n + greedy) <= N - 1
            hi = min((N - 1) // k - (1 if greedy else 0), top)
            if hi >= first_bin:
                total += hi - first_bin + 1
    return total


def line_bytes_sum(lengths, H, greedy, elem, first_bin=1, fundamental_end=0):
    """Bytes moved from L2 to the CUs at cache-line granularity (128 B lines,
    waves of 64 consecutive fundamentals): a fundamental-step at harmonic k
    moves about min(k elem, 128) bytes, summed over every step."""
    total = 0
    for N in lengths:
        N = int(N)
        top = N - 1 if not fundamental_end else min(N, int(fundamental_end)) - 1
        for k in range(1, H + 1):
            hi = min((N - 1) // k - (1 if greedy else 0), top)
            if hi >= first_bin:
                total += (hi - first_bin + 1) * min(k * elem, 128)
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


def plane_2d_leg(hs, torch, dev, steps, warmup, error=True, kernel="auto"):
    """The f-fdot plane (2^21 columns x 201 rows, z = -100..100, H = 16, dense
    outputs), FP32 and FP16 storage, simple and greedy sums; with ``error`` the
    FP16 outputs are compared with the FP32 GPU outputs on the whole plane and
    with the float64 oracle on the original FP32 plane at sampled rows."""
    import synthetic
    plane, _ = synthetic.config4(threads=16)
    n_z, n_r = plane.shape
    z_min, z_max, h2 = -100, 100, 16
    p32 = torch.from_numpy(plane).to(dev)
    p16 = torch.empty(plane.shape, dtype=torch.int16, device=dev)
    scale = float(np.float32(plane.mean(dtype=np.float64)))
    hs.hs_quantize_f16(p32, plane.size, scale, p16)
    outs = {}
    for dname in ("f32", "f16"):
        outs[dname] = (torch.empty((n_z, n_r), dtype=torch.float32, device=dev),
                       torch.empty((n_z, n_r), dtype=torch.uint8, device=dev),
                       torch.empty((n_z, n_r), dtype=torch.uint8, device=dev))
    out = {"workload": "f-fdot plane %d x %d (z = %d..%d), H=%d, dense snr/harm/drift" % (n_r, n_z, z_min, z_max, h2),
           "kernel": kernel}
    mu_sigma = torch.zeros(2, dtype=torch.float64, device=dev)
    # the rate of a plain elementwise read-write kernel on this machine, measured
    # here: the ceiling for the bytes the plane kernels move (they read the
    # plane and write three outputs)
    tmp = outs["f32"][0]
    for _ in range(3):
        torch.neg(p32, out=tmp)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        torch.neg(p32, out=tmp)
    e1.record()
    torch.cuda.synchronize()
    rw_gbs = 2 * p32.numel() * 4 / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9
    out["elementwise_rw_gbs"] = rw_gbs
    for mname, mode in (("standard", hs.HS_STANDARD), ("greedy", hs.HS_GREEDY)):
        for dname, dt, pin, eb in (("f32", hs.HS_F32, p32, 4), ("f16", hs.HS_F16, p16, 2)):
            snr, harm, drift = outs[dname]
            plan = hs.Plan(harmonics=h2, mode=mode, dtype=dt, kernel={"auto": hs.HS_KERNEL_AUTO, "plain": hs.HS_KERNEL_PLAIN,
                                                                     "persistent": hs.HS_KERNEL_PERSISTENT}[kernel])
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
            hs.hs_plan_set_timing(plan.handle, False)
            if dname == "f32":
                hs.hs_get_norm(plan.handle, 1, mu_sigma)
            plan.close()
            work = keff_sum_2d(n_r, z_min, z_max, h2, mode == hs.HS_GREEDY)
            comp = n_z * n_r * (eb + 6)
            sum_ms = sm / max(1, c)
            kern = "k_sum_2d<%d, %s, %s>" % (h2, "true" if mode == hs.HS_GREEDY else "false",
                                                "true" if dname == "f16" else "false")
            rec = read_counters(kern) if kernel != "persistent" else None
            moved = rec["fetch_bytes"] + rec["write_bytes"] if rec and "fetch_bytes" in rec and \
                "write_bytes" in rec else None
            roof = {"bound": "hbm", "kernel": kern, "achieved": comp / (sum_ms * 1e-3) / 1e9,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": comp / (sum_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "traffic": moved}
            if moved:
                mv = moved / (sum_ms * 1e-3) / 1e9
                roof["moved"] = {"achieved": mv, "peak": rw_gbs, "unit": "GB/s", "frac": mv / rw_gbs,
                                 "what": "bytes fetched and written (committed FETCH_SIZE + WRITE_SIZE) vs an "
                                         "elementwise read-write kernel's rate measured in this run"}
            out["%s_%s" % (dname, mname)] = {
                "value": work / el, "unit": "bin·harmonics/s", "ms_per_step": 1e3 * el,
                "stage_ms": {"normalisation": nm / max(1, c), "harmonic_sum": sum_ms},
                "sum_kernel_gbs_compulsory": comp / (sum_ms * 1e-3) / 1e9,
                "sum_kernel_frac_compulsory": comp / (sum_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "roofline": roof}
        if error:
            torch.cuda.synchronize()
            ms = mu_sigma.cpu().numpy()
            rows = [0, 40, 99, 100, 101, 150, 200]
            out["f16_error_" + mname] = fp16_error_stats(
                torch, outs["f32"], outs["f16"], 6.0,
                sample=[(plane[i], (outs["f16"][0][i], outs["f16"][1][i], outs["f16"][2][i]),
                         (outs["f32"][0][i], outs["f32"][1][i], outs["f32"][2][i]), i) for i in rows],
                oracle_call=lambda row_plane, i, m=mode: plane_row_oracle(plane, z_min, z_max, h2, m, i,
                                                                          (float(ms[0]), float(ms[1]))),
                sample_label="plane rows %s (z = %s), float64 oracle with the FP32 plane's (mu1, sigma1)" % (
                    rows, [z_min + i for i in rows]))
    del plane
    return out


def plane_row_oracle(plane, z_min, z_max, H, mode, i, norm):
    """Float64 oracle outputs of plane row i (every column) on the FP32 plane."""
    import oracle
    n_r = plane.shape[1]
    idx = np.arange(i * n_r, (i + 1) * n_r, dtype=np.int64)
    return oracle.hs_2d(plane, z_min, z_max, H, oracle.GREEDY if mode == 1 else oracle.STANDARD, norm=norm,
                        idx=idx, precision="f64")


def fp16_error_stats(torch, o32, o16, thr, sample, oracle_call, sample_label):
    """What FP16 storage costs: (a) FP16 vs FP32 GPU outputs on every bin --
    bins whose harmonic count or drift differ (a flipped greedy comparison or
    argmax), SNR difference on the other bins, and the candidate sets at
    ``thr``; (b) FP16 GPU outputs vs the float64 oracle on the original FP32
    data for ``sample`` = [(data, fp16 outputs, fp32 outputs, label)], with the
    FP32 GPU path's own error beside it.  ``oracle_call(data, label)`` returns
    the oracle's float64 outputs of one sample item."""
    s32, h32, d32 = (t.reshape(-1) for t in o32)
    s16, h16, d16 = (t.reshape(-1) for t in o16)
    path = (h32 != h16) | (d32 != d16)
    same = ~path
    ds = (s16 - s32).abs() / s32.abs().clamp(min=1.0)
    c32 = (s32 > thr) & (h32 > 0)
    c16 = (s16 > thr) & (h16 > 0)
    res = {"vs_fp32_gpu": {
        "bins": int(s32.numel()),
        "harm_diff": int((h32 != h16).sum().item()), "drift_diff": int((d32 != d16).sum().item()),
        "harm_or_drift_diff": int(path.sum().item()),
        "max_rel_dsnr_same_harm_drift": float(ds[same].max().item()) if bool(same.any()) else 0.0,
        "max_rel_dsnr_all": float(ds.max().item()),
        "candidates_fp32": int(c32.sum().item()), "candidates_fp16": int(c16.sum().item()),
        "only_fp32": int((c32 & ~c16).sum().item()), "only_fp16": int((c16 & ~c32).sum().item()),
        "rel": "abs(snr16 - snr32) / max(1, abs(snr32))"}}
    del path, same, ds, c32, c16
    agg = {"bins": 0, "max_rel_dsnr": 0.0, "max_rel_dsnr_same_harm_drift": 0.0, "harm_diff": 0, "drift_diff": 0,
           "over_quantisation_bound": 0, "fp32_gpu_max_rel_dsnr": 0.0, "fp32_gpu_harm_or_drift_diff": 0}
    errs = []
    for data, g16, g32, lab in sample:
        w = oracle_call(data, lab)
        s64, hh, dd = w["snr"].reshape(-1), w["harm"].reshape(-1), w["drift"].reshape(-1)
        a16 = [t.reshape(-1).cpu().numpy() for t in g16]
        a32 = [t.reshape(-1).cpu().numpy() for t in g32]
        e = np.abs(a16[0].astype(np.float64) - s64) / np.maximum(1.0, np.abs(s64))
        sm = (a16[1] == hh) & (a16[2] == dd)
        mu, sg = w["mu1"], w["sigma1"]
        # first-order worst case of storage rounding (relative 2^-11 per value, statistics included)
        bound = 2.0 ** -11 * (2.0 * np.sqrt(np.maximum(hh, 1)) * mu / sg + np.abs(s64) * (2.0 + 2.0 * mu * mu / (sg * sg))) \
            + 1e-5 * np.maximum(1.0, np.abs(s64))
        e32 = np.abs(a32[0].astype(np.float64) - s64) / np.maximum(1.0, np.abs(s64))
        agg["bins"] += int(s64.size)
        agg["max_rel_dsnr"] = max(agg["max_rel_dsnr"], float(e.max(initial=0.0)))
        agg["max_rel_dsnr_same_harm_drift"] = max(agg["max_rel_dsnr_same_harm_drift"], float(e[sm].max(initial=0.0)))
        agg["harm_diff"] += int((a16[1] != hh).sum())
        agg["drift_diff"] += int((a16[2] != dd).sum())
        agg["over_quantisation_bound"] += int((np.abs(a16[0].astype(np.float64) - s64) > bound).sum())
        agg["fp32_gpu_max_rel_dsnr"] = max(agg["fp32_gpu_max_rel_dsnr"], float(e32.max(initial=0.0)))
        agg["fp32_gpu_harm_or_drift_diff"] += int(((a32[1] != hh) | (a32[2] != dd)).sum())
        errs.append(e)
    if errs:
        e = np.concatenate(errs)
        agg["p99_rel_dsnr"] = float(np.quantile(e, 0.99))
        agg["p999_rel_dsnr"] = float(np.quantile(e, 0.999))
        agg["mean_rel_dsnr"] = float(e.mean())
    agg["sample"] = sample_label
    agg["bound"] = ("abs(dsnr) <= 2^-11 (2 sqrt(harm) mu1/sigma1 + abs(snr64) (2 + 2 mu1^2/sigma1^2)) + 1e-5 max(1, abs(snr64))"
                    " on a path the rounding does not change")
    res["vs_fp64_oracle_on_fp32_data"] = agg
    return res


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
    counters = profile_records(TABLE2_FILE)
    modes = (("greedy", hs.HS_GREEDY), ("presto", hs.HS_PRESTO), ("presto_all", hs.HS_PRESTO_ALL),
             ("presto_plus", hs.HS_PRESTO_PLUS))
    for mname, mode in modes:
        res = {}
        for h in (4, 8, 16, 32):
            plan = hs.Plan(harmonics=h, mode=mode, dtype=hs.HS_F32, max_spectra=B)
            if mode == hs.HS_GREEDY:
                hs.hs_plan_tune_batched(plan.handle, xt, ot, B, None, snr, harm, None, None, 0, None, None, stream)
                fl = hs.hs_plan_get_launch(plan.handle)[0]
                kern = "k_sum_xcd<%d, true, false, %d>" % (h, fl) if fl else "k_sum_1d<%d, true, false>" % h
            else:
                kern = "k_presto<%d, %d, false>" % (h, mode)
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
            rec = counters.get((os.path.basename(TABLE2_FILE), kern))
            r["kernel"] = kern
            hbm_frac = comp / (sum_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
            if rec and "valu" in rec and "fetch_bytes" in rec and "write_bytes" in rec:
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


def single_spectrum_leg(hs, torch, dev, steps, copies=32):
    """One long spectrum (2^22 FP32 bins, Exp(1) noise + 50 pulse trains with
    fundamentals below N/32, H = 32), simple and greedy sums, dense outputs
    (6 B per bin): hs_sum_1d per call (the plain kernel, the single-spectrum
    default), cycling over `copies` copies of the input and outputs (32 x 40
    MiB, twice the 256 MB MALL) so every call starts from HBM; HIP events on
    the launch stream."""
    import synthetic
    x, _ = synthetic.config2()
    n = int(x.size)
    xs = torch.from_numpy(x).to(dev).repeat(copies, 1)
    snr = torch.empty((copies, n), dtype=torch.float32, device=dev)
    harm = torch.empty((copies, n), dtype=torch.uint8, device=dev)
    drift = torch.empty((copies, n), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    out = {"workload": "one spectrum of %d FP32 bins, H=32, dense snr/harm/drift, %d rotating copies" % (n, copies)}
    for mname, mode in (("standard", hs.HS_STANDARD), ("greedy", hs.HS_GREEDY)):
        plan = hs.Plan(harmonics=H, mode=mode, dtype=hs.HS_F32)
        i = [0]

        def call():
            c = i[0] % copies
            i[0] += 1
            hs.hs_sum_1d(plan.handle, xs[c], n, None, snr[c], harm[c], drift[c], None, stream)
        ms = _event_ms(torch, stream, call, max(steps, copies))
        plan.close()
        comp = 10.0 * n
        work = keff_sum([n], H, mode == hs.HS_GREEDY)
        out[mname] = {"ms_per_call": ms, "value": work / (ms * 1e-3), "unit": "bin·harmonics/s",
                      "gbin_s": n / (ms * 1e-3) / 1e9, "hbm_gbs_compulsory": comp / (ms * 1e-3) / 1e9,
                      "hbm_frac_compulsory": comp / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "l2_to_cu_tbs": line_bytes_sum([n], H, mode == hs.HS_GREEDY, 4) / (ms * 1e-3) / 1e12}
    del xs, snr, harm, drift
    return out


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


PROBE_K = 32
PROBE_LINE_BYTES = sum(min(4 * k, 128) for k in range(1, PROBE_K + 1))   # per fundamental (waves of 64)
PROBE_SETS = (("l2_resident", 1 << 19), ("mall_resident", 1 << 24), ("beyond_l2", 1 << 28))


def probe_leg(torch, dev, reps=10):
    """Gather ceilings of this device (libhs_probe.so): the greedy walk's
    stride-k pair gather (32 harmonics, waves of 64 consecutive fundamentals,
    no arithmetic beyond the compare) over a 2 MB set that every XCD's L2
    holds, a 64 MB set and a 1 GB set.  Line bytes = per fundamental the sum
    over k of min(4 k, 128) B, the L2-to-CU traffic of 128-byte lines; HIP
    events on the launch stream, median of ``reps`` launches."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2202_12817_amd", "libhs_probe.so"))
    lib.hsp_gather.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                               ctypes.c_void_p]
    lib.hsp_gather.restype = ctypes.c_int
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    blocks = 8 * n_cu
    n_fund = 1 << 24
    stream = torch.cuda.current_stream(dev)
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    res = {"pattern": "greedy pair gather, K=%d harmonics, %d fundamentals per launch, %d workgroups of 256"
                      % (PROBE_K, n_fund, blocks),
           "line_bytes_per_fundamental": PROBE_LINE_BYTES}
    for name, n in PROBE_SETS:
        x = torch.rand(n + 2, dtype=torch.float32, device=dev)

        def call():
            rc = lib.hsp_gather(x.data_ptr(), n - 1, n_fund, blocks, out.data_ptr(), stream.cuda_stream)
            if rc:
                raise RuntimeError("hsp_gather failed: %d" % rc)
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            call()
            b.record(stream)
            ts.append((a, b))
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in ts]))
        clk = n_cu * 2.4e9 * ms * 1e-3
        res[name] = {"set_bytes": 4 * n, "ms": ms, "line_gbs": n_fund * PROBE_LINE_BYTES / (ms * 1e-3) / 1e9,
                     "steps_per_clk_per_cu": n_fund * PROBE_K / clk,
                     "kernel": "k_probe_gather<%d>" % ({1 << 19: 0, 1 << 24: 1, 1 << 28: 2}[n])}
        rec = read_counters(res[name]["kernel"])
        if rec and "fetch_bytes" in rec:
            res[name]["fetch_gbs"] = rec["fetch_bytes"] / (ms * 1e-3) / 1e9
            res[name]["fetch_bytes"] = rec["fetch_bytes"]
        del x
    del out
    return res


def fp16_error_batched(hs, torch, x, off, xt, x16, ot, B, stream, sample):
    """FP16 storage error on the batched workload: dense FP32 and FP16 GPU
    outputs of every spectrum compared bin by bin, and the FP16 outputs of the
    ``sample`` spectra compared with the float64 oracle run on the original
    FP32 spectra (one thread per spectrum)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    n = int(x.size)
    o = {}
    for name, dt, xin in (("f32", hs.HS_F32, xt), ("f16", hs.HS_F16, x16)):
        snr = torch.empty(n, dtype=torch.float32, device=xt.device)
        harm = torch.empty(n, dtype=torch.uint8, device=xt.device)
        drift = torch.empty(n, dtype=torch.uint8, device=xt.device)
        plan = hs.Plan(harmonics=H, mode=hs.HS_GREEDY, dtype=dt, max_spectra=B, threshold=THRESHOLD)
        hs.hs_sum_batched(plan.handle, xin, ot, B, None, snr, harm, drift, None, 0, None, stream)
        torch.cuda.synchronize()
        plan.close()
        o[name] = (snr, harm, drift)
    with ThreadPoolExecutor(max(1, min(len(sample), cpu_threads()))) as ex:
        ref = dict(zip(sample, ex.map(lambda s: oracle.hs_1d(x[off[s]:off[s + 1]], H, oracle.GREEDY, precision="f64"),
                                      sample)))
    items = [(s, tuple(t[int(off[s]):int(off[s + 1])] for t in o["f16"]),
              tuple(t[int(off[s]):int(off[s + 1])] for t in o["f32"]), s) for s in sample]
    res = fp16_error_stats(torch, o["f32"], o["f16"], THRESHOLD, items, lambda d, s: ref[s],
                           "spectra %s (%d bins), float64 oracle on the FP32 spectra" % (
                               list(sample), int(sum(off[s + 1] - off[s] for s in sample))))
    del o
    return res


def cpu_threads():
    """Host threads the CPU legs use: the process's CPU set, at most 16 (the
    share of one GPU on a GPU host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_leg(x, off, lengths, sample_n, single_n, reps=3):
    """The oracle as it stands (float mirror: exact statistics in Python, the
    per-fundamental C loops, candidate selection) on the host: a thread pool
    over the first ``sample_n`` spectra (the C loops release the interpreter
    lock), wall-clock median of ``reps`` runs, and one thread on the first
    ``single_n`` spectra."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    def one(s):
        r = oracle.hs_1d(x[off[s]:off[s + 1]], H, oracle.GREEDY)
        oracle.candidates(r["snr"], r["harm"], r["drift"], THRESHOLD, spectrum=s)

    th = cpu_threads()
    sample = list(range(sample_n))
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        with ThreadPoolExecutor(th) as ex:
            list(ex.map(one, sample))
        ts.append(time.perf_counter() - t0)
    multi = float(np.median(ts))
    single = list(range(single_n))
    ts1 = []
    for _ in range(reps):
        t0 = time.perf_counter()
        for s in single:
            one(s)
        ts1.append(time.perf_counter() - t0)
    one_s = float(np.median(ts1))
    work = keff_sum(lengths[sample], H, True)
    work1 = keff_sum(lengths[single], H, True)
    return {"value": work / multi, "unit": "bin·harmonics/s", "cores": th, "kind": "oracle",
            "sample": "first %d spectra of the same batch (%d bins), float mirror: exact statistics, per-fundamental "
                      "C loops and candidate selection, one spectrum per thread, %d threads, median of %d runs"
                      % (len(sample), int(lengths[sample].sum()), th, reps),
            "ms_per_run": 1e3 * multi, "single_core_value": work1 / one_s,
            "single_core_sample": "first %d spectra (%d bins), median of %d runs" % (
                len(single), int(lengths[single].sum()), reps),
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def roofline_entry(kernel, comp_bytes, line_bytes, kernel_ms, probe, traffic_file=None):
    """Roofline of a harmonic-sum kernel: the HBM roofline of its compulsory
    bytes (input read once, outputs written once), plus the two on-chip
    resources the walk is bound by -- line traffic from L2 to the CUs against
    the probe's L2-resident ceiling, and traffic fetched beyond the L2 (the
    kernel's FETCH_SIZE from the committed counters) against the probe's
    beyond-L2 ceiling -- and which of the three is closest to its ceiling."""
    t = kernel_ms * 1e-3
    ach = comp_bytes / t / 1e9
    rec = read_counters(kernel, traffic_file)
    traffic = rec["fetch_bytes"] + rec["write_bytes"] if rec and "fetch_bytes" in rec and "write_bytes" in rec else None
    r = {"bound": "hbm", "kernel": kernel, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": ach / HBM_PEAK_GBS, "traffic": traffic}
    fr = {"hbm": ach / HBM_PEAK_GBS}
    if probe:
        g = line_bytes / t / 1e9
        r["gather"] = {"achieved": g, "peak": probe["l2_resident"]["line_gbs"], "unit": "GB/s",
                       "frac": g / probe["l2_resident"]["line_gbs"],
                       "what": "128-byte lines from L2 to the CUs (sum over steps of min(k s, 128) B) vs the "
                               "probe's L2-resident pair gather"}
        fr["gather"] = r["gather"]["frac"]
        beyond = probe["beyond_l2"]
        peak = beyond.get("fetch_gbs")
        if rec and "fetch_bytes" in rec and peak:
            f = rec["fetch_bytes"] / t / 1e9
            r["fabric"] = {"achieved": f, "peak": peak, "unit": "GB/s", "frac": f / peak,
                           "fetch_bytes": rec["fetch_bytes"],
                           "what": "bytes fetched beyond the L2 (FETCH_SIZE, committed counters) vs the probe's "
                                   "1 GB-set pair gather (its own FETCH_SIZE)"}
            fr["fabric"] = r["fabric"]["frac"]
    r["binding"] = max(fr, key=fr.get)
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--spectra", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip every leg but the headline step")
    ap.add_argument("--cpu-sample", type=int, default=96, help="spectra of the threaded CPU oracle run")
    ap.add_argument("--cpu-single", type=int, default=4, help="spectra of the one-thread CPU oracle run")
    ap.add_argument("--tune-cache", default=None, help="launch-shape cache file of the tuner (default: tune afresh)")
    ap.add_argument("--launch", default=None, metavar="F,W",
                    help="fixed launch shape (fundamentals per lane, workgroups per CU) instead of tuning")
    ap.add_argument("--no-plane", action="store_true", help="skip the f-fdot plane leg (2^21 x 201, H=16)")
    ap.add_argument("--leg", choices=["table2", "plane_2d", "gather", "single"], default=None,
                    help="run only this leg and print its JSON object (profiling aid)")
    ap.add_argument("--fp16", action="store_true", help="headline step on FP16 storage (profiling aid)")
    ap.add_argument("--plane-kernel", choices=["auto", "plain", "persistent"], default="auto",
                    help="kernel choice of the plane leg (profiling aid)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="also run a 1 GiB read + 1 GiB write elementwise kernel (reference for rocprofv3 byte counters)")
    ap.add_argument("--pmc-summary", nargs="+", metavar="DIR",
                    help="summarise rocprofv3 output directories (kernel trace and --pmc CSV) and exit (no GPU work)")
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
                "plane_2d": lambda: plane_2d_leg(hs, torch, dev, args.steps, args.warmup, error=False,
                                                 kernel=args.plane_kernel),
                "gather": lambda: probe_leg(torch, dev),
                "single": lambda: single_spectrum_leg(hs, torch, dev, args.steps)}
        print(json.dumps({args.leg: legs[args.leg]()}))
        return
    x, off = synthetic.config3(n_spectra=args.spectra, threads=16)
    lengths = np.diff(off)
    n_bins = int(x.size)
    xt = torch.from_numpy(x).to(dev)
    ot = torch.from_numpy(off).to(dev)
    B = args.spectra
    work = keff_sum(lengths, H, True)
    stream = torch.cuda.current_stream(dev)
    x16 = None
    if args.fp16 or not args.no_extra:
        # FP16 storage with a per-spectrum scale (the spectrum's mean)
        x16 = torch.empty(n_bins, dtype=torch.int16, device=dev)
        for s in range(B):
            scale = float(np.float32(x[off[s]:off[s + 1]].mean(dtype=np.float64)))
            hs.hs_quantize_f16(xt.data_ptr() + 4 * int(off[s]), int(lengths[s]), scale,
                               x16.data_ptr() + 2 * int(off[s]), stream)
        torch.cuda.synchronize()

    cap = 1 << 24
    cand = torch.empty((cap, 4), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)

    def step(p, xin):
        hs.hs_sum_batched(p.handle, xin, ot, B, None, None, None, None, cand, cap, count, stream)

    def timed(dtype, xin, fundamental_end=0, graph=False):
        """Tune the launch shape on this batch (unless fixed), warm up, time the steps."""
        plan = hs.Plan(harmonics=H, mode=hs.HS_GREEDY, dtype=dtype, max_spectra=B, threshold=THRESHOLD,
                       fundamental_end=fundamental_end)
        if args.launch:
            hs.hs_plan_set_launch(plan.handle, *[int(v) for v in args.launch.split(",")])
        else:
            hs.hs_plan_tune_batched(plan.handle, xin, ot, B, None, None, None, None, cand, cap, count,
                                    args.tune_cache, stream)
        shape = hs.hs_plan_get_launch(plan.handle)
        for _ in range(args.warmup):
            step(plan, xin)
        torch.cuda.synchronize()
        hs.hs_plan_set_timing(plan.handle, True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(plan, xin)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        calls, norm_ms, sum_ms = hs.hs_plan_get_timing(plan.handle)
        hs.hs_plan_set_timing(plan.handle, False)
        r = {"elapsed": elapsed, "shape": shape, "norm_ms": norm_ms / max(1, calls),
             "sum_ms": sum_ms / max(1, calls), "candidates": int(count.item())}
        if graph:
            # the same step replayed as one captured hipGraph per call
            hs.hs_plan_set_graph(plan.handle, True)
            step(plan, xin)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                step(plan, xin)
            torch.cuda.synchronize()
            r["graph_ms"] = 1e3 * (time.perf_counter() - t0) / args.steps
            r["graph_info"] = hs.hs_plan_graph_info(plan.handle)
            hs.hs_plan_set_graph(plan.handle, False)
        plan.close()
        return r

    eb = 2 if args.fp16 else 4
    head = timed(hs.HS_F16 if args.fp16 else hs.HS_F32, x16 if args.fp16 else xt, graph=not args.no_extra)
    ms_step = 1e3 * head["elapsed"] / args.steps
    value = work * args.steps / head["elapsed"]
    shape = head["shape"]
    n_cand = head["candidates"]
    in_bytes = eb * n_bins
    lines = line_bytes_sum(lengths, H, True, eb)
    sum_kernel = ("k_sum_xcd<32, true, %s, %d>" % ("true" if args.fp16 else "false", shape[0])) if shape[0] else \
        "k_sum_1d<32, true, %s>" % ("true" if args.fp16 else "false")
    cand_bytes = 16 * min(n_cand, cap)
    probe = None if args.no_extra else probe_leg(torch, dev)

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
        "dtype": "f16 storage, f32 sums" if args.fp16 else "f32",
        "data": "synthetic",
        "config": {"workload": "batched 1D greedy harmonic sum: %d spectra of 2^20..2^22 %s bins "
                               "(Exp(1) noise + 5 pulse trains each), H=%d, SNR>%g candidate compaction"
                               % (B, "FP16" if args.fp16 else "FP32", H, THRESHOLD),
                   "spectra": B, "bins": n_bins, "H": H, "mode": "greedy", "threshold": THRESHOLD,
                   "bin_harmonics": work, "candidates": n_cand},
        "bins_per_s": n_bins * args.steps / head["elapsed"],
        "hbm_gbs_compulsory": (in_bytes + cand_bytes) / (ms_step * 1e-3) / 1e9,
        "hbm_frac_compulsory": (in_bytes + cand_bytes) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "stage_ms": {"normalisation": head["norm_ms"], "harmonic_sum": head["sum_ms"]},
        "launch": {"fundamentals_per_lane": shape[0], "workgroups_per_cu": shape[1], "tuned": not args.launch},
        "gather": {"touched_bytes": 2 * eb * work, "touched_gbs": 2 * eb * work / (head["sum_ms"] * 1e-3) / 1e9,
                   "l2_to_cu_bytes": lines, "l2_to_cu_tbs": lines / (head["sum_ms"] * 1e-3) / 1e12,
                   "note": "harmonic-sum kernel: 2 s B touched per greedy step (the compared pair); "
                           "min(k s, 128) B per step at cache-line granularity"},
        "roofline": roofline_entry(sum_kernel, in_bytes + cand_bytes, lines, head["sum_ms"], probe, TRAFFIC_FILE),
    }
    if "graph_ms" in head:
        result["graph_replay"] = {"ms_per_step": head["graph_ms"], "value": work / (head["graph_ms"] * 1e-3),
                                  "graphs_recorded": head["graph_info"][0], "replays": head["graph_info"][1]}
    if probe:
        result["gather_ceilings"] = probe

    if args.calibration_copy:
        calibration_copy(torch, dev)

    if not args.no_extra:
        # full-H fundamentals only (reading of the truncation rule: fundamentals
        # below (N-1)/(H+1) of the shortest spectrum, all 32 harmonics each)
        n_hi = (int(lengths.min()) - 1) // (H + 1)
        fh = timed(hs.HS_F32, xt, fundamental_end=n_hi)
        ms_fh = 1e3 * fh["elapsed"] / args.steps
        work_fh = keff_sum(lengths, H, True, fundamental_end=n_hi)
        lines_fh = line_bytes_sum(lengths, H, True, 4, fundamental_end=n_hi)
        result["full_h_fundamentals"] = {
            "fundamental_end": n_hi, "value": work_fh / (ms_fh * 1e-3), "unit": "bin·harmonics/s",
            "ms_per_step": ms_fh, "stage_ms": {"normalisation": fh["norm_ms"], "harmonic_sum": fh["sum_ms"]},
            "bin_harmonics": work_fh, "l2_to_cu_bytes": lines_fh,
            "l2_to_cu_tbs": lines_fh / (fh["sum_ms"] * 1e-3) / 1e12, "candidates": fh["candidates"],
            "launch": {"fundamentals_per_lane": fh["shape"][0], "workgroups_per_cu": fh["shape"][1]},
            "note": "fundamentals [1, %d) of every spectrum (all of them sum 32 harmonics); the statistics "
                    "still cover whole spectra" % n_hi}

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
        del snr, harm, drift
        result["plain_fp32"] = {"value": work / plain_s, "ms_per_step": 1e3 * plain_s,
                                "speedup_batched": plain_s / (ms_step * 1e-3)}
        # FP16 storage, the same step
        h16 = timed(hs.HS_F16, x16)
        e16 = h16["elapsed"] / args.steps
        k16 = ("k_sum_xcd<32, true, true, %d>" % h16["shape"][0]) if h16["shape"][0] else "k_sum_1d<32, true, true>"
        n_cand16 = h16["candidates"]
        result["batched_fp16"] = {
            "value": work / e16, "ms_per_step": 1e3 * e16, "speedup_vs_plain_fp32": plain_s / e16,
            "speedup_vs_batched_fp32": ms_step / (1e3 * e16),
            "hbm_gbs_compulsory": (2 * n_bins + 16 * n_cand16) / e16 / 1e9,
            "stage_ms": {"normalisation": h16["norm_ms"], "harmonic_sum": h16["sum_ms"]},
            "launch": {"fundamentals_per_lane": h16["shape"][0], "workgroups_per_cu": h16["shape"][1]},
            "candidates": n_cand16,
            "roofline": roofline_entry(k16, 2 * n_bins + 16 * n_cand16, line_bytes_sum(lengths, H, True, 2),
                                       h16["sum_ms"], probe),
            "error": fp16_error_batched(hs, torch, x, off, xt, x16, ot, B, stream,
                                        sample=[0, 1, 128, 255, 384, 511][:max(1, min(6, B))] if B > 1 else [0])}

    if x16 is not None:
        del x16
    if not args.no_extra and not args.no_plane:
        result["plane_2d"] = plane_2d_leg(hs, torch, dev, args.steps, args.warmup)
    if not args.no_extra:
        result["single_spectrum"] = single_spectrum_leg(hs, torch, dev, args.steps)
        result["small_1d"] = small_1d_leg(hs, torch, dev)
        result["table2"] = table2_leg(hs, torch, dev, min(args.steps, 10), args.warmup)

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline_leg(x, off, lengths, min(args.cpu_sample, B), min(args.cpu_single, B))
    print(json.dumps(result))


if __name__ == "__main__":
    main()
