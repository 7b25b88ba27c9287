"""Torch-facing helpers around the C ABI: allocate outputs, pick the plan.

Every result is computed by the HIP kernels of ``libhs.so``; these helpers
only allocate device tensors and pass pointers.
"""
from __future__ import annotations

import torch

from . import hs

_MODES = {"standard": hs.HS_STANDARD, "greedy": hs.HS_GREEDY, "presto": hs.HS_PRESTO,
          "presto_all": hs.HS_PRESTO_ALL, "presto_plus": hs.HS_PRESTO_PLUS}
_MODES.update({v: v for v in list(_MODES.values())})


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return hs.HS_F32
    if t.dtype in (torch.float16, torch.uint16, torch.int16):
        return hs.HS_F16
    raise TypeError("powers must be float32 or float16 (or their 16-bit patterns)")


def _check_powers(t: torch.Tensor, name="x"):
    """The library reads ``t`` through its device pointer: it must be a
    contiguous device tensor of 32- or 16-bit powers (checked here, before any
    library call, so a host or strided tensor never reaches a kernel)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a device (cuda) tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    _dtype_code(t)


def _check_offsets(offsets: torch.Tensor, x: torch.Tensor):
    if not isinstance(offsets, torch.Tensor) or not offsets.is_cuda or offsets.device != x.device:
        raise ValueError("offsets must be a device tensor on the device of x")
    if offsets.dtype != torch.int64 or not offsets.is_contiguous() or offsets.dim() != 1 or offsets.numel() < 2:
        raise ValueError("offsets must be a contiguous int64 vector of n_spectra + 1 entries")


def _check_plan_device(plan: hs.Plan, t: torch.Tensor):
    dev = getattr(plan, "device", None)
    if dev is not None and t.device != dev:
        raise ValueError("the tensors are on %s but the plan on %s" % (t.device, dev))


def _mask(ks) -> int:
    m = 0
    for k in ks:
        m |= 1 << (int(k) - 1)
    return m


_KERNELS = {"auto": hs.HS_KERNEL_AUTO, "persistent": hs.HS_KERNEL_PERSISTENT, "plain": hs.HS_KERNEL_PLAIN}


def make_plan(H, mode, dtype=hs.HS_F32, *, first_bin=1, harmonic_mask=0, report_mask=0, fundamental_end=0,
              max_spectra=1, threshold=6.0, kernel="auto", norm_table=False) -> hs.Plan:
    plan = hs.Plan(harmonics=int(H), mode=_MODES[mode], dtype=int(dtype), first_bin=int(first_bin),
                   harmonic_mask=int(harmonic_mask), report_mask=int(report_mask),
                   fundamental_end=int(fundamental_end), max_spectra=int(max_spectra),
                   threshold=float(threshold), kernel=_KERNELS[kernel],
                   norm_kind=hs.HS_NORM_TABLE if norm_table else hs.HS_NORM_MU_SIGMA)
    plan.device = torch.device("cuda", torch.cuda.current_device())
    return plan


def _norm_tensor(norm, n, device, H=None, table=False):
    """(mu1, sigma1) per spectrum, or with ``table`` the per-k (mu_k, sigma_k)
    table [n][2][H] (mu_1..mu_H, then sigma_1..sigma_H), as a float64 device vector."""
    if norm is None:
        return None
    t = torch.as_tensor(norm, dtype=torch.float64).reshape(-1)
    want = 2 * n * H if table else 2 * n
    if t.numel() != want:
        raise ValueError("norm needs %s per spectrum" % ("(mu_k, sigma_k) for k = 1..H" if table else "(mu1, sigma1)"))
    return t.contiguous().to(device)


def sum_1d(x: torch.Tensor, H: int, mode="greedy", *, first_bin=1, harmonic_mask=0, fundamental_end=0,
           report=(), norm=None, norm_table=None, plan: hs.Plan | None = None, stream=None, with_norm=False,
           kernel="auto"):
    """Dense harmonic sum of one spectrum; returns snr/harm/drift (+ partial, norm).

    ``norm``: (mu1, sigma1); ``norm_table``: per-k (mu_k, sigma_k), shape [2, H]
    (the plan, if given, must have been made with ``norm_table=True``)."""
    _check_powers(x)
    if norm is not None and norm_table is not None:
        raise ValueError("give norm or norm_table, not both")
    n = x.numel()
    own = plan is None
    if own:
        plan = make_plan(H, mode, _dtype_code(x), first_bin=first_bin, harmonic_mask=harmonic_mask,
                         report_mask=_mask(report), fundamental_end=fundamental_end, kernel=kernel,
                         norm_table=norm_table is not None)
    _check_plan_device(plan, x)
    dev = x.device
    snr = torch.empty(n, dtype=torch.float32, device=dev)
    harm = torch.empty(n, dtype=torch.uint8, device=dev)
    drift = torch.empty(n, dtype=torch.uint8, device=dev)
    partial = torch.empty((len(report), n), dtype=torch.float32, device=dev) if len(report) else None
    nt = _norm_tensor(norm_table, 1, dev, plan.desc.harmonics, True) if norm_table is not None else \
        _norm_tensor(norm, 1, dev)
    hs.hs_sum_1d(plan.handle, x, n, nt, snr, harm, drift, partial, stream)
    out = dict(snr=snr, harm=harm, drift=drift, partial=partial)
    if with_norm:
        out.update(get_norm(plan, 1, plan.desc.harmonics, dev, stream))
    if own:
        torch.cuda.synchronize(dev)
        plan.close()
    return out


def get_norm(plan: hs.Plan, n: int, H: int, device, stream=None):
    """(mu1, sigma1), float tables [n, 2, H] and validity of the last call's spectra."""
    ms = torch.empty(2 * n, dtype=torch.float64, device=device)
    tab = torch.empty((n, 2, H), dtype=torch.float32, device=device)
    valid = torch.empty(n, dtype=torch.int32, device=device)
    hs.hs_get_norm(plan.handle, n, ms, tab, valid, stream)
    return dict(mu_sigma=ms.view(n, 2), tables=tab, valid=valid)


def sum_batched(x: torch.Tensor, offsets: torch.Tensor, H: int, mode="greedy", threshold=6.0, *, first_bin=1,
                harmonic_mask=0, fundamental_end=0, dense=False, candidates=True, capacity=None, norm=None,
                norm_table=None, plan: hs.Plan | None = None, stream=None, with_norm=False, kernel="auto"):
    """Batch of spectra ``x[offsets[s]:offsets[s+1]]``; candidates and/or dense outputs.

    ``offsets``: int64 device tensor of n_spectra + 1 entries (CSR).  ``norm``:
    (mu1, sigma1) per spectrum; ``norm_table``: [n_spectra, 2, H] per-k tables."""
    _check_powers(x)
    _check_offsets(offsets, x)
    if norm is not None and norm_table is not None:
        raise ValueError("give norm or norm_table, not both")
    B = offsets.numel() - 1
    dev = x.device
    own = plan is None
    if own:
        plan = make_plan(H, mode, _dtype_code(x), first_bin=first_bin, harmonic_mask=harmonic_mask,
                         fundamental_end=fundamental_end, max_spectra=B, threshold=threshold, kernel=kernel,
                         norm_table=norm_table is not None)
    _check_plan_device(plan, x)
    out = {}
    snr = harm = drift = cand = count = None
    if dense:
        snr = torch.empty(x.numel(), dtype=torch.float32, device=dev)
        harm = torch.empty(x.numel(), dtype=torch.uint8, device=dev)
        drift = torch.empty(x.numel(), dtype=torch.uint8, device=dev)
        out.update(snr=snr, harm=harm, drift=drift)
    cap = 0
    if candidates:
        cap = int(capacity) if capacity is not None else max(1024, x.numel() // 64)
        cand = torch.empty((max(cap, 1), hs.CANDIDATE_BYTES // 4), dtype=torch.int32, device=dev)
        count = torch.zeros(1, dtype=torch.int64, device=dev)
        out.update(cand_raw=cand, count=count)
    nt = _norm_tensor(norm_table, B, dev, plan.desc.harmonics, True) if norm_table is not None else \
        _norm_tensor(norm, B, dev)
    hs.hs_sum_batched(plan.handle, x, offsets, B, nt, snr, harm, drift, cand, cap, count, stream)
    if with_norm:
        out.update(get_norm(plan, B, plan.desc.harmonics, dev, stream))
    if own:
        torch.cuda.synchronize(dev)
        plan.close()
    return out


def sum_2d(plane: torch.Tensor, z_min: int, z_max: int, H: int, mode="greedy", *, first_bin=1, harmonic_mask=0,
           fundamental_end=0, dense=True, candidates=False, threshold=6.0, capacity=None, norm=None,
           norm_table=None, plan: hs.Plan | None = None, stream=None, with_norm=False, kernel="auto"):
    """f-fdot plane [n_z, n_r] (row stride from the tensor); dense planes and/or candidates."""
    if not isinstance(plane, torch.Tensor) or not plane.is_cuda or plane.dim() != 2:
        raise ValueError("plane must be a 2-D device (cuda) tensor")
    _dtype_code(plane)
    n_z, n_r = plane.shape
    if n_z != z_max - z_min + 1:
        raise ValueError("plane rows do not match z range")
    if plane.stride(1) != 1:
        raise ValueError("plane columns must be contiguous")
    if norm is not None and norm_table is not None:
        raise ValueError("give norm or norm_table, not both")
    dev = plane.device
    own = plan is None
    if own:
        plan = make_plan(H, mode, _dtype_code(plane), first_bin=first_bin, harmonic_mask=harmonic_mask,
                         fundamental_end=fundamental_end, threshold=threshold, kernel=kernel,
                         norm_table=norm_table is not None)
    _check_plan_device(plan, plane)
    out = {}
    snr = harm = drift = cand = count = None
    if dense:
        snr = torch.empty((n_z, n_r), dtype=torch.float32, device=dev)
        harm = torch.empty((n_z, n_r), dtype=torch.uint8, device=dev)
        drift = torch.empty((n_z, n_r), dtype=torch.uint8, device=dev)
        out.update(snr=snr, harm=harm, drift=drift)
    cap = 0
    if candidates:
        cap = int(capacity) if capacity is not None else max(1024, plane.numel() // 64)
        cand = torch.empty((max(cap, 1), hs.CANDIDATE_BYTES // 4), dtype=torch.int32, device=dev)
        count = torch.zeros(1, dtype=torch.int64, device=dev)
        out.update(cand_raw=cand, count=count)
    nt = _norm_tensor(norm_table, 1, dev, plan.desc.harmonics, True) if norm_table is not None else \
        _norm_tensor(norm, 1, dev)
    hs.hs_sum_2d(plan.handle, plane, n_r, plane.stride(0), z_min, z_max, nt, snr, harm, drift, cand, cap, count,
                 stream)
    if with_norm:
        out.update(get_norm(plan, 1, plan.desc.harmonics, dev, stream))
    if own:
        torch.cuda.synchronize(dev)
        plan.close()
    return out


def interleave(x: torch.Tensor, stream=None) -> torch.Tensor:
    """[B][N] spectra -> the interleaved layout [N][B] (float32 or 16-bit)."""
    _check_powers(x, "spectra")
    if x.dim() != 2:
        raise ValueError("spectra must be [B][N]")
    B, N = x.shape
    out = torch.empty((N, B), dtype=x.dtype, device=x.device)
    hs.hs_interleave(x, N, B, x.element_size(), out, stream)
    return out


def sum_interleaved(x: torch.Tensor, H: int, mode="greedy", threshold=6.0, *, first_bin=1, harmonic_mask=0,
                    fundamental_end=0, dense=True, candidates=False, capacity=None, norm=None,
                    plan: hs.Plan | None = None, stream=None, with_norm=False):
    """Equal-length spectra in the interleaved layout [N][B] (bin-major); outputs [N][B] and/or candidates."""
    _check_powers(x)
    if x.dim() != 2:
        raise ValueError("the interleaved array must be [N][B]")
    N, B = x.shape
    dev = x.device
    own = plan is None
    if own:
        plan = make_plan(H, mode, _dtype_code(x), first_bin=first_bin, harmonic_mask=harmonic_mask,
                         fundamental_end=fundamental_end, max_spectra=B, threshold=threshold)
    _check_plan_device(plan, x)
    out = {}
    snr = harm = drift = cand = count = None
    if dense:
        snr = torch.empty((N, B), dtype=torch.float32, device=dev)
        harm = torch.empty((N, B), dtype=torch.uint8, device=dev)
        drift = torch.empty((N, B), dtype=torch.uint8, device=dev)
        out.update(snr=snr, harm=harm, drift=drift)
    cap = 0
    if candidates:
        cap = int(capacity) if capacity is not None else max(1024, x.numel() // 64)
        cand = torch.empty((max(cap, 1), hs.CANDIDATE_BYTES // 4), dtype=torch.int32, device=dev)
        count = torch.zeros(1, dtype=torch.int64, device=dev)
        out.update(cand_raw=cand, count=count)
    nt = _norm_tensor(norm, B, dev)
    hs.hs_sum_interleaved(plan.handle, x, N, B, nt, snr, harm, drift, cand, cap, count, stream)
    if with_norm:
        out.update(get_norm(plan, B, plan.desc.harmonics, dev, stream))
    if own:
        torch.cuda.synchronize(dev)
        plan.close()
    return out


def power_spectrum(fft: torch.Tensor, interbin=False, scale=1.0, stream=None) -> torch.Tensor:
    """Powers (float32) of complex64 FFT bins, inter-binned (2N - 1 values) or not."""
    if not isinstance(fft, torch.Tensor) or not fft.is_cuda or fft.dtype != torch.complex64 or not fft.is_contiguous():
        raise ValueError("fft must be a contiguous complex64 device tensor")
    n = fft.numel()
    out = torch.empty(2 * n - 1 if interbin else n, dtype=torch.float32, device=fft.device)
    hs.hs_power_spectrum(fft, n, int(bool(interbin)), scale, out, stream)
    return out


def cluster_peaks(snr: torch.Tensor, harm: torch.Tensor, drift, threshold: float, radius: int, offsets=None,
                  capacity=None, stream=None):
    """Peak clustering of dense outputs (one spectrum, or a batch through device offsets)."""
    for t, name, dt in ((snr, "snr", torch.float32), (harm, "harm", torch.uint8), (drift, "drift", torch.uint8)):
        if t is None and name == "drift":
            continue
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous() \
                or t.device != snr.device or t.numel() != snr.numel():
            raise ValueError("%s must be a contiguous %s device tensor like snr" % (name, dt))
    if offsets is not None:
        _check_offsets(offsets, snr)
    n = snr.numel()
    B = 1 if offsets is None else offsets.numel() - 1
    cap = int(capacity) if capacity is not None else max(1024, n // 64)
    cand = torch.empty((max(cap, 1), hs.CANDIDATE_BYTES // 4), dtype=torch.int32, device=snr.device)
    count = torch.zeros(1, dtype=torch.int64, device=snr.device)
    hs.hs_cluster_peaks(snr, harm, drift, offsets, n, B, radius, threshold, cand, cap, count, stream)
    return dict(cand_raw=cand, count=count)


def quantize_f16(x: torch.Tensor, scale: float, stream=None) -> torch.Tensor:
    """FP16 storage of float32 powers (binary16 patterns viewed as float16)."""
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous():
        raise ValueError("x must be a contiguous float32 device tensor")
    out = torch.empty(x.numel(), dtype=torch.int16, device=x.device)
    hs.hs_quantize_f16(x, x.numel(), scale, out, stream)
    return out.view(torch.float16)


def candidates_numpy(out, limit=None):
    """Copy candidate records to a numpy structured array (host)."""
    import numpy as np
    dt = np.dtype([("spectrum", "<u4"), ("bin", "<u4"), ("snr", "<f4"), ("harm", "<u2"), ("drift", "<u2")])
    n = int(out["count"].item())
    m = min(n, out["cand_raw"].shape[0]) if limit is None else min(n, limit)
    raw = out["cand_raw"][:m].cpu().numpy()
    return raw.view(dt).reshape(-1), n
