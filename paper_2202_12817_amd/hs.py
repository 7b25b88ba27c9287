"""ctypes binding of ``libhs.so`` (the C ABI of ``include/hs.h``).

Argument marshalling only: every function here forwards to the C entry point
of the same name.  Array arguments may be torch tensors (their device
``data_ptr()`` is passed), plain integer device addresses, or ``None`` for a
NULL pointer; ``stream`` may be a ``torch.cuda.Stream``, an integer
``hipStream_t`` or ``None`` (torch's current stream).  A non-OK status raises
:class:`HsError`.  The library must have been built (``build()`` of
``__graft_entry__`` or ``python -m paper_2202_12817_amd.build``): there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhs.so")

HS_OK, HS_ERR_ARG, HS_ERR_UNSUPPORTED, HS_ERR_HIP, HS_ERR_NOMEM, HS_ERR_INTERNAL = 0, 1, 2, 3, 4, 5
HS_STANDARD, HS_GREEDY = 0, 1
HS_PRESTO, HS_PRESTO_ALL, HS_PRESTO_PLUS = 2, 3, 4
HS_F32, HS_F16 = 0, 1
HS_KERNEL_AUTO, HS_KERNEL_PERSISTENT, HS_KERNEL_PLAIN = 0, 1, 2
HS_NORM_MU_SIGMA, HS_NORM_TABLE = 0, 1
HS_MAX_HARMONICS = 64

EXPORTED = ["hs_plan_desc_init", "hs_plan_create", "hs_plan_create_in", "hs_plan_workspace_bytes",
            "hs_plan_destroy", "hs_sum_1d", "hs_sum_batched", "hs_sum_2d", "hs_get_norm", "hs_quantize_f16",
            "hs_plan_set_timing", "hs_plan_get_timing", "hs_plan_set_graph", "hs_plan_graph_info",
            "hs_plan_set_launch", "hs_plan_get_launch", "hs_plan_tune_batched", "hs_status_string",
            "hs_last_error", "hs_sum_interleaved", "hs_interleave", "hs_power_spectrum", "hs_cluster_peaks",
            "hs_sum_batched_static"]


class HsPlanDesc(ctypes.Structure):
    _fields_ = [("harmonics", ctypes.c_int32), ("mode", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("first_bin", ctypes.c_int32), ("harmonic_mask", ctypes.c_uint64),
                ("report_mask", ctypes.c_uint64), ("fundamental_end", ctypes.c_int64),
                ("max_spectra", ctypes.c_int32), ("threshold", ctypes.c_float), ("kernel", ctypes.c_int32),
                ("norm_kind", ctypes.c_int32)]


class HsCandidate(ctypes.Structure):
    _fields_ = [("spectrum", ctypes.c_uint32), ("bin", ctypes.c_uint32), ("snr", ctypes.c_float),
                ("harm", ctypes.c_uint16), ("drift", ctypes.c_uint16)]


CANDIDATE_BYTES = ctypes.sizeof(HsCandidate)


class HsError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__("%s: %s (%s)" % (where, _status_string(status), message))
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load ``libhs.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("libhs.so is not built (%s); run __graft_entry__.build()" % path)
        lib = ctypes.CDLL(path)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.hs_plan_desc_init.argtypes = [ctypes.POINTER(HsPlanDesc)]
        lib.hs_plan_desc_init.restype = None
        lib.hs_plan_create.argtypes = [ctypes.POINTER(HsPlanDesc), ctypes.POINTER(vp)]
        lib.hs_plan_create_in.argtypes = [ctypes.POINTER(HsPlanDesc), vp, ctypes.c_size_t, ctypes.POINTER(vp)]
        lib.hs_plan_workspace_bytes.argtypes = [ctypes.POINTER(HsPlanDesc), ctypes.POINTER(ctypes.c_size_t)]
        lib.hs_plan_destroy.argtypes = [vp]
        lib.hs_sum_1d.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp]
        lib.hs_sum_batched.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp, i64, vp, vp]
        lib.hs_sum_2d.argtypes = [vp, vp, i64, i64, i32, i32, vp, vp, vp, vp, vp, i64, vp, vp]
        lib.hs_sum_batched_static.argtypes = [ctypes.POINTER(HsPlanDesc), vp, vp, i32, vp, vp, vp, vp, vp, i64, vp,
                                              vp]
        lib.hs_get_norm.argtypes = [vp, i32, vp, vp, vp, vp]
        lib.hs_sum_interleaved.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp, vp, i64, vp, vp]
        lib.hs_interleave.argtypes = [vp, i64, i32, i32, vp, vp]
        lib.hs_power_spectrum.argtypes = [vp, i64, i32, ctypes.c_float, vp, vp]
        lib.hs_cluster_peaks.argtypes = [vp, vp, vp, vp, i64, i32, i32, ctypes.c_float, vp, i64, vp, vp]
        lib.hs_quantize_f16.argtypes = [vp, i64, ctypes.c_float, vp, vp]
        lib.hs_plan_set_timing.argtypes = [vp, i32]
        lib.hs_plan_get_timing.argtypes = [vp, vp, vp, vp]
        lib.hs_plan_set_graph.argtypes = [vp, i32]
        lib.hs_plan_graph_info.argtypes = [vp, vp, vp]
        lib.hs_plan_set_launch.argtypes = [vp, i32, i32]
        lib.hs_plan_get_launch.argtypes = [vp, vp, vp]
        lib.hs_plan_tune_batched.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp, i64, vp, ctypes.c_char_p, vp]
        lib.hs_status_string.argtypes = [ctypes.c_int]
        lib.hs_status_string.restype = ctypes.c_char_p
        lib.hs_last_error.argtypes = []
        lib.hs_last_error.restype = ctypes.c_char_p
        for name in ("hs_plan_create", "hs_plan_create_in", "hs_plan_workspace_bytes", "hs_plan_destroy",
                     "hs_sum_1d", "hs_sum_batched", "hs_sum_2d", "hs_get_norm", "hs_quantize_f16", "hs_plan_set_timing", "hs_plan_get_timing",
                     "hs_plan_set_graph", "hs_plan_graph_info", "hs_plan_set_launch", "hs_plan_get_launch",
                     "hs_plan_tune_batched", "hs_sum_interleaved", "hs_interleave", "hs_power_spectrum",
                     "hs_cluster_peaks", "hs_sum_batched_static"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _status_string(status):
    try:
        return load().hs_status_string(status).decode()
    except Exception:  # noqa: BLE001 - only used to format an error
        return "status %d" % status


def _check(status, where):
    if status != HS_OK:
        raise HsError(status, where, load().hs_last_error().decode())


def _p(a):
    if a is None:
        return None
    if isinstance(a, int):
        return a
    return a.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def hs_plan_desc_init(**overrides) -> HsPlanDesc:
    d = HsPlanDesc()
    load().hs_plan_desc_init(ctypes.byref(d))
    for k, v in overrides.items():
        setattr(d, k, v)
    return d


def hs_plan_create(desc: HsPlanDesc) -> int:
    h = ctypes.c_void_p()
    _check(load().hs_plan_create(ctypes.byref(desc), ctypes.byref(h)), "hs_plan_create")
    return h.value


def hs_plan_workspace_bytes(desc: HsPlanDesc) -> int:
    n = ctypes.c_size_t()
    _check(load().hs_plan_workspace_bytes(ctypes.byref(desc), ctypes.byref(n)), "hs_plan_workspace_bytes")
    return n.value


def hs_plan_create_in(desc: HsPlanDesc, workspace, nbytes: int) -> int:
    h = ctypes.c_void_p()
    _check(load().hs_plan_create_in(ctypes.byref(desc), _p(workspace), int(nbytes), ctypes.byref(h)),
           "hs_plan_create_in")
    return h.value


def hs_plan_destroy(plan: int) -> None:
    _check(load().hs_plan_destroy(plan), "hs_plan_destroy")


def hs_sum_1d(plan, x, n_bins, norm, snr, harm, drift, partial=None, stream=None):
    _check(load().hs_sum_1d(plan, _p(x), int(n_bins), _p(norm), _p(snr), _p(harm), _p(drift), _p(partial),
                            _stream(stream)), "hs_sum_1d")


def hs_sum_batched(plan, x, offsets, n_spectra, norm, snr, harm, drift, cand, cand_capacity, cand_count,
                   stream=None):
    _check(load().hs_sum_batched(plan, _p(x), _p(offsets), int(n_spectra), _p(norm), _p(snr), _p(harm),
                                 _p(drift), _p(cand), int(cand_capacity), _p(cand_count), _stream(stream)),
           "hs_sum_batched")


def hs_sum_batched_static(desc, x, offsets, n_spectra, norm, snr, harm, drift, cand, cand_capacity, cand_count,
                          stream=None):
    _check(load().hs_sum_batched_static(ctypes.byref(desc), _p(x), _p(offsets), int(n_spectra), _p(norm), _p(snr),
                                        _p(harm), _p(drift), _p(cand), int(cand_capacity), _p(cand_count),
                                        _stream(stream)), "hs_sum_batched_static")


def hs_sum_2d(plan, plane, n_r, row_stride, z_min, z_max, norm, snr, harm, drift, cand=None, cand_capacity=0,
              cand_count=None, stream=None):
    _check(load().hs_sum_2d(plan, _p(plane), int(n_r), int(row_stride), int(z_min), int(z_max), _p(norm),
                            _p(snr), _p(harm), _p(drift), _p(cand), int(cand_capacity), _p(cand_count),
                            _stream(stream)), "hs_sum_2d")


def hs_sum_interleaved(plan, x, n_bins, n_spectra, norm, snr, harm, drift, cand=None, cand_capacity=0,
                       cand_count=None, stream=None):
    _check(load().hs_sum_interleaved(plan, _p(x), int(n_bins), int(n_spectra), _p(norm), _p(snr), _p(harm),
                                     _p(drift), _p(cand), int(cand_capacity), _p(cand_count), _stream(stream)),
           "hs_sum_interleaved")


def hs_interleave(x, n_bins, n_spectra, elem_bytes, out, stream=None) -> None:
    _check(load().hs_interleave(_p(x), int(n_bins), int(n_spectra), int(elem_bytes), _p(out), _stream(stream)),
           "hs_interleave")


def hs_power_spectrum(fft, n_bins, interbin, scale, out, stream=None) -> None:
    _check(load().hs_power_spectrum(_p(fft), int(n_bins), int(interbin), float(scale), _p(out), _stream(stream)),
           "hs_power_spectrum")


def hs_cluster_peaks(snr, harm, drift, offsets, n_bins, n_spectra, radius, threshold, cand, cand_capacity,
                     cand_count, stream=None) -> None:
    _check(load().hs_cluster_peaks(_p(snr), _p(harm), _p(drift), _p(offsets), int(n_bins), int(n_spectra),
                                   int(radius), float(threshold), _p(cand), int(cand_capacity), _p(cand_count),
                                   _stream(stream)), "hs_cluster_peaks")


def hs_get_norm(plan, n, mu_sigma, tables=None, valid=None, stream=None):
    _check(load().hs_get_norm(plan, int(n), _p(mu_sigma), _p(tables), _p(valid), _stream(stream)),
           "hs_get_norm")


def hs_quantize_f16(x, n, scale, out, stream=None):
    _check(load().hs_quantize_f16(_p(x), int(n), float(scale), _p(out), _stream(stream)), "hs_quantize_f16")


def hs_plan_set_timing(plan, enable: bool) -> None:
    _check(load().hs_plan_set_timing(plan, 1 if enable else 0), "hs_plan_set_timing")


def hs_plan_get_timing(plan):
    """(calls, norm_ms, sum_ms) summed over the timed calls since the last read."""
    c, a, b = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
    _check(load().hs_plan_get_timing(plan, ctypes.byref(c), ctypes.byref(a), ctypes.byref(b)), "hs_plan_get_timing")
    return c.value, a.value, b.value


def hs_plan_set_graph(plan, enable: bool) -> None:
    _check(load().hs_plan_set_graph(plan, 1 if enable else 0), "hs_plan_set_graph")


def hs_plan_graph_info(plan):
    """(graphs recorded, replays) since the plan was created."""
    c, r = ctypes.c_int64(), ctypes.c_int64()
    _check(load().hs_plan_graph_info(plan, ctypes.byref(c), ctypes.byref(r)), "hs_plan_graph_info")
    return c.value, r.value


def hs_plan_set_launch(plan, fundamentals_per_lane: int, workgroups_per_cu: int) -> None:
    _check(load().hs_plan_set_launch(plan, int(fundamentals_per_lane), int(workgroups_per_cu)), "hs_plan_set_launch")


def hs_plan_get_launch(plan):
    """(fundamentals per lane, workgroups per CU) of the persistent kernel."""
    f, w = ctypes.c_int32(), ctypes.c_int32()
    _check(load().hs_plan_get_launch(plan, ctypes.byref(f), ctypes.byref(w)), "hs_plan_get_launch")
    return f.value, w.value


def hs_plan_tune_batched(plan, x, offsets, n_spectra, norm, snr, harm, drift, cand=None, cand_capacity=0,
                         cand_count=None, cache_path=None, stream=None):
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(load().hs_plan_tune_batched(plan, _p(x), _p(offsets), int(n_spectra), _p(norm), _p(snr), _p(harm),
                                       _p(drift), _p(cand), int(cand_capacity), _p(cand_count), path,
                                       _stream(stream)), "hs_plan_tune_batched")


def hs_status_string(status: int) -> str:
    return load().hs_status_string(status).decode()


def hs_last_error() -> str:
    return load().hs_last_error().decode()


class Plan:
    """Owns one ``hs_plan``; ``desc`` fields as keyword arguments."""

    def __init__(self, workspace=None, **desc):
        """``workspace``: None (the plan allocates its own) or a device buffer
        (a torch tensor of at least ``hs_plan_workspace_bytes`` bytes, 256-byte
        aligned) that the plan uses instead and that must outlive it."""
        self.desc = hs_plan_desc_init(**desc)
        if workspace is None:
            self.handle = hs_plan_create(self.desc)
        else:
            nbytes = workspace.numel() * workspace.element_size() if hasattr(workspace, "numel") else None
            if nbytes is None:
                raise TypeError("workspace must be a device tensor")
            self.handle = hs_plan_create_in(self.desc, workspace, nbytes)
        self.workspace = workspace

    def close(self):
        if self.handle:
            hs_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
