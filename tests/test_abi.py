"""The C-ABI libraries load and export every entry point their headers
declare: libhs.so for include/hs.h, libhs_probe.so (the gather-ceiling probe
of the benchmark) for include/hs_probe.h.

No compute call is made here (no GPU in this environment): only symbol
presence and the argument checks that return before any HIP call.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2202_12817_amd import hs
    return hs.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hs_plan_create", "hs_sum_1d", "hs_sum_2d", "hs_sum_batched"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2202_12817_amd import hs
    names = declared_functions()
    assert set(names) == set(hs.EXPORTED)
    for name in names:
        assert hasattr(lib, name), name


def test_probe_library_exports_its_header():
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "hs_probe.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(hsp_[a-z0-9_]+)\s*\(", text)))
    assert names == ["hsp_gather"]
    probe = ctypes.CDLL(os.path.join(ROOT, "paper_2202_12817_amd", "libhs_probe.so"))
    for name in names:
        assert hasattr(probe, name), name
    f = probe.hsp_gather
    f.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    # argument checks return before any HIP call: null pointers, a set that is no power of two or too large
    assert f(None, 1023, 64, 1, None, None) != 0
    assert f(8, 1000, 64, 1, 8, None) != 0
    assert f(8, (1 << 28), 64, 1, 8, None) != 0
    assert f(8, 1023, 0, 1, 8, None) != 0


def test_static_entry_rejects_on_the_host(lib):
    from paper_2202_12817_amd import hs
    d = hs.hs_plan_desc_init()
    for n in (0, 1025):
        with pytest.raises(hs.HsError) as e:
            hs.hs_sum_batched_static(d, 16, 16, n, None, 16, 16, None, None, 0, None, stream=0)
        assert e.value.status == hs.HS_ERR_ARG
    with pytest.raises(hs.HsError) as e:
        hs.hs_sum_batched_static(hs.hs_plan_desc_init(harmonics=65), 16, 16, 1, None, 16, 16, None, None, 0, None,
                                 stream=0)
    assert e.value.status == hs.HS_ERR_UNSUPPORTED
    with pytest.raises(hs.HsError) as e:
        hs.hs_sum_batched_static(d, 16, 16, 1, None, None, None, None, None, 0, None, stream=0)
    assert e.value.status == hs.HS_ERR_ARG


def test_struct_layouts_match_header():
    from paper_2202_12817_amd import hs
    assert ctypes.sizeof(hs.HsCandidate) == 16
    assert ctypes.sizeof(hs.HsPlanDesc) == 56


def test_desc_defaults(lib):
    from paper_2202_12817_amd import hs
    d = hs.hs_plan_desc_init()
    assert (d.harmonics, d.mode, d.dtype, d.first_bin) == (32, hs.HS_GREEDY, hs.HS_F32, 1)
    assert d.harmonic_mask == 0 and d.report_mask == 0 and d.fundamental_end == 0
    assert d.max_spectra == 1024 and d.threshold == pytest.approx(6.0) and d.kernel == hs.HS_KERNEL_AUTO
    assert d.norm_kind == hs.HS_NORM_MU_SIGMA


def test_harmonic_limits(lib):
    # H = 1..64 for the simple and greedy sums; the PRESTO-style sums stop at 32
    from paper_2202_12817_amd import hs
    n = ctypes.c_size_t()
    for mode in (hs.HS_STANDARD, hs.HS_GREEDY):
        for H in (1, 32, 33, 48, 64):
            d = hs.hs_plan_desc_init(mode=mode, harmonics=H, harmonic_mask=1 << (H - 1), report_mask=1 << (H - 1))
            assert lib.hs_plan_workspace_bytes(ctypes.byref(d), ctypes.byref(n)) == hs.HS_OK, (mode, H)
            d = hs.hs_plan_desc_init(mode=mode, harmonics=H, norm_kind=hs.HS_NORM_TABLE)
            assert lib.hs_plan_workspace_bytes(ctypes.byref(d), ctypes.byref(n)) == hs.HS_OK, (mode, H)
        d = hs.hs_plan_desc_init(mode=mode, harmonics=65)
        assert lib.hs_plan_workspace_bytes(ctypes.byref(d), ctypes.byref(n)) == hs.HS_ERR_UNSUPPORTED
    for mode in (hs.HS_PRESTO, hs.HS_PRESTO_ALL, hs.HS_PRESTO_PLUS):
        d = hs.hs_plan_desc_init(mode=mode, harmonics=32)
        assert lib.hs_plan_workspace_bytes(ctypes.byref(d), ctypes.byref(n)) == hs.HS_OK
        d = hs.hs_plan_desc_init(mode=mode, harmonics=33)
        assert lib.hs_plan_workspace_bytes(ctypes.byref(d), ctypes.byref(n)) == hs.HS_ERR_UNSUPPORTED
    assert lib.hs_status_string(hs.HS_ERR_INTERNAL) == b"internal error"


@pytest.mark.parametrize("field,value,status", [
    ("harmonics", 0, 1), ("harmonics", 65, 2), ("mode", 7, 1), ("dtype", 5, 1), ("first_bin", 0, 1),
    ("max_spectra", 0, 1), ("max_spectra", 70000, 1), ("fundamental_end", -1, 1), ("kernel", 3, 1),
    ("norm_kind", 2, 1), ("norm_kind", -1, 1),
])
def test_plan_create_rejects_bad_desc(lib, field, value, status):
    from paper_2202_12817_amd import hs
    d = hs.hs_plan_desc_init(**{field: value})
    h = ctypes.c_void_p()
    assert lib.hs_plan_create(ctypes.byref(d), ctypes.byref(h)) == status
    assert h.value is None
    assert lib.hs_last_error()


def test_presto_modes_validation(lib):
    # the PRESTO-style modes accept the plain kernel only and report no partial sums
    from paper_2202_12817_amd import hs
    n = ctypes.c_size_t()
    for mode in (hs.HS_PRESTO, hs.HS_PRESTO_ALL, hs.HS_PRESTO_PLUS):
        for kernel in (hs.HS_KERNEL_AUTO, hs.HS_KERNEL_PLAIN):
            d = hs.hs_plan_desc_init(mode=mode, kernel=kernel)
            assert lib.hs_plan_workspace_bytes(ctypes.byref(d), ctypes.byref(n)) == hs.HS_OK
        d = hs.hs_plan_desc_init(mode=mode, kernel=hs.HS_KERNEL_PERSISTENT)
        assert lib.hs_plan_workspace_bytes(ctypes.byref(d), ctypes.byref(n)) == hs.HS_ERR_UNSUPPORTED
        d = hs.hs_plan_desc_init(mode=mode, report_mask=1)
        assert lib.hs_plan_workspace_bytes(ctypes.byref(d), ctypes.byref(n)) == hs.HS_ERR_UNSUPPORTED
    d = hs.hs_plan_desc_init(mode=5)
    assert lib.hs_plan_workspace_bytes(ctypes.byref(d), ctypes.byref(n)) == hs.HS_ERR_ARG


def test_interleave_argument_checks_on_host(lib):
    # argument checks of the transpose run before anything is enqueued
    from paper_2202_12817_amd import hs
    buf = ctypes.create_string_buffer(64)
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert lib.hs_interleave(None, 4, 4, 4, p, None) == hs.HS_ERR_ARG
    assert lib.hs_interleave(p, 4, 4, 3, p, None) == hs.HS_ERR_ARG
    assert lib.hs_interleave(p, 4, 4, 4, p, None) == hs.HS_ERR_ARG          # overlap
    assert lib.hs_interleave(p, 0, 4, 4, p, None) == hs.HS_ERR_ARG


def test_pipeline_argument_checks_on_host(lib):
    # argument checks of the pipeline calls run before anything is enqueued
    from paper_2202_12817_amd import hs
    buf = ctypes.create_string_buffer(256)
    p = ctypes.cast(buf, ctypes.c_void_p)
    q = ctypes.c_void_p(p.value + 1)
    assert lib.hs_power_spectrum(None, 4, 0, 1.0, p, None) == hs.HS_ERR_ARG
    assert lib.hs_power_spectrum(p, 4, 1, 1.0, p, None) == hs.HS_ERR_ARG        # overlap
    assert lib.hs_power_spectrum(q, 4, 0, 1.0, p, None) == hs.HS_ERR_ARG        # misaligned
    assert lib.hs_power_spectrum(p, 0, 0, 1.0, p, None) == hs.HS_ERR_ARG
    assert lib.hs_power_spectrum(p, 4, 0, -1.0, p, None) == hs.HS_ERR_ARG
    assert lib.hs_cluster_peaks(None, p, None, None, 4, 1, 1, 1.0, p, 1, p, None) == hs.HS_ERR_ARG
    assert lib.hs_cluster_peaks(p, p, None, None, 4, 1, -1, 1.0, p, 1, p, None) == hs.HS_ERR_ARG
    assert lib.hs_cluster_peaks(p, p, None, None, 4, 2, 1, 1.0, p, 1, p, None) == hs.HS_ERR_ARG
    assert lib.hs_cluster_peaks(p, p, None, p, 4, 0, 1, 1.0, p, 1, p, None) == hs.HS_ERR_ARG


def test_masks_must_fit_h(lib):
    from paper_2202_12817_amd import hs
    h = ctypes.c_void_p()
    d = hs.hs_plan_desc_init(harmonics=4, report_mask=1 << 5)
    assert lib.hs_plan_create(ctypes.byref(d), ctypes.byref(h)) == hs.HS_ERR_ARG
    d = hs.hs_plan_desc_init(harmonics=4, harmonic_mask=1 << 10)
    assert lib.hs_plan_create(ctypes.byref(d), ctypes.byref(h)) == hs.HS_ERR_ARG


def test_null_plan_and_pointers_rejected(lib):
    from paper_2202_12817_amd import hs
    assert lib.hs_sum_1d(None, 16, 100, None, 16, 16, None, None, None) == hs.HS_ERR_ARG
    assert lib.hs_sum_batched(None, 16, 16, 1, None, 16, 16, None, None, 0, None, None) == hs.HS_ERR_ARG
    assert lib.hs_sum_2d(None, 16, 10, 10, 0, 0, None, 16, 16, None, None, 0, None, None) == hs.HS_ERR_ARG
    assert lib.hs_get_norm(None, 1, 16, None, None, None) == hs.HS_ERR_ARG
    assert lib.hs_plan_destroy(None) == hs.HS_ERR_ARG
    assert lib.hs_plan_create(None, None) == hs.HS_ERR_ARG


def test_workspace_bytes_and_caller_workspace_checks(lib):
    from paper_2202_12817_amd import hs
    sizes = []
    for b in (1, 64, 1024, 65535):
        n = hs.hs_plan_workspace_bytes(hs.hs_plan_desc_init(max_spectra=b))
        assert n % 256 == 0 and n > 0
        sizes.append(n)
    assert sizes == sorted(sizes) and sizes[-1] > sizes[0]
    bad = hs.hs_plan_desc_init(harmonics=65)
    n = ctypes.c_size_t()
    assert lib.hs_plan_workspace_bytes(ctypes.byref(bad), ctypes.byref(n)) == hs.HS_ERR_UNSUPPORTED
    assert lib.hs_plan_workspace_bytes(None, ctypes.byref(n)) == hs.HS_ERR_ARG
    d = hs.hs_plan_desc_init()
    need = hs.hs_plan_workspace_bytes(d)
    h = ctypes.c_void_p()
    # rejected before any device work: NULL, misaligned or too small buffers
    assert lib.hs_plan_create_in(ctypes.byref(d), None, need, ctypes.byref(h)) == hs.HS_ERR_ARG
    assert lib.hs_plan_create_in(ctypes.byref(d), 4096 + 16, need, ctypes.byref(h)) == hs.HS_ERR_ARG
    assert lib.hs_plan_create_in(ctypes.byref(d), 4096, need - 256, ctypes.byref(h)) == hs.HS_ERR_ARG
    assert h.value is None


def test_quantize_argument_checks(lib):
    from paper_2202_12817_amd import hs
    assert lib.hs_quantize_f16(16, 10, ctypes.c_float(0.0), 16, None) == hs.HS_ERR_ARG
    assert lib.hs_quantize_f16(16, 10, ctypes.c_float(float("inf")), 16, None) == hs.HS_ERR_ARG
    assert lib.hs_quantize_f16(None, 10, ctypes.c_float(1.0), 16, None) == hs.HS_ERR_ARG
    assert lib.hs_quantize_f16(16, -1, ctypes.c_float(1.0), 16, None) == hs.HS_ERR_ARG
    assert lib.hs_quantize_f16(16, 0, ctypes.c_float(1.0), 16, None) == hs.HS_OK


def test_status_strings(lib):
    from paper_2202_12817_amd import hs
    for s in range(5):
        assert hs.hs_status_string(s)
    assert hs.hs_status_string(99) == "unknown status"


def test_missing_library_fails_loudly(tmp_path):
    from paper_2202_12817_amd import hs
    saved = hs._lib
    try:
        hs._lib = None
        with pytest.raises(RuntimeError, match="not built"):
            hs.load(str(tmp_path / "absent.so"))
    finally:
        hs._lib = saved


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2202_12817_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "hs_oracle" not in text, f


def test_header_is_c_and_links(lib, tmp_path):
    """include/hs.h compiles as C99 and a C program links against libhs.so and
    calls the host-only entry points (no GPU needed)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = os.path.join(ROOT, "tests", "c_abi_check.c")
    exe = str(tmp_path / "c_abi_check")
    libdir = os.path.join(ROOT, "paper_2202_12817_amd")
    cmd = [gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"), src, "-o", exe,
           "-L", libdir, "-lhs", "-Wl,-rpath," + libdir]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "19 entry points" in r.stdout
