"""Build the HIP libraries in-tree for gfx950 with hipcc: ``libhs.so`` (the
harmonic sum) and ``libhs_probe.so`` (the gather-ceiling probe, a
measurement aid).  Sources compile in parallel into ``_build/`` and are then
linked."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhs.so")
PROBE_LIB = os.path.join(HERE, "libhs_probe.so")
SOURCES = ["hs_api.hip", "hs_stats.hip", "hs_sum.hip", "hs_sum_xcd.hip", "hs_sum_2d_ray.hip", "hs_presto.hip",
           "hs_interleaved.hip", "hs_pipeline.hip"]
PROBE_SOURCES = ["hs_probe.hip"]

# -ffp-contract=off: every float operation is the single rounding written in
# the source (the SNR's fma is explicit).  Packed FP32 instructions are
# disabled on the device.  -Wno-pass-failed: an unroll request the compiler
# declines (large harmonic buckets) leaves a correct loop.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-pass-failed"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + out)
    return out


def _compile(src):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    tmp = obj + ".tmp%d" % os.getpid()
    out = _run(["hipcc"] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", "-o", tmp,
                                   os.path.join(CSRC, src)])
    os.replace(tmp, obj)
    return obj, out


def _link(objs, lib):
    tmp = lib + ".tmp%d" % os.getpid()
    out = _run(["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs)
    os.replace(tmp, lib)
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = max(1, min(8, os.cpu_count() or 1))
    with ThreadPoolExecutor(jobs) as ex:
        res = list(ex.map(_compile, SOURCES + PROBE_SOURCES))
    objs = [o for o, _ in res]
    outs = [t for _, t in res]
    outs.append(_link(objs[:len(SOURCES)], LIB))
    outs.append(_link(objs[len(SOURCES):], PROBE_LIB))
    if verbose:
        for t in outs:
            if t.strip():
                print(t)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
