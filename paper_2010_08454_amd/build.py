"""Build step of libppl: compiles the HIP sources for gfx950 into libppl.so (in-tree),
and the rate micro-benchmarks (csrc/peaks/) into libppl_peaks.so.

Run as ``python paper_2010_08454_amd/build.py`` (by path: importing the package
loads the library it builds).  Packed-FP32 instructions are disabled
(-packed-fp32-ops) for every HIP translation unit.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libppl.so")
PEAKS_OUT = os.path.join(HERE, "libppl_peaks.so")

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-command-line-argument"]
OBJ_DIR = os.path.join(HERE, "_build")
NOISE = "packed-fp32-ops"   # the host pass does not know the device feature: harmless


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if NOISE not in ln and ln.strip()]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))


def _hipcc(srcs, out, verbose):
    """Each translation unit is compiled to an object on its own (in parallel;
    every unit carries its own device code, no relocatable device code), then
    the objects are linked into the shared library."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    stem = os.path.splitext(os.path.basename(out))[0]
    objs = [os.path.join(OBJ_DIR, stem + "_" + os.path.splitext(os.path.basename(s))[0] + ".o") for s in srcs]
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 16))
    with ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda so: _run([hipcc] + HIPCC_FLAGS + ["-c", "-o", so[1], so[0]], verbose), zip(srcs, objs)))
    tmp = out + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, out)
    return out


def build(verbose=False):
    _hipcc(sorted(glob.glob(os.path.join(HERE, "csrc", "peaks", "*.hip"))), PEAKS_OUT, verbose)
    return _hipcc(sources(), OUT, verbose)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
