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

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-command-line-argument"]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _hipcc(srcs, out, verbose):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + ["-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"   # the host pass does not know the device feature: harmless
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if noise not in ln and ln.strip()]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, out)
    return out


def build(verbose=False):
    _hipcc(sorted(glob.glob(os.path.join(HERE, "csrc", "peaks", "*.hip"))), PEAKS_OUT, verbose)
    return _hipcc(sources(), OUT, verbose)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
