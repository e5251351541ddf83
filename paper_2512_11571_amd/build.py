"""Builds libcemtamp.so (the HIP library behind include/cemtamp.h) in-tree, for gfx950.

    python -m paper_2512_11571_amd.build

Every call recompiles.  Translation units whose results must be bit-exact
(sampling, select/refit) are compiled with -ffp-contract=off; packed FP32
instructions are disabled for all device code.
"""
import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libcemtamp.so")
ARCH = os.environ.get("CEM_OFFLOAD_ARCH", "gfx950")

SOURCES = {
    "api.hip": [],
    "sampler.hip": ["-ffp-contract=off"],
    "select_refit.hip": ["-ffp-contract=off"],
    # no sinking of common code out of branches: merging the two in-register
    # accumulations of the articulated-body pass into one store through a
    # selected pointer would move those values to scratch memory
    "rollout.hip": ["-mllvm", "-simplifycfg-sink-common=false"],
    "mlp.hip": [],
    "peak.hip": [],
}

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c


def _compile(name):
    src = os.path.join(CSRC, name)
    obj = os.path.join(BUILD, name + ".o")
    cmd = [_hipcc(), "-c", src, "-o", obj] + COMMON + SOURCES[name]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (name, " ".join(cmd), r.stderr))
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, sorted(SOURCES)))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
