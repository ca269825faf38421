"""Build the HIP library libhfe.so for gfx950 in-tree.

Every .hip / .cpp source under csrc/ is compiled with hipcc for gfx950, except the
quad-precision Gaussian table (hfe_cdt.cpp), which is plain host C++ built with g++
against libquadmath.  Objects go to _build/ at the repository root; the shared library is
written next to this file.

The same call builds the tests' host harness of the exact-arithmetic helpers
(tests/native/libhfe_exact_check.so from tests/native/exact_check.cpp, host code only), which
the CPU tests load to check those helpers against exact integers.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhfe.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")]
HIP_SOURCES = ["k_ntt.hip", "k_ntt_big.hip", "k_misc.hip", "k_gemm.hip", "k_batch.hip", "k_rns.hip", "k_p2.hip", "k_chain.hip", "k_fswitch.hip", "k_fold.hip", "k_probe.hip", "hfe_noalloc.hip", "hfe_api.cpp", "hfe_host.cpp", "hfe_server.cpp",
               "hfe_store.cpp", "hfe_fswitch.cpp", "hfe_fold.cpp"]
GXX_SOURCES = ["hfe_cdt.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + out)
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        lang = [] if src.endswith(".hip") else ["-x", "hip"] if src.startswith("k_") else []
        jobs.append(([HIPCC] + HIP_FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj], obj))
    for src in GXX_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((["g++", "-O2", "-fPIC", "-std=c++17", "-c", os.path.join(CSRC, src), "-o", obj], obj))
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(lambda j: _run(j[0]), jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + [o for _, o in jobs] + ["-lquadmath"])
    os.replace(tmp, OUT)
    build_exact_check()
    return OUT


CHECK_SRC = os.path.join(ROOT, "tests", "native", "exact_check.cpp")
CHECK_OUT = os.path.join(ROOT, "tests", "native", "libhfe_exact_check.so")


def build_exact_check() -> str:
    """Host build of the exact-arithmetic helpers for the CPU tests."""
    tmp = CHECK_OUT + ".tmp"
    _run([HIPCC] + HIP_FLAGS + ["-x", "hip", "-shared", CHECK_SRC, "-o", tmp])
    os.replace(tmp, CHECK_OUT)
    return CHECK_OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
