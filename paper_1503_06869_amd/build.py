"""Build the gfx950 shared library paper_1503_06869_amd/liblbmfib.so with hipcc.

    python -m paper_1503_06869_amd.build        (or build() from Python)

Every HIP translation unit is compiled with packed-FP32 instructions
disabled; the particle and host units also with contraction off, so that
the FP64 cell predicate and quaternion arithmetic round exactly as written
(the batched unit gets the same through a pragma after its sweep code).
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbmfib.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")

SOURCES = {
    "sweep.hip": [],
    # boundary update with the default contraction of the sweep (the integer
    # link sums of the second half do no floating-point arithmetic)
    "boundary.hip": [],
    "particles.hip": ["-ffp-contract=off"],
    "api.hip": ["-ffp-contract=off"],
    # the sweep part keeps the default contraction of sweep.hip; the particle
    # part and the host code follow a contraction-off pragma in the header
    "batched.hip": [],
    "stab.hip": [],
    "check.hip": [],
    "features.hip": [],
    "mlp.hip": [],
    "sbf.hip": [],
}
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-result", "-I" + os.path.join(HERE, "..", "include")]


def _compile(src, extra, verbose):
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-6000:]))
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda kv: _compile(kv[0], kv[1], verbose), SOURCES.items()))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
