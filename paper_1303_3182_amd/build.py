"""Builds libtqr.so (HIP kernels for gfx950 + host C++ scheduling layer)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libtqr.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + CSRC, "-I" + INCLUDE, "-I/opt/rocm/include", "-Wall", "-Wno-unused-result"]
# Device code: never emit packed FP32 instructions (some of their forms have
# given silently wrong results on this hardware).
# MFMA accumulators in VGPRs: avoids AGPR<->VGPR copies around guarded MFMA blocks.
# No implicit FMA contraction: every fused multiply-add is written out, so two
# inlined copies of a tile kernel round identically, and the compensated sums
# of the refinement stay exact.
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=off", "-mllvm", "-amdgpu-mfma-vgpr-form"]
HOST_SOURCES = ["graph.cpp", "api.cpp", "configs.cpp"]
DEVICE_SOURCES = ["kernels.hip"]
SHARED_DEVICE_SOURCES = ["refine.hip", "gmres.hip", "mlp.hip", "noalloc.hip", "cholinv.hip", "zqr.hip"]  # compiled once
# (nb, ib) tile configurations; kernels.hip is compiled once per entry
# (the list must match TQR_CONFIGS in configs.cpp).
CONFIGS = [(32, 16), (64, 16), (64, 32), (128, 32), (256, 32)]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r


def build(verbose=False, jobs=8):
    """Compile every source and link libtqr.so in the package directory."""
    os.makedirs(BUILD, exist_ok=True)
    procs, objs = [], []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        procs.append([HIPCC, "-x", "c++", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON +
                     ["-D__HIP_PLATFORM_AMD__"])
    for src in DEVICE_SOURCES:
        for nb, ib in CONFIGS:
            obj = os.path.join(BUILD, "%s.%d_%d.o" % (src, nb, ib))
            objs.append(obj)
            procs.append([HIPCC, "-c", os.path.join(CSRC, src), "-o", obj, "-DTQR_CFG_NB=%d" % nb,
                          "-DTQR_CFG_IB=%d" % ib] + COMMON + DEVICE)
    for src in SHARED_DEVICE_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        procs.append([HIPCC, "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + DEVICE)
    running = []
    for cmd in procs:
        if verbose:
            print(" ".join(cmd))
        running.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        if len(running) >= jobs:
            _wait(running.pop(0))
    for item in running:
        _wait(item)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", "-o", tmp] + objs + ["--offload-arch=" + ARCH, "-L/opt/rocm/lib", "-lamdhip64"])
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    cmd, p = item
    out, err = p.communicate()
    if p.returncode != 0:
        sys.stderr.write(out + err)
        raise RuntimeError("build failed: " + " ".join(cmd))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
