"""Build libpe.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpe.so")
SOURCES = ["api.hip", "gemm.hip", "kernels.hip", "cem.hip"]
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
         # no packed FP32 instructions in generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # matrix-core accumulators in ordinary vector registers: the
         # grouped FP32 product then needs 96 of them and, with 32 KB of LDS
         # per work-group, runs five work-groups per CU
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-Wall", "-Wno-unused-function"]
# the peak probes are compiled as a separate object
PROBE_SOURCE = "probe.hip"
PROBE_FLAGS = []


def _run(cmd, verbose):
    if verbose:
        print("[build]", " ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [line for line in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in line]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs), flush=True)


def build(verbose=True):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = OUT + ".tmp"
    obj = os.path.join(HERE, "probe.o")
    cflags = [f for f in FLAGS if f != "-shared"]
    _run([hipcc] + cflags + PROBE_FLAGS + ["-c", "-o", obj, os.path.join(CSRC, PROBE_SOURCE)], verbose)
    # "-x none": the object after the HIP sources is linked, not compiled
    _run([hipcc] + FLAGS + ["-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES] + ["-x", "none", obj], verbose)
    os.remove(obj)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
