"""Build libfp.so (HIP kernels for gfx950 + C ABI + host enumerator) in-tree."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfp.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-Wall"]
# packed FP32 instructions stay disabled in all device code
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    enum_o = os.path.join(OUT_DIR, "fp_enum.o")
    lib_o = os.path.join(OUT_DIR, "fp_lib.o")
    _run([HIPCC, *COMMON, "-ffp-contract=off", "-pthread", "-c", os.path.join(CSRC, "fp_enum.cpp"), "-o", enum_o],
         verbose)
    _run([HIPCC, *COMMON, *DEVICE, "-c", os.path.join(CSRC, "fp_lib.hip"), "-o", lib_o], verbose)
    _run([HIPCC, "-shared", "--offload-arch=gfx950", "-pthread", "-o", LIB + ".tmp", lib_o, enum_o], verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
