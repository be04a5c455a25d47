"""Build the in-tree HIP library paper_2309_14085_amd/libh2s.so for gfx950.

Host C++ (tree, lists, ACA/NCA, operators, the C ABI) is compiled with g++ and
OpenMP; the MVP kernels with hipcc for gfx950.  Every call rebuilds.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libh2s.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = os.environ.get("H2S_OFFLOAD_ARCH", "gfx950")

HOST_SRC = ["h2s_host_build.cpp", "h2s_api.cpp", "h2s_solve.cpp"]
HIP_SRC = ["h2s_kernels.hip", "h2s_kernels_batch.hip", "h2s_blas.hip", "h2s_eval_rate.hip"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    procs, objs = [], []
    for src in HOST_SRC:
        obj = os.path.join(BUILD, src + ".o")
        cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include")] + inc + \
              ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for src in HIP_SRC:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [os.path.join(ROCM, "bin", "hipcc"), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"] + inc + \
              ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for cmd, p in procs:
        if verbose:
            print(" ".join(cmd), flush=True)
        if p.wait() != 0:
            raise RuntimeError("compile failed: " + " ".join(cmd))
    _run(["g++", "-shared", "-fPIC", "-fopenmp", "-o", LIB + ".tmp"] + objs +
         ["-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")], verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
