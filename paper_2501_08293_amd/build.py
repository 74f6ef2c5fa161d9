"""Builds the HIP library in-tree for gfx950:
    python -m paper_2501_08293_amd.build
produces paper_2501_08293_amd/libopf_admm.so (host C++ set-up, HIP kernels,
C-ABI of include/opf_admm.h)."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libopf_admm.so")
SOURCES = ["setup.cpp", "tune_cache.cpp", "metrics.cpp", "setup_device.hip", "admm_step.hip", "admm_persistent.hip", "admm_tiled.hip", "admm_batch.hip", "admm_multi.hip", "api.hip", "api_batch.hip",
           "api_server.hip"]
ARCH = os.environ.get("OPF_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_flags() -> list:
    """hipcc flags of every translation unit (device code for ARCH only)."""
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include")]


def device_assembly(src: str, out: str) -> str:
    """gfx950 assembly of one HIP source of csrc/ (with the compiler's
    per-kernel resource comments: registers, occupancy, scratch)."""
    cmd = [hipcc()] + compile_flags() + ["-x", "hip", "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
    subprocess.run(cmd, check=True, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return out


def build(verbose: bool = False) -> str:
    objs = []
    common = compile_flags()
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(bdir, src + ".o")
        cmd = [hipcc()] + common + (["-x", "hip"] if src.endswith(".hip") else []) + \
            ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp] + objs + \
        ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
