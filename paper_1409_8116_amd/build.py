"""Build libmpois.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpois.so")
SOURCES = ["aux.hip", "dispatch.cpp", "mpois.cpp", "tune.cpp"]
NUM_SHAPES = 16  # entries of cfgs.h (MPOIS_NUM_CFGS); lp_inst.hip is compiled once per shape
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed FP32 instructions anywhere in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def build(verbose=False, jobs=None):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    cmds, objs = [], []
    for i in range(NUM_SHAPES):
        obj = os.path.join(objdir, f"lp_inst_{i}.o")
        cmds.append([HIPCC] + FLAGS + [f"-DMPOIS_CFG={i}", "-c", os.path.join(CSRC, "lp_inst.hip"), "-o", obj])
        objs.append(obj)
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmds.append([HIPCC] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    running = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        running.append(subprocess.Popen(cmd))
        while len([p for p in running if p.poll() is None]) >= jobs:
            running[0].wait() if running[0].poll() is None else None
            import time
            time.sleep(0.2)
    for p in running:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print("built", LIB)
