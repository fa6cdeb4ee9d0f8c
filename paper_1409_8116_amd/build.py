"""Build libmpois.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc."""
import glob
import hashlib
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpois.so")
SOURCES = ["aux.hip", "proj.hip", "pl_inst.hip", "dispatch.cpp", "mpois.cpp", "tune.cpp"]
def _count(header, macro):
    import re
    with open(os.path.join(CSRC, header)) as fh:
        return int(re.search(r"#define\s+" + macro + r"\s+(\d+)", fh.read()).group(1))


# lp_inst.hip is compiled once per generic shape (cfgs.h), sp_inst.hip once per
# specialised kernel (specs.h)
NUM_SHAPES = _count("cfgs.h", "MPOIS_NUM_CFGS")
NUM_SPECS = _count("specs.h", "MPOIS_NUM_SPECS")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed FP32 instructions anywhere in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _inputs():
    return sorted(glob.glob(os.path.join(CSRC, "*")) + [os.path.join(ROOT, "include", "mpois.h")])


def build_id():
    """Hash of every source the library is built from (keys the tuner cache)."""
    h = hashlib.sha256()
    for f in _inputs():
        if os.path.isfile(f):
            with open(f, "rb") as fh:
                h.update(os.path.basename(f).encode() + fh.read())
    return h.hexdigest()[:12]


def build(verbose=False, jobs=None, incremental=False):
    """Compile every object and link libmpois.so.  incremental=True skips
    objects newer than every source (a developer convenience; the default
    rebuilds everything)."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    newest = max(os.path.getmtime(f) for f in _inputs() if os.path.isfile(f))
    bid = ["-DMPOIS_BUILD_ID=\"" + build_id() + "\""]
    cmds, objs = [], []
    for i in range(NUM_SHAPES):
        obj = os.path.join(objdir, f"lp_inst_{i}.o")
        objs.append(obj)
        if incremental and os.path.exists(obj) and os.path.getmtime(obj) > newest:
            continue
        cmds.append([HIPCC] + FLAGS + [f"-DMPOIS_CFG={i}", "-c", os.path.join(CSRC, "lp_inst.hip"), "-o", obj])
    for i in range(NUM_SPECS):
        obj = os.path.join(objdir, f"sp_inst_{i}.o")
        objs.append(obj)
        if incremental and os.path.exists(obj) and os.path.getmtime(obj) > newest:
            continue
        cmds.append([HIPCC] + FLAGS + [f"-DMPOIS_SPEC={i}", "-c", os.path.join(CSRC, "sp_inst.hip"), "-o", obj])
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        if incremental and src != "tune.cpp" and os.path.exists(obj) and os.path.getmtime(obj) > newest:
            continue
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmds.append([HIPCC] + FLAGS + bid + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
    running = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        while sum(p.poll() is None for p, _ in running) >= jobs:
            time.sleep(0.2)
        # the compiler's resource-usage remarks of every kernel go to a log next
        # to the object, checked below
        log = open(cmd[-1] + ".usage", "w")
        running.append((subprocess.Popen(cmd + ["-Rpass-analysis=kernel-resource-usage"], stderr=log), log))
    for p, log in running:
        rc = p.wait()
        log.close()
        if rc != 0:
            raise RuntimeError("hipcc failed: " + open(log.name).read()[-4000:])
    small, large = scratch_kernels(objs)
    if small and verbose:
        print("kernels with a few spilled registers: " + ", ".join(small), flush=True)
    if large:
        raise RuntimeError("kernels that keep data in scratch memory (a demoted array or struct, or heavy "
                           "register spills): " + ", ".join(large))
    tmp = LIB + ".tmp"
    # roctx (rocprofiler-sdk) for the MPOIS_TRACE ranges
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def scratch_kernels(objs, limit=64):
    """Kernels whose resource-usage remark reports scratch (private) memory:
    (those with at most `limit` bytes per lane, those with more).  The
    kernels keep their data in registers and LDS; a few spilled registers
    (the FP64 shapes held to 128 registers) cost little, but an array or
    struct demoted to scratch costs several times the kernel's time, so the
    build refuses that."""
    import re
    bad = []
    for obj in objs:
        path = obj + ".usage"
        if not os.path.exists(path):
            continue
        name = None
        for line in open(path):
            m = re.search(r"Function Name: (\S+)", line)
            if m:
                name = m.group(1)
            m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
            if m and int(m.group(1)) > 0 and name:
                bad.append((f"{name} ({m.group(1)} B/lane)", int(m.group(1))))
    return [b for b, v in bad if v <= limit], [b for b, v in bad if v > limit]


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv)
    print("built", LIB)
