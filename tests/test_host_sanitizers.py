"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The plan layer (mpois.cpp), the kernel dispatch (dispatch.cpp) and the tuner
(tune.cpp) are rebuilt with the sanitizers on their host side only (the GPU
code of the kernels is the library's own, unchanged objects), linked with
tests/host/abi_driver.c, and run: every validation path, the axis tables and
plans over thousands of lengths with exactly sized output buffers, and the
NULL-argument paths.  Any out-of-bounds access, use after free, signed
overflow or misaligned access fails the test.  No GPU needed.
"""

import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1409_8116_amd")
CSRC = os.path.join(PKG, "csrc")
OBJS = os.path.join(PKG, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _kernel_objects():
    objs = sorted(glob.glob(os.path.join(OBJS, "lp_inst_*.o")) + glob.glob(os.path.join(OBJS, "sp_inst_*.o")))
    for name in ("pl_inst.hip.o", "aux.hip.o", "proj.hip.o"):
        objs.append(os.path.join(OBJS, name))
    return objs


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    kobjs = _kernel_objects()
    if not all(os.path.exists(o) for o in kobjs):
        pytest.skip("library objects not built (run the build first)")
    procs, objs = [], []
    for src in ("mpois.cpp", "dispatch.cpp", "tune.cpp"):
        obj = str(tmp_path / (src + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC] + FLAGS + HOST_SAN + ["-x", "hip", "-c", os.path.join(CSRC, src),
                                                                    "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    drv = str(tmp_path / "abi_driver.o")
    procs.append(subprocess.Popen([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                                   "-I" + os.path.join(ROOT, "include"), "-c",
                                   os.path.join(ROOT, "tests", "host", "abi_driver.c"), "-o", drv],
                                  stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out.decode()[-3000:]
    exe = str(tmp_path / "abi_driver")
    link = [HIPCC, "--offload-arch=gfx950", "-fsanitize=address,undefined", "-fno-gpu-sanitize", "-o", exe, drv] + \
        objs + kobjs + ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-lm"]
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, timeout=600)
    assert r.returncode == 0, r.stdout.decode()[-3000:]
    env = dict(os.environ)
    # the HIP runtime keeps process-lifetime allocations: leaks are not checked
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, env=env, timeout=600)
    text = r.stdout.decode()
    assert r.returncode == 0 and "ok" in text.split(), text[-4000:]
    assert "runtime error" not in text and "AddressSanitizer" not in text, text[-4000:]
    shutil.rmtree(tmp_path, ignore_errors=True)
