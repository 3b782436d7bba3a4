"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
the sources that hold the ABI's validation, workspace plans and batched plan
(abi.hip), the tuning table and its JSON reader (tune.hip) and the launch probes
(runtime.hip) are compiled with host-side sanitizers (device code is built as
usual), linked with the library's other objects and the driver
tests/abi_sanitize_driver.c, and run without a GPU: every call the driver makes
is host-only (sizes, plans, rejected arguments, the tuning table, including
malformed table files).  Out-of-bounds accesses, leaks, use after free or
undefined arithmetic there fail this test."""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1504_06443_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
SANITIZED = ["abi.hip", "tune.hip", "runtime.hip"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


def _objects():
    from paper_1504_06443_amd import build
    objs = sorted(glob.glob(os.path.join(build.OBJ, "*.o")))
    names = {os.path.basename(o) for o in objs}
    if not all(s.replace(".hip", ".o") in names for s in build.SOURCES):
        build.build()
        objs = sorted(glob.glob(os.path.join(build.OBJ, "*.o")))
    return objs


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs ROCm clang")
def test_abi_host_code_under_sanitizers(tmp_path):
    plain = [o for o in _objects() if os.path.basename(o).replace(".o", ".hip") not in SANITIZED]

    def compile_one(src):
        obj = str(tmp_path / src.replace(".hip", ".o"))
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN,
               "-c", os.path.join(PKG, "csrc", src), "-o", obj]
        subprocess.run(cmd, check=True, capture_output=True)
        return obj

    with ThreadPoolExecutor(len(SANITIZED)) as ex:
        san = list(ex.map(compile_one, SANITIZED))
    drv = str(tmp_path / "driver.o")
    subprocess.check_call([CLANG, "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-c",
                           os.path.join(ROOT, "tests", "abi_sanitize_driver.c"), "-o", drv])
    exe = str(tmp_path / "abi_san")
    subprocess.check_call([CLANG + "++", "-fsanitize=address,undefined", drv, *san, *plain,
                           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-lm",
                           "-o", exe])
    scratch = tmp_path / "scratch"
    scratch.mkdir()
    # verify_asan_link_order=0: the run environment may preload libraries of its own
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("GEP_TUNE_FILE", None)
    r = subprocess.run([exe, os.path.join(PKG, "tuning.json"), str(scratch)], capture_output=True,
                       text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert "sanitized abi run ok" in r.stdout
