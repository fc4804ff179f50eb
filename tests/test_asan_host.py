"""The host code of libofv under AddressSanitizer (and LeakSanitizer).

ofv_api.cpp (validation, planning, the backward's workspace layout, the
tuning-table parser) is rebuilt with the sanitizer on its host code only, linked
with the kernel objects of the regular build, and driven by tests/asan_driver.c
through every entry point on a validation-only handle (device -1: nothing is
launched, so no GPU is needed)."""
import os
import shutil
import subprocess

import pytest

from paper_2509_25924_amd import _build

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(_build.BUILD, "asan")
LLVM = "/opt/rocm/lib/llvm"


def _asan_runtime():
    base = os.path.join(LLVM, "lib", "clang")
    if not os.path.isdir(base):
        return None
    for v in sorted(os.listdir(base)):
        d = os.path.join(base, v, "lib", "linux")
        if os.path.exists(os.path.join(d, "libclang_rt.asan-x86_64.so")):
            return d
    return None


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.fixture(scope="module")
def driver():
    if _asan_runtime() is None or shutil.which(_build.hipcc()) is None and not os.path.exists(_build.hipcc()):
        pytest.skip("no ROCm clang with the AddressSanitizer runtime")
    if not _build.built():
        _build.build()
    os.makedirs(OUT, exist_ok=True)
    flags = [f for f in _build.COMMON_FLAGS if f != "-O3"]
    obj = os.path.join(OUT, "ofv_api.asan.o")
    # host code only: each sanitizer flag goes to the host pass
    _run([_build.hipcc(), "-c", os.path.join(_build.CSRC, "ofv_api.cpp"), "-o", obj, "-x", "hip", "-O1", "-g",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"] + flags)
    objs = [os.path.join(_build.BUILD, os.path.basename(s) + ".o") for s in _build.SOURCES if s != "ofv_api.cpp"]
    lib = os.path.join(OUT, "libofv_asan.so")
    _run([_build.hipcc(), "-shared", "-fPIC", f"--offload-arch={_build.ARCH}", "-o", lib, obj] + objs)
    exe = os.path.join(OUT, "asan_driver")
    _run([os.path.join(LLVM, "bin", "clang"), "-g", "-O1", "-Xarch_host", "-fsanitize=address",
          os.path.join(HERE, "asan_driver.c"), "-o", exe, f"-I{_build.INCLUDE}", lib, f"-Wl,-rpath,{OUT}"])
    return exe


def test_host_code_under_address_sanitizer(driver, tmp_path):
    supp = tmp_path / "lsan.supp"
    # allocations the ROCm runtime makes at load time and keeps for the process
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:librocprofiler\nleak:libamd_comgr\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               LSAN_OPTIONS=f"suppressions={supp}")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "all statuses as expected" in r.stdout
