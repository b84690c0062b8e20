"""The library's host code (argument validation, frame geometry, workspace layout) under clang's AddressSanitizer
and UndefinedBehaviorSanitizer: a copy of libwt is built into a temporary folder with the sanitizers on its host
half only (the device code is compiled as usual and never launched here), and the C ABI tests run against it in a
child process with the sanitizer runtime preloaded. No GPU is needed: every call in those tests stops at
validation or sizing."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"


def _asan_runtime():
    try:
        p = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True,
                           check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(not os.path.exists(HIPCC) or _asan_runtime() is None, reason="hipcc or clang's ASan runtime missing")
def test_abi_under_host_sanitizers(tmp_path):
    lib = tmp_path / "libwt_san.so"
    sources = sorted(glob.glob(os.path.join(ROOT, "paper_2201_00094_amd", "csrc", "*.hip")))
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san, "-shared-libsan",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2201_00094_amd", "csrc"), "-o", str(lib), *sources],
                          stderr=subprocess.DEVNULL)
    runner = ("import sys; sys.path.insert(0, %r); import paper_2201_00094_amd._lib as L; L.LIB_PATH = %r; "
              "import pytest; sys.exit(pytest.main(['-q', '-s', '-x', '-p', 'no:cacheprovider', %r, '-k', "
              "'not missing_library']))" % (ROOT, str(lib), os.path.join(ROOT, "tests", "test_abi.py")))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               LD_PRELOAD=_asan_runtime())
    res = subprocess.run([sys.executable, "-c", runner], cwd=str(tmp_path), env=env, capture_output=True, text=True,
                         timeout=600)
    assert res.returncode == 0, (res.stdout[-3000:], res.stderr[-3000:])
    assert " passed" in res.stdout
