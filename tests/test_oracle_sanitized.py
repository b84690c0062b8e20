"""The oracle's C code under gcc's AddressSanitizer and UndefinedBehaviorSanitizer: a sanitized copy of
``oracle/wt_oracle.c`` is built into a temporary folder and the oracle pins run against it in a child process
(the sanitizer runtimes preloaded, leak checking off since the interpreter keeps its allocations), so an
out-of-bounds access or undefined operation anywhere the pins reach fails this test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    try:
        p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(shutil.which("gcc") is None or _runtime("libasan.so") is None or _runtime("libubsan.so") is None,
                    reason="gcc with the sanitizer runtimes is not available")
def test_oracle_pins_under_sanitizers(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", str(lib),
                           os.path.join(ROOT, "oracle", "wt_oracle.c"), "-lm"])
    runner = ("import sys; sys.path.insert(0, %r); import oracle; oracle._LIB = %r; import pytest; "
              "sys.exit(pytest.main(['-q', '-s', '-x', '-p', 'no:cacheprovider', '-m', 'not gpu', %r]))"
              % (ROOT, str(lib), os.path.join(ROOT, "tests", "test_oracle_pins.py")))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               LD_PRELOAD=" ".join([_runtime("libasan.so"), _runtime("libubsan.so")]))
    res = subprocess.run([sys.executable, "-c", runner], cwd=str(tmp_path), env=env, capture_output=True, text=True,
                         timeout=900)
    assert res.returncode == 0, (res.stdout[-3000:], res.stderr[-3000:])
    assert " passed" in res.stdout
