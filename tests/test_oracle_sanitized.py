"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer:
amr_oracle.c is built with both (gcc, every UB check fatal) and the CPU pin
tests run in a child process that loads that build through ORACLE_LIB with
the ASan runtime preloaded.  Any out-of-bounds access, use after free,
signed overflow, bad shift or misaligned load in the oracle ends the child
with a report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "amr_oracle.c")


def _runtime(name):
    r = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liborc_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-o", lib, SRC, "-lm"], check=True)
    env = dict(os.environ)
    env.update({"ORACLE_LIB": lib, "LD_PRELOAD": asan,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=99",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1:exitcode=98"})
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout[-3000:] + r.stderr[-6000:]
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, out
