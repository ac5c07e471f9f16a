"""The CPU oracle built with AddressSanitizer + UndefinedBehaviorSanitizer and
with ThreadSanitizer (gcc, host code only), driven by oracle/sanitize_main.c
over every entry point, single- and multi-threaded."""
import pathlib
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
GCC = shutil.which("gcc")


@pytest.mark.parametrize("flags", [["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                                   ["-fsanitize=thread"]], ids=["asan_ubsan", "tsan"])
def test_oracle_under_sanitizer(tmp_path, flags):
    if GCC is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "oracle_san"
    cmd = [GCC, "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", *flags, "-o", str(exe),
           str(ROOT / "oracle" / "sanitize_main.c"), str(ROOT / "oracle" / "ecc_oracle.c"), "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
    assert "ERROR: " not in r.stderr and "WARNING: ThreadSanitizer" not in r.stderr, r.stderr
