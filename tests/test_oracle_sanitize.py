"""The oracle's pins under AddressSanitizer and UBSan (no GPU).

The oracle's C source is built a second time with -fsanitize=address,undefined
(oracle.build(variant="san")) and the pin tests of tests/test_oracle_pins.py
and tests/test_oracle_adjoint.py run against that build in a child process
with the ASan runtime preloaded; any out-of-bounds access, use after free or
undefined behaviour (UBSan does not recover) fails the child.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _libasan():
    try:
        p = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(_libasan() is None, reason="gcc's AddressSanitizer runtime not found")
def test_oracle_pins_clean_under_sanitizers():
    import oracle
    oracle.build(force=True, variant="san")
    env = dict(os.environ)
    env["LBM_ORACLE_VARIANT"] = "san"
    env["LD_PRELOAD"] = _libasan()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_oracle_pins.py"), os.path.join(ROOT, "tests", "test_oracle_adjoint.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1800)
    tail = (r.stdout + r.stderr)[-3000:]
    print(tail)
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
