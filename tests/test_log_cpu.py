"""ZM_LOG diagnostics on the CPU: with level 1 every failure is echoed to
stderr as one "zm: error: <text>" line carrying the zm_last_error text; with
the variable unset the library writes nothing.  Only argument checks that
fail before any device call are exercised, so no GPU is needed."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2304_14492_amd", "libzm.so")

PROBE = f"""
import ctypes
lib = ctypes.CDLL({LIB!r})
lib.zm_last_error.restype = ctypes.c_char_p
assert lib.zm_destroy(None) == -1
assert lib.zm_count_nonfinite(None, None, 1, None, None) == -1
print(lib.zm_last_error().decode())
"""


def _run(level):
    env = dict(os.environ)
    env.pop("ZM_LOG", None)
    if level is not None:
        env["ZM_LOG"] = level
    return subprocess.run([sys.executable, "-c", PROBE], env=env, capture_output=True, text=True, timeout=120)


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(LIB):
        pytest.skip("libzm.so not built")


def test_errors_logged_at_level_1():
    r = _run("1")
    assert r.returncode == 0, r.stderr
    lines = [l for l in r.stderr.splitlines() if l.startswith("zm: ")]
    assert lines == ["zm: error: null plan", "zm: error: null plan"], r.stderr
    assert r.stdout.strip() == "null plan"


def test_silent_by_default_and_at_level_0():
    for level in (None, "0"):
        r = _run(level)
        assert r.returncode == 0, r.stderr
        assert "zm: " not in r.stderr, r.stderr
