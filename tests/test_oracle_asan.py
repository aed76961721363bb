"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): tests/asan_oracle_driver.c runs every stage on small boxes,
the bounded-memory pipeline in pieces, the subhalos and the argument
checks; any out-of-bounds access, leak or undefined operation fails it.
A planted out-of-bounds read shows that the sanitizer is active."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-std=c11", "-ffp-contract=off", "-Wno-unknown-pragmas"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _gcc():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    return gcc


def _build(tmp_path, name, sources):
    exe = str(tmp_path / name)
    r = subprocess.run([_gcc(), *FLAGS, "-o", exe, *sources, "-lm"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def test_sanitizer_is_active(tmp_path):
    src = tmp_path / "oob.c"
    src.write_text("#include <stdlib.h>\n"
                   "int main(void) { volatile int *p = malloc(4 * sizeof(int)); int v = p[4];\n"
                   "free((void *)p); return v == 12345; }\n")
    exe = _build(tmp_path, "oob", [str(src)])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60, env=ENV)
    assert r.returncode != 0
    # (the undefined-behaviour checker's object-size check may see it first)
    assert "AddressSanitizer" in r.stderr or "runtime error" in r.stderr, r.stderr[-2000:]


def test_oracle_is_clean_under_sanitizers(tmp_path):
    exe = _build(tmp_path, "asan_oracle",
                 [os.path.join(ROOT, "tests", "asan_oracle_driver.c"),
                  os.path.join(ROOT, "oracle", "hop_oracle.c")])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=ENV)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "asan driver: ok" in r.stdout
