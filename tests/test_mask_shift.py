"""Why a candidate mask must be widened before it is shifted (CPU).

The kNN kernels mark the candidates of a 64-particle batch in a 64-bit
mask, 16 candidates at a time.  Collecting 16 bits in a narrower word and
shifting that word by 32 or 48 into place is undefined in C++: the word is
promoted to a 32-bit int, and a shift count at or above the width of the
promoted type has no defined result (the compiler may produce any value).
This test compiles both forms for the host under the undefined-behaviour
sanitizer: the narrow form is reported, the widened form (the kernels')
runs clean and equals the per-bit definition.
"""
import os
import shutil
import subprocess

import pytest

SRC = r"""
#include <cstdint>
#include <cstdio>
#include <cstdlib>

// the kernels' form: each bit widened to 64 bits before the shift
static uint64_t widened(const bool *ok)
{
    uint64_t pass = 0;
    for (int k0 = 0; k0 < 64; k0 += 16)
        for (int k = 0; k < 16; k++) pass |= (uint64_t)(ok[k0 + k] ? 1u : 0u) << (k0 + k);
    return pass;
}

// 16 bits collected first, the 16-bit word shifted into place unwidened
static uint64_t narrow(const bool *ok)
{
    uint64_t pass = 0;
    for (int k0 = 0; k0 < 64; k0 += 16) {
        uint16_t m = 0;
        for (int k = 0; k < 16; k++) m |= (uint16_t)((ok[k0 + k] ? 1 : 0) << k);
        pass |= m << k0;
    }
    return pass;
}

int main(int argc, char **argv)
{
    const bool use_narrow = argc > 1;
    srand(7);
    for (int trial = 0; trial < 1000; trial++) {
        bool ok[64];
        uint64_t ref = 0;
        for (int i = 0; i < 64; i++) {
            ok[i] = (rand() & 3) == 0;
            if (ok[i]) ref |= 1ull << i;
        }
        const uint64_t got = use_narrow ? narrow(ok) : widened(ok);
        if (!use_narrow && got != ref) {
            printf("mismatch\n");
            return 1;
        }
    }
    printf("done\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_narrow_mask_shift_is_undefined_and_widened_is_exact(tmp_path):
    src = tmp_path / "mask.cpp"
    exe = tmp_path / "mask"
    src.write_text(SRC)
    subprocess.run(["g++", "-O1", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
                    "-o", str(exe), str(src)], check=True)
    env = dict(os.environ, UBSAN_OPTIONS="print_stacktrace=0")
    good = subprocess.run([str(exe)], capture_output=True, text=True, env=env)
    assert good.returncode == 0 and "done" in good.stdout, good.stdout + good.stderr
    bad = subprocess.run([str(exe), "narrow"], capture_output=True, text=True, env=env)
    assert bad.returncode != 0
    assert "shift exponent" in bad.stderr and "too large" in bad.stderr, bad.stderr
