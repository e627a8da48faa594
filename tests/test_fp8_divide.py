"""The FP8 encoder's divide by a channel scale (binary32 reciprocal, one
Markstein correction step) against the correctly rounded quotient, on the
CPU: tests/fp8_divide_check.c built with gcc and run over every 4099th
binary32 pattern on 26 scales (the full check runs it over all 2^32
patterns), and the same program with the correction step dropped must
report mismatches."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fp8_divide_check.c")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


def _build(tmp_path, *defs):
    exe = str(tmp_path / ("check" + "".join(defs)))
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", *[f"-D{d}" for d in defs], "-o", exe, SRC,
                    "-lm"], check=True)
    return exe


def test_corrected_reciprocal_product_gives_the_correctly_rounded_code(tmp_path):
    r = subprocess.run([_build(tmp_path), "4099", "8", "1"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "26 scales, stride 4099: 0 mismatches" in r.stdout


def test_the_check_fails_without_the_correction_step(tmp_path):
    r = subprocess.run([_build(tmp_path, "DROP_CORRECTION"), "4099", "8", "1"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 1
    assert " 0 mismatches" not in r.stdout.splitlines()[-1]
