"""The C oracle under gcc's AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): tests/oracle_sanitize_main.c drives every entry point on small
cases (ragged sizes, Parareal with learning and with given fractions, a
point mass through the resample branch, the adjoint with every coefficient,
the rotator's wrapped trigonometric field, the Burgers drift); the build
includes the oracle as one translation unit, so its static helpers are
instrumented as well."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_runs_clean_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not installed")
    exe = str(tmp_path / "oracle_sanitized")
    flags = ["-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-ffp-contract=off",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    b = subprocess.run([gcc, *flags, os.path.join(HERE, "oracle_sanitize_main.c"), "-lm", "-o", exe],
                       capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.stdout.startswith("oracle entry points ran")
