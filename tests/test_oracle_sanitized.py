"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(out-of-bounds and use-after-free accesses, signed overflow, misaligned or
invalid arithmetic in its hand-indexed loops) runs the oracle's own pins
(P1-P9: Yee dispersion and energy, Lorentz susceptibility, rate equations,
growth rate, Philox, monitors, Mur, adjoint) without a report.  CPU only; the
sanitizer runtime is preloaded into a child interpreter, which loads the
sanitized library through MB_ORACLE_LIB."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_yee.py", "tests/test_oracle_bloch.py", "tests/test_oracle_rng.py",
        "tests/test_oracle_monitors.py", "tests/test_oracle_adjoint.py", "tests/test_oracle_modes.py"]


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_pass_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for gcc here")
    lib = tmp_path / "libmboracle_san.so"
    srcs = [os.path.join(ROOT, "oracle", f) for f in ("mb_oracle.c", "pack_oracle.c")]
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-o", str(lib), *srcs, "-lm"], check=True)
    env = dict(os.environ, MB_ORACLE_LIB=str(lib), LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-n", "4", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    out = r.stdout[-3000:] + r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out
    assert r.returncode == 0, out
