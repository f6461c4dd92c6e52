"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize/oracle_driver.c calls every entry of oracle/oracle.c on a
small seeded two-view scene (ragged image sizes, culled Gaussians, a
non-finite parameter); it is built here with gcc's address and undefined
behaviour sanitizers (leak detection on) and must run without a report. A
toolchain check first confirms that such a build does report an
out-of-bounds write, so a sanitizer that is silently unavailable cannot let
the oracle's run pass."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-std=c11", "-D_GNU_SOURCE", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-fopenmp", "-ffp-contract=off"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
           OMP_NUM_THREADS="2")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")


def _build(tmp_path, name, sources):
    exe = str(tmp_path / name)
    r = subprocess.run(["gcc", *FLAGS, "-o", exe, *sources, "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_sanitizer_reports_an_out_of_bounds_write(tmp_path):
    src = tmp_path / "oob.c"
    src.write_text("#include <stdlib.h>\nint main(void) { int *a = malloc(4 * sizeof(int)); volatile int i = 4;\n"
                   "a[i] = 1; free(a); return 0; }\n")
    r = subprocess.run([_build(tmp_path, "oob", [str(src)])], capture_output=True, text=True, env=ENV, timeout=60)
    # (the undefined-behaviour checks may name the bad store before AddressSanitizer does)
    assert r.returncode != 0 and ("AddressSanitizer" in r.stderr or "runtime error" in r.stderr), r.stderr


def test_oracle_runs_clean_under_sanitizers(tmp_path):
    exe = _build(tmp_path, "oracle_driver", [os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                                              os.path.join(ROOT, "oracle", "oracle.c")])
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=120)
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    assert r.returncode == 0, r.stdout + r.stderr
    assert "tiled vs brute max diff 0," in r.stdout, r.stdout
