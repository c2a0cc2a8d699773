"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code.

The oracle's C sources and the library's host-side numerics (``csrc/host.cpp``:
graded mesh, coarsening, dual widths, the 1-D eigen-decompositions of the
direct solve) are built with the host compiler alone, with both sanitizers and
no recovery, and driven by the programs under ``tests/sanitize/``: an
out-of-bounds access, a use after free, a leak or an undefined operation ends
the run with a non-zero status. No GPU code is built this way."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


def _build_and_run(tmp_path, cmd, exe):
    subprocess.run(cmd + ["-o", str(exe)], check=True, capture_output=True, text=True)
    return subprocess.run([str(exe)], capture_output=True, text=True, env=ENV, timeout=300)


def test_sanitizers_catch_a_planted_overflow(tmp_path):
    """The sanitizer build works here: an overflow by one element fails."""
    src = tmp_path / "planted.c"
    src.write_text("#include <stdlib.h>\nint main(void) { volatile double* p = malloc(4 * sizeof(double));"
                   " p[4] = 1.0; free((void*)p); return 0; }\n")
    r = _build_and_run(tmp_path, ["gcc"] + SAN + [str(src)], tmp_path / "planted")
    # UBSan's object-size check or ASan's redzone, whichever sees it first
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr or "runtime error: store to address" in r.stderr


def test_oracle_entry_points_clean_under_sanitizers(tmp_path):
    srcs = [os.path.join(HERE, "oracle_driver.c")] + [os.path.join(ROOT, "oracle", f)
                                                      for f in ("oracle.c", "sphere.c", "basis.c")]
    r = _build_and_run(tmp_path, ["gcc", "-std=c11", "-fopenmp"] + SAN + srcs + ["-lm"], tmp_path / "odrv")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ran clean" in r.stdout


def test_library_host_numerics_clean_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_0806_1723_amd", "csrc")
    srcs = [os.path.join(HERE, "host_driver.cpp"), os.path.join(csrc, "host.cpp")]
    r = _build_and_run(tmp_path, ["g++", "-std=c++17", "-I", csrc] + SAN + srcs, tmp_path / "hdrv")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ran clean" in r.stdout
