"""Host code under the address and undefined-behaviour sanitizers (CPU only).

* The library's host-side logic (chunk planners, plan queries, host CSR
  validation, the triangle-count relabelling) is rebuilt from csrc/ with the
  sanitizers on the host code only, linked with tests/sanitize/host_driver.cpp
  and run on random shapes; no GPU call is made.
* The C oracle is built with gcc's sanitizers and driven by
  tests/sanitize/oracle_driver.c over random products and graphs.

Each driver exits non-zero on a failed check; a sanitizer report aborts it."""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1804_00695_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")

pytestmark = pytest.mark.slow


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ...\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_library_host_code_sanitized(tmp_path):
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    srcs.append(os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops"] + SAN + ["-x", "hip", "-c", src, "-o", obj], str(tmp_path))
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "host_driver")
    _run([HIPCC, "--offload-arch=gfx950"] + SAN + objs + ["-o", exe], str(tmp_path))
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failed checks" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_sanitized(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
          "-fopenmp", os.path.join(ROOT, "oracle", "oracle.c"),
          os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", exe], str(tmp_path))
    r = subprocess.run([exe], capture_output=True, text=True,
                       env=dict(ENV, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"), timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failed checks" in r.stdout
