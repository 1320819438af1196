"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU:

* the whole library rebuilt with its host code instrumented (device code
  unchanged) and the C-ABI tests (tests/test_abi.py: configuration
  validation, workspace layout, batch-plan and argument checks) run against
  it with the sanitizer runtime preloaded into a fresh interpreter;
* the float64 cosmology (cosmo.cpp) driven by a host-only program built
  with both sanitizers (every P(k) kind, growth, step factors of every
  integrator);
* the sort's index algebra (tile numbering, keys, paint bins, the first
  sort's lattice walk, the periodic wrap of pm_device.h) run on the host,
  its host code built with both sanitizers.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_11847_amd", "csrc")


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="no hipcc")
def test_abi_under_host_sanitizers():
    from paper_2010_11847_amd import build as b
    lib = b.build_host_sanitized()
    rt = b.sanitizer_runtime()
    assert os.path.exists(rt), rt
    env = dict(os.environ)
    env.update(PM_LIBRARY=lib, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")], env=env, capture_output=True, text=True,
                       cwd=ROOT, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_host_cosmology_under_sanitizers(tmp_path):
    exe = tmp_path / "host_cosmo_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(ROOT, "tests", "host_cosmo_check.cpp"), os.path.join(CSRC, "cosmo.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host cosmology check ok" in r.stdout


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="no hipcc")
def test_sort_index_algebra_on_host(tmp_path):
    exe = tmp_path / "host_order_check"
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "-std=c++17", "-O1", "-g", "--offload-arch=gfx950",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined",
           f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(ROOT, "tests", "host_order_check.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sort index algebra ok" in r.stdout
