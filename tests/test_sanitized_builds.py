"""CPU builds with AddressSanitizer and UndefinedBehaviorSanitizer.

* The FP64 oracle: every routine on small periodic and outflow/isolated grids
  (tests/oracle_sanitize_driver.c, built with gcc, leak checking on). A
  planted out-of-bounds read in the driver must be reported, which shows that
  the instrumentation is live.
* The library's host code: vp_api.hip compiled with the sanitizers on its host
  side only, driven through every host-validation path of the C ABI
  (tests/host_sanitize_driver.cpp). No call reaches a device, so this runs
  without a GPU; the kernels come from the built libvp.so.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = {"UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _gcc_oracle(tmp_path, extra=()):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not installed")
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wno-alloc-size-larger-than", "-I", os.path.join(ROOT, "oracle"),
           *extra, os.path.join(HERE, "oracle_sanitize_driver.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe, leaks):
    env = dict(os.environ, **SAN_ENV)
    env["ASAN_OPTIONS"] = "detect_leaks=%d:abort_on_error=0" % (1 if leaks else 0)
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)


def test_oracle_is_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    r = _run(_gcc_oracle(tmp_path), leaks=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert r.stdout.startswith("checksum ")


def test_sanitizer_reports_a_planted_out_of_bounds_read(tmp_path):
    r = _run(_gcc_oracle(tmp_path, extra=("-DPLANT_OOB",)), leaks=False)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr


def test_library_host_code_is_clean_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc is not installed")
    from paper_1206_6152_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    libdir = os.path.dirname(_lib.LIB_PATH)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1206_6152_amd", "csrc")]
    # host-side instrumentation only: each sanitizer flag follows -Xarch_host
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
              "-packed-fp32-ops", "-Wno-unused-command-line-argument"]
    api_o, main_o, exe = (str(tmp_path / n) for n in ("vp_api_san.o", "main_san.o", "host_san"))
    steps = [
        [HIPCC, *common, *inc, *san, "-c", os.path.join(ROOT, "paper_1206_6152_amd", "csrc", "vp_api.hip"),
         "-o", api_o],
        [HIPCC, *common, *inc, *san, "-c", os.path.join(HERE, "host_sanitize_driver.cpp"), "-o", main_o],
        # the sanitized vp_* definitions in the executable take precedence over
        # the library's; the kernels and their launchers come from libvp.so
        [HIPCC, "--offload-arch=gfx950", *san, main_o, api_o, "-L", libdir, "-lvp", "-Wl,-rpath," + libdir,
         "-o", exe],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, " ".join(cmd) + "\n" + r.stderr
    # the HIP runtime keeps allocations until exit, so leak checking is off
    r = _run(exe, leaks=False)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "0 failures" in r.stdout
