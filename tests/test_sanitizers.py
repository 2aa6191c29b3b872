"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (gcc/g++, CPU only).

* tests/sanitize/vco_san_driver.c calls every entry point of the CPU oracle for each layout,
  mode and magnitude rounding;
* tests/sanitize/emu_san_driver.cpp runs the host build of the device codec (vc_device.hpp and
  the codec resolution of vc_params.hpp, as tests/hostemu compiles them) for every codec the
  library accepts, and the exact magnitude path directly.
Both feed edge-case vectors (zeros, infinities, NaN, subnormals, the float32 range limits),
random bit patterns and arbitrary codes.  The sanitizers abort on an out-of-bounds access, a
signed overflow, a bad shift or an out-of-range float-to-integer conversion.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer", "-ffp-contract=off"]


def _build_and_run(cmd, exe):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip(f"cannot build with the sanitizers here: {r.stderr.strip()[:300]}")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", OMP_NUM_THREADS="1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    return r.stdout


def test_oracle_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "vco_san")
    cmd = ["gcc", "-std=c11", *SAN, "-fopenmp", os.path.join(ROOT, "tests", "sanitize", "vco_san_driver.c"),
           os.path.join(ROOT, "oracle", "vco.c"), "-o", exe, "-lm"]
    assert "codecs run: 32" in _build_and_run(cmd, exe)


def test_device_codec_host_build_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "emu_san")
    cmd = ["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "sanitize", "emu_san_driver.cpp"),
           os.path.join(ROOT, "tests", "hostemu", "vc_hostemu.cpp"), "-o", exe]
    # 4 layouts x 2 roundings x 2 precisions plain, 4 fractional split at each of two level
    # counts (163840 and the largest accepted, 2^24), 8 companded (both precisions)
    assert "codecs run: 32" in _build_and_run(cmd, exe)
