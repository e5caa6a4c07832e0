"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU): the CPU oracle's C
entry points, and the device generator's quadrature compiled for the host, each driven on small
inputs by an executable of its own.  The sanitizers stop the run at the first invalid access or
undefined operation, so a clean exit is the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stderr[-2000:]
    assert "checksum" in p.stdout
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    src = [os.path.join(ROOT, "oracle", f) for f in ("kquad.c", "direct.c", "pairs.c")]
    src.append(os.path.join(HERE, "host", "oracle_sanitize.c"))
    subprocess.check_call([gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp"] + SAN + src + ["-lm", "-o", exe])
    _run(exe, {"ASAN_OPTIONS": "detect_leaks=1", "OMP_NUM_THREADS": "2"})


def test_generator_host_code_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "gen_san")
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]          # host code only; the device side is built as usual
    cmd = [hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + host_san + [
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2407_03323_amd", "csrc"),
           os.path.join(HERE, "host", "gen_sanitize.cpp"), "-o", exe]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    # the HIP runtime that the executable links keeps allocations until exit
    _run(exe, {"ASAN_OPTIONS": "detect_leaks=0"})
