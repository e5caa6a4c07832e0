"""The device kernel generator's quadrature, compiled for the host and run serially,
against the oracle's independent quadrature (no GPU needed).  This checks the generator's
logic -- shell moments, B-spline lag combination, parity folding, off-grid offsets -- apart
from code generation for gfx950, which the GPU tests cover."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import mot

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def gen_host():
    out_dir = os.path.join(HERE, ".cache")
    os.makedirs(out_dir, exist_ok=True)
    lib = os.path.join(out_dir, "libgen_host.so")
    src = os.path.join(HERE, "host", "gen_host.cpp")
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    cmd = [hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "-x", "hip", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2407_03323_amd", "csrc"),
           src, "-o", lib]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    L = ctypes.CDLL(lib)
    L.host_kernels.argtypes = [ctypes.c_double] * 6 + [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]

    def run(D, kmax, nq=16, r=1.0, hv=(1.0, 1.0, 1.0)):
        assert hv[0] == 1.0
        out = np.zeros((kmax + 1, 6))
        L.host_kernels(float(D[0]), float(D[1]), float(D[2]), float(r), float(hv[1]), float(hv[2]), nq, kmax,
                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return out
    return run


OFFSETS = [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, -1, 0), (-3, 2, 1), (5, 4, -3), (0, 0, 9), (12, -7, 3),
           (1.3, -0.7, 0.45), (2.61, 1.17, -0.38), (4.37, -2.81, 1.55), (0.0, 0.0, 1.75)]


@pytest.mark.parametrize("D", OFFSETS)
def test_generator_on_host_matches_oracle(gen_host, D):
    b = np.sqrt(sum((abs(d) + 1) ** 2 for d in D))
    kmax = int(b) + 3
    got = gen_host(D, kmax)
    ngl = 16 if all(float(d).is_integer() for d in D) else 24
    ref = np.array([mot.kernel_entry(k, D, ngl=ngl) for k in range(kmax + 1)])
    assert np.abs(got - ref).max() <= 3e-12 * np.abs(ref).max()


@pytest.mark.parametrize("r", [0.5, 0.7, 0.3])
@pytest.mark.parametrize("D", [(0, 0, 0), (1, 0, 0), (1, 1, 1), (-3, 2, 1), (5, 4, -3), (1.3, -0.7, 0.45)])
def test_generator_on_host_matches_oracle_short_step(gen_host, D, r):
    """c dt = r h < h: shells r wide, more lags per offset, B'' / r^2 on the time-derivative term."""
    b = np.sqrt(sum((abs(d) + 1) ** 2 for d in D))
    kmax = int(b / r) + 3
    got = gen_host(D, kmax, r=r)
    ngl = 16 if all(float(d).is_integer() for d in D) else 24
    ref = np.array([mot.kernel_entry(k, D, ngl=ngl, r=r) for k in range(kmax + 1)])
    # an off-centre overlap of the two voxels puts 1/R's singularity inside the box away from
    # every symmetry plane, where the oracle's quadrature is good to ~1e-9 only
    tol = 3e-12 if all(float(d).is_integer() for d in D) else 1e-10
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("hv,r", [((1.0, 0.7, 1.3), 0.7), ((1.0, 1.5, 2.0), 0.6)])
@pytest.mark.parametrize("D", [(0, 0, 0), (1, 0, 0), (0, 1, 1), (1, 1, 1), (-3, 2, 1), (5, 4, -3), (1.3, -0.7, 0.45)])
def test_generator_on_host_matches_oracle_prism_voxels(gen_host, D, hv, r):
    """hx x hy x hz voxels: planes and sub-boxes scaled per axis, 1/h_a on the second differences."""
    b = np.sqrt(sum(((abs(d) + 1) * h) ** 2 for d, h in zip(D, hv)))
    kmax = int(b / r) + 3
    got = gen_host(D, kmax, r=r, hv=hv)
    ngl = 16 if all(float(d).is_integer() for d in D) else 24
    ref = np.array([mot.kernel_entry(k, D, ngl=ngl, r=r, hv=hv) for k in range(kmax + 1)])
    tol = 3e-12 if all(float(d).is_integer() for d in D) else 1e-10
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
