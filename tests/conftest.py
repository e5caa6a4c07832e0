import hashlib
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)

CACHE = os.path.join(TESTS, ".cache")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X; runs the HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def _oracle_digest():
    h = hashlib.sha1()
    for f in ("kquad.c", "direct.c", "pairs.c"):
        with open(os.path.join(ROOT, "oracle", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def oracle_kernel_table(U, V, W, kmax, ngl=16, r=1.0, hv=None):
    """Oracle kernel table (c dt = r, voxel edges hv, default cubic), cached on disk per oracle
    source version (the cache is only a speed-up: it is recomputed from oracle/ whenever missing)."""
    from oracle import mot
    os.makedirs(CACHE, exist_ok=True)
    tag = "" if r == 1.0 else "_r%.6g" % r
    if hv is not None and tuple(hv) != (1.0, 1.0, 1.0):
        tag += "_h%.6g_%.6g_%.6g" % tuple(hv)
    path = os.path.join(CACHE, "K_%s_%dx%dx%d_k%d_n%d%s.npy" % (_oracle_digest(), U, V, W, kmax, ngl, tag))
    if os.path.exists(path):
        return np.load(path)
    K = mot.kernel_table(U, V, W, kmax, ngl, r, hv=hv)
    tmp = path + ".tmp%d.npy" % os.getpid()
    np.save(tmp, K)
    os.replace(tmp, path)
    return K


@pytest.fixture(scope="session")
def c1_oracle():
    """Oracle run of the 8^3 eps_r = 4 cube (200 steps, no FIR)."""
    import workloads as wl
    from oracle import mot
    p = wl.config("C1")
    ell = mot.ell(p.U, p.V, p.W)
    K = oracle_kernel_table(p.U, p.V, p.W, ell)
    o = mot.Oracle(p, K=K)
    J = o.run(p.n_steps)
    return p, o, J
