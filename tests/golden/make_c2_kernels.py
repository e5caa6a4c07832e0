"""Writes tests/golden/c2_kernels.npz: the oracle's interaction kernels K_k(C), k = 0..ell, at the
canonical offsets C (sorted |D|) that the 32^3 sphere's march-equation check needs for its
sampled target voxels (12 within 6 h of the centre, 4 near the surface; seed 2), every entry
computed by oracle/ (kquad.c through oracle.mot.kernel_list, Huygens support applied).  Only
non-zero entries are stored: keys [n][4] = (k, C0, C1, C2), values [n][6] = xx yy zz xy xz yz.

    python tests/golden/make_c2_kernels.py        (about 2 minutes on 8 cores)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
OUT = os.path.join(HERE, "c2_kernels.npz")


def spot_targets(prob):
    """Target voxels (u, v, w) of the check: 12 sphere voxels within 6 h of the centre and 4
    within 1.5 h of the surface."""
    src = np.argwhere(prob.eps > 1.0)[:, ::-1]
    d = np.linalg.norm(src + 0.5 - prob.U / 2.0, axis=1)
    rng = np.random.default_rng(2)
    inner, surf = src[d < 6.0], src[d > 13.5]
    return np.concatenate([inner[rng.choice(len(inner), 12, replace=False)],
                           surf[rng.choice(len(surf), 4, replace=False)]])


def needed_canonical(prob, targets):
    from oracle import mot
    src = np.argwhere(prob.eps > 1.0)[:, ::-1]
    C = set()
    for t in targets:
        C |= set(map(tuple, np.unique(mot.canonical_offsets(t[None, :] - src), axis=0)))
    return np.array(sorted(C))


def main():
    import workloads as wl
    from oracle import mot
    prob = wl.config("C2")
    L = mot.ell(prob.U, prob.V, prob.W)
    C = needed_canonical(prob, spot_targets(prob))
    lags = np.repeat(np.arange(L + 1), len(C))
    offs = np.tile(C, (L + 1, 1))
    K = mot.kernel_list(lags, offs)
    nz = np.any(K != 0.0, axis=1)
    keys = np.concatenate([lags[nz, None], offs[nz]], axis=1).astype(np.int32)
    np.savez(OUT, keys=keys, vals=K[nz])
    print("%d canonical offsets, %d non-zero entries -> %s" % (len(C), int(nz.sum()), OUT))


if __name__ == "__main__":
    main()
