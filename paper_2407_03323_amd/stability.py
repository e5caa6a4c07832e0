"""Stability toolkit for the FIR-regularised march (Sec. 6), for choosing a filter before a long run.

Off the per-step path: it assembles the interaction matrices of a *small* grid from the kernels the
library generates on the device (mj_kernel_values) and analyses them on the host with dense linear
algebra, so it is meant for grids of a few hundred unknowns.

* `fir_magnitude`, `fir_report`: the FIR-regularisation magnitude |sum_n delta_n e^{-j n theta}|
  (eq:FIRmagnitude), the value at theta = pi that eq:RegReq1 fixes, and the group delay of a
  linear-phase filter.
* `interaction_matrices`: Z^delta_k, k = 0..L, with Z_k J = c_k J - chi K_k (*) J and
  c_k = T(k dt)/eps + delta_k (eq:Z with Sec. 6.1's taps), restricted to the voxels with chi > 0
  and scaled row-wise by 1/chi, which makes every matrix symmetric and leaves the recursion's
  solutions unchanged.
* `companion_dominant`: the largest-modulus eigenvalue of the companion matrix of
  sum_k Z_k J_{n-k} = 0; the march is stable when its modulus is below 1 (Sec. 6).
* `pdsa_minima`: the smallest eigenvalue of each PDSA matrix
  D_n = sum_{j=0}^{n} (-1)^j C(L - j, L - n) Z_j, n = 0..L (eq:Dn as read here; D_L = sum_j (-1)^j Z_j
  is the matrix that eq:Regularization shifts by delta).  All of them positive guarantees that no
  eigenvalue on the negative real axis leaves the unit circle; it says nothing about the others,
  which is why Sec. 6.1 adds its third requirement.
"""
from __future__ import annotations

from math import comb

import numpy as np


def fir_magnitude(taps, theta) -> np.ndarray:
    """|sum_n delta_n exp(-j n theta)| for normalised frequencies theta (eq:FIRmagnitude)."""
    taps = np.asarray(taps, dtype=float)
    th = np.atleast_1d(np.asarray(theta, dtype=float))
    n = np.arange(len(taps))
    return np.abs(np.exp(-1j * np.outer(th, n)) @ taps)


def fir_report(taps) -> dict:
    """delta = sum (-1)^n delta_n (eq:RegReq1), the largest magnitude for theta in [0, 0.9 pi], and
    the group delay (taps - 1)/2 steps when the taps are symmetric or antisymmetric."""
    taps = np.asarray(taps, dtype=float)
    n = len(taps)
    sym = bool(n) and (np.allclose(taps, taps[::-1]) or np.allclose(taps, -taps[::-1]))
    return {
        "delta": float(np.sum(taps * (-1.0) ** np.arange(n))),
        "max_magnitude_below_0.9pi": float(fir_magnitude(taps, np.linspace(0.0, 0.9 * np.pi, 181)).max()) if n else 0.0,
        "linear_phase": sym,
        "group_delay_steps": (n - 1) / 2.0 if sym else None,
    }


def _tbasis(k: int) -> float:
    """T(k dt) of the causal quadratic B-spline basis T(t) = B(t/dt + 1): 1/2, 1/2, then 0."""
    return 0.5 if k in (0, 1) else 0.0


def interaction_matrices(solver, eps, taps) -> list:
    """Dense Z^delta_k / chi (row-scaled), k = 0..L with L = max(ell, taps - 1), for the voxels of
    `solver`'s grid with eps > 1.  The kernels K_k come from the solver's device generator."""
    U, V, W = solver.U, solver.V, solver.W
    eps = np.asarray(eps, dtype=float).reshape(W, V, U)
    taps = np.asarray(taps, dtype=float)
    ell = solver.ell
    L = max(ell, len(taps) - 1)
    w, v, u = np.nonzero(eps > 1.0)
    pos = np.stack([u, v, w], axis=1)
    nv = len(pos)
    if nv == 0:
        raise ValueError("no voxel with eps > 1")
    chi = (eps[w, v, u] - 1.0) / eps[w, v, u]
    D = (pos[:, None, :] - pos[None, :, :]).reshape(-1, 3)
    uniq, inv = np.unique(D, axis=0, return_inverse=True)
    inv = inv.ravel()
    comp = ((0, 3, 4), (3, 1, 5), (4, 5, 2))
    Z = []
    for k in range(L + 1):
        ck = _tbasis(k) / eps[w, v, u] + (taps[k] if k < len(taps) else 0.0)
        Zk = np.diag(np.tile(ck / chi, 3))
        if k <= ell:
            Kv = solver.kernel_values(np.full(len(uniq), k, dtype=np.int32), uniq)[inv].reshape(nv, nv, 6)
            for a in range(3):
                for b in range(3):
                    Zk[a * nv:(a + 1) * nv, b * nv:(b + 1) * nv] -= Kv[:, :, comp[a][b]]
        Z.append(Zk)
    return Z


def companion_dominant(Z) -> complex:
    """Largest-modulus eigenvalue of the companion matrix of Z_0 J_n = -sum_{k>=1} Z_k J_{n-k}."""
    L, n = len(Z) - 1, Z[0].shape[0]
    Zi = np.linalg.inv(Z[0])
    C = np.zeros((n * L, n * L))
    for k in range(1, L + 1):
        C[:n, (k - 1) * n:k * n] = -Zi @ Z[k]
    C[n:, :-n] = np.eye(n * (L - 1))
    ev = np.linalg.eigvals(C)
    return complex(ev[np.argmax(np.abs(ev))])


def pdsa_minima(Z) -> np.ndarray:
    """Smallest eigenvalue of D_n = sum_{j=0}^{n} (-1)^j C(L - j, L - n) Z_j for n = 0..L."""
    L = len(Z) - 1
    out = np.zeros(L + 1)
    for n in range(L + 1):
        Dn = sum(((-1) ** j) * comb(L - j, L - n) * Z[j] for j in range(n + 1))
        out[n] = np.linalg.eigvalsh(0.5 * (Dn + Dn.T))[0]
    return out
