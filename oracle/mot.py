"""ORACLE -- test infrastructure, not product code.

The FFT-free MOT-JVIE marched step by step exactly as Sec. 2.4 writes it:

    Z_0 J_n = E_n - P_{n-1},      P_{n-1} = sum_{k=1}^{ell} Z_k J_{n-k}      (eq:MOTInversion, eq:PnMOT)

with the elements of eq:Z, the excitation of eq:E and the FIR regularisation
Z_k -> Z_k + delta_k I of Sec. 6.1.  Z_0 is assembled as a sparse matrix and factorised
directly (scipy's sparse LU); the history sum is the direct triple sum of direct.c.
Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use it.

Units: the x edge of a voxel is 1; the voxel edges (1, hy, hz) and c dt <= min(edges) come from
the Problem (the configurations in workloads/ use cubic voxels and c dt = h).
Vectors are stored per component: J[a][w][v][u]  (the paper's eq:CurrentVector
interleaves the three components per voxel; the two orders hold the same numbers).
"""
from __future__ import annotations

import ctypes
from math import floor, sqrt

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dptr, iptr, lib

# (b, a) -> stored component of the symmetric 3x3 kernel: xx, yy, zz, xy, xz, yz
COMP = ((0, 3, 4), (3, 1, 5), (4, 5, 2))


def ell(U: int, V: int, W: int, h: float = 1.0, c_dt: float = 1.0, hy=None, hz=None) -> int:
    """Number of non-zero lags beyond Z_0 (eq:Ell); voxel edges h, hy, hz (default h)."""
    hy = h if hy is None else hy
    hz = h if hz is None else hz
    return int(floor(sqrt((U * h) ** 2 + (V * hy) ** 2 + (W * hz) ** 2) / c_dt)) + 2


def _edges(hv) -> np.ndarray:
    return np.ascontiguousarray(np.ones(3) if hv is None else np.asarray(hv, dtype=np.float64).reshape(3))


def tbasis(t_over_dt: float) -> float:
    """Temporal basis T(t) = B(t/dt + 1): the causal quadratic B-spline with knots
    -dt, 0, dt, 2 dt (reading of Sec. 2.3, which defers T to an earlier paper)."""
    return lib().or_bspline(float(t_over_dt) + 1.0)


def kernel_entry(k: int, D, ngl: int = 16, r: float = 1.0, hv=None) -> np.ndarray:
    """K_k(D) for an offset D in voxel steps, c dt = r and voxel edges hv (default 1, 1, 1)."""
    out = np.zeros(6)
    lib().or_kernel_entry_h(r, dptr(_edges(hv)), int(k), float(D[0]), float(D[1]), float(D[2]), int(ngl), dptr(out))
    return out


def kernel_table(U: int, V: int, W: int, kmax: int, ngl: int = 16, r: float = 1.0,
                 skip_outside: bool = True, hv=None) -> np.ndarray:
    """K[k][6][2W-1][2V-1][2U-1] for k = 0..kmax (offset D at index D + (U-1, V-1, W-1))."""
    K = np.zeros((kmax + 1, 6, 2 * W - 1, 2 * V - 1, 2 * U - 1))
    lib().or_kernel_table_h(r, dptr(_edges(hv)), U, V, W, kmax, ngl, 1 if skip_outside else 0, dptr(K))
    return K


def chi_of(eps: np.ndarray) -> np.ndarray:
    """chi_m = (eps_m - 1) / eps_m  (the contrast factor of eq:TDJVIE)."""
    return (eps - 1.0) / eps


def local_coefficients(eps: np.ndarray, fir: np.ndarray, kmax: int) -> np.ndarray:
    """c_k(m) = T(k dt)/eps_m + delta_k for k = 0..kmax: the identity part of Z_k
    (eq:Z tested at its own voxel, with 1 - chi = 1/eps) plus the FIR tap (Sec. 6.1)."""
    c = np.zeros((kmax + 1,) + eps.shape)
    for k in range(kmax + 1):
        d = fir[k] if k < len(fir) else 0.0
        c[k] = tbasis(k) / eps + d
    return c


def excitation(U, V, W, eps, wave, n: int, nquad: int = 8, r: float = 1.0, hv=None) -> np.ndarray:
    """E_n(m) = chi_m (1/|V_m|) Int_{V_m} E^i(r, n dt) dV  (eq:E, test voxel m and step n),
    the voxel average taken with an nquad^3 Gauss-Legendre rule; c dt = r, voxel edges hv."""
    return chi_of(eps)[None] * incident_average(U, V, W, wave, n, nquad, r, hv)


def incident_average(U, V, W, wave, n: int, nquad: int = 8, r: float = 1.0, hv=None) -> np.ndarray:
    """<E^i>_m(n dt) = (1/|V_m|) Int_{V_m} E^i(r, n dt) dV, [3][W][V][U].  Lengths in the unit of
    the voxel edges hv (default 1, 1, 1); t0 and width are c t0 and the pulse width as lengths;
    c n dt = n r."""
    wz, wy, wx = np.meshgrid(np.arange(W), np.arange(V), np.arange(U), indexing="ij")
    return _wave_average(wx, wy, wz, wave, n, nquad, r, hv)


def incident_average_voxels(voxels, wave, n: int, nquad: int = 8, r: float = 1.0, hv=None) -> np.ndarray:
    """<E^i>_m(n dt) as incident_average, at a list of voxels [nv][3] (u, v, w): [3][nv]."""
    v = np.asarray(voxels, dtype=np.int64).reshape(-1, 3)
    return _wave_average(v[:, 0], v[:, 1], v[:, 2], wave, n, nquad, r, hv)


def _wave_average(wx, wy, wz, wave, n, nquad, r, hv):
    """Voxel averages of the plane wave at voxel indices (wx, wy, wz) (arrays of one shape)."""
    hx, hy, hz = _edges(hv)
    x, w = np.polynomial.legendre.leggauss(nquad)
    x = 0.5 * x
    w = 0.5 * w
    k = np.asarray(wave.khat, float)
    p = np.asarray(wave.pol, float)
    rr = np.asarray(wave.r_ref, float)
    # tau at the voxel centre, and the projections of the quadrature offsets on khat
    tc = float(n) * r - wave.t0 - (((wx + 0.5) * hx - rr[0]) * k[0] + ((wy + 0.5) * hy - rr[1]) * k[1] +
                                    ((wz + 0.5) * hz - rr[2]) * k[2])
    avg = np.zeros(tc.shape)
    for i in range(nquad):
        for j in range(nquad):
            for l in range(nquad):
                s = x[i] * hx * k[0] + x[j] * hy * k[1] + x[l] * hz * k[2]
                avg += w[i] * w[j] * w[l] * np.exp(-((tc - s) / wave.width) ** 2)
    avg *= wave.amp
    return np.stack([avg * p[0], avg * p[1], avg * p[2]])


def kernel_list(lags, offsets, ngl: int = 16, r: float = 1.0, hv=None, skip_outside: bool = True) -> np.ndarray:
    """K_k(D) for a list of lags [n] and offsets [n][3] (voxel steps): [n][6]; entries outside
    the Huygens support are exactly 0 when skip_outside (the dense table's rule)."""
    k = np.ascontiguousarray(np.asarray(lags, dtype=np.int32))
    D = np.ascontiguousarray(np.asarray(offsets, dtype=np.float64).reshape(-1, 3))
    out = np.zeros((len(k), 6))
    lib().or_kernel_list_h(r, dptr(_edges(hv)), len(k), iptr(k), dptr(D), int(ngl), 1 if skip_outside else 0,
                           dptr(out))
    return out


def canonical_offsets(offsets) -> np.ndarray:
    """Sorted absolute values of integer offsets [n][3]: the representative of each class of
    offsets that the symmetries used by kernel_values_by_symmetry relate."""
    return np.sort(np.abs(np.asarray(offsets, dtype=np.int64).reshape(-1, 3)), axis=1)


def kernel_values_by_symmetry(lags, offsets, canon) -> np.ndarray:
    """K_k(D) [n][6] for cubic voxels from values at canonical offsets (sorted |D|), by the
    symmetries of eq:Z that the oracle's pins check on directly computed entries: K^aa is even in
    every D_i, K^ab (a != b) is odd in D_a and in D_b and even in the third, and permuting the
    axes of D permutes the components alike.  canon[k][C0][C1][C2][6] holds K_k at the
    canonical offsets C0 <= C1 <= C2 (zero where not needed)."""
    D = np.asarray(offsets, dtype=np.int64).reshape(-1, 3)
    k = np.broadcast_to(np.asarray(lags, dtype=np.int64), (len(D),))
    a = np.abs(D)
    order = np.argsort(a, axis=1, kind="stable")      # canonical axis j is axis order[:, j] of D
    C = np.take_along_axis(a, order, axis=1)
    pos = np.argsort(order, axis=1)                   # axis x of D is canonical axis pos[:, x]
    Kc = canon[k, C[:, 0], C[:, 1], C[:, 2]]          # [n][6]
    sg = np.where(D < 0, -1.0, 1.0)
    comp = np.array(COMP)
    out = np.zeros((len(D), 6))
    for x in range(3):
        for y in range(x, 3):
            v = np.take_along_axis(Kc, comp[pos[:, x], pos[:, y]][:, None], axis=1)[:, 0]
            out[:, comp[x][y]] = v if x == y else v * sg[:, x] * sg[:, y]
    return out


def restricted_march(prob, voxels, n_steps: int, rhs: int = 0, ngl: int = 16) -> np.ndarray:
    """The march of eq:MOTInversion on the unknowns of a list of voxels [nv][3] (u, v, w) that holds
    every voxel with eps_r != 1.  Any other voxel has chi = 0: its row of every Z_k reduces to
    c_k J(m) = E_n(m) = 0 (eq:E carries the factor chi), so its current vanishes at every step,
    and its column multiplies that zero; dropping both leaves the listed voxels' currents
    unchanged.  Z_k over the listed voxels is dense, c_k(m) on the diagonal minus
    chi_m K_k(r_m - r_m') (eq:Z with Sec. 6.1's taps); the history sum of eq:PnMOT is one
    dense product per lag and Z_0 is solved densely.  Returns J [n_steps][3][nv]."""
    vox = np.asarray(voxels, dtype=np.int64).reshape(-1, 3)
    nv = len(vox)
    hv = problem_edges(prob)
    assert prob.h == 1.0
    r = float(prob.c_dt)
    L = ell(prob.U, prob.V, prob.W, 1.0, r, hv[1], hv[2])
    eps = prob.eps[vox[:, 2], vox[:, 1], vox[:, 0]]
    chi = chi_of(eps)
    assert np.all(np.delete(prob.eps.ravel(), vox[:, 0] + prob.U * (vox[:, 1] + prob.V * vox[:, 2])) == 1.0), \
        "every voxel with eps_r != 1 must be listed"
    fir = np.asarray(prob.fir, float)
    # kernel values of every ordered pair and lag: offsets r_m - r_m' in voxel steps
    D = (vox[:, None, :] - vox[None, :, :]).reshape(-1, 3)
    uniq, inv = np.unique(D, axis=0, return_inverse=True)
    inv = inv.ravel()
    lags = np.repeat(np.arange(L + 1), len(uniq))
    Kv = kernel_list(lags, np.tile(uniq, (L + 1, 1)), ngl, r, hv).reshape(L + 1, len(uniq), 6)
    comp = np.array(COMP)                                   # [b][a] -> stored component
    Z = np.zeros((L + 1, 3, nv, 3, nv))
    for k in range(L + 1):
        Kk = Kv[k][inv].reshape(nv, nv, 6)                  # [m][m'][6]
        ck = tbasis(k) / eps + (fir[k] if k < len(fir) else 0.0)
        for b in range(3):
            for a in range(3):
                Z[k, b, :, a, :] = -chi[:, None] * Kk[:, :, comp[b][a]]
            Z[k, b, np.arange(nv), b, np.arange(nv)] += ck
    Z = Z.reshape(L + 1, 3 * nv, 3 * nv)
    depth = max(L, len(fir) - 1, 1)
    J = np.zeros((n_steps + 1, 3 * nv))
    Z0inv_lu = scipy_lu_factor(Z[0])
    for n in range(1, n_steps + 1):
        P = np.zeros(3 * nv)
        for k in range(1, min(depth, n - 1) + 1):
            if k <= L:
                P += Z[k] @ J[n - k]
            else:   # a FIR tap beyond the kernel's support acts on the voxel's own current
                P += fir[k] * J[n - k]
        E = chi[None, :] * incident_average_voxels(vox, prob.waves[rhs], n, r=r, hv=hv)
        J[n] = scipy_lu_solve(Z0inv_lu, E.ravel() - P)
    return J[1:].reshape(n_steps, 3, nv)


def scipy_lu_factor(A):
    import scipy.linalg as sla
    return sla.lu_factor(A)


def scipy_lu_solve(lu, b):
    import scipy.linalg as sla
    return sla.lu_solve(lu, b)


def conv(K: np.ndarray, Jh: np.ndarray, targets=None) -> np.ndarray:
    """sum_{k=1}^{nlag} K_k (*) J_{n-k}: K[1..nlag] from a table K[0..], Jh[k-1] = J_{n-k}.
    Returns [3][W][V][U], or [3][len(targets)] for a list of voxel indices."""
    nlag = Jh.shape[0]
    _, _, W, V, U = Jh.shape
    Kl = np.ascontiguousarray(K[1:nlag + 1])
    assert Kl.shape[0] == nlag
    Jc = np.ascontiguousarray(Jh, dtype=np.float64)
    if targets is None:
        out = np.zeros((3, W, V, U))
        lib().or_conv(U, V, W, nlag, dptr(Kl), dptr(Jc), None, 0, dptr(out))
        return out
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    out = np.zeros((3, len(t)))
    lib().or_conv(U, V, W, nlag, dptr(Kl), dptr(Jc), t.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                  len(t), dptr(out))
    return out


def conv_pairs(targets, sources, Js: np.ndarray, ngl: int = 16, r: float = 1.0, hv=None) -> np.ndarray:
    """sum_{k=1}^{nlag} sum_s K_k(r_t - r_s) J_{n-k}(s) for integer voxel coordinates
    targets [nt][3], sources [ns][3] and source currents Js[k-1][3][ns] = J_{n-k};
    every kernel value is computed on the spot.  Returns [3][nt]."""
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
    s = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
    J = np.ascontiguousarray(Js, dtype=np.float64)
    out = np.zeros((3, len(t)))
    lib().or_conv_pairs(r, dptr(_edges(hv)), J.shape[0], iptr(t), len(t), iptr(s), len(s), dptr(J), ngl, dptr(out))
    return out


def probe_kernels(probes, sources, kmax: int, ngl: int = 16, r: float = 1.0, hv=None) -> np.ndarray:
    """Kp[p][s][k][6] = K_k(r_p - r_s), k = 0..kmax, for probe points [np][3] (voxel steps per
    axis from the grid corner) and integer source voxels [ns][3] (centres at +1/2): eq:Z tested
    on a virtual voxel centred at the probe."""
    P = np.ascontiguousarray(np.asarray(probes, dtype=np.float64).reshape(-1, 3))
    s = np.ascontiguousarray(np.asarray(sources, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((len(P), len(s), kmax + 1, 6))
    lib().or_probe_kernels(r, dptr(_edges(hv)), int(kmax), dptr(P), len(P), iptr(s), len(s), int(ngl), dptr(out))
    return out


def probe_field(Kp: np.ndarray, J: np.ndarray, sources) -> np.ndarray:
    """Scattered field at the probes, E^s_p(n) = sum_{k=0}^{kmax} sum_s K_k(r_p - r_s) J_{n-k}(s)
    for n = 1..N (eps_0 = 1; J_{n'} = 0 for n' <= 0).  The scattered field of the
    formulation (Sec. 2.1) is -J + S(J); the tested kernel K of eq:Z is S minus its local
    part J, so K alone gives E^s at any test voxel, inside the scatterer or not.
    J[n-1] = J_n with shape [N][3][W][V][U]; returns [N][np][3]."""
    src = np.asarray(sources, dtype=np.int64).reshape(-1, 3)
    Js = J[:, :, src[:, 2], src[:, 1], src[:, 0]]            # [N][3][ns]
    N = J.shape[0]
    kmax = Kp.shape[2] - 1
    # full symmetric 3x3 per (p, s, k)
    Kf = Kp[..., np.array(COMP).ravel()].reshape(Kp.shape[:3] + (3, 3))   # [np][ns][k][b][a]
    E = np.zeros((N, Kp.shape[0], 3))
    for n in range(1, N + 1):
        for k in range(0, min(kmax, n - 1) + 1):
            E[n - 1] += np.einsum("psba,as->pb", Kf[:, :, k], Js[n - 1 - k])
    return E


def history_sum(K: np.ndarray, Jh: np.ndarray, eps: np.ndarray, fir: np.ndarray, ell_: int) -> np.ndarray:
    """P_{n-1} = sum_{k>=1} Z^delta_k J_{n-k} (eq:PnMOT with Sec. 6.1's taps) for a history
    Jh[k-1] = J_{n-k}, k = 1..depth (missing lags count as zero currents):
      P = sum_k c_k J_{n-k} - chi * sum_{k=1}^{ell} K_k (*) J_{n-k}."""
    depth = Jh.shape[0]
    chi = chi_of(eps)
    nl = min(ell_, depth)
    P = -chi[None] * conv(K, Jh[:nl])
    c = local_coefficients(eps, fir, depth)
    for k in range(1, depth + 1):
        P += c[k][None] * Jh[k - 1]
    return P


def z0_matrix(K0: np.ndarray, eps: np.ndarray, fir: np.ndarray) -> sp.csr_matrix:
    """Z^delta_0 as a sparse 3M x 3M matrix in the per-component order (b*M + m):
    rows  c_0(m) J^b(m) - chi_m sum_{m',a} K^{ba}_0(m - m') J^a(m')."""
    W, V, U = eps.shape
    M = U * V * W
    chi = chi_of(eps).ravel()
    c0 = local_coefficients(eps, fir, 0)[0].ravel()
    rows, cols, vals = [], [], []
    idx = np.arange(M).reshape(W, V, U)
    nz, ny, nx = K0.shape[1:]
    for dz in range(-(W - 1), W):
        for dy in range(-(V - 1), V):
            for dx in range(-(U - 1), U):
                kv = K0[:, dz + W - 1, dy + V - 1, dx + U - 1]
                if not np.any(kv):
                    continue
                # target m = source m' + D
                zs = slice(max(0, -dz), W - max(0, dz)); zt = slice(max(0, dz), W - max(0, -dz))
                ys = slice(max(0, -dy), V - max(0, dy)); yt = slice(max(0, dy), V - max(0, -dy))
                xs = slice(max(0, -dx), U - max(0, dx)); xt = slice(max(0, dx), U - max(0, -dx))
                src = idx[zs, ys, xs].ravel()
                tgt = idx[zt, yt, xt].ravel()
                for b in range(3):
                    for a in range(3):
                        v = kv[COMP[b][a]]
                        if v == 0.0:
                            continue
                        rows.append(b * M + tgt)
                        cols.append(a * M + src)
                        vals.append(-chi[tgt] * v)
    for b in range(3):
        rows.append(b * M + np.arange(M))
        cols.append(b * M + np.arange(M))
        vals.append(c0)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(3 * M, 3 * M))
    A.sum_duplicates()
    return A


def problem_edges(prob) -> np.ndarray:
    """Voxel edges (h, hy, hz) of a Problem; hy, hz of 0 (or absent) mean h."""
    hy = getattr(prob, "hy", 0.0) or prob.h
    hz = getattr(prob, "hz", 0.0) or prob.h
    return np.array([prob.h, hy, hz], dtype=np.float64)


class Oracle:
    """Direct MOT-JVIE march for one Problem (workloads.Problem) and one right-hand side."""

    def __init__(self, prob, K=None, ngl: int = 16):
        # lengths in units of the x edge; c dt <= every edge keeps K_0 on the 27 nearest offsets
        assert prob.h == 1.0, "the oracle works in units of h = 1"
        self.r = float(prob.c_dt)
        self.hv = problem_edges(prob)
        assert 0.0 < self.r <= self.hv.min(), "the oracle takes c dt <= every voxel edge"
        self.p = prob
        self.ell = ell(prob.U, prob.V, prob.W, 1.0, self.r, self.hv[1], self.hv[2])
        self.K = kernel_table(prob.U, prob.V, prob.W, self.ell, ngl, self.r, hv=self.hv) if K is None else K
        self.fir = np.asarray(prob.fir, float)
        self.depth = max(self.ell, len(self.fir) - 1, 1)
        self.Z0 = z0_matrix(self.K[0], prob.eps, self.fir).tocsc()
        self.lu = spla.splu(self.Z0)

    def run(self, n_steps: int, rhs: int = 0, return_P: bool = False, excite=None):
        """J_1..J_n for the Problem's plane wave `rhs`, or for excite(n) -> E_n [3][W][V][U]."""
        p = self.p
        W, V, U = p.W, p.V, p.U
        J = np.zeros((n_steps + 1, 3, W, V, U))      # J[0] = 0 (J_{n'} = 0 for n' <= 0)
        Ps = []
        for n in range(1, n_steps + 1):
            lo = max(0, n - self.depth)
            Jh = J[lo:n][::-1]                       # Jh[k-1] = J_{n-k}
            P = history_sum(self.K, np.ascontiguousarray(Jh), p.eps, self.fir, self.ell)
            E = excite(n) if excite is not None else excitation(U, V, W, p.eps, p.waves[rhs], n, r=self.r, hv=self.hv)
            b = (E - P).ravel()
            J[n] = self.lu.solve(b).reshape(3, W, V, U)
            if return_P:
                Ps.append(P)
        if return_P:
            return J[1:], np.array(Ps)
        return J[1:]

    # ------------------------------------------------------------------ adjoint
    def adjoint(self, g: np.ndarray) -> np.ndarray:
        """lambda_1..lambda_N of the transposed march for adjoint sources g[j-1] = g_j:
        the march is the block lower-triangular Toeplitz system sum_k Z_k J_{n-k} = E_n, so
        its transpose runs backward,
            Z_0^T lambda_j = g_j - sum_{k=1}^{ell} Z_k^T lambda_{j+k},
        with Z_k^T = diag(c_k) - K_k (*) (chi .) because every K_k is a symmetric operator
        (K^ab(D) = K^ba(D) = K^ab(-D), reciprocity of eq:Z).  lambda_j = 0 for j > N."""
        p = self.p
        W, V, U = p.W, p.V, p.U
        N = g.shape[0]
        chi = chi_of(p.eps)
        c = local_coefficients(p.eps, self.fir, self.depth)
        lu_t = spla.splu(self.Z0.T.tocsc())
        lam = np.zeros((N + 2 + self.depth, 3, W, V, U))     # lam[j] = lambda_j, zero beyond N
        for j in range(N, 0, -1):
            b = g[j - 1].copy()
            for k in range(1, self.depth + 1):
                if j + k > N:
                    break
                b -= c[k][None] * lam[j + k]
            kk = min(self.ell, N - j)
            if kk >= 1:
                nu = np.ascontiguousarray(np.array([chi[None] * lam[j + k] for k in range(1, kk + 1)]))
                b += conv(self.K[: kk + 1], nu)
            lam[j] = lu_t.solve(b.ravel()).reshape(3, W, V, U)
        return lam[1:N + 1]

    def gradient_terms(self, J: np.ndarray, rhs: int = 0) -> np.ndarray:
        """B_n(m) = <E^i>_m(n) + sum_{k=0}^{ell} (T(k dt) J_{n-k}(m) + (K_k (*) J_{n-k})(m)), the
        factor of lambda_n(m) / eps_m^2 in dPhi/deps_m (derivative of eq:Z and eq:E in eps:
        d c_k/d eps = -T(k dt)/eps^2, d chi/d eps = 1/eps^2)."""
        p = self.p
        N = J.shape[0]
        B = np.zeros_like(J)
        K0 = np.ascontiguousarray(np.stack([self.K[0], self.K[0]]))
        for n in range(1, N + 1):
            lo = max(0, n - 1 - self.ell)
            Jh = np.ascontiguousarray(J[lo:n - 1][::-1])          # Jh[k-1] = J_{n-k}, k >= 1
            Bn = incident_average(p.U, p.V, p.W, p.waves[rhs], n, r=self.r, hv=self.hv)
            Bn = Bn + tbasis(0) * J[n - 1] + conv(K0, np.ascontiguousarray(J[n - 1:n]))
            if n >= 2:
                Bn = Bn + tbasis(1) * J[n - 2]
                Bn = Bn + conv(self.K[: len(Jh) + 1], Jh)
            B[n - 1] = Bn
        return B

    def probe_objective_gradient(self, n_steps: int, probes, rhs: int = 0):
        """Phi = sum_n sum_p |E^s_p(n)|^2 over the march and dPhi/deps_m for every voxel,
        by the discrete adjoint: g_j = dPhi/dJ_j = 2 sum_k sum_p K_k(r_p - r_m) E^s_p(j+k),
        lambda from adjoint(), dPhi/deps_m = sum_n lambda_n(m) . B_n(m) / eps_m^2.
        Returns (Phi, grad[W][V][U], E^s[N][np][3])."""
        p = self.p
        W, V, U = p.W, p.V, p.U
        J = self.run(n_steps, rhs)
        src = [(u, v, w) for w in range(W) for v in range(V) for u in range(U)]
        Kp = probe_kernels(probes, src, self.ell, r=self.r, hv=self.hv)
        E = probe_field(Kp, J, src)
        phi = float((E ** 2).sum())
        Kf = Kp[..., np.array(COMP).ravel()].reshape(Kp.shape[:3] + (3, 3))   # [np][M][k][b][a]
        N = n_steps
        g = np.zeros((N, 3, W, V, U))
        for j in range(1, N + 1):
            acc = np.zeros((3, len(src)))
            for k in range(0, min(self.ell, N - j) + 1):
                acc += 2.0 * np.einsum("pmba,pb->am", Kf[:, :, k], E[j + k - 1])
            g[j - 1] = acc.reshape(3, W, V, U)
        lam = self.adjoint(g)
        B = self.gradient_terms(J, rhs)
        grad = (lam * B).sum(axis=(0, 1)) / p.eps ** 2
        return phi, grad, E

