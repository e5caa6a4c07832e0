"""Stability of the regularised march (Sec. 6): the companion matrix of the MOT recursion on a
3^3 cube, assembled from the oracle's operators, and its spectral radius for the FIR filters
used here and printed in the paper.

Sec. 6.1 asks three things of the taps delta_n: they add delta at theta = pi (eq:RegReq1), they
keep the other frequencies nearly unchanged, and they move no eigenvalue with argument theta < pi
out of the unit circle.  These tests pin the reading of delta for the 17-tap binomial filter of
the workloads: 0.01 pulls the alternating mode (theta = pi) inward; 0.1 pushes a mode with
theta < pi outward (the third requirement fails), which the oracle's own march confirms."""
import numpy as np
import pytest

import workloads as wl

U = 3


@pytest.fixture(scope="module")
def kernels():
    from oracle import mot
    return mot.kernel_table(U, U, U, mot.ell(U, U, U))


def z_matrices(eps_r, fir, K):
    """Dense Z^delta_k, k = 0..L (L = max(ell, taps - 1)), of a homogeneous U^3 cube:
    Z_k J = c_k J - chi K_k (*) J with c_k = T(k dt)/eps + delta_k (eq:Z, Sec. 6.1), the
    convolution taken column by column with the oracle's direct sum; Z_0 from the oracle."""
    from oracle import mot
    eps = np.full((U, U, U), eps_r)
    chi = (eps - 1.0) / eps
    ell = mot.ell(U, U, U)
    fir = np.asarray(fir, float)
    L = max(ell, len(fir) - 1)
    c = mot.local_coefficients(eps, fir, L)
    n = 3 * U ** 3
    Z = [mot.z0_matrix(K[0], eps, fir).toarray()]
    for k in range(1, L + 1):
        Zk = np.diag(np.tile(c[k].ravel(), 3))
        if k <= ell:
            for j in range(n):
                Jh = np.zeros((k, n))
                Jh[k - 1, j] = 1.0
                Zk[:, j] -= (chi[None] * mot.conv(K, Jh.reshape(k, 3, U, U, U))).ravel()
        Z.append(Zk)
    return Z


def dominant_eigenvalue(Z):
    """Largest-modulus eigenvalue of the companion matrix of Z_0 J_n = -sum_k Z_k J_{n-k}."""
    L, n = len(Z) - 1, Z[0].shape[0]
    Zi = np.linalg.inv(Z[0])
    C = np.zeros((n * L, n * L))
    for k in range(1, L + 1):
        C[:n, (k - 1) * n:k * n] = -Zi @ Z[k]
    C[n:, :-n] = np.eye(n * (L - 1))
    ev = np.linalg.eigvals(C)
    return ev[np.argmax(np.abs(ev))]


def test_unregularised_alternating_mode_is_marginal(kernels):
    """Without a filter the dominant mode is the per-step alternating one (theta = pi), just
    inside the unit circle: the margin that element errors eat away (Sec. 6)."""
    lam = dominant_eigenvalue(z_matrices(12.0, np.zeros(17), kernels))
    assert abs(abs(np.angle(lam)) - np.pi) < 1e-6
    assert 0.99 < abs(lam) < 1.0


def test_17_taps_at_delta_001_pull_the_alternating_mode_in(kernels):
    lam = dominant_eigenvalue(z_matrices(12.0, wl.binomial_highpass(17, 0.01), kernels))
    assert abs(lam) < 0.99
    assert abs(abs(np.angle(lam)) - np.pi) < 1e-6


def test_17_taps_at_delta_01_fail_the_third_requirement(kernels):
    """The 17-tap filter (group delay 8 steps) at delta = 0.1 pushes a mode with theta < pi out
    of the unit circle."""
    lam = dominant_eigenvalue(z_matrices(12.0, wl.binomial_highpass(17, 0.1), kernels))
    assert abs(lam) > 1.001
    assert abs(np.angle(lam)) < np.pi - 0.1


@pytest.mark.parametrize("name", ["FIR2", "FIR3"])
def test_paper_filters_at_delta_01_are_stable(kernels, name):
    """eq:FIR2 and eq:FIR3 at delta = 0.1 (their low group delay meets the third requirement)."""
    import os
    taps = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "fir_taps_paper.txt")):
        if line.strip() and not line.startswith("#"):
            parts = line.split()
            taps[parts[0]] = [float(x) for x in parts[1:]]
    lam = dominant_eigenvalue(z_matrices(12.0, 0.1 * np.array(taps[name]), kernels))
    assert abs(lam) < 1.0


def test_companion_growth_rate_matches_the_oracle_march(kernels):
    """The dominant eigenvalue predicts the oracle's own march (direct sums and a sparse LU of
    Z_0, a separate code path): with delta = 0.1 the current grows by |lambda| per step."""
    from oracle import mot
    fir = wl.binomial_highpass(17, 0.1)
    lam = dominant_eigenvalue(z_matrices(12.0, fir, kernels))
    N = 2400
    prob = wl.homogeneous_cube(U, 12.0, N, 2.0, fir=fir)
    J = mot.Oracle(prob, K=kernels).run(N)
    nrm = np.linalg.norm(J.reshape(N, -1), axis=1)
    # envelope over windows longer than the oscillation period 2 pi / theta
    env = np.array([nrm[i:i + 50].max() for i in range(N - 600, N - 50, 50)])
    rate = np.exp(np.polyfit(np.arange(len(env)) * 50.0, np.log(env), 1)[0])
    assert abs(rate - abs(lam)) < 2e-4 * abs(lam), (rate, abs(lam))


def test_pdsa_regularisation_shifts_D_L_by_delta(kernels):
    """eq:Regularization: the taps add delta I to D_L = sum_j (-1)^j Z_j (eq:RegReq1), so with the
    rows scaled by 1/chi its smallest eigenvalue moves by exactly delta/chi; every D_n stays
    positive definite here, although delta = 0.1 is unstable (a theta < pi mode, above)."""
    from paper_2407_03323_amd import stability as st
    chi = 11.0 / 12.0
    m0 = st.pdsa_minima([z / chi for z in z_matrices(12.0, np.zeros(17), kernels)])
    for delta in (0.01, 0.1):
        m = st.pdsa_minima([z / chi for z in z_matrices(12.0, wl.binomial_highpass(17, delta), kernels)])
        assert abs((m[-1] - m0[-1]) - delta / chi) < 1e-12
        assert (m > 0).all()
