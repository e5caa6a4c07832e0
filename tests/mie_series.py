"""Mie series for a homogeneous, non-magnetic dielectric sphere (test reference; the paper
compares its sphere run with this series in Sec. 7.2).  Written from the textbook solution
(Bohren & Huffman, Absorption and Scattering of Light by Small Particles, ch. 4), with time
dependence exp(-i w t), an x-polarised plane wave E0 exp(i k z) x_hat of unit amplitude at the
sphere centre, relative index m = sqrt(eps_r) and size parameter x = k a."""
from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def n_terms(x: float) -> int:
    """Terms kept: the usual x + 4 x^(1/3) + 2, plus a margin."""
    return int(x + 4.0 * x ** (1.0 / 3.0) + 8)


def coefficients(eps_r: float, x: float, nmax: int | None = None):
    """Scattering coefficients a_n, b_n, n = 1..nmax, from the Riccati-Bessel functions
    psi_n(r) = r j_n(r) and xi_n(r) = r h_n(r) (h_n = j_n + i y_n), matching the tangential
    fields on the surface."""
    m = np.sqrt(eps_r)
    nmax = n_terms(x) if nmax is None else nmax
    a = np.zeros(nmax, complex)
    b = np.zeros(nmax, complex)
    for n in range(1, nmax + 1):
        jx, djx = spherical_jn(n, x), spherical_jn(n, x, derivative=True)
        yx, dyx = spherical_yn(n, x), spherical_yn(n, x, derivative=True)
        jm, djm = spherical_jn(n, m * x), spherical_jn(n, m * x, derivative=True)
        psi, dpsi = x * jx, jx + x * djx
        psim, dpsim = m * x * jm, jm + m * x * djm
        h, dh = jx + 1j * yx, djx + 1j * dyx
        xi, dxi = x * h, h + x * dh
        a[n - 1] = (m * psim * dpsi - psi * dpsim) / (m * psim * dxi - xi * dpsim)
        b[n - 1] = (psim * dpsi - m * psi * dpsim) / (psim * dxi - m * xi * dpsim)
    return a, b


def forward_amplitude(eps_r: float, x: float) -> complex:
    """S(0) = sum_n (2n + 1)/2 (a_n + b_n)."""
    a, b = coefficients(eps_r, x)
    n = np.arange(1, len(a) + 1)
    return complex(np.sum((2 * n + 1) / 2.0 * (a + b)))


def axis_field(eps_r: float, radius: float, k: float, r: float) -> complex:
    """x component of the scattered field at distance r > radius on the +z axis (the forward
    direction), per unit incident amplitude at the centre.  On the axis the angular functions
    are pi_n = tau_n = n (n + 1)/2, so the expansion sum_n E_n (i a_n N_e1n - b_n M_o1n) with
    E_n = i^n (2n + 1)/(n (n + 1)) reduces to
        sum_n i^n (2n + 1)/2 [i a_n (rho h_n(rho))'/rho - b_n h_n(rho)],   rho = k r."""
    a, b = coefficients(eps_r, k * radius)
    rho = k * r
    tot = 0j
    for n in range(1, len(a) + 1):
        h = spherical_jn(n, rho) + 1j * spherical_yn(n, rho)
        dh = spherical_jn(n, rho, derivative=True) + 1j * spherical_yn(n, rho, derivative=True)
        tot += (1j) ** n * (2 * n + 1) / 2.0 * (1j * a[n - 1] * (h + rho * dh) / rho - b[n - 1] * h)
    return tot


def internal_coefficients(eps_r: float, x: float, nmax: int | None = None):
    """Internal-field coefficients c_n, d_n, n = 1..nmax (the field inside is
    sum_n E_n (c_n M_o1n - i d_n N_e1n) with j_n(m k r) radial functions), from the same
    tangential-field matching as coefficients(), non-magnetic sphere:
        c_n = [j_n(x) xi_n'(x) - h_n(x) psi_n'(x)] / [j_n(mx) xi_n'(x) - h_n(x) psi_n'(mx)]
        d_n = m [j_n(x) xi_n'(x) - h_n(x) psi_n'(x)] / [m^2 j_n(mx) xi_n'(x) - h_n(x) psi_n'(mx)]
    with psi_n(r) = r j_n(r), xi_n(r) = r h_n(r) and ' the derivative in r."""
    m = np.sqrt(eps_r)
    nmax = n_terms(x) if nmax is None else nmax
    c = np.zeros(nmax, complex)
    d = np.zeros(nmax, complex)
    for n in range(1, nmax + 1):
        jx, djx = spherical_jn(n, x), spherical_jn(n, x, derivative=True)
        yx, dyx = spherical_yn(n, x), spherical_yn(n, x, derivative=True)
        jm, djm = spherical_jn(n, m * x), spherical_jn(n, m * x, derivative=True)
        dpsi = jx + x * djx
        dpsim = jm + m * x * djm
        h, dh = jx + 1j * yx, djx + 1j * dyx
        dxi = h + x * dh
        num = jx * dxi - h * dpsi
        c[n - 1] = num / (jm * dxi - h * dpsim)
        d[n - 1] = m * num / (m * m * jm * dxi - h * dpsim)
    return c, d


def centre_field(eps_r: float, x: float) -> complex:
    """Field at the sphere's centre per unit incident amplitude, along the polarisation: only the
    n = 1 electric term is non-zero there, and N_e11(0) = (2/3) x_hat with E_1 = 3i/2, so the
    field is d_1 (the static limit 3/(eps_r + 2) is the Clausius-Mossotti factor)."""
    _, d = internal_coefficients(eps_r, x, 1)
    return complex(d[0])
