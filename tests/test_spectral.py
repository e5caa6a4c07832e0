"""Frequency-domain post-processing (Sec. 7.1, eq:Halpha) and the Mie internal field used to
check it (no GPU)."""
import numpy as np
import pytest
from scipy.special import spherical_jn, spherical_yn

import mie_series as mie
from paper_2407_03323_amd import spectral


def test_tapered_cosine_window():
    w = spectral.tapered_cosine_window(100, 0.2)
    assert np.all(w[:80] == 1.0)
    assert np.all(np.diff(w[79:]) < 0) and 0.0 < w[-1] < 0.01
    assert np.all(spectral.tapered_cosine_window(10, 0.0) == 1.0)


def test_gaussian_pulse_spectrum_against_quadrature():
    amp, width, s0 = 1.7, 3.0, 40.0
    s = np.linspace(0.0, 80.0, 160001)
    g = amp * np.exp(-((s - s0) / width) ** 2)
    for f in (0.0, 0.05, 0.11, 0.2):
        num = abs(np.trapezoid(g * np.exp(-2j * np.pi * f * s), s))
        assert abs(num - spectral.gaussian_pulse_spectrum(f, amp, width)) < 1e-10


def _bspline(x):
    return np.where((x <= 0) | (x >= 3), 0.0,
                    np.where(x < 1, 0.5 * x * x, np.where(x < 2, 0.5 * (-2 * x * x + 6 * x - 3), 0.5 * (3 - x) ** 2)))


@pytest.mark.parametrize("c_dt", [1.0, 0.5])
def test_march_spectrum_is_the_transform_of_the_spline_expansion(c_dt):
    """The spectrum of sum_n J_n T(t - n dt), T(t) = B(t/dt + 1), evaluated on a fine grid and
    integrated numerically, against the closed form (basis factor and half-step phase)."""
    rng = np.random.default_rng(5)
    N = 40
    J = rng.standard_normal(N)
    t = np.linspace(-2.0 * c_dt, (N + 3) * c_dt, 200001)
    Jt = sum(J[n - 1] * _bspline(t / c_dt - n + 1.0) for n in range(1, N + 1))
    for f in (0.0, 0.03, 0.17, 0.4):
        num = np.trapezoid(Jt * np.exp(-2j * np.pi * f * t), t)
        got = spectral.march_spectrum(J, c_dt, f)[0]
        assert abs(num - got) < 1e-8 * max(1.0, abs(num))


def test_magnitude_response_finds_a_damped_resonance():
    c_dt, f0, tau = 1.0, 0.0123, 4000.0
    n = np.arange(1, 40001)
    J = np.stack([np.exp(-n / tau) * np.sin(2 * np.pi * f0 * n), 0 * n, 0 * n], axis=1)
    f = np.linspace(0.005, 0.02, 3001)
    H = spectral.magnitude_response(J, c_dt, 5.0, 1.0, 10.0, f)
    assert abs(f[np.argmax(H[:, 0])] - f0) < 1e-5
    assert np.all(H[:, 1:] == 0.0)


@pytest.mark.parametrize("eps_r,x", [(4.0, 0.3), (100.0, 0.2), (100.0, 0.45), (12.0, 1.3)])
def test_internal_coefficients_match_the_boundary_conditions(eps_r, x):
    """Tangential E across the surface (Bohren & Huffman 4.52, non-magnetic):
    j_n(mx) c_n + h_n(x) b_n = j_n(x) and m j_n(mx) d_n + h_n(x) a_n = j_n(x)."""
    m = np.sqrt(eps_r)
    a, b = mie.coefficients(eps_r, x)
    c, d = mie.internal_coefficients(eps_r, x, len(a))
    for n in range(1, len(a) + 1):
        jx, jm = spherical_jn(n, x), spherical_jn(n, m * x)
        h = jx + 1j * spherical_yn(n, x)
        assert abs(jm * c[n - 1] + h * b[n - 1] - jx) < 1e-10 * max(1.0, abs(jx))
        assert abs(m * jm * d[n - 1] + h * a[n - 1] - jx) < 1e-10 * max(1.0, abs(jx))


@pytest.mark.parametrize("eps_r", [4.0, 100.0])
def test_centre_field_static_limit(eps_r):
    assert abs(mie.centre_field(eps_r, 1e-5) - 3.0 / (eps_r + 2.0)) < 1e-8
