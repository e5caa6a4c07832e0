"""Frequency-domain view of a march (Sec. 7.1, eq:Halpha), on the host.

Time and frequency are measured in the length unit of the grid: a sample n sits at c t = n c dt,
and a frequency f counts cycles per unit of c t (multiply by c over the length unit for Hz).

* `tapered_cosine_window`: ones, with the last `fraction` of the samples rolled off by a
  half cosine, the taper Sec. 7.1 applies to a record that ends before the response has died out.
* `gaussian_pulse_spectrum`: |e^i(f)| of amp exp(-((c t - c t0) / width)^2), in closed form.
* `march_spectrum`: the Fourier transform of J(t) = sum_n J_n T(t - n dt) at f, with T the
  causal quadratic B-spline of the march (its transform has modulus dt |sinc(f dt)|^3).
* `magnitude_response`: |H^alpha|(f) = |alpha . j(f)| / ((eps_r - 1) |e^i(f)|) (eq:Halpha with
  eps_0 = 1), for each component of a sampled current.
"""
from __future__ import annotations

import numpy as np


def tapered_cosine_window(n: int, fraction: float = 0.2) -> np.ndarray:
    """w[i] = 1 for i < n0 and 0.5 (1 + cos(pi (i - n0 + 1) / (n - n0 + 1))) from n0 = n - round(fraction n)
    on, so the last sample is small but the window never jumps."""
    w = np.ones(n)
    nt = int(round(fraction * n))
    if nt > 0:
        i = np.arange(nt) + 1
        w[n - nt:] = 0.5 * (1.0 + np.cos(np.pi * i / (nt + 1)))
    return w


def gaussian_pulse_spectrum(f, amp: float, width: float) -> np.ndarray:
    """|Int amp exp(-((s - s0)/width)^2) exp(-2 pi i f s) ds| = amp width sqrt(pi) exp(-(pi f width)^2)."""
    f = np.asarray(f, dtype=float)
    return amp * width * np.sqrt(np.pi) * np.exp(-(np.pi * f * width) ** 2)


def march_spectrum(samples, c_dt: float, f, window=None) -> np.ndarray:
    """Complex spectrum at f of the current represented by the samples J_1..J_N (axis 0) on the
    march's temporal basis: c_dt sinc^3(f c_dt) e^{-2 pi i f c_dt / 2} sum_n w_n J_n e^{-2 pi i f n c_dt}.
    The B-spline T(t) = B(t/dt + 1) is centred at t = dt/2, hence the half-step phase."""
    J = np.asarray(samples, dtype=float)
    n = np.arange(1, J.shape[0] + 1)
    if window is not None:
        J = J * np.asarray(window).reshape((-1,) + (1,) * (J.ndim - 1))
    f = np.atleast_1d(np.asarray(f, dtype=float))
    E = np.exp(-2j * np.pi * np.outer(f, n) * c_dt)             # [nf][N]
    S = np.tensordot(E, J, axes=(1, 0))                        # [nf][...]
    basis = c_dt * np.sinc(f * c_dt) ** 3 * np.exp(-1j * np.pi * f * c_dt)
    return S * basis.reshape((-1,) + (1,) * (S.ndim - 1))


def magnitude_response(samples, c_dt: float, eps_r: float, amp: float, width: float, f,
                       taper: float = 0.2) -> np.ndarray:
    """|H^alpha|(f) for samples [N][3] of one voxel's J: the tapered record's spectrum over
    (eps_r - 1) times the incident pulse's.  Returns [nf][3]."""
    J = np.asarray(samples, dtype=float)
    w = tapered_cosine_window(J.shape[0], taper)
    S = np.abs(march_spectrum(J, c_dt, f, w))
    E = gaussian_pulse_spectrum(f, amp, width)
    return S / ((eps_r - 1.0) * E[:, None])
