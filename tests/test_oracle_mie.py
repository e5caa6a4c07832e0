"""The oracle against the physics of a homogeneous sphere: the time-domain march of a
voxelised dielectric sphere, its scattered field at a probe on the forward axis taken to the
frequency domain, against the Mie series (the paper makes the same comparison in Sec. 7.2).
The series itself is pinned first by identities it must satisfy."""
import numpy as np
import pytest

import mie_series as mie


# ----------------------------------------------------------------------------- the series
@pytest.mark.parametrize("eps_r,x", [(4.0, 0.3), (4.0, 1.5), (12.0, 0.8), (100.0, 0.4), (2.25, 5.0)])
def test_mie_optical_theorem(eps_r, x):
    """A lossless sphere absorbs nothing: extinction (forward amplitude) equals scattering,
    sum (2n+1) Re(a_n + b_n) = sum (2n+1) (|a_n|^2 + |b_n|^2)."""
    a, b = mie.coefficients(eps_r, x)
    n = np.arange(1, len(a) + 1)
    ext = np.sum((2 * n + 1) * (a + b).real)
    sca = np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    assert abs(ext - sca) <= 1e-10 * sca


def test_mie_no_contrast_scatters_nothing():
    a, b = mie.coefficients(1.0, 2.0)
    assert np.abs(a).max() < 1e-14 and np.abs(b).max() < 1e-14


@pytest.mark.parametrize("eps_r", [4.0, 12.0])
def test_mie_static_limit_is_the_clausius_mossotti_dipole(eps_r):
    """k -> 0: a sphere of radius a in a uniform field is a dipole p = 4 pi a^3 (eps-1)/(eps+2)
    along x; on the z axis its field is -p / (4 pi r^3) x_hat (the series departs from it
    linearly in k r)."""
    a_, r = 1.0, 3.0
    E = mie.axis_field(eps_r, a_, 1e-6, r)
    ref = -a_ ** 3 * (eps_r - 1) / (eps_r + 2) / r ** 3
    assert abs(E - ref) <= 1e-6 * abs(ref)


@pytest.mark.parametrize("eps_r,x", [(4.0, 0.7), (12.0, 1.3)])
def test_mie_far_field_is_the_forward_amplitude(eps_r, x):
    """k r -> infinity: E_s -> S(0) exp(i k r) / (-i k r)."""
    k, rho = 1.0, 2e5
    E = mie.axis_field(eps_r, x / k, k, rho / k)
    ref = mie.forward_amplitude(eps_r, x) * np.exp(1j * rho) / (-1j * rho)
    assert abs(E - ref) <= 1e-4 * abs(ref)


# ----------------------------------------------------------------------------- the oracle
def test_oracle_sphere_matches_mie_series():
    """eps_r = 4 sphere of radius 3.5 h voxelised on an 8^3 grid (160 voxels), x-polarised
    Gaussian pulse along +z (sigma = 3 dt), 17-tap FIR (delta = 0.01), 256 steps.  The scattered field at
    30 h on the forward axis (oracle probe operator), transformed, over the incident field at the
    centre, against the series for the sphere of equal volume.  Up to k a = 1 the staircase
    costs a few percent (1-3 % seen); a wrong factor or sign anywhere in the chain costs far
    more.  The cross-polarised component vanishes by symmetry."""
    import workloads as wl
    from conftest import oracle_kernel_table
    from oracle import mot
    U, R0, eps_r, N, dist = 8, 3.5, 4.0, 256, 30.0
    c = U / 2.0
    X, Y, Z = wl.voxel_centres(U, U, U)
    inside = (X - c) ** 2 + (Y - c) ** 2 + (Z - c) ** 2 <= R0 ** 2
    eps = np.where(inside, eps_r, 1.0)
    a_eq = (3.0 * inside.sum() / (4.0 * np.pi)) ** (1.0 / 3.0)
    wave = wl.gaussian_wave(U, U, U, (0, 0, 1), (1, 0, 0), 3.0)
    prob = wl.Problem("sphere", U, U, U, eps, [wave], N, fir=wl.binomial_highpass(17, wl.FIR17_DELTA))
    J = mot.Oracle(prob, K=oracle_kernel_table(U, U, U, mot.ell(U, U, U))).run(N)
    src = np.argwhere(inside)[:, ::-1]
    probe = np.array([[c, c, c + dist]])
    kmax = int(np.ceil(dist + np.sqrt(3.0) * R0)) + 3
    E = mot.probe_field(mot.probe_kernels(probe, src, kmax), J, src)[:, 0, :]
    n = np.arange(1, N + 1)
    Ei = wave.amp * np.exp(-((n - (wave.t0 + c - wave.r_ref[2])) / wave.width) ** 2)
    assert np.abs(E[-16:]).max() < 1e-4 * np.abs(E).max()     # the record holds the response
    for w in (0.05, 0.1, 0.15, 0.2, 0.25, 0.3):
        ph = np.exp(1j * w * n)
        H = (E[:, 0] * ph).sum() / (Ei * ph).sum()
        Hm = mie.axis_field(eps_r, a_eq, w, dist)
        assert abs(H - Hm) <= 0.05 * abs(Hm), (w, H, Hm)
        assert abs((E[:, 1] * ph).sum()) <= 1e-10 * abs((E[:, 0] * ph).sum())
        assert abs((E[:, 2] * ph).sum()) <= 1e-10 * abs((E[:, 0] * ph).sum())
