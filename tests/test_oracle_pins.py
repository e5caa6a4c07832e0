"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test compares the oracle with something other than itself: closed forms (Newell's
demagnetising tensor, erf voxel averages, Clausius-Mossotti, B-spline identities),
independent quadratures of smooth integrands, brute-force nested quadrature, library
routines (numpy/scipy), invariants (symmetry, support, trace) and the paper's printed
taps.
"""
import os
from math import comb, erf, pi, sqrt

import numpy as np
import pytest
from scipy.integrate import quad

import pins
import workloads as wl
from oracle import lib, mot

RNG = np.random.default_rng(12345)


# ----------------------------------------------------------------------------- basics
def test_gauss_legendre_matches_library():
    import ctypes
    for n in (4, 8, 16, 24):
        x = np.zeros(n)
        w = np.zeros(n)
        lib().or_gauss_legendre(n, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        xr, wr = np.polynomial.legendre.leggauss(n)
        assert np.abs(np.sort(x) - xr).max() < 1e-15
        assert np.abs(w[np.argsort(x)] - wr).max() < 1e-15


def test_bspline_identities():
    """Causal quadratic B-spline basis: partition of unity and the closed-form moments
    sum_k k T(k - s) = s + 1/2, sum_k k^2 T(k - s) = s^2 + s + 1/2 (s = R / (c dt))."""
    for s in RNG.uniform(0.0, 50.0, 40):
        ks = np.arange(0, 60)
        T = np.array([mot.tbasis(k - s) for k in ks])
        assert abs(T.sum() - 1.0) < 1e-14
        assert abs((ks * T).sum() - (s + 0.5)) < 1e-12
        assert abs((ks ** 2 * T).sum() - (s * s + s + 0.5)) < 1e-10
    assert mot.tbasis(0.0) == 0.5 and mot.tbasis(1.0) == 0.5
    assert mot.tbasis(-1.0) == 0.0 and mot.tbasis(2.0) == 0.0
    assert abs(mot.tbasis(0.5) - 0.75) < 1e-16


def test_ell_formula():
    """eq:Ell for the grids used here."""
    assert mot.ell(8, 8, 8) == 15
    assert mot.ell(32, 32, 32) == 57
    assert mot.ell(48, 48, 48) == 85
    assert mot.ell(64, 64, 64) == 112
    assert mot.ell(104, 104, 104) == 182
    assert mot.ell(3, 4, 12) == 15          # diagonal exactly 13
    assert mot.ell(1, 1, 1) == 3


# ----------------------------------------------------------------------------- kernels
NEAR = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (1, 1, 1), (2, 1, 0), (2, 2, 1),
        (-1, 2, 0), (3, 1, -2), (2, -2, 2)]
FAR = [(3, 2, 2), (5, 3, 2), (-6, 0, 0), (10, 4, 3), (4, -7, 5), (12, 12, 2)]


def lag_window(D):
    a = sum(max(abs(d) - 1, 0) ** 2 for d in D) ** 0.5
    b = sum((abs(d) + 1) ** 2 for d in D) ** 0.5
    return a, b


def kernel_lags(D, extra=2):
    """All lags 0..kmax computed (no support shortcut), with kmax past the window."""
    _, b = lag_window(D)
    kmax = int(np.floor(b)) + 2 + extra
    return np.array([mot.kernel_entry(k, D) for k in range(kmax + 1)])


@pytest.mark.parametrize("D", NEAR)
def test_static_sum_equals_newell(D):
    """sum_k K_k(D) = -N(D): the partition of unity of T turns the lag sum into the static
    kernel, the demagnetising tensor of two cubes (Newell, Williams & Dunlop 1993)."""
    Ks = kernel_lags(D)
    N = pins.newell_tensor(D)
    assert np.abs(Ks.sum(0) + N).max() < 2e-14


@pytest.mark.parametrize("D", FAR)
def test_static_sum_far_field(D):
    """Same identity, referenced by tensor Gauss-Legendre of d_a d_b (1/4 pi R) over Lam."""
    Ks = kernel_lags(D)
    ref = pins.overlap_gl(D, pins.static_second_derivative)     # = -N(D)
    scale = np.abs(Ks).max()
    assert np.abs(Ks.sum(0) - ref).max() < 1e-11 * scale


@pytest.mark.parametrize("D", NEAR[:6] + FAR[:3])
def test_first_moment(D):
    """sum_k k K_k = (1/2) sum_k K_k (from sum_k k T(k - s) = s + 1/2 and Int d_a d_b Lam = 0)."""
    Ks = kernel_lags(D)
    k = np.arange(len(Ks))[:, None]
    assert np.abs((k * Ks).sum(0) - 0.5 * Ks.sum(0)).max() < 1e-11 * np.abs(Ks).max()


@pytest.mark.parametrize("D", FAR)
def test_second_moment_far_field(D):
    """sum_k k^2 K_k = -N/2 - Int (d_ab + dhat_a dhat_b)/(4 pi R) Lam(d - D) dd; this pins the
    time-derivative (gbar) term, which drops out of the two identities above."""
    Ks = kernel_lags(D)
    k = np.arange(len(Ks))[:, None]
    static = pins.overlap_gl(D, pins.static_second_derivative)     # = sum_k K_k = -N(D)
    ref = 0.5 * static - pins.overlap_gl(D, pins.second_moment_integrand)
    assert np.abs((k ** 2 * Ks).sum(0) - ref).max() < 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("D", NEAR + FAR[:2])
def test_trace_identity(D):
    """tr sum_k K_k(D) = -delta_{D,0} (the Laplacian of 1/(4 pi R) is -delta)."""
    Ks = kernel_lags(D)
    tr = Ks.sum(0)[:3].sum()
    want = -1.0 if D == (0, 0, 0) else 0.0
    assert abs(tr - want) < 1e-13


def test_symmetries():
    """Reciprocity and parity: K^aa even in every D_i, K^ab odd in D_a and D_b and even in
    the third; an axis permutation permutes the components.  Checked on integer and
    non-integer (probe-like) offsets without any symmetry used in the oracle."""
    cases = [(2, 1, 0, 4), (3, -2, 1, 5), (1, 1, 1, 2), (2.3, -1.7, 4.1, 6), (-5.5, 2.25, 0.4, 7)]
    for Dx, Dy, Dz, k in cases:
        K = mot.kernel_entry(k, (Dx, Dy, Dz))
        for sx in (-1, 1):
            for sy in (-1, 1):
                for sz in (-1, 1):
                    Kf = mot.kernel_entry(k, (sx * Dx, sy * Dy, sz * Dz))
                    want = K * np.array([1, 1, 1, sx * sy, sx * sz, sy * sz])
                    assert np.abs(Kf - want).max() < 1e-14 * max(1e-3, np.abs(K).max()) + 1e-17
        # swap x <-> y: xx<->yy, xz<->yz
        Kp = mot.kernel_entry(k, (Dy, Dx, Dz))
        want = K[[1, 0, 2, 3, 5, 4]]
        assert np.abs(Kp - want).max() < 1e-13 * np.abs(K).max() + 1e-17
        # cyclic x -> y -> z -> x
        Kc = mot.kernel_entry(k, (Dz, Dx, Dy))
        want = K[[2, 0, 1, 4, 5, 3]]
        assert np.abs(Kc - want).max() < 1e-13 * np.abs(K).max() + 1e-17


def test_support_and_stencil():
    """Causality/Huygens support (eq:Ell of Sec. 2.3; the leading zero blocks of Sec. 5.1): K_k(D) vanishes unless the lag window
    (k-2, k+1) c dt meets the distances between the two voxels; K_0 is the 27-point
    stencil when c dt = h; eq:Ell is the last lag reached by the farthest pair."""
    for D in [(0, 0, 0), (1, 1, 1), (2, 0, 0), (3, 2, 1), (7, 7, 7)]:
        Ks = kernel_lags(D, extra=3)
        a, b = lag_window(D)
        scale = np.abs(Ks).max()
        for k in range(len(Ks)):
            active = (k + 1 > a) and (k - 2 < b)
            if not active:
                assert np.abs(Ks[k]).max() < 1e-13 * scale + 1e-15
            else:
                assert np.abs(Ks[k]).max() > 1e-9 * scale or (k + 1 - a) < 1e-2 or (b - (k - 2)) < 0.5
    # K_0 non-zero exactly on the 27-point stencil
    for D in [(1, 1, 1), (1, 0, 1), (0, 0, 0)]:
        assert np.abs(mot.kernel_entry(0, D)).max() > 1e-3
    for D in [(2, 0, 0), (2, 1, 1), (0, 2, 2)]:
        assert np.abs(mot.kernel_entry(0, D)).max() < 1e-15
    # farthest pair of an 8^3 grid reaches exactly lag ell = 15
    Dfar = (7, 7, 7)
    assert np.abs(mot.kernel_entry(15, Dfar)).max() > 1e-8
    assert np.abs(mot.kernel_entry(16, Dfar)).max() < 1e-15


# brute force: nested adaptive quadrature, innermost split exactly at the knot spheres
_gx, _gw = np.polynomial.legendre.leggauss(24)


def _bs(x):
    return np.where((x <= 0) | (x >= 3), 0.0,
                    np.where(x < 1, 0.5 * x * x, np.where(x < 2, 0.5 * (-2 * x * x + 6 * x - 3), 0.5 * (3 - x) ** 2)))


def _bs2(x):
    return np.where((x <= 0) | (x >= 3), 0.0, np.where(x < 1, 1.0, np.where(x < 2, -2.0, 1.0)))


def _inner(fun, lo, hi, knots, x, y):
    pts = [lo, hi]
    for R in knots:
        q = R * R - x * x - y * y
        if q > 0:
            for t in (sqrt(q), -sqrt(q)):
                if lo < t < hi:
                    pts.append(t)
    pts.sort()
    tot = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        z = 0.5 * (a + b) + 0.5 * (b - a) * _gx
        tot += 0.5 * (b - a) * np.sum(_gw * fun(x, y, z))
    return tot


@pytest.mark.slow
@pytest.mark.parametrize("k,D,s,which", [(3, (2, 1, 0), (1, -1, 1), 0), (5, (3, 2, 1), (-1, 1, 1), 1),
                                         (7, (6, 0, 0), (1, 1, -1), 0)])
def test_brute_force_box_integrals(k, D, s, which):
    """Cube integrals (gbar * Lam, and g * lam' lam' lam for xy) against nested adaptive
    quadrature in Cartesian coordinates."""
    lo = [D[i] if s[i] > 0 else D[i] - 1 for i in range(3)]
    hi = [v + 1 for v in lo]
    knots = [k - 2, k - 1, k, k + 1]

    def f(x, y, z):
        R = np.sqrt(x * x + y * y + z * z)
        l0, l1, l2 = 1 - s[0] * (x - D[0]), 1 - s[1] * (y - D[1]), 1 - s[2] * (z - D[2])
        if which == 0:
            return _bs2(k + 1 - R) / (4 * pi * R) * l0 * l1 * l2
        return _bs(k + 1 - R) / (4 * pi * R) * s[0] * s[1] * l2

    def mid(x):
        return quad(lambda y: _inner(f, lo[2], hi[2], knots, x, y), lo[1], hi[1],
                    epsabs=1e-15, epsrel=1e-12, limit=100)[0]

    ref = quad(mid, lo[0], hi[0], epsabs=1e-15, epsrel=1e-12, limit=100)[0]
    out = np.zeros(4)
    lib().or_box_integrals(1.0, k, float(D[0]), float(D[1]), float(D[2]), s[0], s[1], s[2], 16,
                           out.ctypes.data_as(__import__("ctypes").POINTER(__import__("ctypes").c_double)))
    got = out[0] if which == 0 else out[1]
    assert abs(got - ref) < 1e-11 * max(abs(ref), 1e-3)


@pytest.mark.slow
@pytest.mark.parametrize("k,D,a,sp,s1,s2", [(2, (1, 0, 0), 0, 0, 1, -1), (6, (4, 2, 1), 1, -1, 1, 1),
                                            (4, (0, 3, 1), 2, 1, -1, 1)])
def test_brute_force_plane_integrals(k, D, a, sp, s1, s2):
    """Plane terms of K^aa against nested adaptive quadrature."""
    a1, a2 = (a + 1) % 3, (a + 2) % 3
    c = D[a] + sp
    lo1 = D[a1] if s1 > 0 else D[a1] - 1
    lo2 = D[a2] if s2 > 0 else D[a2] - 1
    knots = [k - 2, k - 1, k, k + 1]

    def f(u, v, w):  # u along a1 (outer), w along a2 (inner, vectorised)
        R = np.sqrt(c * c + u * u + w * w)
        return _bs(k + 1 - R) / (4 * pi * R) * (1 - s1 * (u - D[a1])) * (1 - s2 * (w - D[a2]))

    def inner(u):
        # treat c as the "y" of _inner's sphere crossing: R^2 - u^2 - c^2 = w^2
        return _inner(lambda x, y, z: f(x, None, z), lo2, lo2 + 1, knots, u, c)

    ref = quad(inner, lo1, lo1 + 1, epsabs=1e-15, epsrel=1e-12, limit=100)[0]
    got = lib().or_plane_integral(1.0, k, float(D[0]), float(D[1]), float(D[2]), a, sp, s1, s2, 16)
    assert abs(got - ref) < 1e-11 * max(abs(ref), 1e-3)


# ----------------------------------------------------------------------------- excitation
def test_excitation_axis_wave_closed_form():
    """Voxel average of a Gaussian plane wave along +z equals the erf closed form."""
    p = wl.homogeneous_cube(4, 5.0, 10, 4.0)
    wave = p.waves[0]
    chi = 4.0 / 5.0
    for n in (1, 12, 20, 27, 40):
        E = mot.excitation(4, 4, 4, p.eps, wave, n)
        for w in range(4):
            tc = n - wave.t0 - (w + 0.5)
            ref = chi * wave.amp * pins.axis_wave_voxel_average(tc, wave.width)
            assert np.allclose(E[0, w], ref, rtol=1e-13, atol=1e-300)
            assert np.all(E[1:] == 0.0)


def _perp(k, seed_vec):
    """A unit vector orthogonal to k (Gram-Schmidt of seed_vec)."""
    k = np.asarray(k, float)
    v = np.asarray(seed_vec, float) - np.dot(seed_vec, k) * k
    return tuple(v / np.linalg.norm(v))


S2 = sqrt(2.0)
OBLIQUE_CASES = [
    # khat, polarisation seed, voxel edges, c dt, reference point of the pulse (None: the box
    # corner the front reaches first, as the workloads choose it)
    ((0.0, 0.6, 0.8), (1.0, 0.0, 0.0), (1.0, 1.0, 1.0), 1.0, None),
    ((-0.48, 0.6, -0.64), (0.0, 0.0, 1.0), (1.0, 1.0, 1.0), 1.0, None),
    ((-0.5, -0.5, -S2 / 2), (0.5, 0.5, -S2 / 2), (1.0, 0.7, 1.3), 0.7, (0.0, 0.0, 0.0)),   # the paper's sphere
    ((2.0 / 3, -1.0 / 3, 2.0 / 3), (0.0, 1.0, 0.0), (1.0, 0.7, 1.3), 0.7, None),
    ((0.6, 0.0, -0.8), (0.0, 1.0, 1.0), (1.0, 0.7, 1.3), 0.5, None),
]


@pytest.mark.parametrize("case", range(len(OBLIQUE_CASES)))
def test_excitation_oblique_wave_closed_form(case):
    """Voxel average of an obliquely incident Gaussian plane wave (eq:E with a pulse of the
    eq:GaussPlaneWave form) against the exact box average of tests/pins.py: the retarded time
    taken at each voxel's lower corner, the three edge projections khat_i L_i as differences of
    the Gaussian's repeated antiderivatives.  Directions with negative components, one with a
    zero component and the paper's (-1, -1, -sqrt 2)/2; cubic and 1 x 0.7 x 1.3 voxels;
    polarisations along no axis.  Every component of every voxel to 1e-12 of the largest."""
    khat, pseed, hv, r, rref = OBLIQUE_CASES[case]
    U, V, W = 4, 3, 5
    pol = _perp(khat, pseed)
    if rref is None:
        # the box corner with the smallest r.khat
        rref = tuple(0.0 if khat[i] >= 0 else (U, V, W)[i] * hv[i] for i in range(3))
    wave = wl.PlaneWave(khat=khat, pol=pol, width=S2 * 3.0, t0=18.0, amp=1.7, r_ref=rref)
    worst = 0.0
    for n in (4, 19, 27, 33, 41):
        got = mot.incident_average(U, V, W, wave, n, r=r, hv=hv)
        ref = np.zeros_like(got)
        for w in range(W):
            for v in range(V):
                for u in range(U):
                    lo = (u * hv[0], v * hv[1], w * hv[2])
                    tau0 = n * r - wave.t0 - sum((lo[i] - rref[i]) * khat[i] for i in range(3))
                    c = tuple(khat[i] * hv[i] for i in range(3))
                    a = wave.amp * pins.box_wave_average(tau0, c, wave.width)
                    ref[:, w, v, u] = a * np.asarray(pol)
        worst = max(worst, np.abs(got - ref).max() / np.abs(ref).max())
    assert worst <= 1e-12, worst


def test_workload_wave_reference_corner():
    """The workloads' pulse reaches its reference point first: over the box corners,
    min (r - r_ref).khat = 0 for every direction, so every voxel sees the pulse peak at or
    after t0 (the excitation arrives after t = 0, Sec. 2.1)."""
    U, V, W = 5, 4, 3
    for k, p in wl.random_directions(12, 7) + [((-0.5, -0.5, -S2 / 2), (0.5, 0.5, -S2 / 2))]:
        wave = wl.gaussian_wave(U, V, W, k, p, 2.0)
        corners = [np.array([x, y, z], float) for x in (0, U) for y in (0, V) for z in (0, W)]
        proj = [np.dot(c - np.asarray(wave.r_ref), k) for c in corners]
        assert abs(min(proj)) < 1e-12


# ----------------------------------------------------------------------------- FIR
def _paper_taps():
    taps = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "fir_taps_paper.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, *vals = line.split()
            taps[name] = np.array([float(v) for v in vals])
    return taps


def test_fir_taps_against_paper():
    """Binomial high-pass taps reproduce FIR2 and FIR3 (eq:FIR2, eq:FIR3) and satisfy
    eq:RegReq1 with zero DC gain; the printed FIR4 (eq:FIR4) has alternating sum 3/4 delta,
    so its last tap is read as -delta/8 (the binomial order-3 filter)."""
    t = _paper_taps()
    assert np.allclose(wl.binomial_highpass(2, 1.0), t["FIR2"], atol=0)
    assert np.allclose(wl.binomial_highpass(3, 1.0), t["FIR3"], atol=0)
    alt = lambda d: sum((-1) ** k * v for k, v in enumerate(d))
    assert abs(alt(t["FIR4"]) - 0.75) < 1e-15
    b4 = wl.binomial_highpass(4, 1.0)
    assert np.allclose(b4[:3], t["FIR4"][:3]) and b4[3] == -t["FIR4"][3]
    for n in (2, 3, 4, 17):
        d = wl.binomial_highpass(n, 0.1)
        assert abs(alt(d) - 0.1) < 1e-15            # eq:RegReq1
        assert abs(d.sum()) < 1e-15                 # no low-frequency change at theta = 0
        th = np.linspace(0, pi, 50)
        H = np.abs(np.exp(-1j * np.outer(th, np.arange(n))) @ d)
        assert np.allclose(H, 0.1 * np.sin(th / 2) ** (n - 1), atol=1e-15)


# ----------------------------------------------------------------------------- direct sum
def test_conv_against_library_convolution():
    """Direct history convolution equals scipy's full linear convolution restricted to the grid."""
    from scipy.signal import fftconvolve
    U, V, W, nlag = 5, 4, 3, 3
    K = RNG.standard_normal((nlag + 1, 6, 2 * W - 1, 2 * V - 1, 2 * U - 1))
    Jh = RNG.standard_normal((nlag, 3, W, V, U))
    out = mot.conv(K, Jh)
    ref = np.zeros((3, W, V, U))
    for k in range(1, nlag + 1):
        for b in range(3):
            for a in range(3):
                full = fftconvolve(K[k, mot.COMP[b][a]], Jh[k - 1, a])
                ref[b] += full[W - 1:2 * W - 1, V - 1:2 * V - 1, U - 1:2 * U - 1]
    assert np.abs(out - ref).max() < 1e-12
    # the same through the sparse-target path
    t = [0, 7, 59]
    assert np.abs(mot.conv(K, Jh, t) - out.reshape(3, -1)[:, t]).max() < 1e-14


def test_conv_pairs_matches_table_conv():
    U = V = W = 4
    ell = mot.ell(U, V, W)
    K = mot.kernel_table(U, V, W, ell)
    Jh = RNG.standard_normal((ell, 3, W, V, U))
    full = mot.conv(K, Jh)
    src = [(u, v, w) for w in range(W) for v in range(V) for u in range(U)]
    tgt = [(0, 0, 0), (3, 3, 3), (1, 2, 3)]
    Js = Jh.reshape(ell, 3, -1)
    got = mot.conv_pairs(tgt, src, Js)
    for i, (u, v, w) in enumerate(tgt):
        assert np.abs(got[:, i] - full[:, w, v, u]).max() < 1e-14


# ----------------------------------------------------------------------------- march
def _constant_excitation(p, E0):
    chi = mot.chi_of(p.eps)
    E = np.stack([chi * E0[0], chi * E0[1], chi * E0[2]])
    return lambda n: E


@pytest.mark.parametrize("eps", [2.0, 12.0])
def test_one_voxel_clausius_mossotti(eps):
    """One voxel under a constant field: the march settles at J = 3 (eps-1)/(eps+2) E
    (the static Clausius-Mossotti response; sum_k Z_k = 1/eps + chi/3)."""
    p = wl.homogeneous_cube(1, eps, 10, 4.0)
    o = mot.Oracle(p)
    J = o.run(400, excite=_constant_excitation(p, (1.0, 0.0, 0.0)))
    assert abs(J[-1, 0, 0, 0, 0] - 3 * (eps - 1) / (eps + 2)) < 1e-12
    assert np.abs(J[-1, 1:]).max() < 1e-14


@pytest.mark.slow
@pytest.mark.parametrize("use_fir", [False, True])
def test_steady_state_against_newell(use_fir):
    """3^3 heterogeneous block under a uniform field ramped up to a constant: the march settles at
    (I/eps + chi N) J = chi E with N the Newell tensor (the binomial FIR has zero DC gain)."""
    U = 3
    eps = wl.random_eps(U, U, U, 7, 2.0, 6.0)
    p = wl.Problem("ss", U, U, U, eps, [], 10, fir=wl.binomial_highpass(3, 0.1) if use_fir else np.zeros(0))
    o = mot.Oracle(p)
    E0 = np.array([1.0, 0.5, -0.25])
    const = _constant_excitation(p, E0)
    # smooth ramp (rise >> ell dt) that starts from zero to rounding, so the slowly decaying
    # per-step alternating mode (theta = pi) is not excited
    J = o.run(600, excite=lambda n: const(n) * 0.5 * (1.0 + erf((n - 100.0) / 12.0)))
    M = U ** 3
    chi = mot.chi_of(eps).ravel()
    A = np.zeros((3 * M, 3 * M))
    coords = [(u, v, w) for w in range(U) for v in range(U) for u in range(U)]
    for i, ci in enumerate(coords):
        for j, cj in enumerate(coords):
            N = pins.newell_tensor(tuple(ci[t] - cj[t] for t in range(3)))
            for b in range(3):
                for a in range(3):
                    A[b * M + i, a * M + j] += chi[i] * N[mot.COMP[b][a]]
    for b in range(3):
        A[b * M:(b + 1) * M, b * M:(b + 1) * M] += np.diag(1.0 / eps.ravel())
    rhs = np.concatenate([chi * E0[b] for b in range(3)])
    Jinf = np.linalg.solve(A, rhs)
    assert np.abs(J[-1].reshape(-1) - Jinf).max() < 1e-10 * np.abs(Jinf).max()


def test_time_shift_invariance():
    """Delaying the pulse by an integer number of steps delays J exactly (Toeplitz in time)."""
    p = wl.homogeneous_cube(3, 6.0, 80, 3.0)
    p.waves[0].t0 = 30.0          # pulse negligible (< 1e-20) at the first steps
    o = mot.Oracle(p)
    J1 = o.run(80)
    p.waves[0].t0 += 5.0
    J2 = o.run(80)
    assert np.abs(J2[5:] - J1[:-5]).max() < 1e-13 * np.abs(J1).max()
    assert np.abs(J2[:5]).max() < 1e-6 * np.abs(J1).max()


def test_z0_matrix_matches_conv():
    """The assembled Z_0 acts as c_0 J - chi K_0 (*) J."""
    U = 4
    eps = wl.random_eps(U, U, U, 3, 1.0, 9.0)
    K = mot.kernel_table(U, U, U, 1)
    fir = wl.binomial_highpass(3, 0.1)
    Z0 = mot.z0_matrix(K[0], eps, fir)
    J = RNG.standard_normal((3, U, U, U))
    Kshift = np.stack([K[0], K[0]])     # conv() reads lags 1.., so place K_0 at index 1
    ref = mot.local_coefficients(eps, fir, 0)[0][None] * J - mot.chi_of(eps)[None] * mot.conv(Kshift, J[None])
    assert np.abs(Z0 @ J.ravel() - ref.ravel()).max() < 1e-14


@pytest.mark.slow
def test_c1_march_is_stable_and_bounded(c1_oracle):
    p, o, J = c1_oracle
    assert o.ell == 15
    amp = np.abs(J).reshape(len(J), -1).max(1)
    assert amp.max() < 10.0 and amp[-20:].max() < 1e-2 * amp.max()


@pytest.mark.slow
def test_fir17_stabilises_without_distorting():
    """FIR with the 17-tap binomial high-pass (delta = 0.1) on a high-contrast block stays
    bounded over 5 ell steps, and its low-frequency effect on J is small."""
    p0 = wl.homogeneous_cube(4, 12.0, 0, 4.0)
    p1 = wl.homogeneous_cube(4, 12.0, 0, 4.0, fir=wl.binomial_highpass(17, 0.1))
    o0 = mot.Oracle(p0)
    o1 = mot.Oracle(p1, K=o0.K)
    n = 5 * o0.ell + 40
    J0 = o0.run(n)
    J1 = o1.run(n)
    a0 = np.abs(J0).max()
    assert np.abs(J1).max() < 1.5 * a0
    assert np.abs(J1[-10:]).max() < 0.2 * a0
    assert np.abs(J1 - J0).max() < 0.05 * a0


# ----------------------------------------------------------------------------- off-grid offsets
# Probes see the grid from a virtual test voxel at an arbitrary point, so the kernels are
# needed at non-integer offsets D.  The same identities pin them there.
NEAR_REAL = [(1.3, -0.7, 0.45), (2.61, 1.17, -0.38), (0.0, 0.0, 1.75)]
# the virtual voxel overlapping a source voxel off-centre: 1/R is singular inside the
# overlap away from every symmetry plane and the quadrature reaches only ~1e-9 there
OVERLAP_REAL = (0.5, 0.25, 0.0)
FAR_REAL = [(4.37, -2.81, 1.55), (7.2, 3.9, -5.45), (11.5, 0.5, 0.5)]


@pytest.mark.parametrize("D", NEAR_REAL + FAR_REAL[:1])
def test_static_sum_equals_newell_offgrid(D):
    Ks = kernel_lags(D)
    N = pins.newell_tensor(D)
    assert np.abs(Ks.sum(0) + N).max() < 5e-14


@pytest.mark.parametrize("D", FAR_REAL)
def test_static_sum_far_field_offgrid(D):
    Ks = kernel_lags(D)
    ref = pins.overlap_gl(D, pins.static_second_derivative)
    assert np.abs(Ks.sum(0) - ref).max() < 1e-11 * np.abs(Ks).max()


@pytest.mark.parametrize("D", NEAR_REAL + FAR_REAL)
def test_first_moment_offgrid(D):
    Ks = kernel_lags(D)
    k = np.arange(len(Ks))[:, None]
    assert np.abs((k * Ks).sum(0) - 0.5 * Ks.sum(0)).max() < 1e-11 * np.abs(Ks).max()


@pytest.mark.parametrize("D", FAR_REAL)
def test_second_moment_far_field_offgrid(D):
    Ks = kernel_lags(D)
    k = np.arange(len(Ks))[:, None]
    static = pins.overlap_gl(D, pins.static_second_derivative)
    ref = 0.5 * static - pins.overlap_gl(D, pins.second_moment_integrand)
    assert np.abs((k ** 2 * Ks).sum(0) - ref).max() < 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("D", NEAR_REAL + FAR_REAL[:1])
def test_trace_identity_offgrid(D):
    """tr sum_k K_k(D) = -Lam(D): the delta of the Laplacian picks the overlap of the cubes."""
    Ks = kernel_lags(D)
    lam = np.prod([max(1.0 - abs(d), 0.0) for d in D])
    assert abs(Ks.sum(0)[:3].sum() + lam) < 1e-13


def test_offgrid_parity_and_continuity():
    """K^aa is even and K^ab odd in D_a and D_b at any offset; K is continuous in D, so an
    offset 1e-9 from a grid point gives the grid point's values."""
    D = (2.3, -1.4, 0.6)
    for k in range(0, 7):
        K = mot.kernel_entry(k, D)
        Km = mot.kernel_entry(k, (-D[0], D[1], D[2]))
        assert np.allclose(Km, K * np.array([1, 1, 1, -1, -1, 1]), rtol=0, atol=1e-15 * max(1, np.abs(K).max()))
    for k in range(0, 6):
        a = mot.kernel_entry(k, (3, 1, 2))
        b = mot.kernel_entry(k, (3 + 1e-9, 1 - 1e-9, 2 + 1e-9))
        assert np.abs(a - b).max() < 1e-7 * max(np.abs(a).max(), 1e-3)


def test_overlapping_offgrid_reduced_accuracy():
    Ks = kernel_lags(OVERLAP_REAL)
    N = pins.newell_tensor(OVERLAP_REAL)
    assert np.abs(Ks.sum(0) + N).max() < 5e-9 * np.abs(N).max()
    lam = np.prod([max(1.0 - abs(d), 0.0) for d in OVERLAP_REAL])
    assert abs(Ks.sum(0)[:3].sum() + lam) < 5e-9


def test_probe_field_at_voxel_centres_closes_the_march_equation():
    """A probe at the centre of a grid voxel m sees E^s = K (*) J; the march solves
    sum_k c_k J_{n-k} = chi (<E^i> + K (*) J) there (c_k = T(k dt)/eps + delta_k), so
    E^s_m(n) = (1/chi) sum_k c_k J_{n-k}(m) - <E^i>_m(n).  This pins the probe path (centres,
    the k = 0 term, the contraction) against the march itself."""
    U, V, W, n = 4, 4, 3, 30
    eps = wl.random_eps(U, V, W, 8, 2.0, 9.0)
    k, p = wl.XPOL_PLUS_Z
    fir = wl.binomial_highpass(3, 0.1)
    prob = wl.Problem("probe-pin", U, V, W, eps, [wl.gaussian_wave(U, V, W, k, p, 2.0)], n, fir=fir)
    o = mot.Oracle(prob)
    J = o.run(n)
    cells = [(1, 2, 1), (3, 0, 2), (0, 3, 0)]
    probes = [(u + 0.5, v + 0.5, w + 0.5) for u, v, w in cells]
    src = [(u, v, w) for w in range(W) for v in range(V) for u in range(U)]
    Kp = mot.probe_kernels(probes, src, o.ell)
    E = mot.probe_field(Kp, J, src)
    c = mot.local_coefficients(eps, fir, o.ell)
    chi = mot.chi_of(eps)
    err = 0.0
    for n_ in range(1, n + 1):
        Ei = mot.excitation(U, V, W, eps, prob.waves[0], n_)
        for ip, (u, v, w) in enumerate(cells):
            lhs = sum(c[kk][w, v, u] * J[n_ - 1 - kk][:, w, v, u] for kk in range(min(n_, len(c))))
            ref = lhs / chi[w, v, u] - Ei[:, w, v, u] / chi[w, v, u]
            err = max(err, np.abs(E[n_ - 1, ip] - ref).max() / (np.abs(ref).max() + 1e-300))
    assert err < 1e-9


# ----------------------------------------------------------------------------- adjoint
def _adjoint_problem():
    U, V, W, n = 4, 3, 3, 30
    eps = wl.random_eps(U, V, W, 3, 2.0, 9.0)
    k, p = wl.XPOL_PLUS_Z
    prob = wl.Problem("adj", U, V, W, eps, [wl.gaussian_wave(U, V, W, k, p, 2.0)], n,
                      fir=wl.binomial_highpass(3, 0.1))
    return prob, wl.fibonacci_sphere(4, 4.0, (2.0, 1.5, 1.5))


def test_adjoint_dot_product():
    """<lambda, E> = <g, J> for the march Z J = E and its transpose Z^T lambda = g, random
    E and g: the backward recursion is the exact transpose of the forward one."""
    prob, _ = _adjoint_problem()
    o = mot.Oracle(prob)
    N = 25
    rng = np.random.default_rng(11)
    E = rng.standard_normal((N, 3, prob.W, prob.V, prob.U))
    g = rng.standard_normal((N, 3, prob.W, prob.V, prob.U))
    J = o.run(N, excite=lambda n: E[n - 1])
    lam = o.adjoint(g)
    a, b = float((lam * E).sum()), float((g * J).sum())
    assert abs(a - b) < 1e-11 * max(abs(a), abs(b))


def test_adjoint_gradient_matches_finite_differences():
    """dPhi/deps_m of Phi = sum_n sum_p |E^s_p(n)|^2 against central differences (delta 1e-6)
    of the forward march at three voxels."""
    prob, probes = _adjoint_problem()
    o = mot.Oracle(prob)
    n = prob.n_steps
    phi, grad, _ = o.probe_objective_gradient(n, probes)
    src = [(u, v, w) for w in range(prob.W) for v in range(prob.V) for u in range(prob.U)]
    Kp = mot.probe_kernels(probes, src, o.ell)
    for (u, v, w) in [(0, 0, 0), (2, 1, 1), (3, 2, 2)]:
        vals = []
        for sgn in (1.0, -1.0):
            e2 = prob.eps.copy()
            e2[w, v, u] += sgn * 1e-6
            p2 = wl.Problem("adj", prob.U, prob.V, prob.W, e2, prob.waves, n, fir=prob.fir)
            J = mot.Oracle(p2, K=o.K).run(n)
            vals.append(float((mot.probe_field(Kp, J, src) ** 2).sum()))
        fd = (vals[0] - vals[1]) / 2e-6
        assert abs(fd - grad[w, v, u]) < 1e-6 * np.abs(grad).max()


def test_adjoint_gradient_local_form():
    """With the forward equation satisfied, the gradient term reduces to a local one:
    dPhi/deps_m = 1/(eps (eps - 1)) sum_n lambda_n(m) . sum_k (T(k dt) + delta_k) J_{n-k}(m)."""
    prob, probes = _adjoint_problem()
    o = mot.Oracle(prob)
    n = prob.n_steps
    phi, grad, E = o.probe_objective_gradient(n, probes)
    J = o.run(n)
    src = [(u, v, w) for w in range(prob.W) for v in range(prob.V) for u in range(prob.U)]
    Kp = mot.probe_kernels(probes, src, o.ell)
    Kf = Kp[..., np.array(mot.COMP).ravel()].reshape(Kp.shape[:3] + (3, 3))
    g = np.zeros_like(J)
    for j in range(1, n + 1):
        acc = np.zeros((3, len(src)))
        for k in range(0, min(o.ell, n - j) + 1):
            acc += 2.0 * np.einsum("pmba,pb->am", Kf[:, :, k], E[j + k - 1])
        g[j - 1] = acc.reshape(J.shape[1:])
    lam = o.adjoint(g)
    fir = np.asarray(prob.fir)
    loc = np.zeros_like(J)
    for m in range(1, n + 1):
        for k in range(0, min(m, max(3, len(fir)))):
            w_ = mot.tbasis(k) + (fir[k] if k < len(fir) else 0.0)
            loc[m - 1] += w_ * J[m - 1 - k]
    eps = prob.eps
    ref = (lam * loc).sum(axis=(0, 1)) / (eps * (eps - 1.0))
    assert np.abs(ref - grad).max() < 1e-9 * np.abs(grad).max()


# ----------------------------------------------------------------------------- c dt < h
# The same identities at c dt = r h, r < 1: the time basis is a partition of unity at any step,
# so the lag sum is still the static kernel; the moment identities carry the step through
# s = R / (c dt) (sum_k k^2 T(k dt - R/c) = s^2 + s + 1/2 gives the 1/r^2 on the second moment).
SHORT = [0.5, 0.7, 0.3]


def kernel_lags_r(D, r, extra=2):
    _, b = lag_window(D)
    kmax = int(np.floor(b / r)) + 2 + extra
    return np.array([mot.kernel_entry(k, D, r=r) for k in range(kmax + 1)])


@pytest.mark.parametrize("r", SHORT)
@pytest.mark.parametrize("D", [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 1, 0), (3, 1, -2)])
def test_short_step_static_sum_equals_newell(D, r):
    Ks = kernel_lags_r(D, r)
    assert np.abs(Ks.sum(0) + pins.newell_tensor(D)).max() < 5e-14


@pytest.mark.parametrize("r", SHORT[:2])
@pytest.mark.parametrize("D", [(1, 0, 0), (1, 1, 1), (3, 2, 2), (5, 3, 2)])
def test_short_step_first_moment(D, r):
    Ks = kernel_lags_r(D, r)
    k = np.arange(len(Ks))[:, None]
    assert np.abs((k * Ks).sum(0) - 0.5 * Ks.sum(0)).max() < 1e-11 * np.abs(Ks).max()


@pytest.mark.parametrize("r", SHORT[:2])
@pytest.mark.parametrize("D", [(3, 2, 2), (5, 3, 2), (-6, 0, 0)])
def test_short_step_second_moment_far_field(D, r):
    """sum_k k^2 K_k = -N/2 - (1/r^2) Int (d_ab + dhat_a dhat_b)/(4 pi R) Lam(d - D) dd."""
    Ks = kernel_lags_r(D, r)
    k = np.arange(len(Ks))[:, None]
    static = pins.overlap_gl(D, pins.static_second_derivative)
    ref = 0.5 * static - pins.overlap_gl(D, pins.second_moment_integrand) / (r * r)
    assert np.abs((k ** 2 * Ks).sum(0) - ref).max() < 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("r", SHORT)
def test_short_step_support_and_stencil(r):
    """K_k(D) vanishes unless (k - 2, k + 1) r meets [R_min, R_max]; for r <= 1 K_0 stays on the
    27-point stencil; the farthest pair of an 8^3 grid reaches the last lag of eq:Ell."""
    for D in [(0, 0, 0), (1, 1, 1), (2, 0, 0), (3, 2, 1)]:
        Ks = kernel_lags_r(D, r, extra=3)
        a, b = lag_window(D)
        scale = np.abs(Ks).max()
        for k in range(len(Ks)):
            if not ((k + 1) * r > a and (k - 2) * r < b):
                assert np.abs(Ks[k]).max() < 1e-13 * scale + 1e-15
    for D in [(1, 1, 1), (1, 0, 1), (0, 0, 0)]:
        assert np.abs(mot.kernel_entry(0, D, r=r)).max() > 1e-6
    for D in [(2, 0, 0), (2, 1, 1), (0, 2, 2)]:
        assert np.abs(mot.kernel_entry(0, D, r=r)).max() < 1e-15
    L = mot.ell(8, 8, 8, 1.0, r)
    assert L == int(np.floor(8 * sqrt(3) / r)) + 2
    Dfar = (7, 7, 7)
    assert np.abs(mot.kernel_entry(L, Dfar, r=r)).max() > 1e-12
    assert np.abs(mot.kernel_entry(L + 1, Dfar, r=r)).max() < 1e-15


def test_short_step_excitation_axis_wave_closed_form():
    """c n dt = n r in the retarded time of the voxel average."""
    r = 0.5
    p = wl.homogeneous_cube(4, 5.0, 10, 4.0)
    wave = p.waves[0]
    for n in (3, 24, 41, 55):
        E = mot.excitation(4, 4, 4, p.eps, wave, n, r=r)
        for w in range(4):
            tc = n * r - wave.t0 - (w + 0.5)
            ref = 0.8 * wave.amp * pins.axis_wave_voxel_average(tc, wave.width)
            assert np.allclose(E[0, w], ref, rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("r", [0.5, 0.8])
def test_short_step_one_voxel_clausius_mossotti(r):
    eps = 6.0
    p = wl.homogeneous_cube(1, eps, 10, 4.0)
    p.c_dt = r
    J = mot.Oracle(p).run(600, excite=_constant_excitation(p, (1.0, 0.0, 0.0)))
    assert abs(J[-1, 0, 0, 0, 0] - 3 * (eps - 1) / (eps + 2)) < 1e-12


@pytest.mark.slow
def test_short_step_steady_state_against_newell():
    """The 3^3 block of the c dt = h test at c dt = h/2: the static limit does not depend on dt."""
    U = 3
    eps = wl.random_eps(U, U, U, 7, 2.0, 6.0)
    p = wl.Problem("ss", U, U, U, eps, [], 10, fir=np.zeros(0), c_dt=0.5)
    o = mot.Oracle(p)
    E0 = np.array([1.0, 0.5, -0.25])
    const = _constant_excitation(p, E0)
    J = o.run(1200, excite=lambda n: const(n) * 0.5 * (1.0 + erf((n - 200.0) / 24.0)))
    M = U ** 3
    chi = mot.chi_of(eps).ravel()
    A = np.zeros((3 * M, 3 * M))
    coords = [(u, v, w) for w in range(U) for v in range(U) for u in range(U)]
    for i, ci in enumerate(coords):
        for j, cj in enumerate(coords):
            N = pins.newell_tensor(tuple(ci[t] - cj[t] for t in range(3)))
            for b in range(3):
                for a in range(3):
                    A[b * M + i, a * M + j] += chi[i] * N[mot.COMP[b][a]]
    for b in range(3):
        A[b * M:(b + 1) * M, b * M:(b + 1) * M] += np.diag(1.0 / eps.ravel())
    rhs = np.concatenate([chi * E0[b] for b in range(3)])
    Jinf = np.linalg.solve(A, rhs)
    assert np.abs(J[-1].reshape(-1) - Jinf).max() < 1e-10 * np.abs(Jinf).max()


def test_short_step_time_shift_invariance():
    p = wl.homogeneous_cube(3, 6.0, 80, 3.0)
    p.c_dt = 0.5
    p.waves[0].t0 = 30.0
    o = mot.Oracle(p)
    J1 = o.run(140)
    p.waves[0].t0 += 2.5            # five steps of c dt = 1/2
    J2 = o.run(140)
    assert np.abs(J2[5:] - J1[:-5]).max() < 1e-13 * np.abs(J1).max()


# ----------------------------------------------------------------------------- unequal voxel edges
# Voxels hx x hy x hz (hx = 1 sets the unit).  The identities keep their form with Newell's
# prism tensor, the overlap of two prisms and the distance range of two prisms.
HV = (1.0, 0.7, 1.3)


def lag_window_h(D, hv):
    a = sum((max(abs(d) - 1, 0) * h) ** 2 for d, h in zip(D, hv)) ** 0.5
    b = sum(((abs(d) + 1) * h) ** 2 for d, h in zip(D, hv)) ** 0.5
    return a, b


def kernel_lags_h(D, r, hv, extra=2):
    _, b = lag_window_h(D, hv)
    kmax = int(np.floor(b / r)) + 2 + extra
    return np.array([mot.kernel_entry(k, D, r=r, hv=hv) for k in range(kmax + 1)])


@pytest.mark.parametrize("r", [0.7, 0.5])
@pytest.mark.parametrize("D", [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1), (2, -1, 0), (3, 1, -2)])
def test_prism_static_sum_equals_newell(D, r):
    Ks = kernel_lags_h(D, r, HV)
    assert np.abs(Ks.sum(0) + pins.newell_tensor_h(D, HV)).max() < 5e-14


@pytest.mark.parametrize("D", [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 1, 0)])
def test_prism_trace_identity(D):
    Ks = kernel_lags_h(D, 0.7, HV)
    want = -1.0 if D == (0, 0, 0) else 0.0
    assert abs(Ks.sum(0)[:3].sum() - want) < 1e-13


@pytest.mark.parametrize("D", [(1, 1, 1), (3, 2, 2), (5, -3, 2)])
def test_prism_first_and_second_moments(D):
    r = 0.6
    Ks = kernel_lags_h(D, r, HV)
    k = np.arange(len(Ks))[:, None]
    assert np.abs((k * Ks).sum(0) - 0.5 * Ks.sum(0)).max() < 1e-11 * np.abs(Ks).max()
    if D != (1, 1, 1):
        static = pins.overlap_gl_h(D, HV, pins.static_second_derivative)
        assert np.abs(Ks.sum(0) - static).max() < 1e-10 * np.abs(static).max()
        ref = 0.5 * static - pins.overlap_gl_h(D, HV, pins.second_moment_integrand) / (r * r)
        assert np.abs((k ** 2 * Ks).sum(0) - ref).max() < 1e-9 * np.abs(ref).max()


def test_prism_axis_swap():
    """Swapping two axes together with their edges permutes the components."""
    r = 0.6
    for D, k in [((2, 1, 0), 4), ((3, -2, 1), 6), ((1.3, 0.4, -2.2), 5)]:
        K = mot.kernel_entry(k, D, r=r, hv=HV)
        Ks = mot.kernel_entry(k, (D[1], D[0], D[2]), r=r, hv=(HV[1], HV[0], HV[2]))
        assert np.abs(Ks - K[[1, 0, 2, 3, 5, 4]]).max() < 1e-13 * np.abs(K).max()


def test_prism_support_and_stencil():
    r = 0.7          # = the shortest edge: K_0 still on the 27 nearest offsets
    for D in [(0, 0, 0), (1, 1, 1), (0, 2, 0), (3, 2, 1)]:
        Ks = kernel_lags_h(D, r, HV, extra=3)
        a, b = lag_window_h(D, HV)
        scale = np.abs(Ks).max()
        for k in range(len(Ks)):
            if not ((k + 1) * r > a and (k - 2) * r < b):
                assert np.abs(Ks[k]).max() < 1e-13 * scale + 1e-15
    for D in [(1, 1, 1), (0, 1, 0), (0, 0, 0)]:
        assert np.abs(mot.kernel_entry(0, D, r=r, hv=HV)).max() > 1e-4
    for D in [(2, 0, 0), (0, 2, 0), (0, 0, 2), (2, 1, 1)]:
        assert np.abs(mot.kernel_entry(0, D, r=r, hv=HV)).max() < 1e-15
    assert mot.ell(5, 4, 3, 1.0, r, HV[1], HV[2]) == int(np.floor(sqrt(25 + (4 * 0.7) ** 2 + (3 * 1.3) ** 2) / r)) + 2


def test_prism_excitation_axis_wave_closed_form():
    hv = (1.0, 0.7, 1.3)
    p = wl.homogeneous_cube(4, 5.0, 10, 4.0)
    wave = p.waves[0]
    for n in (3, 14, 22):
        E = mot.excitation(4, 4, 4, p.eps, wave, n, r=0.7, hv=hv)
        for w in range(4):
            tc = n * 0.7 - wave.t0 - (w + 0.5) * hv[2]
            ref = 0.8 * wave.amp * pins.axis_wave_voxel_average(tc, wave.width, hv[2])
            assert np.allclose(E[0, w], ref, rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_prism_one_voxel_static_limit(axis):
    """One hx x hy x hz voxel under a constant field along an axis settles at
    J = chi E / (1/eps + chi N_aa(0)) with Newell's self factor of the prism."""
    eps = 6.0
    p = wl.homogeneous_cube(1, eps, 10, 4.0)
    p.c_dt, p.hy, p.hz = 0.7, HV[1], HV[2]
    E0 = [0.0, 0.0, 0.0]
    E0[axis] = 1.0
    J = mot.Oracle(p).run(500, excite=_constant_excitation(p, E0))
    chi = (eps - 1) / eps
    N = pins.newell_tensor_h((0, 0, 0), HV)[axis]
    assert abs(J[-1, axis, 0, 0, 0] - chi / (1 / eps + chi * N)) < 1e-12


# ----------------------------------------------------------------------------- restricted march
def test_restricted_march_matches_full_oracle():
    """The oracle's dense march on the listed voxels (every voxel with eps_r != 1) gives the
    full-grid oracle march's currents there, and the full march's currents vanish exactly at
    every other voxel (chi = 0): dropping the vacuum voxels from the system is exact.  Oblique
    wave, 3-tap FIR, scatterer voxels far apart and adjacent."""
    from conftest import oracle_kernel_table
    U, V, W, n = 6, 5, 4, 60
    eps = np.ones((W, V, U))
    vox = np.array([[0, 0, 0], [1, 0, 0], [5, 4, 3], [2, 3, 1], [4, 1, 3]])   # (u, v, w)
    for i, (u, v, w) in enumerate(vox):
        eps[w, v, u] = 2.0 + 2.5 * i
    k = (0.48, -0.6, 0.64)
    wave = wl.gaussian_wave(U, V, W, k, _perp(k, (1.0, 0.0, 0.0)), 2.0)
    prob = wl.Problem("restricted", U, V, W, eps, [wave], n, fir=wl.binomial_highpass(3, 0.1))
    K = oracle_kernel_table(U, V, W, mot.ell(U, V, W))
    J = mot.Oracle(prob, K=K).run(n)
    Jr = mot.restricted_march(prob, vox, n)
    got = J[:, :, vox[:, 2], vox[:, 1], vox[:, 0]]
    assert np.abs(got - Jr).max() <= 1e-12 * np.abs(got).max()
    mask = np.ones((W, V, U), bool)
    mask[vox[:, 2], vox[:, 1], vox[:, 0]] = False
    assert np.all(J[:, :, mask] == 0.0)


def test_kernel_values_by_symmetry_match_direct_entries():
    """kernel_values_by_symmetry, fed canonical entries only, reproduces directly computed
    entries at offsets with every sign pattern and axis order."""
    rng = np.random.default_rng(77)
    offs = [np.array(d) for d in ([3, -1, 2], [-2, 0, 5], [0, 4, -4], [-1, -3, 0], [2, 2, -1])]
    lags, D = [], []
    for d in offs:
        for k in (int(np.linalg.norm(d)), int(np.linalg.norm(d)) + 1):
            for perm in ([0, 1, 2], [2, 0, 1], [1, 2, 0]):
                lags.append(k)
                D.append(d[perm] * rng.choice([-1, 1], 3))
    D = np.array(D)
    C = mot.canonical_offsets(D)
    uniq = sorted(set((k,) + tuple(c) for k, c in zip(lags, C)))
    vals = mot.kernel_list([u[0] for u in uniq], [u[1:] for u in uniq])
    canon = np.zeros((max(lags) + 1, 6, 6, 6, 6))
    for u, v in zip(uniq, vals):
        canon[u] = v
    got = mot.kernel_values_by_symmetry(lags, D, canon)
    ref = mot.kernel_list(lags, D, skip_outside=False)
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
