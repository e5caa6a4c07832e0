"""Independent references used to pin the oracle (no code shared with oracle/ or the HIP library).

* Newell, Williams & Dunlop (1993) closed form of the demagnetising tensor between two
  rectangular prisms: the static sum of the interaction kernels over all lags.
* Tensor Gauss-Legendre integration of smooth (kink-free) static integrands over the
  voxel-overlap function, for offsets whose overlap box stays away from the origin.
* Closed-form voxel average of a Gaussian plane wave travelling along a grid axis.
"""
from __future__ import annotations

from math import asinh, atan, erf, pi, sqrt

import numpy as np


def _asinh_ratio(a, b2):
    # asinh(a / sqrt(b2)) with the b2 -> 0 limit handled (a * 0 factor outside makes it vanish)
    if b2 <= 0.0:
        return 0.0
    return asinh(a / sqrt(b2))


def _atan_ratio(num, den):
    if den == 0.0:
        return 0.0
    return atan(num / den)


def newell_f(x, y, z):
    """Newell's f:  d^2/dy^2 d^2/dz^2 f = 1/R."""
    x, y, z = abs(x), abs(y), abs(z)
    R = sqrt(x * x + y * y + z * z)
    t = 0.0
    if y > 0:
        t += 0.5 * y * (z * z - x * x) * _asinh_ratio(y, x * x + z * z)
    if z > 0:
        t += 0.5 * z * (y * y - x * x) * _asinh_ratio(z, x * x + y * y)
    if x > 0 and y > 0 and z > 0:
        t -= x * y * z * _atan_ratio(y * z, x * R)
    t += (2 * x * x - y * y - z * z) * R / 6.0
    return t


def newell_g(x, y, z):
    """Newell's g:  d/dx d/dy d^2/dz^2 g = 1/R (sign-adjusted for negative x, y)."""
    sgn = np.sign(x) * np.sign(y)
    if sgn == 0:
        return 0.0
    x, y, z = abs(x), abs(y), abs(z)
    R = sqrt(x * x + y * y + z * z)
    t = 0.0
    if z > 0:
        t += x * y * z * _asinh_ratio(z, x * x + y * y)
    t += y / 6.0 * (3 * z * z - y * y) * _asinh_ratio(x, y * y + z * z)
    t += x / 6.0 * (3 * z * z - x * x) * _asinh_ratio(y, x * x + z * z)
    if z > 0:
        t -= z ** 3 / 6.0 * _atan_ratio(x * y, z * R)
        t -= z * y * y / 2.0 * _atan_ratio(x * z, y * R)
        t -= z * x * x / 2.0 * _atan_ratio(y * z, x * R)
    t -= x * y * R / 3.0
    return sgn * t


def _sixth_difference(fun, X, Y, Z):
    s = 0.0
    w = {-1: 1.0, 0: -2.0, 1: 1.0}
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                s += w[i] * w[j] * w[k] * fun(X + i, Y + j, Z + k)
    return s


def newell_tensor(D):
    """Demagnetising tensor N(D) between two unit cubes at offset D:
    N_ab = -(1/V) Int Int d_a d_b (1/(4 pi |r - r'|)), so that N(0) = I/3.
    Returns (xx, yy, zz, xy, xz, yz)."""
    X, Y, Z = (float(v) for v in D)
    c = -1.0 / (4.0 * pi)
    nxx = c * _sixth_difference(newell_f, X, Y, Z)
    nyy = c * _sixth_difference(lambda a, b, d: newell_f(b, d, a), X, Y, Z)
    nzz = c * _sixth_difference(lambda a, b, d: newell_f(d, a, b), X, Y, Z)
    nxy = c * _sixth_difference(newell_g, X, Y, Z)
    nxz = c * _sixth_difference(lambda a, b, d: newell_g(a, d, b), X, Y, Z)
    nyz = c * _sixth_difference(lambda a, b, d: newell_g(b, d, a), X, Y, Z)
    return np.array([nxx, nyy, nzz, nxy, nxz, nyz])


def newell_tensor_h(D, h):
    """Demagnetising tensor between two hx x hy x hz prisms whose centres are D_i h_i apart
    (Newell, Williams & Dunlop 1993 for unequal edges: the sixth differences step by h_i and
    the volume is hx hy hz).  Returns (xx, yy, zz, xy, xz, yz); its trace is 1 at D = 0."""
    hx, hy, hz = (float(v) for v in h)
    X, Y, Z = float(D[0]) * hx, float(D[1]) * hy, float(D[2]) * hz
    c = -1.0 / (4.0 * pi * hx * hy * hz)
    w = {-1: 1.0, 0: -2.0, 1: 1.0}

    def diff(fun, sx, sy, sz):
        t = 0.0
        for i in (-1, 0, 1):
            for j in (-1, 0, 1):
                for k in (-1, 0, 1):
                    t += w[i] * w[j] * w[k] * fun(X + i * sx, Y + j * sy, Z + k * sz)
        return t
    nxx = c * diff(newell_f, hx, hy, hz)
    nyy = c * diff(lambda a, b, d: newell_f(b, d, a), hx, hy, hz)
    nzz = c * diff(lambda a, b, d: newell_f(d, a, b), hx, hy, hz)
    nxy = c * diff(newell_g, hx, hy, hz)
    nxz = c * diff(lambda a, b, d: newell_g(a, d, b), hx, hy, hz)
    nyz = c * diff(lambda a, b, d: newell_g(b, d, a), hx, hy, hz)
    return np.array([nxx, nyy, nzz, nxy, nxz, nyz])


PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def overlap_gl(D, integrand, n=16):
    """Int F(d) Lam(d - D) dd by tensor Gauss-Legendre over the 8 sub-boxes where Lam is a
    polynomial; F is vector-valued (shape (6,) per point).  Accurate only when F is smooth on
    the box [D-1, D+1]^3 (origin outside it)."""
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    D = np.asarray(D, float)
    total = np.zeros(6)
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                s = np.array([sx, sy, sz], float)
                # local coordinate t in [0,1]: d_i = D_i + s_i t_i, Lam = prod (1 - t_i)
                tx, ty, tz = np.meshgrid(x, x, x, indexing="ij")
                wt = (w[:, None, None] * w[None, :, None] * w[None, None, :])
                d = np.stack([D[0] + sx * tx, D[1] + sy * ty, D[2] + sz * tz])
                lam = (1 - tx) * (1 - ty) * (1 - tz)
                F = integrand(d)
                total += np.array([np.sum(F[c] * lam * wt) for c in range(6)])
    return total


def overlap_gl_h(D, h, integrand, n=16):
    """(1/(hx hy hz)) Int F(d) Lam(d - D h) dd for prisms of edges h (Lam the overlap volume),
    by tensor Gauss-Legendre over the 8 sub-boxes; F smooth on the box as for overlap_gl."""
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    h = np.asarray(h, float)
    P = np.asarray(D, float) * h
    total = np.zeros(6)
    tx, ty, tz = np.meshgrid(x, x, x, indexing="ij")
    wt = (w[:, None, None] * w[None, :, None] * w[None, None, :])
    lam = (1 - tx) * (1 - ty) * (1 - tz)
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                d = np.stack([P[0] + sx * h[0] * tx, P[1] + sy * h[1] * ty, P[2] + sz * h[2] * tz])
                F = integrand(d)
                # dd = hx hy hz dt and Lam / (hx hy hz) = prod (1 - t_i)
                total += np.array([np.sum(F[c] * lam * wt) for c in range(6)]) * h.prod()
    return total


def static_second_derivative(d):
    """d_a d_b (1/(4 pi R)) = (3 d_a d_b - delta_ab R^2) / (4 pi R^5) away from the origin."""
    R2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
    R5 = R2 ** 2.5
    out = []
    for a, b in PAIRS:
        v = 3 * d[a] * d[b] - (R2 if a == b else 0.0)
        out.append(v / (4 * pi * R5))
    return out


def second_moment_integrand(d):
    """(delta_ab + dhat_a dhat_b) / (4 pi R): the kink-free remainder of sum_k k^2 K_k."""
    R2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
    R = np.sqrt(R2)
    out = []
    for a, b in PAIRS:
        v = (1.0 if a == b else 0.0) + d[a] * d[b] / R2
        out.append(v / (4 * pi * R))
    return out


def axis_wave_voxel_average(tau_centre, width, hz=1.0):
    """(1/hz) Int_{-hz/2}^{hz/2} exp(-((tau_centre - z)/width)^2) dz in closed form (erf)."""
    from math import erfc
    a = (tau_centre + 0.5 * hz) / width
    b = (tau_centre - 0.5 * hz) / width
    # erf(a) - erf(b) written with erfc on the side away from zero (no cancellation in the tails)
    if b >= 0:
        d = erfc(b) - erfc(a)
    elif a <= 0:
        d = erfc(-a) - erfc(-b)
    else:
        d = erf(a) - erf(b)
    return 0.5 * width * sqrt(pi) * d / hz


def box_wave_average(tau0, c, width):
    """Average over the box [0,1]^3 (coordinates eta) of exp(-((tau0 - sum_i c_i eta_i)/width)^2).

    tau0 is the pulse's retarded argument at the box's lower corner and c_i = khat_i L_i the
    change of the argument along edge i (L_i the edge).  Averaging over one uniform eta is a
    backward difference of an antiderivative: (1/c) Int_0^c g(t - s) ds = (F(t) - F(t - c)) / c.
    Three of them give the third difference of the third antiderivative of the Gaussian,
    written with erf: with x = t / width,
        F_1 = width (sqrt(pi)/2) erf x,
        F_2 = width^2 (sqrt(pi)/2) (x erf x + exp(-x^2)/sqrt(pi)),
        F_3 = width^3 (sqrt(pi)/2) ((x^2/2 + 1/4) erf x + x exp(-x^2)/(2 sqrt(pi))).
    Edges with c_i = 0 drop out (the average over them is the identity).  Evaluated with 50
    digits (mpmath), so that the differences of nearly equal values lose nothing in double."""
    import mpmath as mp
    with mp.workdps(50):
        w = mp.mpf(width)
        sp = mp.sqrt(mp.pi)

        def F(order, t):
            x = t / w
            if order == 0:
                return mp.exp(-x * x)
            if order == 1:
                return w * sp / 2 * mp.erf(x)
            if order == 2:
                return w ** 2 * sp / 2 * (x * mp.erf(x) + mp.exp(-x * x) / sp)
            return w ** 3 * sp / 2 * ((x * x / 2 + mp.mpf(1) / 4) * mp.erf(x) + x * mp.exp(-x * x) / (2 * sp))

        cs = [mp.mpf(ci) for ci in c if ci != 0.0]
        m = len(cs)
        tot = mp.mpf(0)
        # sum over the 2^m corners of the difference stencil
        for mask in range(1 << m):
            shift = mp.mpf(0)
            sign = 1
            for i in range(m):
                if mask >> i & 1:
                    shift += cs[i]
                    sign = -sign
            tot += sign * F(m, mp.mpf(tau0) - shift)
        den = mp.mpf(1)
        for ci in cs:
            den *= ci
        return float(tot / den)
