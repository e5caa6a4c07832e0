/*
 * ORACLE -- test infrastructure, not product code.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load,
 * call or link this file.  It shares no code with the HIP library.
 *
 * Plain CPU evaluation of the space-time Galerkin interaction kernels of the
 * MOT-JVIE, one lag and one voxel offset at a time.
 *
 * What is computed (Sec. 2.3, eq:Z with eq:TestOperator and eq:SpatialBasis;
 * the temporal basis is read as the causal uniform quadratic B-spline with knots
 * (n'-1, n', n'+1, n'+2) dt, because the paper defers its definition):
 *
 *   Z^{ba}_{m,m',k} = d_ab d_mm' T(k dt)/eps_m - chi_m K^{ba}_k(D),   D = r_m - r_m'
 *
 *   K^{ba}_k(D) = (1/(hx hy hz)) [ Int g_k(d) d_a d_b Lam(d - D) dd
 *                                  - d_ab c^-2 Int gbar_k(d) Lam(d - D) dd ]
 *
 *   g_k(d)    = T(k dt - |d|/c) / (4 pi |d|),   gbar_k(d) = T''(k dt - |d|/c) / (4 pi |d|)
 *   Lam(x)    = prod_i (h_i - |x_i|)_+   (overlap volume of two voxels at offset x)
 *
 * The curl-curl of the retarded potential is split with grad(div) - Laplacian
 * and the wave equation, and both spatial derivatives are moved onto Lam
 * (distributional derivatives):
 *   a != b : d_a d_b Lam = lam'(x_a) lam'(x_b) lam(x_c)  -- bounded, cube integrals
 *   a == b : d_a^2 lam   = (delta(s+h_a) - 2 delta(s) + delta(s-h_a)) / h_a -- plane integrals
 * with lam(x) = 1 - |x|/h_i per axis (Lam / (hx hy hz) = prod_i lam(x_i)).
 *
 * Units: lengths in the unit of h = (hx, hy, hz) (1, 1, 1 for cubic voxels), r = c dt in the
 * same unit; offsets D are given in voxel steps per axis.  K is dimensionless.
 *
 * Quadrature (every integrand is analytic between the spheres |d| = knot radius):
 *  - a cube integral of F = phi(|d|) P(d) (P polynomial) is turned into face
 *    integrals by the divergence theorem with V = y Psi(y)/|y|^3,
 *    Psi(y) = Int_0^{|y|} phi(u) P(u y/|y|) u^2 du  (so div V = F);
 *    Psi is a piecewise polynomial in u, integrated exactly by 4-point
 *    Gauss-Legendre per B-spline piece;
 *  - a face (unit square in a plane |y_ax| = const) is split into four signed
 *    triangles with apex at the foot of the perpendicular from the origin; each
 *    triangle is parametrised by (s along its edge, tau along the ray), and
 *    split in s and tau where the knot spheres cut the plane;
 *    n x n Gauss-Legendre on every cell.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXGL 48

/* Gauss-Legendre nodes and weights on [-1,1], Newton iteration in long double. */
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; i++) {
        long double z = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
        long double dp = 1.0L;
        for (int it = 0; it < 100; it++) {
            long double p0 = 1.0L, p1 = z;
            for (int j = 2; j <= n; j++) {
                long double p2 = ((2.0L * j - 1.0L) * z * p1 - (j - 1.0L) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        {
            long double p0 = 1.0L, p1 = z;
            for (int j = 2; j <= n; j++) {
                long double p2 = ((2.0L * j - 1.0L) * z * p1 - (j - 1.0L) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
        }
        x[i] = (double)(-z);
        w[i] = (double)(2.0L / ((1.0L - z * z) * dp * dp));
    }
}

/* Uniform quadratic B-spline on [0,3] and its second derivative. */
static double bspl(double x)
{
    if (x <= 0.0 || x >= 3.0) return 0.0;
    if (x < 1.0) return 0.5 * x * x;
    if (x < 2.0) return 0.5 * (-2.0 * x * x + 6.0 * x - 3.0);
    return 0.5 * (3.0 - x) * (3.0 - x);
}
static double bspl2(double x)
{
    if (x <= 0.0 || x >= 3.0) return 0.0;
    if (x < 1.0) return 1.0;
    if (x < 2.0) return -2.0;
    return 1.0;
}

double or_bspline(double x) { return bspl(x); }

/* ------------------------------------------------------------------------- */
/* Oracle context for one lag k and one offset D.                             */
/* ------------------------------------------------------------------------- */
typedef struct {
    double r;          /* c dt */
    int k;             /* lag */
    double h[3];       /* voxel edges */
    double D[3];       /* offset as a length: voxel steps times h */
    int ngl;
    double glx[MAXGL], glw[MAXGL];
    double g4x[4], g4w[4];
    double knot[4];    /* r(k-2), r(k-1), r k, r(k+1) */
} octx;

/* Radial profile times u^2:  u^2 * g_k(u) = B(k+1-u/r) u / (4 pi) (kind 0),
 *                           u^2 * c^-2 gbar_k(u) = B''(k+1-u/r) u / (4 pi r^2) (kind 1). */
static double radial_u2(const octx *o, int kind, double u)
{
    double x = o->k + 1.0 - u / o->r;
    if (kind == 0) return bspl(x) * u / (4.0 * M_PI);
    return bspl2(x) * u / (4.0 * M_PI * o->r * o->r);
}

/* Sub-box polynomial weights.  Box sign s[i] = +1 for [D_i, D_i+h_i], -1 for [D_i-h_i, D_i].
 * lam(x) = 1 - |x|/h_i = 1 - s x / h_i on the box;  lam'(x) = -s / h_i.  */
typedef struct { int s[3]; } boxw;

/* wfun: 0 = Lam = lam lam lam;  1 = xy: lam' lam' lam;  2 = xz;  3 = yz */
static double box_weight(const octx *o, const boxw *b, int wfun, const double p[3])
{
    double l[3], dl[3];
    for (int i = 0; i < 3; i++) {
        l[i] = 1.0 - b->s[i] * (p[i] - o->D[i]) / o->h[i];
        dl[i] = -(double)b->s[i] / o->h[i];
    }
    switch (wfun) {
    case 0: return l[0] * l[1] * l[2];
    case 1: return dl[0] * dl[1] * l[2];
    case 2: return dl[0] * l[1] * dl[2];
    default: return l[0] * dl[1] * dl[2];
    }
}

/* Psi(y) = Int_0^{|y|} phi(u) P(u yhat) u^2 du, exact per B-spline piece.
 * Evaluated for the four box weights at once:
 *   out[0] = Lam with the gbar profile, out[1..3] = xy, xz, yz with the g profile. */
static void cone_psi4(const octx *o, const boxw *b, const double y[3], double ny, double out[4])
{
    double yhat[3] = {y[0] / ny, y[1] / ny, y[2] / ny};
    double lo = o->knot[0] > 0.0 ? o->knot[0] : 0.0;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    for (int piece = 0; piece < 3; piece++) {
        double a = o->knot[piece], c = o->knot[piece + 1];
        if (a < lo) a = lo;
        if (c > ny) c = ny;
        if (c <= a) continue;
        double hm = 0.5 * (c - a), hc = 0.5 * (c + a);
        double s[4] = {0, 0, 0, 0};
        for (int q = 0; q < 4; q++) {
            double u = hc + hm * o->g4x[q];
            double p[3] = {u * yhat[0], u * yhat[1], u * yhat[2]};
            double rg = o->g4w[q] * radial_u2(o, 0, u);
            double rb = o->g4w[q] * radial_u2(o, 1, u);
            s[0] += rb * box_weight(o, b, 0, p);
            s[1] += rg * box_weight(o, b, 1, p);
            s[2] += rg * box_weight(o, b, 2, p);
            s[3] += rg * box_weight(o, b, 3, p);
        }
        for (int i = 0; i < 4; i++) out[i] += hm * s[i];
    }
}

/* Integrand on a face at point y (3-D); up to four values at once.
 * mode 0: cone fluxes of one sub-box (values of cone_psi4, times y.n/|y|^3);
 * mode 1: plane term g_k(|y|) lam(y_a1 - D_a1) lam(y_a2 - D_a2) on one sub-square. */
typedef struct {
    const octx *o;
    int mode;
    const boxw *b;
    double ndoty;      /* y . n, constant on the face */
    int pa1, pa2, ps1, ps2;
} fctx;

static int face_integrand(const fctx *f, const double y[3], double v[4])
{
    const octx *o = f->o;
    double ny = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    if (f->mode == 0) {
        if (ny <= 0.0) { v[0] = v[1] = v[2] = v[3] = 0.0; return 4; }
        cone_psi4(o, f->b, y, ny, v);
        double sc = f->ndoty / (ny * ny * ny);
        for (int i = 0; i < 4; i++) v[i] *= sc;
        return 4;
    }
    if (ny <= 0.0) { v[0] = 0.0; return 1; }
    double x = o->k + 1.0 - ny / o->r;
    double g = bspl(x) / (4.0 * M_PI * ny);
    double l1 = 1.0 - f->ps1 * (y[f->pa1] - o->D[f->pa1]) / o->h[f->pa1];
    double l2 = 1.0 - f->ps2 * (y[f->pa2] - o->D[f->pa2]) / o->h[f->pa2];
    v[0] = g * l1 * l2;
    return 1;
}

static int cmpd(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Integral over the square {y_ax = c, y_a1 in [lo1,hi1], y_a2 in [lo2,hi2]};
 * accumulates nv values into res. */
static void face_quad(const fctx *f, int ax, double c, double lo1, double hi1, double lo2, double hi2,
                      int nv, double *res)
{
    const octx *o = f->o;
    int a1 = (ax + 1) % 3, a2 = (ax + 2) % 3;
    double rho[4];
    int nr = 0;
    for (int j = 0; j < 4; j++) {
        double R = o->knot[j];
        if (R > fabs(c)) rho[nr++] = sqrt(R * R - c * c);
    }
    qsort(rho, nr, sizeof(double), cmpd);

    /* Each edge: signed distance p from the foot (outward normal), the range of
     * the edge coordinate s, and which in-plane coordinate is fixed on the edge. */
    struct { double p; double s0, s1; int fixed_is_1; double fixed; } e[4] = {
        {-lo2, lo1, hi1, 0, lo2},  /* y_a2 = lo2, s runs along a1 */
        { hi1, lo2, hi2, 1, hi1},  /* y_a1 = hi1, s runs along a2 */
        { hi2, lo1, hi1, 0, hi2},  /* y_a2 = hi2 */
        {-lo1, lo2, hi2, 1, lo1},  /* y_a1 = lo1 */
    };
    for (int ie = 0; ie < 4; ie++) {
        double p = e[ie].p;
        if (p == 0.0) continue;
        double ap = fabs(p), sg = p > 0 ? 1.0 : -1.0;
        double sp[16];
        int ns = 0;
        sp[ns++] = e[ie].s0;
        for (int j = 0; j < nr; j++) {
            if (rho[j] > ap) {
                double t = sqrt(rho[j] * rho[j] - p * p);
                if (t > e[ie].s0 && t < e[ie].s1) sp[ns++] = t;
                if (-t > e[ie].s0 && -t < e[ie].s1) sp[ns++] = -t;
            }
        }
        sp[ns++] = e[ie].s1;
        qsort(sp, ns, sizeof(double), cmpd);
        double esum[4] = {0, 0, 0, 0};
        for (int is = 0; is + 1 < ns; is++) {
            double sa = sp[is], sb = sp[is + 1];
            if (sb <= sa) continue;
            double shm = 0.5 * (sb - sa), shc = 0.5 * (sb + sa);
            double sacc[4] = {0, 0, 0, 0};
            for (int i = 0; i < o->ngl; i++) {
                double s = shc + shm * o->glx[i];
                double L = sqrt(p * p + s * s);
                double tp[24];
                int nt = 0;
                tp[nt++] = 0.0;
                for (int j = 0; j < nr; j++) {
                    double t = rho[j] / L;
                    if (t > 0.0 && t < 1.0) tp[nt++] = t;
                }
                /* |y| = sqrt(c^2 + tau^2 L^2) makes the integrand singular at
                 * tau = +-i|c|/L; where the integrand is not identically zero near
                 * the foot (first knot inside the plane's distance), grade the
                 * tau cells geometrically towards the foot. */
                if (o->knot[0] <= fabs(c)) {
                    for (double t = fabs(c) / L; t < 1.0 && nt < 22; t *= 3.0) tp[nt++] = t;
                }
                tp[nt++] = 1.0;
                qsort(tp, nt, sizeof(double), cmpd);
                double e1 = e[ie].fixed_is_1 ? e[ie].fixed : s;
                double e2 = e[ie].fixed_is_1 ? s : e[ie].fixed;
                double tacc[4] = {0, 0, 0, 0};
                for (int it = 0; it + 1 < nt; it++) {
                    double ta = tp[it], tb = tp[it + 1];
                    if (tb <= ta) continue;
                    double thm = 0.5 * (tb - ta), thc = 0.5 * (tb + ta);
                    double pacc[4] = {0, 0, 0, 0};
                    for (int q = 0; q < o->ngl; q++) {
                        double tau = thc + thm * o->glx[q];
                        double y[3], v[4];
                        y[ax] = c;
                        y[a1] = tau * e1;
                        y[a2] = tau * e2;
                        face_integrand(f, y, v);
                        for (int m = 0; m < nv; m++) pacc[m] += o->glw[q] * tau * v[m];
                    }
                    for (int m = 0; m < nv; m++) tacc[m] += thm * pacc[m];
                }
                for (int m = 0; m < nv; m++) sacc[m] += o->glw[i] * tacc[m];
            }
            for (int m = 0; m < nv; m++) esum[m] += shm * sacc[m];
        }
        for (int m = 0; m < nv; m++) res[m] += sg * ap * esum[m];
    }
}

/* Cube integrals over sub-box b of  c^-2 gbar_k * Lam  (res[0]) and of
 * g_k * d_a d_b Lam for ab = xy, xz, yz (res[1..3]), by the divergence theorem
 * (a face with y.n = 0 carries no flux). */
static void box_integrals(const octx *o, const boxw *b, double res[4])
{
    double lo[3], hi[3];
    for (int i = 0; i < 3; i++) {
        if (b->s[i] > 0) { lo[i] = o->D[i]; hi[i] = o->D[i] + o->h[i]; }
        else { lo[i] = o->D[i] - o->h[i]; hi[i] = o->D[i]; }
    }
    res[0] = res[1] = res[2] = res[3] = 0.0;
    for (int ax = 0; ax < 3; ax++) {
        int a1 = (ax + 1) % 3, a2 = (ax + 2) % 3;
        for (int side = 0; side < 2; side++) {
            double c = side ? hi[ax] : lo[ax];
            if (c == 0.0) continue;
            fctx f = {o, 0, b, side ? c : -c, 0, 0, 0, 0};
            face_quad(&f, ax, c, lo[a1], hi[a1], lo[a2], hi[a2], 4, res);
        }
    }
}

static void octx_init(octx *o, double r, const double h[3], int k, const double D[3], int ngl)
{
    o->r = r;
    o->k = k;
    for (int i = 0; i < 3; i++) {
        o->h[i] = h[i];
        o->D[i] = D[i] * h[i];
    }
    if (ngl < 2) ngl = 2;
    if (ngl > MAXGL) ngl = MAXGL;
    o->ngl = ngl;
    gauss_legendre(ngl, o->glx, o->glw);
    gauss_legendre(4, o->g4x, o->g4w);
    for (int j = 0; j < 4; j++) o->knot[j] = r * (k - 2 + j);
}

/*
 * K_k(D) for one lag and one (real-valued) offset D in voxel steps, voxel edges h, c dt = r;
 * out = {xx, yy, zz, xy, xz, yz}.
 */
void or_kernel_entry_h(double r, const double *h, int k, double Dx, double Dy, double Dz, int ngl, double *out)
{
    octx o;
    const double Dv[3] = {Dx, Dy, Dz};
    octx_init(&o, r, h, k, Dv, ngl);
    const double *D = o.D;
    for (int i = 0; i < 6; i++) out[i] = 0.0;

    /* a == b: second difference across the planes y_a = D_a + s h_a, weights (1,-2,1)/h_a */
    for (int a = 0; a < 3; a++) {
        int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
        for (int s = -1; s <= 1; s++) {
            double ws = ((s == 0) ? -2.0 : 1.0) / h[a];
            double c = D[a] + s * h[a];
            for (int s1 = -1; s1 <= 1; s1 += 2) {
                for (int s2 = -1; s2 <= 1; s2 += 2) {
                    double lo1 = s1 > 0 ? D[a1] : D[a1] - h[a1], hi1 = lo1 + h[a1];
                    double lo2 = s2 > 0 ? D[a2] : D[a2] - h[a2], hi2 = lo2 + h[a2];
                    fctx f = {&o, 1, NULL, 0.0, a1, a2, s1, s2};
                    double v = 0.0;
                    face_quad(&f, a, c, lo1, hi1, lo2, hi2, 1, &v);
                    out[a] += ws * v;
                }
            }
        }
    }
    /* a != b (cube terms) and the d_ab gbar term, over the 8 sub-boxes */
    for (int sx = -1; sx <= 1; sx += 2)
        for (int sy = -1; sy <= 1; sy += 2)
            for (int sz = -1; sz <= 1; sz += 2) {
                boxw b = {{sx, sy, sz}};
                double res[4];
                box_integrals(&o, &b, res);
                out[0] -= res[0];
                out[1] -= res[0];
                out[2] -= res[0];
                out[3] += res[1];
                out[4] += res[2];
                out[5] += res[3];
            }
}

static const double unit_h[3] = {1.0, 1.0, 1.0};

/* Cubic voxels of edge 1, c dt = r. */
void or_kernel_entry(double r, int k, double Dx, double Dy, double Dz, int ngl, double *out)
{
    or_kernel_entry_h(r, unit_h, k, Dx, Dy, Dz, ngl, out);
}

/* Largest and smallest distance between points of two voxels at integer-or-real offset D
 * (voxel steps), edges h. */
static void offset_radii(const double D[3], const double h[3], double *rmin, double *rmax)
{
    double a = 0.0, b = 0.0;
    for (int i = 0; i < 3; i++) {
        double d = fabs(D[i]);
        double m = d - 1.0 > 0.0 ? (d - 1.0) * h[i] : 0.0;
        a += m * m;
        b += (d + 1.0) * (d + 1.0) * h[i] * h[i];
    }
    *rmin = sqrt(a);
    *rmax = sqrt(b);
}

/*
 * Dense table K[k][6][2W-1][2V-1][2U-1] for k = 0..kmax over all offsets
 * D in [-(U-1),U-1] x [-(V-1),V-1] x [-(W-1),W-1] (no symmetry is used).
 * skip_outside != 0: entries whose lag window (r(k-2), r(k+1)) misses the
 * distance range of the two voxels are set to exactly 0 instead of computed.
 */
void or_kernel_table_h(double r, const double *h, int U, int V, int W, int kmax, int ngl, int skip_outside,
                       double *K)
{
    long nx = 2L * U - 1, ny = 2L * V - 1, nz = 2L * W - 1;
    long noff = nx * ny * nz;
    long ntask = (long)(kmax + 1) * noff;
#pragma omp parallel for schedule(dynamic, 4)
    for (long t = 0; t < ntask; t++) {
        int k = (int)(t / noff);
        long rem = t % noff;
        long iz = rem / (nx * ny), iy = (rem / nx) % ny, ix = rem % nx;
        double D[3] = {(double)(ix - (U - 1)), (double)(iy - (V - 1)), (double)(iz - (W - 1))};
        double out[6] = {0, 0, 0, 0, 0, 0};
        int active = 1;
        if (skip_outside) {
            double rmin, rmax;
            offset_radii(D, h, &rmin, &rmax);
            if (!(r * (k + 1) > rmin && r * (k - 2) < rmax)) active = 0;
        }
        if (active) or_kernel_entry_h(r, h, k, D[0], D[1], D[2], ngl, out);
        for (int c = 0; c < 6; c++) K[((long)k * 6 + c) * noff + rem] = out[c];
    }
}

void or_kernel_table(double r, int U, int V, int W, int kmax, int ngl, int skip_outside, double *K)
{
    or_kernel_table_h(r, unit_h, U, V, W, kmax, ngl, skip_outside, K);
}

/* Exposed for tests: Gauss-Legendre rule of this file. */
void or_gauss_legendre(int n, double *x, double *w) { gauss_legendre(n, x, w); }

/* Exposed for tests: the four cube integrals of one sub-box (see box_integrals). */
void or_box_integrals(double r, int k, double Dx, double Dy, double Dz, int sx, int sy, int sz, int ngl, double *out4)
{
    octx o;
    double D[3] = {Dx, Dy, Dz};
    octx_init(&o, r, unit_h, k, D, ngl);
    boxw b = {{sx, sy, sz}};
    box_integrals(&o, &b, out4);
}

/* Exposed for tests: one plane term of K^{aa}_k(D): the integral of g_k(|y|) times the
 * sub-square weight over {y_a = D_a + s, sub-square signs (s1, s2)}. */
double or_plane_integral(double r, int k, double Dx, double Dy, double Dz, int a, int s, int s1, int s2, int ngl)
{
    octx o;
    double D[3] = {Dx, Dy, Dz};
    octx_init(&o, r, unit_h, k, D, ngl);
    int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
    double lo1 = s1 > 0 ? D[a1] : D[a1] - 1.0, hi1 = lo1 + 1.0;
    double lo2 = s2 > 0 ? D[a2] : D[a2] - 1.0, hi2 = lo2 + 1.0;
    fctx f = {&o, 1, NULL, 0.0, a1, a2, s1, s2};
    double v = 0.0;
    face_quad(&f, a, D[a] + s, lo1, hi1, lo2, hi2, 1, &v);
    return v;
}
