// Space-time interaction kernels of the MOT-JVIE on the device (FP64).
//
// For test voxel m, source voxel m', lag k = n - n' and D = r_m - r_m' (lengths in units of
// the x edge: voxel edges h = (1, hy, hz), c dt = r <= min h), eq:Z with the
// piecewise-constant spatial basis (eq:SpatialBasis),
// the voxel-average Dirac-in-time test (eq:TestOperator) and the quadratic-spline
// temporal basis T(t) = B(t/dt + 1) (B the uniform quadratic B-spline on [0,3]) gives
//
//   Z^{ba}_k(m, m') = d_ab d_mm' T(k dt) / eps_m - chi_m K^{ba}_k(D),
//   K^{ba}_k(D) = Int g_k(d) d_a d_b Lam(d - D) dd - d_ab Int gbar_k(d) Lam(d - D) dd,
//   g_k = B(k + 1 - |d|/r) / (4 pi |d|),  gbar_k = B''(k + 1 - |d|/r) / (4 pi r^2 |d|),
//   Lam(x) = prod_i (1 - |x_i| / h_i)_+ ,
//
// the derivatives of Lam taken in the distributional sense (a == b gives the second
// difference across the planes d_a = D_a - h_a, D_a, D_a + h_a, divided by h_a).
//
// Factorisation used here.  On the shell a r <= |d| < (a + 1) r each B-spline piece is
// a quadratic in v = |d|/r - a, so every lag is a fixed combination of the lag-free
// shell moments
//   plane_a,j : sum_s w_s Int_{plane s, shell} lam lam v^j / |d| dS    (a = x, y, z; j = 0..2)
//   cube_ab,j : Int_{shell} d_a d_b Lam v^j / |d| dV                    (ab = xy, xz, yz)
//   gbar      : Int_{shell} Lam / |d| dV
// of the three shells a = k, k - 1, k - 2 (K_k = 0 unless one of them meets the
// distance range of the voxel pair: the causal / Huygens support).
//
// Quadrature.  A volume moment over a sub-box (where Lam and its derivatives are
// polynomials) is turned into face integrals by the divergence theorem with the radial
// field y Psi(y) / |y|^3, Psi(y) = Int_{a r}^{min(|y|, (a+1) r)} P(u yhat) v^j u du (div = P v^j/|y|
// on the shell); Psi is a polynomial in u of degree <= 4 and is integrated exactly by
// 3-point Gauss-Legendre.  Every face or plane integral is taken over a unit square as
// four signed triangles with apex at the foot of the perpendicular from the origin,
// parametrised by (s along the edge, tau along the ray), split where the shell's two
// spheres cut the plane and graded towards the foot where the integrand does not vanish
// there; nq x nq Gauss-Legendre on every cell.  Only the octant D >= 0 is computed; the
// other octants follow from the parity of each component.

#include "mj_internal.h"

#include <cmath>

namespace mj {

namespace {

constexpr int kGenThreads = 64;
constexpr int kMaxQ = 24;
constexpr double kInvFourPi = 0.07957747154594766788;

struct GenArg {
    int Uo, Vo, Wo;
    int nq;
    int ms;                          // shells stored per offset
    double r;                        // c dt
    double hv[3], ih[3];             // voxel edges and their inverses
    double glx[kMaxQ], glw[kMaxQ];   // nq-point rule on [-1, 1]
    double g3x[3], g3w[3];           // 3-point rule on [-1, 1]
};

// Shells a r <= |d| < (a + 1) r, a in [a_lo, a_lo + nsh), that meet the distance range
// [R_min, R_max] of two voxels: a_lo = floor(R_min / r), a_lo + nsh = ceil(R_max / r).  With
// r = 1 the squared radii are integers and the bounds are exact.
__host__ __device__ inline void shell_bounds(double rmin2, double rmax2, double r, int &a_lo, int &nsh)
{
    const double Rmin = sqrt(rmin2), Rmax = sqrt(rmax2);
    int lo = (int)floor(Rmin / r);
    while ((lo + 1) * r <= Rmin) lo++;
    while (lo > 0 && lo * r > Rmin) lo--;
    int hi = (int)ceil(Rmax / r);
    while (hi - 1 > lo && (hi - 1) * r >= Rmax) hi--;
    while (hi * r < Rmax) hi++;
    a_lo = lo;
    nsh = hi - lo;
}

__host__ __device__ inline void shell_range(int dx, int dy, int dz, const double hv[3], double r, int &a_lo,
                                            int &nsh)
{
    const int ex = dx > 0 ? dx - 1 : 0, ey = dy > 0 ? dy - 1 : 0, ez = dz > 0 ? dz - 1 : 0;
    const double rmin2 = (ex * hv[0]) * (ex * hv[0]) + (ey * hv[1]) * (ey * hv[1]) + (ez * hv[2]) * (ez * hv[2]);
    const double rmax2 = ((dx + 1) * hv[0]) * ((dx + 1) * hv[0]) + ((dy + 1) * hv[1]) * ((dy + 1) * hv[1]) +
                         ((dz + 1) * hv[2]) * ((dz + 1) * hv[2]);
    shell_bounds(rmin2, rmax2, r, a_lo, nsh);
}

// Upper bound on the shells of one voxel pair: R_max - R_min <= 2 |h|, plus one shell cut at
// each end and one for rounding.
__host__ __device__ inline int shells_per_offset(double r, const double hv[3])
{
    return (int)(2.0 * sqrt(hv[0] * hv[0] + hv[1] * hv[1] + hv[2] * hv[2]) / r) + 3;
}

// Fixed-size ascending sort with compile-time indices only (values stay in registers).
template <int N>
__host__ __device__ inline void sort_fixed(double *a)
{
#pragma unroll
    for (int i = 0; i < N - 1; i++)
#pragma unroll
        for (int j = 0; j < N - 1 - i; j++) {
            double lo = fmin(a[j], a[j + 1]), hi = fmax(a[j], a[j + 1]);
            a[j] = lo;
            a[j + 1] = hi;
        }
}

// Contribution of one face node y (weight wgt = dA * quadrature weight) on the square of
// plane y_AX = c = D[AX] + s h_AX with sub-square signs (s1, s2) along the in-plane axes.
// Every array index is a compile-time constant.
// ANI = false compiles the cubic-voxel case, where every edge factor is 1.
template <int AX, bool ANI>
__host__ __device__ inline void node_contrib(double m[kMoments], const double y[3], double ny, double wgt, int s,
                                             int s1, int s2, const double D[3], double Ra, double Rb, double inv_r,
                                             const double *ih, const double *g3x, const double *g3w)
{
    constexpr int A1 = (AX + 1) % 3, A2 = (AX + 2) % 3;
    const double c = y[AX];
    const double inv_ny = 1.0 / ny;
    // plane term of component AX: w_s lam lam v^j / |y| on the shell
    if (ny >= Ra && ny < Rb) {
        const double ws = ANI ? ((s == 0) ? -2.0 : 1.0) * ih[AX] : ((s == 0) ? -2.0 : 1.0);
        const double l1 = ANI ? 1.0 - s1 * (y[A1] - D[A1]) * ih[A1] : 1.0 - s1 * (y[A1] - D[A1]);
        const double l2 = ANI ? 1.0 - s2 * (y[A2] - D[A2]) * ih[A2] : 1.0 - s2 * (y[A2] - D[A2]);
        const double v = (ny - Ra) * inv_r;
        const double f = wgt * ws * l1 * l2 * inv_ny;
        m[3 * AX + 0] += f;
        m[3 * AX + 1] += f * v;
        m[3 * AX + 2] += f * v * v;
    }
    if (c == 0.0 || ny <= Ra) return;
    // cone fluxes of the adjacent sub-boxes
    const double hi = ny < Rb ? ny : Rb;
    const double hm = 0.5 * (hi - Ra), hc = 0.5 * (hi + Ra);
    const double yh[3] = {y[0] * inv_ny, y[1] * inv_ny, y[2] * inv_ny};
    const double flux_scale = wgt * inv_ny * inv_ny * inv_ny * hm;
#pragma unroll
    for (int side = 0; side < 2; side++) {
        // s = -1: box sb_AX = -1, lower face (y.n = -c); s = +1: box +1, upper face (y.n = c);
        // s = 0: box -1 upper face (y.n = c) and box +1 lower face (y.n = -c)
        int sbax;
        double ydotn;
        if (s == 0) {
            sbax = side == 0 ? -1 : 1;
            ydotn = side == 0 ? c : -c;
        } else {
            if (side == 1) break;
            sbax = s;
            ydotn = s < 0 ? -c : c;
        }
        int sb[3];
        sb[AX] = sbax;
        sb[A1] = s1;
        sb[A2] = s2;
        double lamI = 0.0, cb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const double u = hc + hm * g3x[q];
            const double wq = g3w[q] * u;
            const double l0 = ANI ? 1.0 - sb[0] * (u * yh[0] - D[0]) * ih[0] : 1.0 - sb[0] * (u * yh[0] - D[0]);
            const double l1 = ANI ? 1.0 - sb[1] * (u * yh[1] - D[1]) * ih[1] : 1.0 - sb[1] * (u * yh[1] - D[1]);
            const double l2 = ANI ? 1.0 - sb[2] * (u * yh[2] - D[2]) * ih[2] : 1.0 - sb[2] * (u * yh[2] - D[2]);
            const double v = (u - Ra) * inv_r;
            lamI += wq * l0 * l1 * l2;
            const double w0 = wq, w1 = wq * v, w2 = wq * v * v;
            const double pxy = ANI ? sb[0] * sb[1] * l2 * (ih[0] * ih[1]) : sb[0] * sb[1] * l2;
            const double pxz = ANI ? sb[0] * sb[2] * l1 * (ih[0] * ih[2]) : sb[0] * sb[2] * l1;
            const double pyz = ANI ? sb[1] * sb[2] * l0 * (ih[1] * ih[2]) : sb[1] * sb[2] * l0;
            cb[0][0] += w0 * pxy; cb[0][1] += w1 * pxy; cb[0][2] += w2 * pxy;
            cb[1][0] += w0 * pxz; cb[1][1] += w1 * pxz; cb[1][2] += w2 * pxz;
            cb[2][0] += w0 * pyz; cb[2][1] += w1 * pyz; cb[2][2] += w2 * pyz;
        }
        const double f = flux_scale * ydotn;
        m[18] += f * lamI;
#pragma unroll
        for (int pr = 0; pr < 3; pr++)
#pragma unroll
            for (int j = 0; j < 3; j++) m[9 + 3 * pr + j] += f * cb[pr][j];
    }
}

constexpr double kSentinel = 1e300;
constexpr int kMaxGrade = 6;   // graded tau points towards the foot (ratio 3)

// One work item of the face quadrature of shell [Ra, Rb) at octant offset D for a unit square in the
// plane y_AX = D[AX] + s h_AX: edge e, s-interval iv of that edge, s-node iq; accumulates into m.
// glx/glw: nq-point rule on [-1,1]; g3x/g3w: 3-point rule.
template <int AX, int E, bool ANI>
__host__ __device__ inline void gen_edge(int nq, const double *glx, const double *glw, const double *g3x,
                                         const double *g3w, const double D[3], double Ra, double Rb, double inv_r,
                                         const double *hv, const double *ih, int s, int s1, int s2, int iv, int iq,
                                         double m[kMoments])
{
    constexpr int A1 = (AX + 1) % 3, A2 = (AX + 2) % 3;
    const double e0_ = ANI ? hv[AX] : 1.0, e1_ = ANI ? hv[A1] : 1.0, e2_ = ANI ? hv[A2] : 1.0;
    const double c = D[AX] + s * e0_;
    const double lo1 = s1 > 0 ? D[A1] : D[A1] - e1_, lo2 = s2 > 0 ? D[A2] : D[A2] - e2_;
    const double hi1 = lo1 + e1_, hi2 = lo2 + e2_;
    // edge e: signed distance p of its line from the foot; range [e0, e1] of the edge coordinate
    // E = 0: y_A2 = lo2 (s along A1); 1: y_A1 = hi1 (s along A2); 2: y_A2 = hi2; 3: y_A1 = lo1
    constexpr bool fixed_is_1 = (E == 1 || E == 3);
    const double p = E == 0 ? -lo2 : (E == 1 ? hi1 : (E == 2 ? hi2 : -lo1));
    const double e0 = fixed_is_1 ? lo2 : lo1, e1 = fixed_is_1 ? hi2 : hi1;
    const double fixed = E == 0 ? lo2 : (E == 1 ? hi1 : (E == 2 ? hi2 : lo1));
    if (p == 0.0) return;
    const double ap = fabs(p);
    const double c2 = c * c;
    // nothing contributes where |y| <= a: skip edges whose farthest point is inside the shell
    const double Lmax2 = p * p + fmax(e0 * e0, e1 * e1);
    if (c2 + Lmax2 <= Ra * Ra) return;
    // in-plane radii of the two spheres (0 when the sphere does not reach the plane)
    const bool haveA = Ra > fabs(c), haveB = Rb > fabs(c);
    const double rhoA = haveA ? sqrt(Ra * Ra - c2) : 0.0;
    const double rhoB = haveB ? sqrt(Rb * Rb - c2) : 0.0;
    // split points of the edge coordinate where the spheres cross the edge
    double sp[6];
    sp[0] = e0;
    sp[1] = sp[2] = sp[3] = sp[4] = kSentinel;
    sp[5] = e1;
    if (haveA && rhoA > ap) {
        const double t = sqrt(rhoA * rhoA - p * p);
        if (t > e0 && t < e1) sp[1] = t;
        if (-t > e0 && -t < e1) sp[2] = -t;
    }
    if (haveB && rhoB > ap) {
        const double t = sqrt(rhoB * rhoB - p * p);
        if (t > e0 && t < e1) sp[3] = t;
        if (-t > e0 && -t < e1) sp[4] = -t;
    }
    sort_fixed<6>(sp);
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int j = 0; j < 5; j++)
        if (j == iv) {
            sa = sp[j];
            sb = sp[j + 1];
        }
    if (!(sb > sa) || sb >= kSentinel) return;
    const double shm = 0.5 * (sb - sa), shc = 0.5 * (sb + sa);
    const double sn = shc + shm * glx[iq];
    const double L = sqrt(p * p + sn * sn);
    const double ey1 = fixed_is_1 ? fixed : sn;
    const double ey2 = fixed_is_1 ? sn : fixed;
    // tau cells: from the inner sphere (nothing inside it), split at the outer one, graded
    // towards the foot when the integrand does not vanish there
    const double tstart = haveA ? rhoA / L : 0.0;
    if (tstart >= 1.0) return;
    constexpr int NT = 4 + kMaxGrade;
    double tp[NT];
#pragma unroll
    for (int j = 0; j < NT; j++) tp[j] = kSentinel;
    tp[0] = tstart;
    tp[1] = 1.0;
    if (haveB) {
        const double t = rhoB / L;
        if (t > tstart && t < 1.0) tp[2] = t;
    }
    if (!haveA && c != 0.0) {
        double t = fabs(c) / L;
#pragma unroll
        for (int g = 0; g < kMaxGrade; g++) {
            if (t > tstart && t < 1.0) tp[3 + g] = t;
            t *= 3.0;
        }
    }
    sort_fixed<NT>(tp);
    const double wsn = glw[iq] * shm * ap * (p > 0 ? 1.0 : -1.0);
#pragma unroll
    for (int jt = 0; jt < NT - 1; jt++) {
        const double ta = tp[jt], tb = tp[jt + 1];
        if (!(tb > ta) || tb > 1.0) continue;
        const double thm = 0.5 * (tb - ta), thc = 0.5 * (tb + ta);
        for (int q = 0; q < nq; q++) {
            const double tau = thc + thm * glx[q];
            double y[3];
            y[AX] = c;
            y[A1] = tau * ey1;
            y[A2] = tau * ey2;
            const double ny = sqrt(c2 + tau * tau * L * L);
            const double wgt = wsn * thm * glw[q] * tau;
            node_contrib<AX, ANI>(m, y, ny, wgt, s, s1, s2, D, Ra, Rb, inv_r, ih, g3x, g3w);
        }
    }
}

template <int AX, bool ANI>
__host__ __device__ inline void gen_square(int nq, const double *glx, const double *glw, const double *g3x,
                                           const double *g3w, const double D[3], double Ra, double Rb, double inv_r,
                                           const double *hv, const double *ih, int s, int s1, int s2, int iv, int iq,
                                           double m[kMoments])
{
    gen_edge<AX, 0, ANI>(nq, glx, glw, g3x, g3w, D, Ra, Rb, inv_r, hv, ih, s, s1, s2, iv, iq, m);
    gen_edge<AX, 1, ANI>(nq, glx, glw, g3x, g3w, D, Ra, Rb, inv_r, hv, ih, s, s1, s2, iv, iq, m);
    gen_edge<AX, 2, ANI>(nq, glx, glw, g3x, g3w, D, Ra, Rb, inv_r, hv, ih, s, s1, s2, iv, iq, m);
    gen_edge<AX, 3, ANI>(nq, glx, glw, g3x, g3w, D, Ra, Rb, inv_r, hv, ih, s, s1, s2, iv, iq, m);
}

// Number of work items per (offset, shell): 36 unit squares x 5 s-intervals x nq s-nodes.
__host__ __device__ inline int gen_items(int nq) { return 36 * 5 * nq; }

// Item index -> (unit square, s-interval, s-node); the four edges of the square are
// handled inside the item.  Dispatch on the plane axis.  Inlined by force: as a called
// function its moment accumulators lived in scratch memory (192 bytes per lane).
template <bool ANI>
__host__ __device__ __attribute__((always_inline)) inline void gen_item(int nq, const double *glx, const double *glw, const double *g3x,
                                         const double *g3w, const double D[3], int a, double r, const double *hv,
                                         const double *ih, int it, double m[kMoments])
{
    const double Ra = a * r, Rb = (a + 1) * r, inv_r = 1.0 / r;
    const int iq = it % nq;
    const int rest = it / nq;
    const int iv = rest % 5;
    const int sq = rest / 5;
    const int ax = sq / 12, rem = sq % 12;
    const int s = rem / 4 - 1;
    const int s1 = (rem & 1) ? 1 : -1, s2 = (rem & 2) ? 1 : -1;
    if (ax == 0) gen_square<0, ANI>(nq, glx, glw, g3x, g3w, D, Ra, Rb, inv_r, hv, ih, s, s1, s2, iv, iq, m);
    else if (ax == 1) gen_square<1, ANI>(nq, glx, glw, g3x, g3w, D, Ra, Rb, inv_r, hv, ih, s, s1, s2, iv, iq, m);
    else gen_square<2, ANI>(nq, glx, glw, g3x, g3w, D, Ra, Rb, inv_r, hv, ih, s, s1, s2, iv, iq, m);
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <bool ANI>
__global__ void __launch_bounds__(kGenThreads) k_gen_moments(double *__restrict__ mom, GenArg ga)
{
    const int idx = blockIdx.x;
    const int dx = idx % ga.Uo, dy = (idx / ga.Uo) % ga.Vo, dz = idx / (ga.Uo * ga.Vo);
    const double D[3] = {dx * ga.hv[0], dy * ga.hv[1], dz * ga.hv[2]};
    int a_lo, nsh;
    shell_range(dx, dy, dz, ga.hv, ga.r, a_lo, nsh);
    double *out = mom + (size_t)idx * ga.ms * kMoments;
    const int nq = ga.nq;
    __shared__ double glx[kMaxQ], glw[kMaxQ], g3x[3], g3w[3];
    for (int i = threadIdx.x; i < kMaxQ; i += kGenThreads) {
        glx[i] = ga.glx[i];
        glw[i] = ga.glw[i];
    }
    if (threadIdx.x < 3) {
        g3x[threadIdx.x] = ga.g3x[threadIdx.x];
        g3w[threadIdx.x] = ga.g3w[threadIdx.x];
    }
    __syncthreads();
    const int nitems = gen_items(nq);
    const double r = ga.r;
    for (int sh = 0; sh < ga.ms; sh++) {
        double m[kMoments];
#pragma unroll
        for (int i = 0; i < kMoments; i++) m[i] = 0.0;
        const int a = a_lo + sh;
        if (sh < nsh) {
            for (int it = threadIdx.x; it < nitems; it += kGenThreads)
                gen_item<ANI>(nq, glx, glw, g3x, g3w, D, a, r, ga.hv, ga.ih, it, m);
        }
#pragma unroll
        for (int i = 0; i < kMoments; i++) {
            double v = wave_sum(m[i]);
            if (threadIdx.x == 0) out[sh * kMoments + i] = v;
        }
    }
}

// K_k at an octant offset >= 0 from the moments of its shells a_lo .. a_lo + nsh - 1.
__host__ __device__ inline void kernel_from_shells(const double *mom_d, int a_lo, int nsh, int k, double r,
                                                   double K[6])
{
    for (int i = 0; i < 6; i++) K[i] = 0.0;
    // B(k+1-|d|/r) on shell k-p as a quadratic in v = |d|/r - a:  p=0: (1-v)^2/2, p=1: (1+2v-2v^2)/2,
    // p=2: v^2/2; the time derivatives bring B'' / r^2
    const double cg[3][3] = {{0.5, -1.0, 0.5}, {0.5, 1.0, -1.0}, {0.0, 0.0, 0.5}};
    const double ir2 = 1.0 / (r * r);
    const double cb[3] = {ir2, -2.0 * ir2, ir2};  // B'' on the three pieces
    for (int p = 0; p < 3; p++) {
        int sh = k - p - a_lo;
        if (sh < 0 || sh >= nsh) continue;
        const double *m = mom_d + sh * kMoments;
        for (int al = 0; al < 3; al++)
            K[al] += cg[p][0] * m[3 * al] + cg[p][1] * m[3 * al + 1] + cg[p][2] * m[3 * al + 2] - cb[p] * m[18];
        for (int pr = 0; pr < 3; pr++)
            K[3 + pr] += cg[p][0] * m[9 + 3 * pr] + cg[p][1] * m[9 + 3 * pr + 1] + cg[p][2] * m[9 + 3 * pr + 2];
    }
    for (int i = 0; i < 6; i++) K[i] *= kInvFourPi;
}

// K_k at integer octant offset (dx,dy,dz) >= 0 from the shell moments.
__host__ __device__ inline void kernel_from_moments(const double *mom_d, int dx, int dy, int dz, int k, double r,
                                                    const double hv[3], double K[6])
{
    int a_lo, nsh;
    shell_range(dx, dy, dz, hv, r, a_lo, nsh);
    kernel_from_shells(mom_d, a_lo, nsh, k, r, K);
    // exact zeros of the odd components on their symmetry planes
    if (dx == 0 || dy == 0) K[3] = 0.0;
    if (dx == 0 || dz == 0) K[4] = 0.0;
    if (dy == 0 || dz == 0) K[5] = 0.0;
}

struct MomView {
    const double *mom;   // [Wo][Vo][Uo][ms][kMoments]
    int Uo, Vo, Wo, ms;
    double r;
    double hv[3];
};

__device__ inline void kernel_at(const MomView &g, int k, int Dx, int Dy, int Dz, double K[6])
{
    int ax = Dx < 0 ? -Dx : Dx, ay = Dy < 0 ? -Dy : Dy, az = Dz < 0 ? -Dz : Dz;
    const double *md = g.mom + ((size_t)(az * g.Vo + ay) * g.Uo + ax) * g.ms * kMoments;
    kernel_from_moments(md, ax, ay, az, k, g.r, g.hv, K);
    double sx = Dx < 0 ? -1.0 : 1.0, sy = Dy < 0 ? -1.0 : 1.0, sz = Dz < 0 ? -1.0 : 1.0;
    K[3] *= sx * sy;
    K[4] *= sx * sz;
    K[5] *= sy * sz;
}

// Periodic embedding on the Nx x Ny x Nz grid: index i holds offset i (i < U) or i - N
// (i > N - U); the remaining indices are zero (Appendix A, first column of the circulant).
__global__ void k_kernel_grid(MomView g, int k, int Nx, int Ny, int Nz, double *__restrict__ grid)
{
    const int Uo = g.Uo, Vo = g.Vo, Wo = g.Wo;
    size_t n = (size_t)Nx * Ny * Nz;
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int ix = (int)(i % Nx), iy = (int)((i / Nx) % Ny), iz = (int)(i / ((size_t)Nx * Ny));
    int Dx = ix < Uo ? ix : (ix > Nx - Uo ? ix - Nx : INT32_MAX);
    int Dy = iy < Vo ? iy : (iy > Ny - Vo ? iy - Ny : INT32_MAX);
    int Dz = iz < Wo ? iz : (iz > Nz - Wo ? iz - Nz : INT32_MAX);
    double K[6] = {0, 0, 0, 0, 0, 0};
    if (Dx != INT32_MAX && Dy != INT32_MAX && Dz != INT32_MAX) kernel_at(g, k, Dx, Dy, Dz, K);
    for (int c = 0; c < 6; c++) grid[c * n + i] = K[c];
}

__global__ void k_kernel_values(MomView g, int n, const int *__restrict__ lag, const int *__restrict__ off,
                                double *__restrict__ out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double K[6];
    kernel_at(g, lag[i], off[3 * i], off[3 * i + 1], off[3 * i + 2], K);
    for (int c = 0; c < 6; c++) out[6 * i + c] = K[c];
}

// ---------------------------------------------------------------------------- off-grid offsets
// Shell range for a real octant offset D >= 0 (the distances between points of the two
// voxels lie in [|max(D - 1, 0)|, |D + 1|]).
// D in voxel steps per axis; edges hv.
__host__ __device__ inline void shell_range_real(const double D[3], const double hv[3], double r, int &a_lo,
                                                 int &nsh)
{
    double a2 = 0.0, b2 = 0.0;
    for (int i = 0; i < 3; i++) {
        const double e = D[i] > 1.0 ? (D[i] - 1.0) * hv[i] : 0.0;
        a2 += e * e;
        b2 += ((D[i] + 1.0) * hv[i]) * ((D[i] + 1.0) * hv[i]);
    }
    shell_bounds(a2, b2, r, a_lo, nsh);
    if (nsh > kShellCap) nsh = kShellCap;   // cannot happen for r >= kMinCdtOverH
}

// K_k for k = kmin .. kmin + nw - 1 at the signed real offset Ds, serially (host checks and
// reference): fold to the octant, quadrature of every shell, parity signs.
__host__ __device__ inline void fold_offset(const double Ds[3], double D[3], double sg[3])
{
    for (int i = 0; i < 3; i++) {
        D[i] = Ds[i] < 0.0 ? -Ds[i] : Ds[i];
        sg[i] = Ds[i] < 0.0 ? -1.0 : 1.0;
    }
}

__host__ __device__ inline void finish_offgrid(const double D[3], const double sg[3], double K[6])
{
    if (D[0] == 0.0 || D[1] == 0.0) K[3] = 0.0;
    if (D[0] == 0.0 || D[2] == 0.0) K[4] = 0.0;
    if (D[1] == 0.0 || D[2] == 0.0) K[5] = 0.0;
    K[3] *= sg[0] * sg[1];
    K[4] *= sg[0] * sg[2];
    K[5] *= sg[1] * sg[2];
}

struct OffgridArg {
    const double *pos;        // [np][3] test-voxel centres, voxel steps per axis from the grid corner
    const int *pair_probe;    // [npairs]
    const int *pair_vox;      // [npairs] source voxel, linear index u + U (v + V w)
    const int *pair_kmin;     // [npairs] first lag of the window
    int U, V;
    double r;                 // c dt
    double hv[3], ih[3];      // voxel edges and their inverses
    int nw;                   // lags per pair
    int kmax;                 // lags above kmax are stored as zero
    long npairs;
    double *out;              // [nw][npairs][6]: for one window slot, consecutive pairs are adjacent
};

// One 64-lane block per (test voxel, source voxel) pair: shell moments by the same face
// quadrature as the grid kernels, then the pair's window of lags.
template <bool ANI>
__global__ void __launch_bounds__(kGenThreads) k_offgrid_table(OffgridArg oa, GenArg ga)
{
    const long i = blockIdx.x;
    const int p = oa.pair_probe[i], vox = oa.pair_vox[i];
    const int u = vox % oa.U, v = (vox / oa.U) % oa.V, w = vox / (oa.U * oa.V);
    const double Ds[3] = {oa.pos[3 * p] - (u + 0.5), oa.pos[3 * p + 1] - (v + 0.5), oa.pos[3 * p + 2] - (w + 0.5)};
    double Dv[3], sg[3];
    fold_offset(Ds, Dv, sg);
    int a_lo, nsh;
    shell_range_real(Dv, oa.hv, oa.r, a_lo, nsh);
    const double D[3] = {Dv[0] * oa.hv[0], Dv[1] * oa.hv[1], Dv[2] * oa.hv[2]};
    const int nq = ga.nq;
    __shared__ double glx[kMaxQ], glw[kMaxQ], g3x[3], g3w[3];
    __shared__ double mom[kShellCap * kMoments];
    for (int t = threadIdx.x; t < kMaxQ; t += kGenThreads) {
        glx[t] = ga.glx[t];
        glw[t] = ga.glw[t];
    }
    if (threadIdx.x < 3) {
        g3x[threadIdx.x] = ga.g3x[threadIdx.x];
        g3w[threadIdx.x] = ga.g3w[threadIdx.x];
    }
    __syncthreads();
    const int nitems = gen_items(nq);
    for (int sh = 0; sh < nsh; sh++) {
        double m[kMoments];
#pragma unroll
        for (int t = 0; t < kMoments; t++) m[t] = 0.0;
        for (int it = threadIdx.x; it < nitems; it += kGenThreads)
            gen_item<ANI>(nq, glx, glw, g3x, g3w, D, a_lo + sh, oa.r, oa.hv, oa.ih, it, m);
#pragma unroll
        for (int t = 0; t < kMoments; t++) {
            const double s_ = wave_sum(m[t]);
            if (threadIdx.x == 0) mom[sh * kMoments + t] = s_;
        }
    }
    __syncthreads();
    for (int wl = threadIdx.x; wl < oa.nw; wl += kGenThreads) {
        const int k = oa.pair_kmin[i] + wl;
        double K[6] = {0, 0, 0, 0, 0, 0};
        if (k <= oa.kmax) {
            kernel_from_shells(mom, a_lo, nsh, k, oa.r, K);
            finish_offgrid(D, sg, K);
        }
        double *o = oa.out + ((long)wl * oa.npairs + i) * 6;
        for (int c = 0; c < 6; c++) o[c] = K[c];
    }
}

// Gauss-Legendre rule on [-1, 1]: roots of P_n by Newton's method from Tricomi's initial
// guesses, in long double; weights 2 / ((1 - x^2) P_n'(x)^2).
void legendre_rule(int n, double *x, double *w)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; i++) {
        long double th = pi * (4.0L * (i + 1) - 1.0L) / (4.0L * n + 2.0L);
        long double z = (1.0L - (n - 1.0L) / (8.0L * n * n * n)) * cosl(th);
        long double dp = 0.0L;
        for (int iter = 0; iter < 60; iter++) {
            long double pm = 1.0L, pc = z;  // P_0, P_1
            for (int j = 1; j < n; j++) {
                long double pn = ((2.0L * j + 1.0L) * z * pc - j * pm) / (j + 1.0L);
                pm = pc;
                pc = pn;
            }
            dp = n * (pm - z * pc) / (1.0L - z * z);
            long double dz = pc / dp;
            z -= dz;
            if (fabsl(dz) <= 1e-19L * fabsl(z) + 1e-30L) break;
        }
        long double pm = 1.0L, pc = z;
        for (int j = 1; j < n; j++) {
            long double pn = ((2.0L * j + 1.0L) * z * pc - j * pm) / (j + 1.0L);
            pm = pc;
            pc = pn;
        }
        dp = n * (pm - z * pc) / (1.0L - z * z);
        x[n - 1 - i] = (double)z;   // ascending order
        w[n - 1 - i] = (double)(2.0L / ((1.0L - z * z) * dp * dp));
    }
}

}  // namespace

static void check_geometry(double r, const double hv[3])
{
    const double hmin = fmin(hv[0], fmin(hv[1], hv[2])), hmax = fmax(hv[0], fmax(hv[1], hv[2]));
    if (!(hmin > 0.0) || !(r <= hmin * (1.0 + 1e-12)) || !(r >= kMinCdtOverH * hmax))
        throw ArgError("c dt must lie in [0.3 max(h), min(h)]");
    if (shells_per_offset(r, hv) > kShellCap) throw ArgError("too many kernel shells per voxel pair");
}

void gen_moments(GenResult &g, int U, int V, int W, double r, const double hv[3], int nquad, const DevAlloc &da,
                 hipStream_t st)
{
    if (nquad < 4 || nquad > kMaxQ) throw ArgError("quad_order must be in [4, 24]");
    check_geometry(r, hv);
    GenArg ga{};
    ga.Uo = U;
    ga.Vo = V;
    ga.Wo = W;
    ga.nq = nquad;
    ga.r = r;
    for (int i = 0; i < 3; i++) {
        ga.hv[i] = hv[i];
        ga.ih[i] = 1.0 / hv[i];
        g.hv[i] = hv[i];
    }
    ga.ms = shells_per_offset(r, hv);
    legendre_rule(nquad, ga.glx, ga.glw);
    legendre_rule(3, ga.g3x, ga.g3w);
    g.Uo = U;
    g.Vo = V;
    g.Wo = W;
    g.ms = ga.ms;
    g.r = r;
    size_t noff = (size_t)U * V * W;
    size_t bytes = noff * g.ms * kMoments * sizeof(double);
    g.moments = (double *)da.get(bytes, "kernel moments");
    MJ_CHECK(hipMemsetAsync(g.moments, 0, bytes, st));
    if (hv[1] != 1.0 || hv[2] != 1.0)
        hipLaunchKernelGGL(k_gen_moments<true>, dim3((unsigned)noff), dim3(kGenThreads), 0, st, g.moments, ga);
    else
        hipLaunchKernelGGL(k_gen_moments<false>, dim3((unsigned)noff), dim3(kGenThreads), 0, st, g.moments, ga);
    MJ_CHECK(hipGetLastError());
}

void gen_kernel_grid(const GenResult &g, int k, int Nx, int Ny, int Nz, double *grid, hipStream_t st)
{
    size_t n = (size_t)Nx * Ny * Nz;
    dim3 blk(256), grd((unsigned)((n + 255) / 256));
    const MomView mv{g.moments, g.Uo, g.Vo, g.Wo, g.ms, g.r, {g.hv[0], g.hv[1], g.hv[2]}};
    hipLaunchKernelGGL(k_kernel_grid, grd, blk, 0, st, mv, k, Nx, Ny, Nz, grid);
    MJ_CHECK(hipGetLastError());
}

void gen_kernel_values(const GenResult &g, int n, const int *lag_dev, const int *off_dev, double *out_dev,
                       hipStream_t st)
{
    if (n <= 0) return;
    const MomView mv{g.moments, g.Uo, g.Vo, g.Wo, g.ms, g.r, {g.hv[0], g.hv[1], g.hv[2]}};
    hipLaunchKernelGGL(k_kernel_values, dim3((n + 127) / 128), dim3(128), 0, st, mv, n, lag_dev, off_dev, out_dev);
    MJ_CHECK(hipGetLastError());
}

void gen_offgrid_table(const double *pos_dev, const int *pair_probe_dev, const int *pair_vox_dev,
                       const int *pair_kmin_dev, long npairs, int U, int V, double r, const double hv[3], int nw,
                       int kmax, int nquad, double *out_dev, hipStream_t st)
{
    if (npairs <= 0) return;
    check_geometry(r, hv);
    if (nquad < 4 || nquad > kMaxQ) throw ArgError("quad_order must be in [4, 24]");
    if (npairs > 0x7fffffffL) throw ArgError("too many probe pairs");
    GenArg ga{};
    ga.nq = nquad;
    legendre_rule(nquad, ga.glx, ga.glw);
    legendre_rule(3, ga.g3x, ga.g3w);
    OffgridArg oa{};
    oa.pos = pos_dev;
    oa.pair_probe = pair_probe_dev;
    oa.pair_vox = pair_vox_dev;
    oa.pair_kmin = pair_kmin_dev;
    oa.U = U;
    oa.V = V;
    oa.r = r;
    for (int i = 0; i < 3; i++) {
        oa.hv[i] = hv[i];
        oa.ih[i] = 1.0 / hv[i];
    }
    oa.nw = nw;
    oa.kmax = kmax;
    oa.npairs = npairs;
    oa.out = out_dev;
    if (hv[1] != 1.0 || hv[2] != 1.0)
        hipLaunchKernelGGL(k_offgrid_table<true>, dim3((unsigned)npairs), dim3(kGenThreads), 0, st, oa, ga);
    else
        hipLaunchKernelGGL(k_offgrid_table<false>, dim3((unsigned)npairs), dim3(kGenThreads), 0, st, oa, ga);
    MJ_CHECK(hipGetLastError());
}

}  // namespace mj
