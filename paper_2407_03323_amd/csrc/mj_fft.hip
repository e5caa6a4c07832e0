// Padded 3-D FFTs of real vector fields (FP64), hand-written for gfx950.
//
// The history sum uses the circulant embedding of the three-level block-Toeplitz
// interaction matrices (Appendix A): fields on the U x V x W voxel box are
// zero-padded to an Nx x Ny x Nz grid with N >= 2U - 1 per axis, transformed,
// multiplied point-wise in the spectral domain and transformed back; only the
// box part of the inverse is kept.
//
// Each 1-D pass loads a tile of pencils into LDS, runs a Stockham autosort FFT
// (decimation in time, natural-order output) stage by stage in place (each stage
// reads its butterflies into registers, synchronises, writes them back), and
// writes the tile back.  Pencils along y and z are strided in
// memory; a tile covers consecutive x-frequencies so every global access is a
// run of consecutive complex values.  The x pass packs two real rows into one
// complex pencil (real and imaginary part) and separates the two half-spectra
// afterwards (and the reverse for the inverse).  Zero padding is never stored:
// the forward passes read only the U (V, W) live inputs, the inverse passes
// write only the box outputs.
//
// Twiddles come from a table W_N^m computed on the host in long double and
// rounded once, so no recurrence error accumulates.

#include "mj_internal.h"

#include <algorithm>
#include <cmath>

namespace mj {

namespace {

constexpr int kThreads = 256;

// Division by a divisor that is the same in every lane (a tile or plan size), by one multiply:
// for x < 2^16 and 1 <= d <= 2^16, floor(x / d) = floor(x m / 2^32) with m = floor(2^32 / d) + 1,
// since x m / 2^32 exceeds x / d by less than 2^-16 and the fraction of x / d is at most
// 1 - 1/d.  Building m is scalar work (d is uniform); the per-element quotient replaces the
// reciprocal-and-correct sequence of a division by a run-time divisor, which dominated the
// integer work of the index arithmetic.  Every index divided here is below 2^16.
struct FastDiv {
    unsigned d;
    unsigned long long m;
    __device__ explicit FastDiv(unsigned dv) : d(dv), m((1ull << 32) / dv + 1) {}
    __device__ unsigned div(unsigned x) const { return (unsigned)(((unsigned long long)x * m) >> 32); }
    __device__ unsigned mod(unsigned x) const { return x - div(x) * d; }
};

__device__ inline double2 tw_at(const double2 *tw, int m, bool inv)
{
    double2 w = tw[m];
    return inv ? make_double2(w.x, -w.y) : w;
}

// cos(2 pi m / R) and sin(2 pi m / R), m = 1 .. (R-1)/2, of the odd radices, interleaved, from
// offset odd_base(R).  They are the same for every N, so they sit in constant memory, where the
// compiler keeps them in scalar registers.
__constant__ double c_odd_cs[2 * (1 + 2 + 3 + 5 + 6)];
constexpr int odd_base(int R) { return R == 3 ? 0 : R == 5 ? 2 : R == 7 ? 6 : R == 11 ? 12 : 22; }

// In-register R-point DFT, v[q] <- sum_t v[t] W_R^{q t} (W_R = exp(-+2 pi i / R)).
template <int R>
__device__ inline void dft_small(double2 *v, const double2 *tw, int N, bool inv)
{
    if constexpr (R == 2) {
        double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        double2 a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
        double2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
        double2 s13 = cadd(a1, a3), d13 = csub(a1, a3);
        // forward: -i * d13 ; inverse: +i * d13
        double2 r = inv ? make_double2(-d13.y, d13.x) : make_double2(d13.y, -d13.x);
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, r);
        v[3] = csub(d02, r);
    } else {
        // odd R: pair inputs t and R - t.  With a_t = v_t + v_{R-t}, b_t = v_t - v_{R-t},
        // c_m = cos(2 pi m / R), s_m = sin(2 pi m / R) and sg = -1 (forward) or +1 (inverse):
        //   out_q     = v_0 + sum_t a_t c_{qt} + i sg sum_t b_t s_{qt}
        //   out_{R-q} = v_0 + sum_t a_t c_{qt} - i sg sum_t b_t s_{qt}     (q, t = 1 .. (R-1)/2)
        static_assert(R % 2 == 1, "even radices other than 2 and 4 are not used");
        constexpr int H = (R - 1) / 2;
        double cm[H + 1], sm[H + 1];
#pragma unroll
        for (int m = 1; m <= H; m++) {
            cm[m] = c_odd_cs[odd_base(R) + 2 * (m - 1)];
            sm[m] = c_odd_cs[odd_base(R) + 2 * (m - 1) + 1];
        }
        double2 a[H + 1], b[H + 1];
        double2 sum = v[0];
#pragma unroll
        for (int t = 1; t <= H; t++) {
            a[t] = cadd(v[t], v[R - t]);
            b[t] = csub(v[t], v[R - t]);
            sum = cadd(sum, a[t]);
        }
        const double sg = inv ? 1.0 : -1.0;
        const double2 v0 = v[0];
        v[0] = sum;
#pragma unroll
        for (int q = 1; q <= H; q++) {
            double2 A = v0, B = make_double2(0.0, 0.0);
#pragma unroll
            for (int t = 1; t <= H; t++) {
                const int m = (q * t) % R;
                // cos is even and sin odd about R/2: fold m into 1 .. H
                const double c = m <= H ? cm[m] : cm[R - m];
                const double sn = m <= H ? sm[m] : -sm[R - m];
                A.x += a[t].x * c;
                A.y += a[t].y * c;
                B.x += b[t].x * sn;
                B.y += b[t].y * sn;
            }
            // i sg B = (-sg B.y, sg B.x)
            const double2 iB = make_double2(-sg * B.y, sg * B.x);
            v[q] = cadd(A, iB);
            v[R - q] = csub(A, iB);
        }
    }
}

// A tile holds at most kTileElems complex values (P pencils of length N, P * N <= kTileElems).
constexpr int kTileElems = 3072;
static_assert(kMaxFftN <= kTileElems, "one pencil must fit a tile");

// One Stockham stage, in place, on P pencils of length N stored with leading dimension ld.
// Every thread first reads and transforms all of its butterflies (at most BF of them), the
// block synchronises, and only then are the results written back over the inputs; the caller
// synchronises again before the next stage.
template <int R>
__device__ void stage(double2 *buf, int N, int Ns, int P, int ld, const double2 *tw, bool inv)
{
    constexpr int BF = (kTileElems / R + kThreads - 1) / kThreads;
    const int nb = N / R;
    const int step = N / (Ns * R);
    const int total = P * nb;
    const FastDiv fnb(nb), fns(Ns);
    double2 v[BF][R];
#pragma unroll
    for (int f = 0; f < BF; f++) {
        const int b = (int)threadIdx.x + f * kThreads;
        if (b < total) {
            const int p = fnb.div(b), j = b - p * nb, jm = fns.mod(j);
            const double2 *s = buf + p * ld;
#pragma unroll
            for (int r = 0; r < R; r++) v[f][r] = s[j + r * nb];
#pragma unroll
            for (int r = 1; r < R; r++) v[f][r] = cmul(v[f][r], tw_at(tw, jm * r * step, inv));
            dft_small<R>(v[f], tw, N, inv);
        }
    }
    __syncthreads();
#pragma unroll
    for (int f = 0; f < BF; f++) {
        const int b = (int)threadIdx.x + f * kThreads;
        if (b < total) {
            const int p = fnb.div(b), j = b - p * nb, jq = fns.div(j), jm = j - jq * Ns;
            const int base = jq * Ns * R + jm;
            double2 *d = buf + p * ld;
#pragma unroll
            for (int r = 0; r < R; r++) d[base + r * Ns] = v[f][r];
        }
    }
}

struct PlanArg {
    int N, nst;
    int radix[kMaxStages];
};

// Radix sets: a kernel instantiated for set MASK holds code (and registers) only for the
// radices in it.  The generic instance kAll serves every plan.
constexpr int kR2 = 1, kR3 = 2, kR4 = 4, kR5 = 8, kR7 = 16, kR11 = 32, kR13 = 64, kAll = 127;

// Stage of radix R for a plan whose radices lie in MASK: tests the radices of MASK in turn;
// the last one is taken without a test (the plan guarantees R is in MASK).
constexpr int kRadixOfBit[7] = {2, 3, 4, 5, 7, 11, 13};
constexpr int lowest_bit(int m) { return (m & 1) ? 0 : 1 + lowest_bit(m >> 1); }

template <int MASK>
__device__ inline void stage_of(int R, double2 *buf, int N, int Ns, int P, int ld, const double2 *tw, bool inv)
{
    constexpr int b = lowest_bit(MASK);
    constexpr int RB = kRadixOfBit[b];
    constexpr int REST = MASK & ~(1 << b);
    if constexpr (REST == 0) {
        stage<RB>(buf, N, Ns, P, ld, tw, inv);
    } else {
        if (R == RB) stage<RB>(buf, N, Ns, P, ld, tw, inv);
        else stage_of<REST>(R, buf, N, Ns, P, ld, tw, inv);
    }
}

// Runs all stages in place on the tile in buf.
template <int MASK>
__device__ void lds_fft(double2 *buf, int P, int ld, const PlanArg &pl, const double2 *tw, bool inv)
{
    int Ns = 1;
    for (int s = 0; s < pl.nst; s++) {
        const int R = pl.radix[s];
        stage_of<MASK>(R, buf, pl.N, Ns, P, ld, tw, inv);
        __syncthreads();
        Ns *= R;
    }
}

__device__ inline void load_twiddles(double2 *tw_s, const double2 *tw, int N)
{
    for (int i = threadIdx.x; i < N; i += blockDim.x) tw_s[i] = tw[i];
}

// Moves a tile from global memory into LDS: every thread first issues kBatch independent
// loads (get(i) for items i = i0 + u * kThreads + tid), then stores them (put(i, v)), so
// that the loads of a thread overlap instead of each waiting out the memory latency.
constexpr int kBatch = 8;
template <typename T, class Get, class Put>
__device__ inline void gather_tile(int total, Get get, Put put)
{
    for (int i0 = 0; i0 < total; i0 += kThreads * kBatch) {
        T v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; u++) {
            const int i = i0 + u * kThreads + (int)threadIdx.x;
            v[u] = i < total ? get(i) : T{};
        }
#pragma unroll
        for (int u = 0; u < kBatch; u++) {
            const int i = i0 + u * kThreads + (int)threadIdx.x;
            if (i < total) put(i, v[u]);
        }
    }
}

// ---------------------------------------------------------------------------- x pass
// Forward: rows of U reals (row r at x + r*U), nrows rows; two rows per pencil.
// Output: rows of Hx complex at X + r*Hp.
template <int MASK>
__global__ void __launch_bounds__(kThreads) k_fft_x_fwd(const double *__restrict__ x, double2 *__restrict__ X,
                                                        int nrows, int U, int Hx, int Hp, PlanArg pl, const double2 *tw,
                                                        int P)
{
    extern __shared__ double2 sm[];
    const int N = pl.N, ld = N + 1;
    double2 *tw_s = sm;
    double2 *a = sm + N;
    load_twiddles(tw_s, tw, N);
    const int row0 = (int)xcd_block(blockIdx.x, gridDim.x) * (2 * P);
    const FastDiv fN(N), fU(U), fH(Hx);
    // load: pencil p takes rows row0 + 2p (real part) and row0 + 2p + 1 (imaginary part)
    for (int i = threadIdx.x; i < P * N; i += blockDim.x) {
        int p = fN.div(i), n = i - p * N;
        a[p * ld + n] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    gather_tile<double>(
        2 * P * U,
        [&](int i) {
            const int rr = fU.div(i), u = i - rr * U, row = row0 + rr;
            return row < nrows ? x[(size_t)row * U + u] : 0.0;
        },
        [&](int i, double v) {
            const int rr = fU.div(i), u = i - rr * U;
            double2 *slot = &a[(rr >> 1) * ld + u];
            if (rr & 1) slot->y = v; else slot->x = v;
        });
    __syncthreads();
    lds_fft<MASK>(a, P, ld, pl, tw_s, false);
    const double2 *res = a;
    // separate: Xa[k] = (Z[k] + conj Z[N-k]) / 2, Xb[k] = (Z[k] - conj Z[N-k]) / (2i)
    for (int i = threadIdx.x; i < 2 * P * Hx; i += blockDim.x) {
        int rr = fH.div(i), k = i - rr * Hx;
        int row = row0 + rr;
        if (row >= nrows) continue;
        const double2 *Z = res + (rr >> 1) * ld;
        double2 z1 = Z[k], z2 = Z[k == 0 ? 0 : N - k];
        double2 o;
        if (rr & 1) o = make_double2(0.5 * (z1.y + z2.y), -0.5 * (z1.x - z2.x));
        else o = make_double2(0.5 * (z1.x + z2.x), 0.5 * (z1.y - z2.y));
        X[(size_t)row * Hp + k] = o;
    }
}

// Inverse: rows of Hx complex half-spectra (pitch Hp) -> rows of U reals (unnormalised).
template <int MASK>
__global__ void __launch_bounds__(kThreads) k_fft_x_inv(const double2 *__restrict__ X, double *__restrict__ y,
                                                        int nrows, int U, int Hx, int Hp, PlanArg pl, const double2 *tw,
                                                        int P)
{
    extern __shared__ double2 sm[];
    const int N = pl.N, ld = N + 1;
    double2 *tw_s = sm;
    double2 *a = sm + N;
    load_twiddles(tw_s, tw, N);
    const int row0 = (int)xcd_block(blockIdx.x, gridDim.x) * (2 * P);
    const FastDiv fN(N), fU(U);
    // Z[k] = Xa[k] + i Xb[k] for k <= N/2, Z[N-k] = conj(Xa[k]) + i conj(Xb[k]) for 0 < k < N/2
    gather_tile<double4>(
        P * N,
        [&](int i) {
            const int p = fN.div(i), n = i - p * N;
            const int ra = row0 + 2 * p, rb = ra + 1;
            const int k = n <= N / 2 ? n : N - n;
            double2 xa = make_double2(0, 0), xb = make_double2(0, 0);
            if (ra < nrows) xa = X[(size_t)ra * Hp + k];
            if (rb < nrows) xb = X[(size_t)rb * Hp + k];
            return make_double4(xa.x, xa.y, xb.x, xb.y);
        },
        [&](int i, double4 v) {
            const int p = fN.div(i), n = i - p * N;
            double2 xa = make_double2(v.x, v.y), xb = make_double2(v.z, v.w);
            if (n > N / 2) {
                xa.y = -xa.y;
                xb.y = -xb.y;
            }
            a[p * ld + n] = make_double2(xa.x - xb.y, xa.y + xb.x);
        });
    __syncthreads();
    lds_fft<MASK>(a, P, ld, pl, tw_s, true);
    const double2 *res = a;
    for (int i = threadIdx.x; i < 2 * P * U; i += blockDim.x) {
        int rr = fU.div(i), u = i - rr * U;
        int row = row0 + rr;
        if (row >= nrows) continue;
        double2 z = res[(rr >> 1) * ld + u];
        y[(size_t)row * U + u] = (rr & 1) ? z.y : z.x;
    }
}

// ---------------------------------------------------------------------------- strided pass
// Pencil groups g = (c, q), c < ncomp, q < nq.  Group g holds Hx pencils (consecutive in
// memory, index kx) with elements at stride es.  Input base c*cs_in + q*qs_in, n_in live
// elements (the rest are zero); output base c*cs_out + q*qs_out, first n_out elements stored.
struct StridedArg {
    int nq, Hx;
    long cs_in, qs_in, es_in, cs_out, qs_out, es_out;
    int n_in, n_out;
};

template <int MASK>
__global__ void __launch_bounds__(kThreads) k_fft_strided(const double2 *__restrict__ in, double2 *__restrict__ out,
                                                          StridedArg g, PlanArg pl, const double2 *tw, int P,
                                                          int inv)
{
    extern __shared__ double2 sm[];
    const int N = pl.N, ld = N + 1;
    double2 *tw_s = sm;
    double2 *a = sm + N;
    load_twiddles(tw_s, tw, N);
    const int ntile = (g.Hx + P - 1) / P;
    const int lb = (int)xcd_block(blockIdx.x, gridDim.x);   // neighbouring tiles share row ends
    const int tile = lb % ntile;
    const int grp = lb / ntile;
    const int c = grp / g.nq, q = grp - c * g.nq;
    const int kx0 = tile * P;
    const int np = min(P, g.Hx - kx0);
    const FastDiv fP(P);
    const double2 *src = in + c * g.cs_in + q * g.qs_in + kx0;
    gather_tile<double2>(
        P * N,
        [&](int i) {
            const int n = fP.div(i), p = i - n * P;
            return (n < g.n_in && p < np) ? src[(long)n * g.es_in + p] : make_double2(0.0, 0.0);
        },
        [&](int i, double2 v) {
            const int n = fP.div(i), p = i - n * P;
            a[p * ld + n] = v;
        });
    __syncthreads();
    lds_fft<MASK>(a, P, ld, pl, tw_s, inv != 0);
    const double2 *res = a;
    double2 *dst = out + c * g.cs_out + q * g.qs_out + kx0;
    for (int i = threadIdx.x; i < P * g.n_out; i += blockDim.x) {
        int n = fP.div(i), p = i - n * P;
        if (p < np) dst[(long)n * g.es_out + p] = res[p * ld + n];
    }
}

PlanArg plan_arg(const FftPlan1D &p)
{
    PlanArg a{};
    a.N = p.N;
    a.nst = p.nst;
    for (int i = 0; i < p.nst; i++) a.radix[i] = p.radix[i];
    return a;
}

int pencils_per_block(int N) { return std::max(1, std::min(16, kTileElems / N)); }

size_t lds_bytes(int N, int P) { return sizeof(double2) * (size_t)(N + P * (N + 1)); }

// Radices of the stages, in order.  The first stage (Ns = 1) writes its R outputs with a stride
// of R complex values in LDS, so an odd radix goes first: a stride of 13 x 16 bytes spreads the
// lanes over every bank, where a stride of 4 x 16 bytes puts four lanes on each bank group.
// Later stages write runs of Ns consecutive values.  Then radix 4 as often as possible, and 2.
bool factor(int N, std::vector<int> &out)
{
    out.clear();
    int n = N;
    for (int r : {13, 11, 7, 5, 3})
        while (n % r == 0) { out.push_back(r); n /= r; }
    while (n % 4 == 0) { out.push_back(4); n /= 4; }
    while (n % 2 == 0) { out.push_back(2); n /= 2; }
    return n == 1 && (int)out.size() <= kMaxStages;
}

}  // namespace

bool fft_size_ok(int N)
{
    std::vector<int> f;
    return N >= 2 && N <= kMaxFftN && N % 2 == 0 && factor(N, f);
}

int fft_pick_size(int nmin)
{
    for (int N = nmin; N <= kMaxFftN; N++)
        if (fft_size_ok(N)) return N;
    throw ArgError("grid too large for the FFT (padded size above " + std::to_string(kMaxFftN) + ")");
}

void fft_plan_init(FftPlan1D &p, int N, const DevAlloc &da)
{
    std::vector<int> f;
    if (!fft_size_ok(N) || !factor(N, f)) throw ArgError("unsupported FFT size " + std::to_string(N));
    p.N = N;
    p.nst = (int)f.size();
    for (int i = 0; i < p.nst; i++) p.radix[i] = f[i];
    std::vector<double2> h(N);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int m = 0; m < N; m++) {
        long double ang = -2.0L * pi * (long double)m / (long double)N;
        h[m] = make_double2((double)cosl(ang), (double)sinl(ang));
    }
    p.tw = (double2 *)da.get(sizeof(double2) * N, "FFT twiddles");
    MJ_CHECK(hipMemcpy(p.tw, h.data(), sizeof(double2) * N, hipMemcpyHostToDevice));
    // the odd-radix constants, rounded the same way (cheap; repeated for every plan so that
    // the device current at plan creation has them)
    double cs[2 * (1 + 2 + 3 + 5 + 6)];
    for (int R : {3, 5, 7, 11, 13})
        for (int m = 1; m <= (R - 1) / 2; m++) {
            long double ang = 2.0L * pi * (long double)m / (long double)R;
            cs[odd_base(R) + 2 * (m - 1)] = (double)cosl(ang);
            cs[odd_base(R) + 2 * (m - 1) + 1] = (double)sinl(ang);
        }
    MJ_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_odd_cs), cs, sizeof(cs)));
}

void fft_plan_free(FftPlan1D &p, const DevAlloc &da)
{
    da.put(p.tw);
    p.tw = nullptr;
}

void fft3d_init(Fft3D &f, int U, int V, int W, int ncomp, int Nx, int Ny, int Nz, const DevAlloc &da)
{
    f.da = da;
    f.U = U; f.V = V; f.W = W;
    f.Nx = Nx; f.Ny = Ny; f.Nz = Nz;
    f.Hx = Nx / 2 + 1;
    f.Hp = spectrum_pitch(f.Hx);
    f.ncomp = ncomp;
    fft_plan_init(f.px, Nx, da);
    fft_plan_init(f.py, Ny, da);
    fft_plan_init(f.pz, Nz, da);
    fft3d_set_pencils(f, 1 << 30);
    size_t na = (size_t)ncomp * W * V * f.Hp, nb = (size_t)ncomp * W * Ny * f.Hp;
    f.bufA = (double2 *)da.get(sizeof(double2) * na, "FFT scratch A");
    f.bufB = (double2 *)da.get(sizeof(double2) * nb, "FFT scratch B");
}

void fft3d_free(Fft3D &f)
{
    fft_plan_free(f.px, f.da);
    fft_plan_free(f.py, f.da);
    fft_plan_free(f.pz, f.da);
    f.da.put(f.bufA);
    f.da.put(f.bufB);
    f.bufA = f.bufB = nullptr;
}

// Radix set of a plan, and the kernel instance that serves it: the sets of the usual padded
// sizes (208 = 13 4 4; powers of two; 3 2^k) have their own instances, any other plan the
// generic one.
static int plan_mask(const FftPlan1D &p)
{
    int m = 0;
    for (int i = 0; i < p.nst; i++) {
        switch (p.radix[i]) {
        case 2: m |= kR2; break;
        case 3: m |= kR3; break;
        case 4: m |= kR4; break;
        case 5: m |= kR5; break;
        case 7: m |= kR7; break;
        case 11: m |= kR11; break;
        default: m |= kR13; break;
        }
    }
    return m;
}

#define MJ_FFT_DISPATCH(mask, KERNEL, ...)                                                        \
    do {                                                                                          \
        switch (mask) {                                                                           \
        case kR4 | kR13: hipLaunchKernelGGL(KERNEL<kR4 | kR13>, __VA_ARGS__); break;              \
        case kR4: hipLaunchKernelGGL(KERNEL<kR4>, __VA_ARGS__); break;                            \
        case kR2 | kR4: hipLaunchKernelGGL(KERNEL<kR2 | kR4>, __VA_ARGS__); break;                \
        case kR3 | kR4: hipLaunchKernelGGL(KERNEL<kR3 | kR4>, __VA_ARGS__); break;                \
        case kR2 | kR3 | kR4: hipLaunchKernelGGL(KERNEL<kR2 | kR3 | kR4>, __VA_ARGS__); break;    \
        default: hipLaunchKernelGGL(KERNEL<kAll>, __VA_ARGS__); break;                            \
        }                                                                                         \
    } while (0)

static void launch_strided(const double2 *in, double2 *out, const StridedArg &g, int ncomp, const FftPlan1D &p,
                           int P, bool inv, hipStream_t st)
{
    int ntile = (g.Hx + P - 1) / P;
    dim3 grid(ncomp * g.nq * ntile);
    MJ_FFT_DISPATCH(plan_mask(p), k_fft_strided, grid, dim3(kThreads), lds_bytes(p.N, P), st, in, out, g,
                    plan_arg(p), p.tw, P, inv ? 1 : 0);
    MJ_CHECK(hipGetLastError());
}

// The six passes; P is the number of pencils per block of the pass (x: 2P real rows).
// x pass forward: rows (c, w, v) of U reals -> A[c][w][v][kx]
static void pass_x_fwd(const Fft3D &f, int ncomp, const double *x, int P, hipStream_t st)
{
    const int nrows = ncomp * f.W * f.V;
    dim3 grid((nrows + 2 * P - 1) / (2 * P));
    MJ_FFT_DISPATCH(plan_mask(f.px), k_fft_x_fwd, grid, dim3(kThreads), lds_bytes(f.Nx, P), st, x, f.bufA, nrows,
                    f.U, f.Hx, f.Hp, plan_arg(f.px), f.px.tw, P);
    MJ_CHECK(hipGetLastError());
}
// y pass forward: groups (c, w); A[c][w][v][kx] -> B[c][w][ky][kx]
static void pass_y_fwd(const Fft3D &f, int ncomp, int P, hipStream_t st)
{
    StridedArg g{};
    g.nq = f.W; g.Hx = f.Hx;
    g.cs_in = (long)f.W * f.V * f.Hp; g.qs_in = (long)f.V * f.Hp; g.es_in = f.Hp;
    g.cs_out = (long)f.W * f.Ny * f.Hp; g.qs_out = (long)f.Ny * f.Hp; g.es_out = f.Hp;
    g.n_in = f.V; g.n_out = f.Ny;
    launch_strided(f.bufA, f.bufB, g, ncomp, f.py, P, false, st);
}
// z pass forward: groups (c, ky); B[c][w][ky][kx] -> X[c][kz][ky][kx]
static void pass_z_fwd(const Fft3D &f, int ncomp, double2 *X, int P, hipStream_t st)
{
    StridedArg g{};
    g.nq = f.Ny; g.Hx = f.Hx;
    g.cs_in = (long)f.W * f.Ny * f.Hp; g.qs_in = f.Hp; g.es_in = (long)f.Ny * f.Hp;
    g.cs_out = (long)f.Nz * f.Ny * f.Hp; g.qs_out = f.Hp; g.es_out = (long)f.Ny * f.Hp;
    g.n_in = f.W; g.n_out = f.Nz;
    launch_strided(f.bufB, X, g, ncomp, f.pz, P, false, st);
}
// z pass inverse: X[c][kz][ky][kx] -> B[c][w][ky][kx], w < W
static void pass_z_inv(const Fft3D &f, int ncomp, const double2 *X, int P, hipStream_t st)
{
    StridedArg g{};
    g.nq = f.Ny; g.Hx = f.Hx;
    g.cs_in = (long)f.Nz * f.Ny * f.Hp; g.qs_in = f.Hp; g.es_in = (long)f.Ny * f.Hp;
    g.cs_out = (long)f.W * f.Ny * f.Hp; g.qs_out = f.Hp; g.es_out = (long)f.Ny * f.Hp;
    g.n_in = f.Nz; g.n_out = f.W;
    launch_strided(X, f.bufB, g, ncomp, f.pz, P, true, st);
}
// y pass inverse: B[c][w][ky][kx] -> A[c][w][v][kx], v < V
static void pass_y_inv(const Fft3D &f, int ncomp, int P, hipStream_t st)
{
    StridedArg g{};
    g.nq = f.W; g.Hx = f.Hx;
    g.cs_in = (long)f.W * f.Ny * f.Hp; g.qs_in = (long)f.Ny * f.Hp; g.es_in = f.Hp;
    g.cs_out = (long)f.W * f.V * f.Hp; g.qs_out = (long)f.V * f.Hp; g.es_out = f.Hp;
    g.n_in = f.Ny; g.n_out = f.V;
    launch_strided(f.bufB, f.bufA, g, ncomp, f.py, P, true, st);
}
// x pass inverse: rows (c, w, v) of Hx -> U reals
static void pass_x_inv(const Fft3D &f, int ncomp, double *y, int P, hipStream_t st)
{
    const int nrows = ncomp * f.W * f.V;
    dim3 grid((nrows + 2 * P - 1) / (2 * P));
    MJ_FFT_DISPATCH(plan_mask(f.px), k_fft_x_inv, grid, dim3(kThreads), lds_bytes(f.Nx, P), st, f.bufA, y, nrows,
                    f.U, f.Hx, f.Hp, plan_arg(f.px), f.px.tw, P);
    MJ_CHECK(hipGetLastError());
}

// ncomp <= the plan's ncomp (the scratch buffers are sized for that)
void fft3d_forward(Fft3D &f, const double *x, double2 *X, int ncomp, hipStream_t st)
{
    if (ncomp < 1 || ncomp > f.ncomp) throw std::logic_error("FFT batch larger than its plan");
    pass_x_fwd(f, ncomp, x, f.Px, st);
    pass_y_fwd(f, ncomp, f.Py, st);
    pass_z_fwd(f, ncomp, X, f.Pz, st);
}

void fft3d_inverse(Fft3D &f, const double2 *X, double *y, int ncomp, hipStream_t st)
{
    if (ncomp < 1 || ncomp > f.ncomp) throw std::logic_error("FFT batch larger than its plan");
    pass_z_inv(f, ncomp, X, f.Pz, st);
    pass_y_inv(f, ncomp, f.Py, st);
    pass_x_inv(f, ncomp, y, f.Px, st);
}

void fft3d_set_pencils(Fft3D &f, int cap)
{
    f.Px = std::max(1, std::min(cap, pencils_per_block(f.Nx)));
    f.Py = std::max(1, std::min(cap, pencils_per_block(f.Ny)));
    f.Pz = std::max(1, std::min(cap, pencils_per_block(f.Nz)));
}

// Picks the pencils per block of each axis pass by timing it.  A pencil's arithmetic does not
// depend on how many pencils share its block, so every choice gives bit-identical transforms;
// only the speed differs (row runs of the strided passes, blocks per compute unit).
// Candidates: the most a tile holds, and 3/4, 1/2 and 1/4 of that; each pass forward and
// inverse, best of three after one warm-up.
void fft3d_autotune(Fft3D &f, hipStream_t st)
{
    const size_t nX = (size_t)f.ncomp * f.Nz * f.Ny * f.Hp;
    double2 *X = (double2 *)f.da.get(sizeof(double2) * nX, "FFT autotune scratch");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    try {
        const size_t na = (size_t)f.ncomp * f.W * f.V * f.Hp, nb = (size_t)f.ncomp * f.W * f.Ny * f.Hp;
        MJ_CHECK(hipMemsetAsync(X, 0, sizeof(double2) * nX, st));
        MJ_CHECK(hipMemsetAsync(f.bufA, 0, sizeof(double2) * na, st));
        MJ_CHECK(hipMemsetAsync(f.bufB, 0, sizeof(double2) * nb, st));
        MJ_CHECK(hipEventCreate(&e0));
        MJ_CHECK(hipEventCreate(&e1));
        // bufB holds at least ncomp W V U reals: real input and output of the x pass
        double *xr = (double *)f.bufB;
        auto run = [&](int axis, int P) {
            if (axis == 0) {
                pass_x_fwd(f, f.ncomp, xr, P, st);
                pass_x_inv(f, f.ncomp, xr, P, st);
            } else if (axis == 1) {
                pass_y_fwd(f, f.ncomp, P, st);
                pass_y_inv(f, f.ncomp, P, st);
            } else {
                pass_z_fwd(f, f.ncomp, X, P, st);
                pass_z_inv(f, f.ncomp, X, P, st);
            }
        };
        const int Ns[3] = {f.Nx, f.Ny, f.Nz};
        int *Ps[3] = {&f.Px, &f.Py, &f.Pz};
        for (int axis = 0; axis < 3; axis++) {
            const int pmax = pencils_per_block(Ns[axis]);
            int cand[4] = {pmax, (3 * pmax) / 4, pmax / 2, pmax / 4};
            float best = 0.0f;
            int bestP = pmax;
            for (int ci = 0; ci < 4; ci++) {
                const int P = cand[ci];
                if (P < 1 || (ci > 0 && std::find(cand, cand + ci, P) != cand + ci)) continue;
                run(axis, P);
                float tmin = 0.0f;
                for (int rep = 0; rep < 3; rep++) {
                    MJ_CHECK(hipEventRecord(e0, st));
                    run(axis, P);
                    MJ_CHECK(hipEventRecord(e1, st));
                    MJ_CHECK(hipEventSynchronize(e1));
                    float ms = 0.0f;
                    MJ_CHECK(hipEventElapsedTime(&ms, e0, e1));
                    if (rep == 0 || ms < tmin) tmin = ms;
                }
                if (ci == 0 || tmin < best) {
                    best = tmin;
                    bestP = P;
                }
            }
            *Ps[axis] = bestP;
        }
    } catch (...) {
        (void)hipStreamSynchronize(st);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        f.da.put(X);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    f.da.put(X);
}

}  // namespace mj
