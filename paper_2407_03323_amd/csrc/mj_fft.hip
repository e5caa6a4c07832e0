// Padded 3-D FFTs of real vector fields (FP64), hand-written for gfx950.
//
// The history sum uses the circulant embedding of the three-level block-Toeplitz
// interaction matrices (Appendix A): fields on the U x V x W voxel box are
// zero-padded to an Nx x Ny x Nz grid with N >= 2U - 1 per axis, transformed,
// multiplied point-wise in the spectral domain and transformed back; only the
// box part of the inverse is kept.
//
// Each 1-D pass loads a tile of pencils into LDS, runs a Stockham autosort FFT
// (decimation in time, natural-order output) stage by stage between two LDS
// buffers, and writes the tile back.  Pencils along y and z are strided in
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

#include <cmath>

namespace mj {

namespace {

constexpr int kThreads = 256;
static const int kRadices[] = {8, 4, 2, 3, 5, 7, 11, 13};

__device__ inline double2 tw_at(const double2 *tw, int m, bool inv)
{
    double2 w = tw[m];
    return inv ? make_double2(w.x, -w.y) : w;
}

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
        const int st = N / R;
        double2 o[R];
#pragma unroll
        for (int q = 0; q < R; q++) {
            double2 acc = v[0];
#pragma unroll
            for (int t = 1; t < R; t++) {
                double2 w = tw_at(tw, ((q * t) % R) * st, inv);
                acc.x += v[t].x * w.x - v[t].y * w.y;
                acc.y += v[t].x * w.y + v[t].y * w.x;
            }
            o[q] = acc;
        }
#pragma unroll
        for (int q = 0; q < R; q++) v[q] = o[q];
    }
}

// One Stockham stage on P pencils of length N stored with leading dimension ld.
template <int R>
__device__ void stage(const double2 *src, double2 *dst, int N, int Ns, int P, int ld, const double2 *tw,
                      bool inv)
{
    const int nb = N / R;
    const int step = N / (Ns * R);
    for (int b = threadIdx.x; b < P * nb; b += blockDim.x) {
        int p = b / nb, j = b - p * nb;
        const double2 *s = src + p * ld;
        double2 v[R];
        int jm = j % Ns;
#pragma unroll
        for (int r = 0; r < R; r++) v[r] = s[j + r * nb];
#pragma unroll
        for (int r = 1; r < R; r++) v[r] = cmul(v[r], tw_at(tw, jm * r * step, inv));
        dft_small<R>(v, tw, N, inv);
        int base = (j / Ns) * Ns * R + jm;
        double2 *d = dst + p * ld;
#pragma unroll
        for (int r = 0; r < R; r++) d[base + r * Ns] = v[r];
    }
}

struct PlanArg {
    int N, nst;
    int radix[kMaxStages];
};

// Runs all stages; returns the LDS buffer holding the result (a or b).
__device__ double2 *lds_fft(double2 *a, double2 *b, int P, int ld, const PlanArg &pl, const double2 *tw, bool inv)
{
    int Ns = 1;
    double2 *src = a, *dst = b;
    for (int s = 0; s < pl.nst; s++) {
        int R = pl.radix[s];
        switch (R) {
        case 2: stage<2>(src, dst, pl.N, Ns, P, ld, tw, inv); break;
        case 3: stage<3>(src, dst, pl.N, Ns, P, ld, tw, inv); break;
        case 4: stage<4>(src, dst, pl.N, Ns, P, ld, tw, inv); break;
        case 5: stage<5>(src, dst, pl.N, Ns, P, ld, tw, inv); break;
        case 7: stage<7>(src, dst, pl.N, Ns, P, ld, tw, inv); break;
        case 8: stage<8>(src, dst, pl.N, Ns, P, ld, tw, inv); break;
        case 11: stage<11>(src, dst, pl.N, Ns, P, ld, tw, inv); break;
        default: stage<13>(src, dst, pl.N, Ns, P, ld, tw, inv); break;
        }
        __syncthreads();
        Ns *= R;
        double2 *t = src;
        src = dst;
        dst = t;
    }
    return src;
}

__device__ inline void load_twiddles(double2 *tw_s, const double2 *tw, int N)
{
    for (int i = threadIdx.x; i < N; i += blockDim.x) tw_s[i] = tw[i];
}

// ---------------------------------------------------------------------------- x pass
// Forward: rows of U reals (row r at x + r*U), nrows rows; two rows per pencil.
// Output: rows of Hx complex at X + r*Hx.
__global__ void __launch_bounds__(kThreads) k_fft_x_fwd(const double *__restrict__ x, double2 *__restrict__ X,
                                                        int nrows, int U, int Hx, PlanArg pl, const double2 *tw, int P)
{
    extern __shared__ double2 sm[];
    const int N = pl.N, ld = N + 1;
    double2 *tw_s = sm;
    double2 *a = sm + N;
    double2 *b = a + P * ld;
    load_twiddles(tw_s, tw, N);
    const int row0 = blockIdx.x * (2 * P);
    // load: pencil p takes rows row0 + 2p (real part) and row0 + 2p + 1 (imaginary part)
    for (int i = threadIdx.x; i < P * N; i += blockDim.x) {
        int p = i / N, n = i - p * N;
        a[p * ld + n] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * P * U; i += blockDim.x) {
        int rr = i / U, u = i - rr * U;
        int row = row0 + rr;
        if (row < nrows) {
            double v = x[(size_t)row * U + u];
            double2 *slot = &a[(rr >> 1) * ld + u];
            if (rr & 1) slot->y = v; else slot->x = v;
        }
    }
    __syncthreads();
    double2 *res = lds_fft(a, b, P, ld, pl, tw_s, false);
    // separate: Xa[k] = (Z[k] + conj Z[N-k]) / 2, Xb[k] = (Z[k] - conj Z[N-k]) / (2i)
    for (int i = threadIdx.x; i < 2 * P * Hx; i += blockDim.x) {
        int rr = i / Hx, k = i - rr * Hx;
        int row = row0 + rr;
        if (row >= nrows) continue;
        const double2 *Z = res + (rr >> 1) * ld;
        double2 z1 = Z[k], z2 = Z[(N - k) % N];
        double2 o;
        if (rr & 1) o = make_double2(0.5 * (z1.y + z2.y), -0.5 * (z1.x - z2.x));
        else o = make_double2(0.5 * (z1.x + z2.x), 0.5 * (z1.y - z2.y));
        X[(size_t)row * Hx + k] = o;
    }
}

// Inverse: rows of Hx complex half-spectra -> rows of U reals (unnormalised).
__global__ void __launch_bounds__(kThreads) k_fft_x_inv(const double2 *__restrict__ X, double *__restrict__ y,
                                                        int nrows, int U, int Hx, PlanArg pl, const double2 *tw, int P)
{
    extern __shared__ double2 sm[];
    const int N = pl.N, ld = N + 1;
    double2 *tw_s = sm;
    double2 *a = sm + N;
    double2 *b = a + P * ld;
    load_twiddles(tw_s, tw, N);
    const int row0 = blockIdx.x * (2 * P);
    // Z[k] = Xa[k] + i Xb[k] for k <= N/2, Z[N-k] = conj(Xa[k]) + i conj(Xb[k]) for 0 < k < N/2
    for (int i = threadIdx.x; i < P * N; i += blockDim.x) {
        int p = i / N, n = i - p * N;
        int ra = row0 + 2 * p, rb = ra + 1;
        double2 xa = make_double2(0, 0), xb = make_double2(0, 0);
        int k = n <= N / 2 ? n : N - n;
        bool conj = n > N / 2;
        if (ra < nrows) xa = X[(size_t)ra * Hx + k];
        if (rb < nrows) xb = X[(size_t)rb * Hx + k];
        if (conj) {
            xa.y = -xa.y;
            xb.y = -xb.y;
        }
        a[p * ld + n] = make_double2(xa.x - xb.y, xa.y + xb.x);
    }
    __syncthreads();
    double2 *res = lds_fft(a, b, P, ld, pl, tw_s, true);
    for (int i = threadIdx.x; i < 2 * P * U; i += blockDim.x) {
        int rr = i / U, u = i - rr * U;
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

__global__ void __launch_bounds__(kThreads) k_fft_strided(const double2 *__restrict__ in, double2 *__restrict__ out,
                                                          StridedArg g, PlanArg pl, const double2 *tw, int P,
                                                          int inv)
{
    extern __shared__ double2 sm[];
    const int N = pl.N, ld = N + 1;
    double2 *tw_s = sm;
    double2 *a = sm + N;
    double2 *b = a + P * ld;
    load_twiddles(tw_s, tw, N);
    const int ntile = (g.Hx + P - 1) / P;
    const int tile = blockIdx.x % ntile;
    const int grp = blockIdx.x / ntile;
    const int c = grp / g.nq, q = grp - c * g.nq;
    const int kx0 = tile * P;
    const int np = min(P, g.Hx - kx0);
    const double2 *src = in + c * g.cs_in + q * g.qs_in + kx0;
    for (int i = threadIdx.x; i < P * N; i += blockDim.x) {
        int n = i / P, p = i - n * P;
        double2 v = make_double2(0.0, 0.0);
        if (n < g.n_in && p < np) v = src[(long)n * g.es_in + p];
        a[p * ld + n] = v;
    }
    __syncthreads();
    double2 *res = lds_fft(a, b, P, ld, pl, tw_s, inv != 0);
    double2 *dst = out + c * g.cs_out + q * g.qs_out + kx0;
    for (int i = threadIdx.x; i < P * g.n_out; i += blockDim.x) {
        int n = i / P, p = i - n * P;
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

int pencils_per_block(int N) { return N <= 64 ? 16 : (N <= 128 ? 12 : 8); }

size_t lds_bytes(int N, int P) { return sizeof(double2) * (size_t)(N + 2 * P * (N + 1)); }

bool factor(int N, std::vector<int> &out)
{
    out.clear();
    int n = N;
    // prefer radix 4 (then 8 for leftovers of 2s), then the odd radices
    while (n % 4 == 0) { out.push_back(4); n /= 4; }
    while (n % 2 == 0) { out.push_back(2); n /= 2; }
    for (int r : {3, 5, 7, 11, 13})
        while (n % r == 0) { out.push_back(r); n /= r; }
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

void fft_plan_init(FftPlan1D &p, int N)
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
    MJ_CHECK(hipMalloc(&p.tw, sizeof(double2) * N));
    MJ_CHECK(hipMemcpy(p.tw, h.data(), sizeof(double2) * N, hipMemcpyHostToDevice));
}

void fft_plan_free(FftPlan1D &p)
{
    if (p.tw) (void)hipFree(p.tw);
    p.tw = nullptr;
}

void fft3d_init(Fft3D &f, int U, int V, int W, int ncomp, int Nx, int Ny, int Nz)
{
    f.U = U; f.V = V; f.W = W;
    f.Nx = Nx; f.Ny = Ny; f.Nz = Nz;
    f.Hx = Nx / 2 + 1;
    f.ncomp = ncomp;
    fft_plan_init(f.px, Nx);
    fft_plan_init(f.py, Ny);
    fft_plan_init(f.pz, Nz);
    size_t na = (size_t)ncomp * W * V * f.Hx, nb = (size_t)ncomp * W * Ny * f.Hx;
    if (hipMalloc(&f.bufA, sizeof(double2) * na) != hipSuccess) throw MemError("FFT scratch A");
    if (hipMalloc(&f.bufB, sizeof(double2) * nb) != hipSuccess) throw MemError("FFT scratch B");
}

void fft3d_free(Fft3D &f)
{
    fft_plan_free(f.px);
    fft_plan_free(f.py);
    fft_plan_free(f.pz);
    if (f.bufA) (void)hipFree(f.bufA);
    if (f.bufB) (void)hipFree(f.bufB);
    f.bufA = f.bufB = nullptr;
}

static void launch_strided(const double2 *in, double2 *out, const StridedArg &g, int ncomp, const FftPlan1D &p,
                           bool inv, hipStream_t st)
{
    int P = pencils_per_block(p.N);
    int ntile = (g.Hx + P - 1) / P;
    dim3 grid(ncomp * g.nq * ntile);
    hipLaunchKernelGGL(k_fft_strided, grid, dim3(kThreads), lds_bytes(p.N, P), st, in, out, g, plan_arg(p), p.tw, P,
                       inv ? 1 : 0);
    MJ_CHECK(hipGetLastError());
}

void fft3d_forward(Fft3D &f, const double *x, double2 *X, int ncomp, hipStream_t st)
{
    const int U = f.U, V = f.V, W = f.W, Hx = f.Hx, Ny = f.Ny, Nz = f.Nz;
    // x pass: rows (c, w, v)
    {
        int nrows = ncomp * W * V;
        int P = pencils_per_block(f.Nx);
        dim3 grid((nrows + 2 * P - 1) / (2 * P));
        hipLaunchKernelGGL(k_fft_x_fwd, grid, dim3(kThreads), lds_bytes(f.Nx, P), st, x, f.bufA, nrows, U, Hx,
                           plan_arg(f.px), f.px.tw, P);
        MJ_CHECK(hipGetLastError());
    }
    // y pass: groups (c, w); A[c][w][v][kx] -> B[c][w][ky][kx]
    {
        StridedArg g{};
        g.nq = W; g.Hx = Hx;
        g.cs_in = (long)W * V * Hx; g.qs_in = (long)V * Hx; g.es_in = Hx;
        g.cs_out = (long)W * Ny * Hx; g.qs_out = (long)Ny * Hx; g.es_out = Hx;
        g.n_in = V; g.n_out = Ny;
        launch_strided(f.bufA, f.bufB, g, ncomp, f.py, false, st);
    }
    // z pass: groups (c, ky); B[c][w][ky][kx] -> X[c][kz][ky][kx]
    {
        StridedArg g{};
        g.nq = Ny; g.Hx = Hx;
        g.cs_in = (long)W * Ny * Hx; g.qs_in = Hx; g.es_in = (long)Ny * Hx;
        g.cs_out = (long)Nz * Ny * Hx; g.qs_out = Hx; g.es_out = (long)Ny * Hx;
        g.n_in = W; g.n_out = Nz;
        launch_strided(f.bufB, X, g, ncomp, f.pz, false, st);
    }
}

void fft3d_inverse(Fft3D &f, const double2 *X, double *y, int ncomp, hipStream_t st)
{
    const int U = f.U, V = f.V, W = f.W, Hx = f.Hx, Ny = f.Ny, Nz = f.Nz;
    // z pass: X[c][kz][ky][kx] -> B[c][w][ky][kx], w < W
    {
        StridedArg g{};
        g.nq = Ny; g.Hx = Hx;
        g.cs_in = (long)Nz * Ny * Hx; g.qs_in = Hx; g.es_in = (long)Ny * Hx;
        g.cs_out = (long)W * Ny * Hx; g.qs_out = Hx; g.es_out = (long)Ny * Hx;
        g.n_in = Nz; g.n_out = W;
        launch_strided(X, f.bufB, g, ncomp, f.pz, true, st);
    }
    // y pass: B[c][w][ky][kx] -> A[c][w][v][kx], v < V
    {
        StridedArg g{};
        g.nq = W; g.Hx = Hx;
        g.cs_in = (long)W * Ny * Hx; g.qs_in = (long)Ny * Hx; g.es_in = Hx;
        g.cs_out = (long)W * V * Hx; g.qs_out = (long)V * Hx; g.es_out = Hx;
        g.n_in = Ny; g.n_out = V;
        launch_strided(f.bufB, f.bufA, g, ncomp, f.py, true, st);
    }
    // x pass: rows (c, w, v) of Hx -> U reals
    {
        int nrows = ncomp * W * V;
        int P = pencils_per_block(f.Nx);
        dim3 grid((nrows + 2 * P - 1) / (2 * P));
        hipLaunchKernelGGL(k_fft_x_inv, grid, dim3(kThreads), lds_bytes(f.Nx, P), st, f.bufA, y, nrows, U, Hx,
                           plan_arg(f.px), f.px.tw, P);
        MJ_CHECK(hipGetLastError());
    }
}

}  // namespace mj
