// C interface and host orchestration of the MOT-JVIE march (see include/motjvie.h).
#include "motjvie.h"
#include "mj_march.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using mj::ArgError;
using mj::HipError;
using mj::MemError;
using mj::UnstableError;

namespace {

thread_local std::string g_err;

// voxels (per right-hand side) up to which z0_solver = 0 takes the Chebyshev solve
constexpr long kChebMaxUnknowns = 1L << 19;
// bytes of solve vectors per group of right-hand sides that the Chebyshev solve takes at once
constexpr size_t kChebGroupBytes = (size_t)320 << 20;

// whether outer_overlap = 0 runs the outer level of three on the second stream
constexpr bool kOverlapDefault = false;
// LDS each block of the second stream's launch claims: above half of a CU's 160 KB, so that a
// CU holds one such block (one wave per SIMD) and keeps room for the march's kernels
constexpr size_t kSideLdsReserve = 96 * 1024;

// ---------------------------------------------------------------------------- static staging
// mj_kernel_values_noalloc stages its requests and results through this file-scope array
// instead of allocating: kNoAllocMax requests, laid out as results [max][6] doubles, then
// lags [max] and offsets [max][3] as int32.  Every GPU the library runs on holds its own copy
// until the process ends.  In host code the name `scratch` is only a stand-in: the array's
// device address is looked up per device with hipGetSymbolAddress (with that device
// current) and kept in g_scratch; host code passes that address, never the name.
constexpr int kNoAllocMax = 65536;
constexpr size_t kNoAllocBytes = (size_t)kNoAllocMax * (6 * sizeof(double) + 4 * sizeof(int32_t));
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;                 // guards g_scratch
std::vector<unsigned char *> g_scratch;  // device address of `scratch` per device id (null: not looked up)
std::mutex g_noalloc_mu;                 // calls of one process take turns on the staging array

// Address of this device's copy of `scratch`; dev must be the current device.
unsigned char *scratch_ptr(int dev)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize((size_t)dev + 1, nullptr);
    if (!g_scratch[(size_t)dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            throw HipError(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[(size_t)dev] = (unsigned char *)ptr;
    }
    return g_scratch[(size_t)dev];
}

__global__ void k_extract_octant(const double2 *__restrict__ X, int Hx, int Hp, int Ny, int Nz, double scale,
                                 double *__restrict__ out)
{
    const int Nyo = Ny / 2 + 1, Nzo = Nz / 2 + 1;
    const long n = (long)Hp * Nyo * Nzo;
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int kx = (int)(t % Hp), qy = (int)((t / Hp) % Nyo), qz = (int)(t / ((long)Hp * Nyo));
    const long plane = (long)Nz * Ny * Hp;
    for (int c = 0; c < 6; c++)
        out[6 * t + c] = kx < Hx ? scale * X[c * plane + ((long)qz * Ny + qy) * Hp + kx].x : 0.0;
}

struct Events {
    std::vector<hipEvent_t> ev;
    void ensure(size_t n)
    {
        while (ev.size() < n) {
            hipEvent_t e;
            MJ_CHECK(hipEventCreate(&e));
            ev.push_back(e);
        }
    }
    ~Events()
    {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

}  // namespace

// n-point Gauss-Legendre rule on [-1/2, 1/2] (Newton on P_n from the Chebyshev-like start),
// weights summing to 1
static void gl_half(int n, double *x, double *w)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; i++) {
        long double zz = cosl(pi * (i + 0.75L) / (n + 0.5L));
        long double dp = 0;
        for (int itn = 0; itn < 50; itn++) {
            long double p0 = 1, p1 = zz;
            for (int j = 2; j <= n; j++) {
                long double p2 = ((2 * j - 1) * zz * p1 - (j - 1) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (zz * p1 - p0) / (zz * zz - 1);
            long double d = p1 / dp;
            zz -= d;
            if (fabsl(d) < 1e-19L) break;
        }
        x[i] = n == 1 ? 0.0 : (double)(0.5L * zz);
        w[i] = n == 1 ? 1.0 : (double)(1.0L / ((1 - zz * zz) * dp * dp));
    }
}

// Gauss-Legendre order for averaging exp(-((T - k h x) / w)^2) over x in [-1/2, 1/2] with spread
// s = |k| h / w: the least n <= 8 (the most the device tables hold) whose remainder bound
// (n!)^4 / ((2n + 1) ((2n)!)^3) s^2n max|H_2n(x) exp(-x^2)|, with Cramer's bound
// |H_m(x)| exp(-x^2 / 2) <= 1.0865 sqrt(2^m m!), stays below 2^-53, or 9 when none does.  0 spread takes the 1-point rule, which is then exact.
static int gl_order(double s)
{
    if (s == 0.0) return 1;
    for (int n = 1; n <= 8; n++) {
        double f = 1.0, f2 = 1.0;
        for (int i = 2; i <= n; i++) f *= i;
        for (int i = 2; i <= 2 * n; i++) f2 *= i;
        const double c = std::pow(f, 4) / ((2 * n + 1) * f2 * f2 * f2) * 1.0865 * std::sqrt(std::ldexp(f2, 2 * n));
        if (c * std::pow(s, 2 * n) <= std::ldexp(1.0, -53)) return n;
    }
    return 9;
}

// The averaging plan of a wave with two or more non-zero direction components on voxels of
// edges (h, hy, hz); see the fields of WaveArg.
static void plan_wave(mj::WaveArg &w, double h, double hy, double hz)
{
    const double kh[3] = {w.k[0] * h, w.k[1] * hy, w.k[2] * hz};
    int ax[3] = {0, 1, 2};
    std::stable_sort(ax, ax + 3, [&](int a, int b) { return std::fabs(kh[a]) > std::fabs(kh[b]); });
    int order[3];
    for (int i = 0; i < 3; i++) {
        w.kh[i] = kh[ax[i]];
        order[i] = gl_order(std::fabs(kh[ax[i]]) / w.width);
        w.nq[i] = std::min(order[i], 8);
    }
    // an erf pair costs about what 5 exponentials do
    w.form = order[1] > 8 ? 2 : order[0] >= 6 ? 1 : 0;
}

struct mj_solver {
    // geometry and configuration
    int U = 0, V = 0, W = 0;
    long M = 0;
    double h = 1.0, hy = 1.0, hz = 1.0, c_dt = 1.0;
    int nrhs = 1, ell = 0;
    int Nx = 0, Ny = 0, Nz = 0, Hx = 0, Hp = 0;
    std::vector<double> fir;
    double cg_rtol = 1e-13;
    int cg_maxit = 200;
    int B = 1;                      // steps per (inner) time block
    int B2 = 0;                     // steps per outer time block (three levels), 0: two levels
    int nquad = 16;
    hipStream_t st = nullptr;
    int nloc = 5, rdepth = 6;
    // degree of the extrapolated initial guess of the Z_0 solve: at 104^3 degree 6 (seven past
    // steps) takes 11.0 CG iterations, 4 takes 13.0 and 10 takes 12.2 (higher degrees amplify
    // the rounding noise of the history)
    int guess_deg = 6;
    // device state
    mj::DevAlloc da;                // hipMalloc, or the caller's allocator (mj_config.alloc)
    size_t bytes = 0;
    std::vector<void *> allocs;
    double *chi = nullptr, *schi = nullptr, *inv_eps = nullptr, *c0 = nullptr;
    double *fir_d = nullptr;
    double *Khat = nullptr;
    double2 *ring = nullptr, *Shat = nullptr, *farbuf = nullptr;
    double2 *gbuf = nullptr;        // outer-block partial sums [B2][nrhs][3][plane] (three levels)
    // Overlapped outer level (three levels): while an outer block marches, a second stream forms
    // the next block's outer sums over the sources before the current block; at the next block
    // start the sources of the block just marched are added on the caller's stream.
    bool overlap = false;
    double2 *hbuf = nullptr;        // those sums [B2][nrhs][3][plane], of the block starting at h_block
    int h_block = 0;                // 0: hbuf holds no block's sums
    hipStream_t side = nullptr;     // the library's second stream (non-blocking, default priority)
    hipEvent_t ev_main = nullptr, ev_side = nullptr;
    bool side_pending = false;      // work on `side` may still run: `st` waits for ev_side first
    static constexpr int kSideTimers = 8;
    hipEvent_t side_t[kSideTimers][2] = {};   // start and end of recent launches on `side`
    bool side_busy[kSideTimers] = {};
    int side_count = 0, side_done = 0;
    double side_ms = 0.0;
    double *S = nullptr, *Jr = nullptr;
    double *rhs = nullptr, *y = nullptr, *p = nullptr, *q = nullptr;
    double *u = nullptr, *uy = nullptr;
    double *parts = nullptr;
    mj::CgScalars *scal = nullptr;
    int cg_guess = 8;
    // Z_0 solver: 0 Chebyshev iteration (needs spectral bounds of M^-1 A), 1 CG
    int z0_method = 0;
    double lam_lo = 0.0, lam_hi = 0.0;   // bounds of the eigenvalues of M^-1 A (0: not estimated)
    double *e2 = nullptr;                // second buffer of s d for the Chebyshev passes (haloed)
    int cheb_pred = 0;                   // passes predicted for the next solve (0: none yet)
    std::vector<double> cheb_rho;        // Chebyshev recurrence scalars by pass index (for lam_lo, lam_hi)
    bool use_graphs = false;             // replay the Chebyshev batches from captured HIP graphs
    hipStream_t cap_st = nullptr;        // the library's own stream, for capturing (never the null stream)
    std::map<long, hipGraphExec_t> cheb_graphs;   // captured batches by (with init, first pass, passes)
    double cheb_rho2 = 0.0;              // observed reduction of |r|^2 per pass
    mj::CgStatus *cgstat = nullptr, *cgstat_h = nullptr;
    mj::WaveArg *waves_d = nullptr;
    bool waves_set = false;
    std::vector<mj::WaveArg> waves;
    mj::Fft3D fft{};
    mj::GenResult gen{};
    double K0_27[27 * 6] = {};
    double *k0_d = nullptr;         // K0_27 on the device (the Z_0 stencil of this solver)
    double *gl_d = nullptr;         // Gauss-Legendre rules of 1..8 points for the excitation
    int nblk = 1;
    int n = 0;
    int dev = 0;                    // device current at mj_create
    std::string err;
    // probes: scattered field at test voxels centred at arbitrary points
    std::vector<double> eps_h;
    int np = 0, nw = 0;
    long npairs = 0;
    double *probe_pos = nullptr, *ptable = nullptr, *ppart = nullptr, *pout = nullptr;
    int *pair_vox = nullptr, *pair_kmin = nullptr, *row_start = nullptr, *pinv = nullptr;
    int *ck_row = nullptr, *ck_lo = nullptr, *ck_hi = nullptr, *ck_start = nullptr;   // probe row chunks
    double *ptable_v = nullptr;   // probe kernel table ordered by voxel (adjoint source)
    int *pkmin_v = nullptr;
    long pnck = 0;
    // transposed march: local history lambda, and the right-hand side before its sqrt(chi) scaling
    double *Lr = nullptr, *bq = nullptr;
    // statistics of the last run
    double t_gen_ms = 0, t_spec_ms = 0, t_probe_ms = 0;
    double t_mac_tune_ms = 0;       // MAC time per step of the timed choice (time_block < 0)
    double stat[21] = {};
    Events events;

    template <class T>
    T *dalloc(size_t count, const char *what)
    {
        size_t b = count * sizeof(T);
        if (b == 0) b = sizeof(T);
        void *ptr = da.get(b, what);
        allocs.push_back(ptr);
        bytes += b;
        return (T *)ptr;
    }

    ~mj_solver()
    {
        if (st) (void)hipStreamSynchronize(st);
        if (side) {
            (void)hipStreamSynchronize(side);
            (void)hipStreamDestroy(side);
        }
        for (hipEvent_t e : {ev_main, ev_side})
            if (e) (void)hipEventDestroy(e);
        for (auto &pr : side_t)
            for (hipEvent_t e : pr)
                if (e) (void)hipEventDestroy(e);
        clear_graphs();
        if (cap_st) (void)hipStreamDestroy(cap_st);
        mj::fft3d_free(fft);
        da.put(gen.moments);
        for (void *a : allocs) da.put(a);
        if (cgstat_h) (void)hipHostFree(cgstat_h);
    }

    void dfree(void *&ptr)
    {
        if (!ptr) return;
        for (size_t i = 0; i < allocs.size(); i++)
            if (allocs[i] == ptr) {
                allocs.erase(allocs.begin() + (long)i);
                break;
            }
        da.put(ptr);
        ptr = nullptr;
    }

    long spec_plane() const { return (long)Nz * Ny * Hp; }
    long koct() const { return (long)Hp * (Ny / 2 + 1) * (Nz / 2 + 1); }
    int slotS(int j) const { return j % ell; }
    int slotR(int j) const { return j % rdepth; }

    void create(const mj_config &c);
    void build_spectra();
    void set_material(const double *eps);
    struct StepIO {
        hipEvent_t *ev = nullptr;       // 7 events, or NULL
        double *Jout = nullptr;         // forward: J_n copy
        double *Pout = nullptr;         // forward: probe field of the step (else the internal buffer)
        bool skip_probes = false;
        double *Bout = nullptr;         // forward: gradient term B_n
        char *far_kind = nullptr;       // 1 far (outer) launch, 2 near launch, 3 middle launch
        bool adjoint = false;           // transposed march
        const double *G = nullptr;      // adjoint: source g_j
        const double *Bj = nullptr;     // adjoint: B_j for the gradient (NULL: none)
        double *grad = nullptr;         // adjoint: gradient accumulator
    };
    mj::EpiArg epi_arg() const;
    const double2 *mac(int n, int *kind);
    void outer_sums(int nb, hipStream_t stream);
    void outer_overlapped(int nb);
    // `st` waits for the work on the second stream
    void join_side()
    {
        if (!side_pending) return;
        MJ_CHECK(hipStreamWaitEvent(st, ev_side, 0));
        side_pending = false;
    }
    // ... and forgets the sums it formed (the march, the ring or the time division changes)
    void drop_side()
    {
        join_side();
        h_block = 0;
    }
    void collect_side_timers(bool wait);
    void mac_autotune();
    void default_time_division();
    // arguments of a time-block MAC launch writing to `out`, first target step nb
    mj::BlockMacArg block_arg(double2 *out, int nb) const
    {
        mj::BlockMacArg a{};
        a.Khat = Khat;
        a.ring_base = ring;
        a.far = out;
        a.Hx = Hx;
        a.Hp = Hp;
        a.Ny = Ny;
        a.Nz = Nz;
        a.nk = ell;
        a.ring = ell;
        a.nb = nb;
        a.nrhs = nrhs;
        a.jmin = 1;
        return a;
    }
    mj::AdjArg adj_arg() const;
    void step(const StepIO &io);
    void check_growth() const;
    void run(int n_steps, double *Jout, double *Pout, int j_every = 1);
    void restart();
    void adjoint_gradient(int n_steps, int ckpt_every, double *phi, double *grad_dev, double *probe_hist);
    size_t state_bytes() const;
    void get_state(void *buf) const;
    void set_state(const void *buf, size_t bytes);
    void set_probes(int n_probes, const double *pos);
    void offgrid_values(int n, const int *probe, const int *vox, const int *lag, double *out);
    void solve_z0();
    mj::CgArg cg_arg() const;
    void solve_z0_chebyshev();
    void estimate_spectrum();
    void clear_graphs()
    {
        for (auto &kv : cheb_graphs) (void)hipGraphExecDestroy(kv.second);
        cheb_graphs.clear();
    }
    void history_sum(const double *Jh, int depth, double *P);
};

void mj_solver::create(const mj_config &c)
{
    if (c.U < 1 || c.V < 1 || c.W < 1) throw ArgError("U, V, W must be >= 1");
    if (!(c.h > 0.0) || !std::isfinite(c.h)) throw ArgError("h must be positive and finite");
    if (!(c.c_dt > 0.0) || !std::isfinite(c.c_dt)) throw ArgError("c_dt must be positive and finite");
    if (!(c.hy >= 0.0) || !(c.hz >= 0.0) || !std::isfinite(c.hy) || !std::isfinite(c.hz))
        throw ArgError("hy, hz must be finite and >= 0 (0: equal to h)");
    {
        // c dt <= every edge keeps K_0 on the 27-point stencil the Z_0 solve is built for
        const double ey = c.hy > 0.0 ? c.hy : c.h, ez = c.hz > 0.0 ? c.hz : c.h;
        const double hmin = std::min(c.h, std::min(ey, ez)), hmax = std::max(c.h, std::max(ey, ez));
        if (!(c.c_dt <= hmin * (1.0 + 1e-12) && c.c_dt >= mj::kMinCdtOverH * hmax))
            throw ArgError("c_dt must lie in [0.3 max(h, hy, hz), min(h, hy, hz)]");
    }
    if (!c.eps_r) throw ArgError("eps_r is NULL");
    if (c.n_fir < 0 || (c.n_fir > 0 && !c.fir)) throw ArgError("bad FIR taps");
    if (c.n_fir > mj::kMaxLocal) throw ArgError("at most 64 FIR taps");
    if (c.n_rhs < 1 || c.n_rhs > 64) throw ArgError("n_rhs must be in [1, 64]");
    if (c.fft_pencils < 0) throw ArgError("fft_pencils must be >= 0 (0: autotune)");
    if ((c.alloc == nullptr) != (c.free_ == nullptr)) throw ArgError("alloc and free_ are given together or not at all");
    if (c.z0_solver < 0 || c.z0_solver > 2) throw ArgError("z0_solver must be 0 (by size), 1 (CG) or 2 (Chebyshev)");
    if (c.outer_overlap < 0 || c.outer_overlap > 2)
        throw ArgError("outer_overlap must be 0 (default), 1 (in line) or 2 (on a second stream)");
    use_graphs = c.z0_graphs != 0;
    da.fn_alloc = c.alloc;
    da.fn_free = c.free_;
    da.ctx = c.alloc_ctx;
    U = c.U;
    V = c.V;
    W = c.W;
    M = (long)U * V * W;
    h = c.h;
    hy = c.hy > 0.0 ? c.hy : c.h;
    hz = c.hz > 0.0 ? c.hz : c.h;
    c_dt = c.c_dt;
    nrhs = c.n_rhs;
    cg_rtol = c.cg_rtol > 0 ? c.cg_rtol : 1e-13;
    cg_maxit = c.cg_maxit > 0 ? c.cg_maxit : 200;
    nquad = c.quad_order > 0 ? c.quad_order : 16;
    st = (hipStream_t)c.stream;
    fir.assign(c.fir, c.fir + c.n_fir);
    for (double d : fir)
        if (!std::isfinite(d)) throw ArgError("FIR taps must be finite");
    std::vector<double> eps(c.eps_r, c.eps_r + M);
    eps_h = eps;
    for (double e : eps)
        if (!(e >= 1.0) || !std::isfinite(e)) throw ArgError("eps_r must be finite and >= 1");
    // eq:Ell
    double diag = std::sqrt((U * h) * (U * h) + (V * hy) * (V * hy) + (W * hz) * (W * hz));
    ell = (int)std::floor(diag / c_dt + 1e-12) + 2;
    // zero padding N >= 2U - 1 per axis (Appendix A)
    Nx = mj::fft_pick_size(2 * U - 1);
    Ny = mj::fft_pick_size(2 * V - 1);
    Nz = mj::fft_pick_size(2 * W - 1);
    Hx = Nx / 2 + 1;
    Hp = mj::spectrum_pitch(Hx);
    const bool tune_mac = c.time_block < 0;
    B = c.time_block > 0 ? c.time_block : 8;
    if (!(B == 1 || B == 4 || B == 32 || (B >= 8 && B <= 16 && B % 2 == 0)))
        throw ArgError("time_block must be -1 (timed), 0 (default), 1, 4, 8, 10, 12, 14, 16 or 32");
    B2 = c.outer_block > 1 ? c.outer_block : 0;
    if (c.time_block == 0 && c.outer_block == 0) default_time_division();
    if (B2 && !(B == 4 || B == 8) ) throw ArgError("outer_block needs time_block 4 or 8");
    if (B2 && !(B2 > B && B2 % B == 0 && B2 >= 8 && B2 <= 16 && B2 % 2 == 0))
        throw ArgError("outer_block must be a multiple of time_block in 8 .. 16 (even), or 0");
    nloc = std::max(guess_deg + 1, (int)fir.size() - 1);   // the initial guess uses guess_deg + 1 steps
    rdepth = nloc + 1;

    // the Z_0 solve: Chebyshev passes cost one launch each against four per CG iteration, which
    // decides on small grids; on large ones CG's fewer iterations win (104^3: 12.9 CG iterations,
    // 1.02 ms, against 24 passes, 1.12 ms; 32^3: 0.48 against 0.19 ms).  A batch shares its
    // launches, so the size that decides is the grid's (16 right-hand sides at 64^3: 26 passes,
    // 5.98-6.07 ms, against 20 CG iterations, 6.23 ms)
    z0_method = c.z0_solver == 1 ? 1 : c.z0_solver == 2 ? 0 : (M <= kChebMaxUnknowns ? 0 : 1);
    MJ_CHECK(hipGetDevice(&dev));
    if (use_graphs) MJ_CHECK(hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking));
    (void)scratch_ptr(dev);   // this device's staging array (mj_kernel_values_noalloc)
    chi = dalloc<double>(M, "chi");
    schi = dalloc<double>(M, "sqrt chi");
    inv_eps = dalloc<double>(M, "1/eps");
    c0 = dalloc<double>(M, "c0");
    fir_d = dalloc<double>(std::max<size_t>(fir.size(), 1), "fir");
    if (!fir.empty()) MJ_CHECK(hipMemcpy(fir_d, fir.data(), fir.size() * 8, hipMemcpyHostToDevice));

    build_spectra();
    set_material(eps.data());

    // march state
    const long sp = spec_plane();
    ring = dalloc<double2>((size_t)ell * nrhs * 3 * sp, "spectral history ring");
    Shat = dalloc<double2>((size_t)nrhs * 3 * sp, "spectral sum");
    // a timed choice of the time division tries blocks of up to 16 steps at both levels
    const int fb_targets = tune_mac ? 16 : B, gb_targets = tune_mac ? 16 : B2;
    if (fb_targets > 1) farbuf = dalloc<double2>((size_t)fb_targets * nrhs * 3 * sp, "time-block partial sums");
    if (gb_targets) gbuf = dalloc<double2>((size_t)gb_targets * nrhs * 3 * sp, "outer-block partial sums");
    const bool want_overlap = c.outer_overlap == 2 || (c.outer_overlap == 0 && kOverlapDefault);
    if (gb_targets && want_overlap) {
        hbuf = dalloc<double2>((size_t)gb_targets * nrhs * 3 * sp, "next outer block's sums");
        MJ_CHECK(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
        MJ_CHECK(hipEventCreateWithFlags(&ev_main, hipEventDisableTiming));
        MJ_CHECK(hipEventCreateWithFlags(&ev_side, hipEventDisableTiming));
        for (auto &pr : side_t)
            for (hipEvent_t &e : pr) MJ_CHECK(hipEventCreate(&e));
    }
    S = dalloc<double>((size_t)nrhs * 3 * M, "convolution");
    Jr = dalloc<double>((size_t)rdepth * nrhs * 3 * M, "current history");
    rhs = dalloc<double>((size_t)nrhs * 3 * M, "cg rhs");
    y = dalloc<double>((size_t)nrhs * 3 * M, "cg y");
    p = dalloc<double>((size_t)nrhs * 3 * M, "cg p");
    q = dalloc<double>((size_t)nrhs * 3 * M, "cg q");
    // the first iteration of every solve scales p and q by beta = 0: they must be finite
    MJ_CHECK(hipMemset(p, 0, sizeof(double) * nrhs * 3 * M));
    MJ_CHECK(hipMemset(q, 0, sizeof(double) * nrhs * 3 * M));
    const size_t Mp = (size_t)(U + 2) * (V + 2) * (W + 2);
    u = dalloc<double>((size_t)nrhs * 3 * Mp, "cg u");
    uy = dalloc<double>((size_t)nrhs * 3 * Mp, "cg uy");
    e2 = dalloc<double>((size_t)nrhs * 3 * Mp, "chebyshev direction");
    // the one-voxel halo of u, uy and e2 is never written and stays zero
    MJ_CHECK(hipMemset(u, 0, sizeof(double) * nrhs * 3 * Mp));
    MJ_CHECK(hipMemset(uy, 0, sizeof(double) * nrhs * 3 * Mp));
    MJ_CHECK(hipMemset(e2, 0, sizeof(double) * nrhs * 3 * Mp));
    nblk = (int)((M + 255) / 256);
    parts = dalloc<double>((size_t)3 * nrhs * nblk, "cg partials");
    scal = dalloc<mj::CgScalars>(nrhs, "cg scalars");
    cgstat = dalloc<mj::CgStatus>(nrhs, "cg status");
    waves_d = dalloc<mj::WaveArg>(nrhs, "waves");
    {
        double rules[9 * 16] = {};
        for (int n = 1; n <= 8; n++) gl_half(n, rules + 16 * n, rules + 16 * n + 8);
        gl_d = dalloc<double>(9 * 16, "quadrature rules");
        MJ_CHECK(hipMemcpy(gl_d, rules, sizeof rules, hipMemcpyHostToDevice));
    }
    MJ_CHECK(hipHostMalloc((void **)&cgstat_h, sizeof(mj::CgStatus) * nrhs, hipHostMallocDefault));
    mj::fft3d_init(fft, U, V, W, 3 * nrhs, Nx, Ny, Nz, da);
    bytes += sizeof(double2) * ((size_t)3 * nrhs * W * V * Hp + (size_t)3 * nrhs * W * Ny * Hp);
    if (c.fft_pencils > 0) mj::fft3d_set_pencils(fft, c.fft_pencils);
    else mj::fft3d_autotune(fft, st);
    if (tune_mac) mac_autotune();
    overlap = hbuf != nullptr && B2 > 0;
    if (z0_method == 0) estimate_spectrum();
    n = 0;
    MJ_CHECK(hipStreamSynchronize(st));
}

// chi, sqrt chi, 1/eps, c_0 = T(0)/eps + delta_0 and the Jacobi preconditioner
// diag(A) = c_0 - chi K_0^{bb}(0) of the symmetrised Z_0 (needs K_0 from build_spectra)
void mj_solver::set_material(const double *eps)
{
    for (long i = 0; i < M; i++)
        if (!(eps[i] >= 1.0) || !std::isfinite(eps[i])) throw ArgError("eps_r must be finite and >= 1");
    eps_h.assign(eps, eps + M);
    std::vector<double> chi_h(M), schi_h(M), ie_h(M), c0_h(M);
    const double d0 = fir.empty() ? 0.0 : fir[0];
    for (long i = 0; i < M; i++) {
        chi_h[i] = (eps[i] - 1.0) / eps[i];
        schi_h[i] = std::sqrt(chi_h[i]);
        ie_h[i] = 1.0 / eps[i];
        c0_h[i] = 0.5 * ie_h[i] + d0;   // T(0)/eps + delta_0
    }
    MJ_CHECK(hipMemcpy(chi, chi_h.data(), M * 8, hipMemcpyHostToDevice));
    MJ_CHECK(hipMemcpy(schi, schi_h.data(), M * 8, hipMemcpyHostToDevice));
    MJ_CHECK(hipMemcpy(inv_eps, ie_h.data(), M * 8, hipMemcpyHostToDevice));
    MJ_CHECK(hipMemcpy(c0, c0_h.data(), M * 8, hipMemcpyHostToDevice));
}

void mj_solver::build_spectra()
{
    auto t0 = std::chrono::steady_clock::now();
    {
        // generator units: the x edge
        const double hv[3] = {1.0, hy / h, hz / h};
        mj::gen_moments(gen, U, V, W, c_dt / h, hv, nquad, da, st);
    }
    bytes += (size_t)M * gen.ms * mj::kMoments * sizeof(double);
    MJ_CHECK(hipStreamSynchronize(st));
    auto t1 = std::chrono::steady_clock::now();
    t_gen_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();

    // K_0 stencil (27 offsets, 6 components) for the Z_0 solve
    {
        std::vector<int> lag(27, 0), off(81);
        int o = 0;
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++, o++) {
                    off[3 * o] = (U > 1 || dx == 0) ? dx : 0;
                    off[3 * o + 1] = (V > 1 || dy == 0) ? dy : 0;
                    off[3 * o + 2] = (W > 1 || dz == 0) ? dz : 0;
                }
        mj::DevTemp tl(da, 27 * sizeof(int), "stencil request");
        mj::DevTemp to(da, 81 * sizeof(int), "stencil request");
        mj::DevTemp tv(da, 162 * sizeof(double), "stencil values");
        int *lag_d = tl.as<int>(), *off_d = to.as<int>();
        double *out_d = tv.as<double>();
        MJ_CHECK(hipMemcpy(lag_d, lag.data(), 27 * sizeof(int), hipMemcpyHostToDevice));
        MJ_CHECK(hipMemcpy(off_d, off.data(), 81 * sizeof(int), hipMemcpyHostToDevice));
        mj::gen_kernel_values(gen, 27, lag_d, off_d, out_d, st);
        MJ_CHECK(hipMemcpyAsync(K0_27, out_d, 162 * sizeof(double), hipMemcpyDeviceToHost, st));
        MJ_CHECK(hipStreamSynchronize(st));
        // offsets that fall outside a one-voxel-thick axis do not couple
        o = 0;
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++, o++)
                    if ((U == 1 && dx != 0) || (V == 1 && dy != 0) || (W == 1 && dz != 0))
                        for (int c = 0; c < 6; c++) K0_27[6 * o + c] = 0.0;
        k0_d = dalloc<double>(27 * 6, "K_0 stencil");
        MJ_CHECK(hipMemcpy(k0_d, K0_27, sizeof K0_27, hipMemcpyHostToDevice));
    }

    // spectra of lags 1..ell on the padded grid, octant only, with 1/(Nx Ny Nz) folded in
    const long ko = koct();
    Khat = dalloc<double>((size_t)ell * 6 * ko, "kernel spectra");
    mj::Fft3D kf{};
    double *grid = nullptr;
    double2 *X = nullptr;
    const size_t ng = (size_t)Nx * Ny * Nz;
    try {
        mj::fft3d_init(kf, Nx, Ny, Nz, 6, Nx, Ny, Nz, da);
        grid = (double *)da.get(6 * ng * sizeof(double), "kernel grid");
        X = (double2 *)da.get(6 * (size_t)Nz * Ny * Hp * sizeof(double2), "kernel spectrum");
        const double scale = 1.0 / ((double)Nx * Ny * Nz);
        for (int k = 1; k <= ell; k++) {
            mj::gen_kernel_grid(gen, k, Nx, Ny, Nz, grid, st);
            mj::fft3d_forward(kf, grid, X, 6, st);
            hipLaunchKernelGGL(k_extract_octant, dim3((unsigned)((ko + 255) / 256)), dim3(256), 0, st, X, Hx, Hp, Ny, Nz,
                               scale, Khat + (size_t)(k - 1) * 6 * ko);
            MJ_CHECK(hipGetLastError());
        }
        MJ_CHECK(hipStreamSynchronize(st));
    } catch (...) {
        mj::fft3d_free(kf);
        da.put(grid);
        da.put(X);
        throw;
    }
    mj::fft3d_free(kf);
    da.put(grid);
    da.put(X);
    auto t2 = std::chrono::steady_clock::now();
    t_spec_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
}

mj::CgArg mj_solver::cg_arg() const
{
    mj::CgArg a{};
    a.M = M;
    a.U = U;
    a.V = V;
    a.W = W;
    a.Mp = (long)(U + 2) * (V + 2) * (W + 2);
    a.nrhs = nrhs;
    a.nblk = nblk;
    a.tol2 = cg_rtol * cg_rtol;
    a.schi = schi;
    a.d0 = fir.empty() ? 0.0 : fir[0];
    a.k0c = K0_27[13 * 6 + 0];
    a.k0 = k0_d;
    a.rhs = rhs;
    a.uy = uy;
    a.y = y;
    a.p = p;
    a.q = q;
    a.u = u;
    a.part = parts;
    a.scal = scal;
    a.stat = cgstat;
    return a;
}

void mj_solver::solve_z0()
{
    if (z0_method == 0 && lam_hi > 0.0) {
        solve_z0_chebyshev();
        return;
    }
    mj::CgArg a = cg_arg();
    mj::launch_cg_init(a, st);   // also clears the status records
    // enqueue as many iterations as the last solve needed before the first look at the
    // convergence flags; kernels after convergence return at once
    int it = 0;
    int batch = std::max(2, std::min(cg_maxit, cg_guess));
    bool all_done = false;
    while (it < cg_maxit && !all_done) {
        int upto = std::min(cg_maxit, it + batch);
        for (; it < upto; it++) {
            mj::launch_cg_a(a, it, st);
            mj::launch_cg_b(a, it, st);
        }
        MJ_CHECK(hipMemcpyAsync(cgstat_h, cgstat, sizeof(mj::CgStatus) * nrhs, hipMemcpyDeviceToHost, st));
        MJ_CHECK(hipStreamSynchronize(st));
        all_done = true;
        for (int i = 0; i < nrhs; i++) all_done = all_done && cgstat_h[i].done;
        batch = 2;
    }
    // the last update of y (a no-op for the right-hand sides whose solve already ended)
    mj::launch_cg_end(a, it, st);
    int mx = 0;
    for (int i = 0; i < nrhs; i++) mx = std::max(mx, cgstat_h[i].iters);
    cg_guess = mx + 1;
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix (diagonal a, off-diagonal
// b, b[0] unused): the Sturm count of the LDL^T pivots.
static int sturm_count(const std::vector<double> &a, const std::vector<double> &b, double x)
{
    int cnt = 0;
    double q = 1.0;
    for (size_t j = 0; j < a.size(); j++) {
        const double off = j ? b[j] * b[j] / q : 0.0;
        q = a[j] - x - off;
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) cnt++;
    }
    return cnt;
}

// Extreme eigenvalues of M^-1 A (M the Jacobi preconditioner) for the Chebyshev solve: a CG run
// on a pseudo-random right-hand side is a Lanczos process, whose tridiagonal matrix
// T (T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_{j,j+1} = sqrt(beta_j)/alpha_j) has extreme
// eigenvalues that approach those of M^-1 A from inside; bisection on its Sturm counts gives
// them.  The bounds used are widened by 10 % below and 5 % above.  A spectrum with nothing in
// it (no voxel with eps != 1) leaves the bounds at 0, which selects the CG solve.
void mj_solver::estimate_spectrum()
{
    lam_lo = lam_hi = 0.0;
    cheb_rho.clear();   // the recurrence scalars and the captured batches hold the old bounds
    clear_graphs();
    mj::CgArg a = cg_arg();
    a.nrhs = 1;
    a.tol2 = 0.0;   // run every iteration
    const size_t Mp = (size_t)(U + 2) * (V + 2) * (W + 2);
    MJ_CHECK(hipMemsetAsync(uy, 0, sizeof(double) * Mp * 3, st));
    mj::launch_fill_trial(schi, M, 1, rhs, y, st);
    mj::launch_cg_init(a, st);
    std::vector<double> alpha, beta;
    mj::CgScalars sc{};
    MJ_CHECK(hipMemcpyAsync(&sc, scal, sizeof sc, hipMemcpyDeviceToHost, st));
    MJ_CHECK(hipStreamSynchronize(st));
    const double rz0 = sc.rz[0];
    if (!(rz0 > 0.0) || !std::isfinite(rz0)) {
        restart();
        return;
    }
    const int m = std::min(40, 3 * (int)std::min<long>(M, 1000));
    for (int it = 0; it < m; it++) {
        mj::launch_cg_a(a, it, st);
        mj::launch_cg_b(a, it, st);
        MJ_CHECK(hipMemcpyAsync(&sc, scal, sizeof sc, hipMemcpyDeviceToHost, st));
        MJ_CHECK(hipStreamSynchronize(st));
        const double rz = sc.rz[it & 1], rzn = sc.rz[(it + 1) & 1], pq = sc.pq;
        if (!(pq > 0.0) || !std::isfinite(pq) || !(rz > 0.0)) break;
        alpha.push_back(rz / pq);
        beta.push_back(rzn / rz);
        // the Krylov space is exhausted (tiny grids): the residual has vanished
        if (!(rzn > 1e-28 * rz0)) break;
    }
    restart();
    const size_t k = alpha.size();
    if (k == 0) return;
    std::vector<double> d(k), e(k, 0.0);
    for (size_t j = 0; j < k; j++) {
        d[j] = 1.0 / alpha[j] + (j ? beta[j - 1] / alpha[j - 1] : 0.0);
        if (j) e[j] = std::sqrt(beta[j - 1]) / alpha[j - 1];
    }
    double lo = 1e300, hi = -1e300;
    for (size_t j = 0; j < k; j++) {   // Gershgorin interval of T
        const double rad = (j ? std::fabs(e[j]) : 0.0) + (j + 1 < k ? std::fabs(e[j + 1]) : 0.0);
        lo = std::min(lo, d[j] - rad);
        hi = std::max(hi, d[j] + rad);
    }
    auto kth = [&](int idx) {   // eigenvalue number idx (0-based, ascending) by bisection
        double l = lo, h = hi;
        for (int b = 0; b < 200 && h - l > 1e-14 * std::max(1.0, std::fabs(h)); b++) {
            const double mid = 0.5 * (l + h);
            if (sturm_count(d, e, mid) > idx) h = mid;
            else l = mid;
        }
        return 0.5 * (l + h);
    };
    const double emin = kth(0), emax = kth((int)k - 1);
    if (!(emin > 0.0) || !(emax >= emin)) return;
    lam_lo = 0.9 * emin;
    lam_hi = 1.05 * emax;
}

// The Z_0 solve by Chebyshev iteration (k_cheb_*): one stencil pass per iteration and no inner
// products, so no reductions inside the iteration.  The passes of a solve are enqueued in
// batches; only the last pass of a batch computes |r|^2, and the host reads the outcome once per
// batch.  The first batch has as many passes as the last solve needed, from its observed
// reduction per pass and its initial residual; without a last solve, the host first reads
// |r_0| / |b| and uses the convergence factor of the Chebyshev polynomials for the estimated
// spectrum.
//
// Right-hand sides are solved in groups, one group after the other, so that the vectors a pass
// streams for its group (y, r and the two directions: about 6 x 3 x 8 bytes per voxel and
// right-hand side) stay within kChebGroupBytes, which the device's last-level cache largely
// holds from one pass to the next.  At 64^3 the solve per right-hand side took 0.27 ms in a
// batch of 8 and 0.41 ms in a batch of 16 (0.31 in 4, 0.42 alone).
void mj_solver::solve_z0_chebyshev()
{
    mj::ChebArg a{};
    a.cg = cg_arg();
    a.r = q;
    const double theta = 0.5 * (lam_hi + lam_lo), delta = 0.5 * (lam_hi - lam_lo);
    a.inv_theta = 1.0 / theta;
    double *ebuf[2] = {u, e2};
    const double kappa = lam_hi / lam_lo;
    const double rho_th = (std::sqrt(kappa) - 1.0) / (std::sqrt(kappa) + 1.0);
    const double tol2 = cg_rtol * cg_rtol;
    // the recurrence scalars by pass index: rho_0 = delta / theta, rho_{k+1} = 1 / (2 theta / delta - rho_k)
    if ((int)cheb_rho.size() < cg_maxit + 1) {
        cheb_rho.assign((size_t)cg_maxit + 1, 0.0);
        cheb_rho[0] = delta / theta;
        for (int k = 0; k < cg_maxit; k++) cheb_rho[(size_t)k + 1] = 1.0 / (2.0 * theta / delta - cheb_rho[(size_t)k]);
    }
    // the kernels of one batch: (the initial residual and) passes T .. T + K - 1, the last with the
    // check; their arguments depend only on (group, T, K), so a captured batch replays unchanged
    auto launch_batch = [&](bool with_init, int T, int K, hipStream_t s_) {
        if (with_init) {
            a.e_out = ebuf[0];
            a.passes = 0;
            mj::launch_cheb_init(a, s_);
        }
        for (int j = 0; j < K; j++) {
            const int k = T + j;
            a.c1 = cheb_rho[(size_t)k + 1] * cheb_rho[(size_t)k];
            a.c2 = 2.0 * cheb_rho[(size_t)k + 1] / delta;
            a.e_in = ebuf[k & 1];
            a.e_out = ebuf[(k + 1) & 1];
            a.want_norm = j == K - 1;
            a.passes = k + 1;
            mj::launch_cheb_pass(a, s_);
        }
    };
    auto enqueue = [&](bool with_init, int T, int K) {
        if (!use_graphs) {
            launch_batch(with_init, T, K, st);
            return;
        }
        const long key = ((long)a.rhs0 << 48) | ((long)with_init << 40) | ((long)T << 20) | K;
        auto it = cheb_graphs.find(key);
        if (it == cheb_graphs.end()) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ex = nullptr;
            MJ_CHECK(hipStreamBeginCapture(cap_st, hipStreamCaptureModeRelaxed));
            try {
                launch_batch(with_init, T, K, cap_st);
            } catch (...) {
                (void)hipStreamEndCapture(cap_st, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            MJ_CHECK(hipStreamEndCapture(cap_st, &g));
            const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            MJ_CHECK(e);
            it = cheb_graphs.emplace(key, ex).first;
        }
        MJ_CHECK(hipGraphLaunch(it->second, st));
    };
    // passes to bring |r|^2 from rr to tol^2 bb at a reduction rho2 per pass
    auto passes_for = [&](double rr, double bb, double rho2) {
        if (!(rr > tol2 * bb) || !(bb > 0.0)) return 0;
        const double k = std::log(tol2 * bb / rr) / std::log(rho2);
        return (int)std::ceil(std::max(1.0, k));
    };
    const size_t per_rhs = (size_t)6 * 3 * M * sizeof(double);
    const int G = (int)std::max<size_t>(1, std::min<size_t>((size_t)nrhs, kChebGroupBytes / per_rhs));
    int pred_all = 1;
    bool predicted = false;   // a group that met its initial test at once leaves no prediction
    for (int g0 = 0; g0 < nrhs; g0 += G) {
        const int g1 = std::min(nrhs, g0 + G);
        a.rhs0 = g0;
        a.nr = g1 - g0;
        auto read_status = [&] {
            MJ_CHECK(hipMemcpyAsync(cgstat_h, cgstat, sizeof(mj::CgStatus) * nrhs, hipMemcpyDeviceToHost, st));
            MJ_CHECK(hipStreamSynchronize(st));
            bool done = true;
            for (int i = g0; i < g1; i++) done = done && cgstat_h[i].done;
            return done;
        };
        int K = std::min(cheb_pred, cg_maxit);
        int total = 0;
        bool done = false;
        if (K <= 0) {
            // no last solve: read |r_0| / |b| first, and use the Chebyshev polynomials' convergence factor
            enqueue(true, 0, 0);
            if (read_status()) continue;
            K = 0;
            for (int i = g0; i < g1; i++)
                K = std::max(K, passes_for(cgstat_h[i].rr0, cgstat_h[i].bb, rho_th * rho_th) + 1);
            K = std::max(1, std::min(K, cg_maxit));
            enqueue(false, 0, K);
        } else {
            enqueue(true, 0, K);
        }
        total = K;
        done = read_status();
        while (!done && total < cg_maxit) {
            // more passes, from the residual reached and the reduction seen so far
            K = 1;
            for (int i = g0; i < g1; i++) {
                const mj::CgStatus &c = cgstat_h[i];
                if (c.done) continue;
                const double rr = c.res * c.res * c.bb;
                double rho2 = rho_th * rho_th;
                if (c.rr0 > 0.0 && rr > 0.0 && rr < c.rr0) rho2 = std::max(rho2, std::pow(rr / c.rr0, 1.0 / total));
                if (!(rho2 < 1.0)) rho2 = 0.9;
                K = std::max(K, passes_for(rr, c.bb, rho2) + 1);
            }
            K = std::min(K, cg_maxit - total);
            enqueue(false, total, K);
            total += K;
            done = read_status();
        }
        // the next solve starts with the passes this one would have needed: its observed
        // reduction per pass applied to its initial residual
        predicted = true;
        for (int i = g0; i < g1; i++) {
            const mj::CgStatus &c = cgstat_h[i];
            const double rr = c.res * c.res * c.bb;
            double rho2 = rho_th * rho_th;
            if (c.rr0 > 0.0 && rr > 0.0 && rr < c.rr0 && total > 0)
                rho2 = std::max(rho2 * 0.25, std::pow(rr / c.rr0, 1.0 / total));
            if (!(rho2 < 1.0)) rho2 = 0.9;
            pred_all = std::max(pred_all, passes_for(c.rr0, c.bb, rho2));
        }
    }
    if (predicted) cheb_pred = pred_all;
}

mj::EpiArg mj_solver::epi_arg() const
{
    mj::EpiArg e{};
    e.k0 = k0_d;
    for (const mj::WaveArg &w : waves)
        if ((w.k[0] != 0.0) + (w.k[1] != 0.0) + (w.k[2] != 0.0) >= 2) e.oblique = 1;
    e.M = M;
    e.U = U;
    e.V = V;
    e.W = W;
    e.nrhs = nrhs;
    e.n = n;
    e.h = h;
    e.hy = hy;
    e.hz = hz;
    e.c_dt = c_dt;
    e.chi = chi;
    e.schi = schi;
    e.inv_eps = inv_eps;
    e.fir = fir_d;
    e.nfir = (int)fir.size();
    e.nloc = nloc;
    for (int k = 1; k <= nloc; k++) e.slot_of[k] = n - k >= 1 ? slotR(n - k) : 0;
    // extrapolation through m = nguess equally spaced past steps to the next one:
    // weight of J_{n-k} is (-1)^(k+1) binomial(m, k)
    e.nguess = std::min(guess_deg + 1, nloc);
    for (int k = 1; k <= e.nguess; k++) {
        double bin = 1.0;
        for (int q = 1; q <= k; q++) bin = bin * (e.nguess - q + 1) / q;
        e.gx[k - 1] = (k & 1) ? bin : -bin;
    }
    e.Jring = Jr;
    e.waves = waves_d;
    gl_half(8, e.glx8, e.glw8);
    e.gl = gl_d;
    e.rhs = rhs;
    e.y = y;
    e.uy = uy;
    return e;
}

// The spectral history sum of step n >= 2 (sources J_1 .. J_{n-1} in the ring), launched as the
// configured time division requires; returns where the step's sum is left.  *kind: 1 far (outer)
// launch, 2 near, 3 middle, 0 none of these (no time blocking).
const double2 *mj_solver::mac(int n, int *kind)
{
    const long sp = spec_plane();
    const double2 *spec = Shat;
    int far_kind = 0;
    if (B == 1) {
        mj::MacArg a{};
        a.Khat = Khat;
        a.ring_base = ring;
        a.Shat = Shat;
        a.Hx = Hx;
        a.Hp = Hp;
        a.Ny = Ny;
        a.Nz = Nz;
        a.nk = std::min(ell, n - 1);
        a.ring = ell;
        a.slot_nm1 = slotS(n - 1);
        a.nrhs = nrhs;
        mj::launch_mac(a, st);
    } else if (B2 == 0) {
        // blocks of B steps starting at n_b = 2, 2 + B, ...: the far part of every step of the
        // block is formed at n_b, when all of its sources are in the ring
        const int t = (n - 2) % B;
        mj::BlockMacArg a = block_arg(farbuf, n - t);
        a.ntarget = B;
        a.t = t;
        if (t == 0) mj::launch_mac_far(a, B, st);
        else mj::launch_mac_near(a, st);
        far_kind = t == 0 ? 1 : 2;
        spec = farbuf + (size_t)t * nrhs * 3 * sp;
    } else {
        // three levels (the Toeplitz division of Sec. 4.1 applied twice): outer blocks of B2
        // steps start at N_b = 2, 2 + B2, ...; each splits into inner blocks of B steps.
        //   outer, at N_b:  G[tau] = sum_{k > tau} Khat_k Jhat_{N_b + tau - k} over sources before N_b
        //   middle, at each inner start n_b > N_b:  F[t] = G[n_b - N_b + t] + the terms of the
        //                   sources N_b .. n_b - 1 (inside the outer block, before the inner one)
        //   near, every step:  + the terms of the sources n_b .. n - 1
        // The first inner block needs no middle part: its sums stay in G.
        const int tau = (n - 2) % B2, t = tau % B, q = tau / B;
        double2 *fb = q == 0 ? gbuf : farbuf;
        if (tau == 0) {
            if (overlap) {
                outer_overlapped(n);
            } else {
                mj::BlockMacArg a = block_arg(gbuf, n);
                a.ntarget = B2;
                mj::launch_mac_win(a, B2, st);
            }
            far_kind = 1;
        } else if (t == 0) {
            mj::BlockMacArg a = block_arg(farbuf, n);
            a.ntarget = B;
            a.jmin = n - tau;
            a.init = gbuf + (size_t)tau * nrhs * 3 * sp;
            mj::launch_mac_win(a, B, st);
            far_kind = 3;
        } else {
            mj::BlockMacArg a = block_arg(fb, n - t);
            a.t = t;
            mj::launch_mac_near(a, st);
            far_kind = 2;
        }
        spec = fb + (size_t)t * nrhs * 3 * sp;
    }
    *kind = far_kind;
    return spec;
}

// The outer sums of the block starting at nb over the sources before nb - B2 (lags above B2),
// into hbuf on `stream`: the work that can run while the block before nb marches.
void mj_solver::outer_sums(int nb, hipStream_t stream)
{
    if (nb - B2 - 1 < 1) throw std::logic_error("outer sums without sources");
    mj::BlockMacArg a = block_arg(hbuf, nb);
    a.ntarget = B2;
    a.jmax = nb - B2 - 1;
    mj::launch_mac_win(a, B2, stream, stream == side ? kSideLdsReserve : 0);
}

// The outer level at the start nb of an outer block, overlapped (Sec. 4.1's division with the
// outer sums split at nb - B2):
//   G[tau] = H[tau] + sum over the sources nb - B2 .. nb - 1 of Khat_k Jhat_{nb + tau - k},
// H being the sums over the sources before nb - B2, formed on the second stream while the block
// before marched (or here, in line, after a restart).  Then the second stream starts on the
// next block's H, over the sources before nb.  It reads ring slots of sources nb + B2 - ell ..
// nb - 1 while this block's steps write the slots of sources nb - ell .. nb + B2 - 1 - ell, and
// writes hbuf, which only the next block start reads, after waiting for it.
void mj_solver::outer_overlapped(int nb)
{
    join_side();
    const bool have_h = nb - B2 - 1 >= 1;
    if (have_h && h_block != nb) outer_sums(nb, st);
    mj::BlockMacArg a = block_arg(gbuf, nb);
    a.ntarget = B2;
    a.jmin = nb - B2;
    a.init = have_h ? hbuf : nullptr;
    mj::launch_mac_win(a, B2, st);
    MJ_CHECK(hipEventRecord(ev_main, st));
    MJ_CHECK(hipStreamWaitEvent(side, ev_main, 0));
    const int slot = side_count % kSideTimers;
    if (side_busy[slot]) {
        MJ_CHECK(hipEventSynchronize(side_t[slot][1]));
        collect_side_timers(false);
    }
    MJ_CHECK(hipEventRecord(side_t[slot][0], side));
    outer_sums(nb + B2, side);
    MJ_CHECK(hipEventRecord(side_t[slot][1], side));
    side_busy[slot] = true;
    side_count++;
    MJ_CHECK(hipEventRecord(ev_side, side));
    side_pending = true;
    h_block = nb + B2;
}

// Adds the durations of the finished launches on the second stream to side_ms (waiting for
// all of them with wait).
void mj_solver::collect_side_timers(bool wait)
{
    for (int i = 0; i < kSideTimers; i++) {
        if (!side_busy[i]) continue;
        if (wait) MJ_CHECK(hipEventSynchronize(side_t[i][1]));
        const hipError_t q = hipEventQuery(side_t[i][1]);
        if (q == hipErrorNotReady) {
            (void)hipGetLastError();   // not an error: keep it from the next launch check
            continue;
        }
        MJ_CHECK(q);
        float ms = 0.0f;
        MJ_CHECK(hipEventElapsedTime(&ms, side_t[i][0], side_t[i][1]));
        side_ms += ms;
        side_done++;
        side_busy[i] = false;
    }
}

// Default time division when the caller sets neither block: three levels, blocks of 4 in
// outer blocks of 16, once the kernel reaches far enough back in time (ell >= 64) for the
// outer level to pay; else two levels with blocks of 8.  At 104^3 (ell = 182) per step:
// 2.85 ms against 3.39 ms for blocks of 8 alone.
void mj_solver::default_time_division()
{
    if (ell >= 64) {
        B = 4;
        B2 = 16;
    } else {
        B = 8;
        B2 = 0;
    }
}

// Picks the time division (time block B, outer block B2) by timing the history sum of one
// period of steps at steady state for each candidate: every lag live (the steps timed lie
// beyond ell), on a cleared ring (the values do not change the time).  The candidates only
// group the terms of eq:PnMOT differently, so results depend on the choice at rounding level.
void mj_solver::mac_autotune()
{
    static const int cand[][2] = {{8, 0}, {12, 0}, {16, 0}, {4, 8}, {4, 12}, {4, 16}, {8, 16}};
    MJ_CHECK(hipMemsetAsync(ring, 0, sizeof(double2) * (size_t)ell * nrhs * 3 * spec_plane(), st));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MJ_CHECK(hipEventCreate(&e0));
    MJ_CHECK(hipEventCreate(&e1));
    double best = -1.0;
    int bestB = 8, bestB2 = 0;
    try {
        for (const auto &cd : cand) {
            B = cd[0];
            B2 = cd[1];
            const int period = B2 ? B2 : B;
            const int n0 = 2 + period * ((ell + period - 1) / period);
            double tmin = -1.0;
            for (int rep = 0; rep < 3; rep++) {
                MJ_CHECK(hipEventRecord(e0, st));
                for (int i = 0; i < period; i++) {
                    int kind = 0;
                    (void)mac(n0 + i, &kind);
                }
                MJ_CHECK(hipEventRecord(e1, st));
                MJ_CHECK(hipEventSynchronize(e1));
                float ms = 0.0f;
                MJ_CHECK(hipEventElapsedTime(&ms, e0, e1));
                if (rep > 0 && (tmin < 0.0 || ms < tmin)) tmin = ms;
            }
            const double per_step = tmin / period;
            if (best < 0.0 || per_step < best) {
                best = per_step;
                bestB = cd[0];
                bestB2 = cd[1];
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    B = bestB;
    B2 = bestB2;
    t_mac_tune_ms = best;
}

// One step n -> n + 1 of the march on the current track: FFT of the newest source, spectral
// history sum (plain or time-blocked), inverse FFT, right-hand side, Z_0 solve, and the
// outputs asked for.  io.adjoint runs the transposed march instead (sources nu, local
// history lambda in Lr, right-hand side from io.G).
void mj_solver::step(const StepIO &io)
{
    const long sp = spec_plane();
    hipEvent_t *ev = io.ev;
    if (ev) MJ_CHECK(hipEventRecord(ev[0], st));
    n += 1;
    const bool hist = n >= 2;
    if (hist) {
        const int j = n - 1;
        mj::fft3d_forward(fft, Jr + (size_t)slotR(j) * nrhs * 3 * M, ring + (size_t)slotS(j) * nrhs * 3 * sp,
                          3 * nrhs, st);
    }
    if (ev) MJ_CHECK(hipEventRecord(ev[1], st));
    int far_kind = 0;
    const double2 *spec = hist ? mac(n, &far_kind) : Shat;
    if (io.far_kind) *io.far_kind = (char)far_kind;
    if (ev) MJ_CHECK(hipEventRecord(ev[2], st));
    if (hist) mj::fft3d_inverse(fft, spec, S, 3 * nrhs, st);
    if (ev) MJ_CHECK(hipEventRecord(ev[3], st));
    mj::EpiArg e = epi_arg();
    e.S = hist ? S : nullptr;
    if (io.adjoint) {
        e.Lring = Lr;
        e.G = io.G;
        e.bq = bq;
        mj::launch_adj_epilogue(e, st);
    } else {
        mj::launch_epilogue(e, st);
    }
    if (ev) MJ_CHECK(hipEventRecord(ev[4], st));
    solve_z0();
    double *Jn = Jr + (size_t)slotR(n) * nrhs * 3 * M;
    mj::launch_cg_finish(y, schi, M, nrhs, Jn, io.Jout, st);
    if (ev) MJ_CHECK(hipEventRecord(ev[5], st));
    if (io.adjoint) {
        mj::AdjArg a = adj_arg();
        a.y = y;
        a.nu = Jn;
        a.bq = bq;
        a.lam = Lr + (size_t)slotR(n) * nrhs * 3 * M;
        mj::launch_adj_lambda(a, st);
        if (io.Bj) {
            a.Bj = io.Bj;
            a.grad = io.grad;
            mj::launch_grad_accum(a, st);
        }
    } else {
        if (np > 0 && !io.skip_probes) {
            mj::ProbeStepArg pa{};
            pa.table = ptable;
            pa.pair_vox = pair_vox;
            pa.pair_kmin = pair_kmin;
            pa.row_start = row_start;
            pa.np = np;
            pa.ell = ell;
            pa.nw = nw;
            pa.nrhs = nrhs;
            pa.n = n;
            pa.M = M;
            pa.npairs = npairs;
            pa.Jring = Jr;
            pa.rdepth = rdepth;
            pa.part = ppart;
            pa.ck_row = ck_row;
            pa.ck_lo = ck_lo;
            pa.ck_hi = ck_hi;
            pa.ck_start = ck_start;
            pa.nck = pnck;
            pa.out = io.Pout ? io.Pout : pout;
            mj::launch_probes(pa, st);
        }
        if (io.Bout)
            mj::launch_grad_term(e, Jn, n >= 2 ? Jr + (size_t)slotR(n - 1) * nrhs * 3 * M : nullptr, io.Bout, st);
    }
    if (ev) MJ_CHECK(hipEventRecord(ev[6], st));
}

// The march grows without bound (Sec. 5.2 and 6: the alternating mode at f = 1/(2 dt)): stop once the
// right-hand side of a Z_0 solve leaves the finite range or passes 1e100 in norm.
void mj_solver::check_growth() const
{
    for (int i = 0; i < nrhs; i++) {
        const double bb = cgstat_h[i].bb;
        if (!std::isfinite(bb) || bb > 1e200 || !std::isfinite(cgstat_h[i].res))
            throw UnstableError("the march is unstable: the Z_0 right-hand side of step " + std::to_string(n) +
                                " exceeds 1e100 in norm or is not finite");
    }
}

mj::AdjArg mj_solver::adj_arg() const
{
    mj::AdjArg a{};
    a.k0 = k0_d;
    a.M = M;
    a.U = U;
    a.V = V;
    a.W = W;
    a.nrhs = nrhs;
    a.table = ptable;
    a.pair_kmin = pair_kmin;
    a.inv = pinv;
    a.table_v = ptable_v;
    a.kmin_v = pkmin_v;
    a.np = np;
    a.nw = nw;
    a.npairs = npairs;
    a.schi = schi;
    a.c0 = c0;
    a.inv_eps = inv_eps;
    return a;
}

// J_n goes to Jout for every j_every-th step of the call (steps s = j_every - 1, 2 j_every - 1, ...
// counted from 0), entry (s + 1) / j_every - 1; the probe field of every step goes to Pout.
void mj_solver::run(int n_steps, double *Jout, double *Pout, int j_every)
{
    if (!waves_set) throw std::logic_error("plane waves not set (mj_set_plane_waves)");
    events.ensure((size_t)7 * std::max(n_steps, 1));
    double cg_iter_sum = 0, cg_res_max = 0, cg_iter_max = 0;
    bool noconv = false;
    std::vector<char> step_far(n_steps, 0);
    side_ms = 0.0;
    side_done = 0;
    for (int s = 0; s < n_steps; s++) {
        StepIO io;
        io.ev = &events.ev[(size_t)7 * s];
        io.Jout = (Jout && (s + 1) % j_every == 0) ? Jout + (size_t)((s + 1) / j_every - 1) * nrhs * 3 * M : nullptr;
        io.Pout = Pout ? Pout + (size_t)s * nrhs * np * 3 : nullptr;
        io.far_kind = &step_far[s];
        step(io);
        check_growth();
        for (int i = 0; i < nrhs; i++) {
            cg_iter_sum += cgstat_h[i].iters;
            cg_iter_max = std::max(cg_iter_max, (double)cgstat_h[i].iters);
            cg_res_max = std::max(cg_res_max, cgstat_h[i].res);
            if (!cgstat_h[i].done) noconv = true;
        }
    }
    MJ_CHECK(hipStreamSynchronize(st));
    double ph[6] = {0, 0, 0, 0, 0, 0}, probe_ms = 0;
    double far_ms = 0, near_ms = 0, mid_ms = 0;
    int nfar = 0, nnear = 0, nmid = 0;
    for (int s = 0; s < n_steps; s++) {
        hipEvent_t *ev = &events.ev[(size_t)7 * s];
        for (int k = 0; k < 5; k++) {
            float ms = 0;
            MJ_CHECK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
            ph[k] += ms;
            if (k == 1 && step_far[s] == 1) { far_ms += ms; nfar++; }
            if (k == 1 && step_far[s] == 2) { near_ms += ms; nnear++; }
            if (k == 1 && step_far[s] == 3) { mid_ms += ms; nmid++; }
        }
        float pms = 0, tot = 0;
        MJ_CHECK(hipEventElapsedTime(&pms, ev[5], ev[6]));
        probe_ms += pms;
        MJ_CHECK(hipEventElapsedTime(&tot, ev[0], ev[6]));
        ph[5] += tot;
    }
    const double ns = std::max(n_steps, 1);
    for (int k = 0; k < 6; k++) stat[k] = ph[k] / ns;
    stat[6] = cg_iter_sum / (ns * nrhs);
    stat[7] = cg_res_max;
    stat[8] = n_steps;
    stat[9] = cg_iter_max;
    stat[10] = nfar ? far_ms / nfar : 0.0;
    stat[11] = nfar;
    stat[12] = nnear ? near_ms / nnear : 0.0;
    stat[13] = probe_ms / ns;
    stat[18] = nmid ? mid_ms / nmid : 0.0;
    if (side) collect_side_timers(false);
    stat[19] = side_done ? side_ms / side_done : 0.0;
    stat[20] = side_done;
    if (noconv) throw std::range_error("Z_0 solve did not converge");
}

// Back to n = 0 with every past current zero.  The search directions p and q enter the first
// iteration of each Z_0 solve multiplied by beta = 0, so they must be finite: a march that ended
// on non-finite values (MJ_EUNSTABLE) would otherwise turn every later solve into NaN through
// 0 * Inf.  They are cleared here, as at mj_create.
void mj_solver::restart()
{
    drop_side();
    const size_t v = sizeof(double) * (size_t)nrhs * 3 * M;
    MJ_CHECK(hipMemsetAsync(p, 0, v, st));
    MJ_CHECK(hipMemsetAsync(q, 0, v, st));
    MJ_CHECK(hipMemsetAsync(y, 0, v, st));
    // the Chebyshev directions: voxels whose eps changed to 1 must read as zero in the stencil
    const size_t vp = sizeof(double) * (size_t)nrhs * 3 * (U + 2) * (V + 2) * (W + 2);
    MJ_CHECK(hipMemsetAsync(u, 0, vp, st));
    MJ_CHECK(hipMemsetAsync(e2, 0, vp, st));
    MJ_CHECK(hipStreamSynchronize(st));
    cg_guess = 8;
    cheb_pred = 0;
    n = 0;
}

void mj_solver::history_sum(const double *Jh, int depth, double *P)
{
    drop_side();
    const long sp = spec_plane();
    const int nfake = ell + 1;
    for (int k = 1; k <= ell; k++) {
        double2 *slot = ring + (size_t)slotS(nfake - k) * nrhs * 3 * sp;
        if (k <= depth) mj::fft3d_forward(fft, Jh + (size_t)(k - 1) * 3 * M, slot, 3, st);
        else MJ_CHECK(hipMemsetAsync(slot, 0, sizeof(double2) * 3 * sp, st));
    }
    const double2 *spec = Shat;
    if (B == 1) {
        mj::MacArg a{};
        a.Khat = Khat;
        a.ring_base = ring;
        a.Shat = Shat;
        a.Hx = Hx;
        a.Hp = Hp;
        a.Ny = Ny;
        a.Nz = Nz;
        a.nk = ell;
        a.ring = ell;
        a.slot_nm1 = slotS(nfake - 1);
        a.nrhs = nrhs;   // ring stride; only right-hand side 0 is meaningful here
        mj::launch_mac(a, st);
    } else {
        // the far part of the first step of a block starting at n = ell + 1 is the whole sum
        mj::BlockMacArg a{};
        a.Khat = Khat;
        a.ring_base = ring;
        a.far = farbuf;
        a.Hx = Hx;
        a.Hp = Hp;
        a.Ny = Ny;
        a.Nz = Nz;
        a.nk = ell;
        a.ring = ell;
        a.nb = nfake;
        a.ntarget = 1;
        a.t = 0;
        a.nrhs = nrhs;
        mj::launch_mac_far(a, B, st);
        spec = farbuf;
    }
    mj::fft3d_inverse(fft, spec, S, 3, st);
    mj::launch_history_local(Jh, depth, S, chi, inv_eps, fir_d, (int)fir.size(), M, P, st);
    MJ_CHECK(hipStreamSynchronize(st));
    n = 0;
}

// Probes: test voxels of side h centred at arbitrary points.  Pairs (probe, scatterer voxel)
// whose lag window [kmin, kmin + nw) meets 0..ell are kept, per probe sorted by kmin, with the
// kernel values of their window generated on the device once.
void mj_solver::set_probes(int n_probes, const double *pos)
{
    if (n != 0) throw std::logic_error("probes are set before the first step (or after mj_reset)");
    if (n_probes < 0 || n_probes > 65536) throw ArgError("n_probes must be in [0, 65536]");
    if (n_probes > 0 && !pos) throw ArgError("probe positions are NULL");
    for (int i = 0; i < 3 * n_probes; i++)
        if (!std::isfinite(pos[i])) throw ArgError("probe positions must be finite");
    // drop a previous set
    dfree((void *&)probe_pos);
    dfree((void *&)ptable);
    dfree((void *&)ppart);
    dfree((void *&)pout);
    dfree((void *&)pair_vox);
    dfree((void *&)pair_kmin);
    dfree((void *&)row_start);
    dfree((void *&)pinv);
    dfree((void *&)ck_row);
    dfree((void *&)ck_lo);
    dfree((void *&)ck_hi);
    dfree((void *&)ck_start);
    dfree((void *&)ptable_v);
    dfree((void *&)pkmin_v);
    pnck = 0;
    np = 0;
    nw = 0;
    npairs = 0;
    if (n_probes == 0) return;
    // probe points in voxel steps per axis; distances in units of the x edge
    const double r = c_dt / h;
    const double edge[3] = {h, hy, hz}, hv[3] = {1.0, hy / h, hz / h};
    std::vector<double> P(3 * (size_t)n_probes);
    for (size_t i = 0; i < P.size(); i++) P[i] = pos[i] / edge[i % 3];
    // every voxel is a source: voxels with eps_r = 1 carry no current in the march, but the
    // transposed march needs the probe kernels there (their lambda enters the eps-gradient)
    std::vector<int> src((size_t)M);
    for (long m = 0; m < M; m++) src[(size_t)m] = (int)m;
    struct Pair {
        int kmin, vox;
    };
    std::vector<int> pp, pv, pk, rs((size_t)n_probes * (ell + 2));
    int nwin = 1;
    for (int p = 0; p < n_probes; p++) {
        std::vector<Pair> list;
        for (int m : src) {
            const int u = m % U, v = (m / U) % V, w = m / (U * V);
            const double d[3] = {P[3 * p] - (u + 0.5), P[3 * p + 1] - (v + 0.5), P[3 * p + 2] - (w + 0.5)};
            double a2 = 0, b2 = 0;
            for (int i = 0; i < 3; i++) {
                const double ad = std::fabs(d[i]);
                const double e = ad > 1.0 ? (ad - 1.0) * hv[i] : 0.0;
                a2 += e * e;
                b2 += ((ad + 1.0) * hv[i]) * ((ad + 1.0) * hv[i]);
            }
            // lags with r(k + 1) > R_min and r(k - 2) < R_max
            const int kmin = std::max(0, (int)std::floor(std::sqrt(a2) / r));
            const int kmax = std::min(ell, (int)std::ceil(std::sqrt(b2) / r + 2.0) - 1);
            if (kmin > kmax) continue;
            nwin = std::max(nwin, kmax - kmin + 1);
            list.push_back({kmin, m});
        }
        std::stable_sort(list.begin(), list.end(), [](const Pair &a, const Pair &b) { return a.kmin < b.kmin; });
        const int base = (int)pp.size();
        size_t q = 0;
        for (int kk = 0; kk <= ell + 1; kk++) {
            while (q < list.size() && list[q].kmin < kk) q++;
            rs[(size_t)p * (ell + 2) + kk] = base + (int)q;
        }
        for (const Pair &x : list) {
            pp.push_back(p);
            pv.push_back(x.vox);
            pk.push_back(x.kmin);
        }
    }
    np = n_probes;
    nw = nwin;
    npairs = (long)pp.size();
    probe_pos = dalloc<double>(P.size(), "probe positions");
    pair_vox = dalloc<int>(std::max<size_t>(pv.size(), 1), "probe pairs");
    pair_kmin = dalloc<int>(std::max<size_t>(pk.size(), 1), "probe windows");
    row_start = dalloc<int>(rs.size(), "probe rows");
    {
        std::vector<int> inv((size_t)n_probes * M, -1);
        for (size_t q = 0; q < pp.size(); q++) inv[(size_t)pp[q] * M + pv[q]] = (int)q;
        pinv = dalloc<int>(inv.size(), "probe pair index");
        MJ_CHECK(hipMemcpy(pinv, inv.data(), sizeof(int) * inv.size(), hipMemcpyHostToDevice));
    }
    int *pair_probe = dalloc<int>(std::max<size_t>(pp.size(), 1), "probe pair owners");
    ptable = dalloc<double>((size_t)std::max<long>(npairs, 1) * nw * 6, "probe kernel table");
    {
        // every row (p, k) cut into chunks of at most kProbeChunk pairs, probe by probe
        std::vector<int> crow, clo, chi_, cst;
        for (int p = 0; p < n_probes; p++) {
            cst.push_back((int)crow.size());
            for (int kk = 0; kk <= ell; kk++) {
                const int lo = rs[(size_t)p * (ell + 2) + std::max(0, kk - nwin + 1)];
                const int hi = rs[(size_t)p * (ell + 2) + kk + 1];
                for (int q = lo; q < hi; q += mj::kProbeChunk) {
                    crow.push_back(p * (ell + 1) + kk);
                    clo.push_back(q);
                    chi_.push_back(std::min(hi, q + mj::kProbeChunk));
                }
            }
        }
        cst.push_back((int)crow.size());
        pnck = (long)crow.size();
        ck_row = dalloc<int>(std::max<size_t>(crow.size(), 1), "probe chunks");
        ck_lo = dalloc<int>(std::max<size_t>(crow.size(), 1), "probe chunks");
        ck_hi = dalloc<int>(std::max<size_t>(crow.size(), 1), "probe chunks");
        ck_start = dalloc<int>(cst.size(), "probe chunks");
        if (pnck > 0) {
            MJ_CHECK(hipMemcpy(ck_row, crow.data(), sizeof(int) * crow.size(), hipMemcpyHostToDevice));
            MJ_CHECK(hipMemcpy(ck_lo, clo.data(), sizeof(int) * clo.size(), hipMemcpyHostToDevice));
            MJ_CHECK(hipMemcpy(ck_hi, chi_.data(), sizeof(int) * chi_.size(), hipMemcpyHostToDevice));
        }
        MJ_CHECK(hipMemcpy(ck_start, cst.data(), sizeof(int) * cst.size(), hipMemcpyHostToDevice));
    }
    ppart = dalloc<double>((size_t)nrhs * std::max<long>(pnck, 1) * 3, "probe partial sums");
    pout = dalloc<double>((size_t)nrhs * np * 3, "probe field");
    MJ_CHECK(hipMemcpy(probe_pos, P.data(), sizeof(double) * P.size(), hipMemcpyHostToDevice));
    MJ_CHECK(hipMemcpy(row_start, rs.data(), sizeof(int) * rs.size(), hipMemcpyHostToDevice));
    if (npairs > 0) {
        MJ_CHECK(hipMemcpy(pair_vox, pv.data(), sizeof(int) * pv.size(), hipMemcpyHostToDevice));
        MJ_CHECK(hipMemcpy(pair_kmin, pk.data(), sizeof(int) * pk.size(), hipMemcpyHostToDevice));
        MJ_CHECK(hipMemcpy(pair_probe, pp.data(), sizeof(int) * pp.size(), hipMemcpyHostToDevice));
        hipEvent_t e0, e1;
        MJ_CHECK(hipEventCreate(&e0));
        MJ_CHECK(hipEventCreate(&e1));
        MJ_CHECK(hipEventRecord(e0, st));
        mj::gen_offgrid_table(probe_pos, pair_probe, pair_vox, pair_kmin, npairs, U, V, gen.r, gen.hv, nw, ell, nquad, ptable, st);
        MJ_CHECK(hipEventRecord(e1, st));
        MJ_CHECK(hipEventSynchronize(e1));
        float ms = 0;
        MJ_CHECK(hipEventElapsedTime(&ms, e0, e1));
        t_probe_ms = ms;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    dfree((void *&)pair_probe);
    // the adjoint source walks the table voxel by voxel: a copy in that order
    ptable_v = dalloc<double>((size_t)nw * n_probes * M * 6, "probe kernel table by voxel");
    pkmin_v = dalloc<int>((size_t)n_probes * M, "probe windows by voxel");
    mj::launch_probe_table_by_voxel(ptable, pair_kmin, pinv, npairs, n_probes, nw, M, ptable_v, pkmin_v, st);
    // the probe rows read J_{n-k} for k = 0..ell from the real-space ring
    if (rdepth < ell + 1) {
        dfree((void *&)Jr);
        rdepth = ell + 1;
        Jr = dalloc<double>((size_t)rdepth * nrhs * 3 * M, "current history");
    }
    MJ_CHECK(hipStreamSynchronize(st));
}

// Kernel values at (probe, voxel, lag) triples through the same off-grid generator.
void mj_solver::offgrid_values(int cnt, const int *probe, const int *vox3, const int *lag, double *out)
{
    if (cnt <= 0) return;
    if (!probe_pos) throw std::logic_error("no probes set");
    std::vector<int> pp(cnt), pv(cnt), pk(cnt);
    for (int i = 0; i < cnt; i++) {
        if (probe[i] < 0 || probe[i] >= np) throw ArgError("probe index out of range");
        const int u = vox3[3 * i], v = vox3[3 * i + 1], w = vox3[3 * i + 2];
        if (u < 0 || u >= U || v < 0 || v >= V || w < 0 || w >= W) throw ArgError("voxel out of range");
        if (lag[i] < 0) throw ArgError("lag < 0");
        pp[i] = probe[i];
        pv[i] = u + U * (v + V * w);
        pk[i] = lag[i];
    }
    int *d_p = nullptr, *d_v = nullptr, *d_k = nullptr;
    double *d_o = nullptr;
    try {
        d_p = (int *)da.get(sizeof(int) * cnt, "probe request");
        d_v = (int *)da.get(sizeof(int) * cnt, "probe request");
        d_k = (int *)da.get(sizeof(int) * cnt, "probe request");
        d_o = (double *)da.get(sizeof(double) * 6 * cnt, "probe values");
        MJ_CHECK(hipMemcpy(d_p, pp.data(), sizeof(int) * cnt, hipMemcpyHostToDevice));
        MJ_CHECK(hipMemcpy(d_v, pv.data(), sizeof(int) * cnt, hipMemcpyHostToDevice));
        MJ_CHECK(hipMemcpy(d_k, pk.data(), sizeof(int) * cnt, hipMemcpyHostToDevice));
        mj::gen_offgrid_table(probe_pos, d_p, d_v, d_k, cnt, U, V, gen.r, gen.hv, 1, 0x7fffffff, nquad, d_o, st);
        MJ_CHECK(hipStreamSynchronize(st));
        MJ_CHECK(hipMemcpy(out, d_o, sizeof(double) * 6 * cnt, hipMemcpyDeviceToHost));
    } catch (...) {
        da.put(d_p);
        da.put(d_v);
        da.put(d_k);
        da.put(d_o);
        throw;
    }
    da.put(d_p);
    da.put(d_v);
    da.put(d_k);
    da.put(d_o);
}

// March state: a fixed header, then the spectral ring, the time block's far sums and the
// real-space history, each copied whole (slots the march does not read yet copy as they are).
namespace {
struct StateHeader {
    char magic[8];
    int32_t version, U, V, W, nrhs, ell, B, rdepth, Nx, Ny, Nz, Hp, B2, cheb_pred;
    int64_t n, ring_bytes, far_bytes, jr_bytes, outer_bytes;
};
constexpr char kStateMagic[8] = {'M', 'J', 'S', 'T', 'A', 'T', 'E', '2'};
}  // namespace

size_t mj_solver::state_bytes() const
{
    const size_t sp = (size_t)spec_plane(), v3 = (size_t)nrhs * 3;
    return sizeof(StateHeader) + sizeof(double2) * (size_t)ell * v3 * sp +
           (farbuf ? sizeof(double2) * (size_t)B * v3 * sp : 0) + (gbuf ? sizeof(double2) * (size_t)B2 * v3 * sp : 0) +
           sizeof(double) * (size_t)rdepth * v3 * M;
}

void mj_solver::get_state(void *buf) const
{
    const size_t sp = (size_t)spec_plane(), v3 = (size_t)nrhs * 3;
    StateHeader h{};
    std::memcpy(h.magic, kStateMagic, 8);
    h.version = 2;
    h.U = U;
    h.V = V;
    h.W = W;
    h.nrhs = nrhs;
    h.ell = ell;
    h.B = B;
    h.rdepth = rdepth;
    h.Nx = Nx;
    h.Ny = Ny;
    h.Nz = Nz;
    h.Hp = Hp;
    h.B2 = B2;
    h.cheb_pred = cheb_pred;   // the next Z_0 solve's first batch of passes (part of its arithmetic)
    h.n = n;
    h.ring_bytes = (int64_t)(sizeof(double2) * (size_t)ell * v3 * sp);
    h.far_bytes = farbuf ? (int64_t)(sizeof(double2) * (size_t)B * v3 * sp) : 0;
    h.jr_bytes = (int64_t)(sizeof(double) * (size_t)rdepth * v3 * M);
    h.outer_bytes = gbuf ? (int64_t)(sizeof(double2) * (size_t)B2 * v3 * sp) : 0;
    char *p = (char *)buf;
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    MJ_CHECK(hipStreamSynchronize(st));
    MJ_CHECK(hipMemcpy(p, ring, (size_t)h.ring_bytes, hipMemcpyDeviceToHost));
    p += h.ring_bytes;
    if (h.far_bytes) MJ_CHECK(hipMemcpy(p, farbuf, (size_t)h.far_bytes, hipMemcpyDeviceToHost));
    p += h.far_bytes;
    MJ_CHECK(hipMemcpy(p, Jr, (size_t)h.jr_bytes, hipMemcpyDeviceToHost));
    p += h.jr_bytes;
    if (h.outer_bytes) MJ_CHECK(hipMemcpy(p, gbuf, (size_t)h.outer_bytes, hipMemcpyDeviceToHost));
}

void mj_solver::set_state(const void *buf, size_t bytes)
{
    StateHeader h;
    if (bytes < sizeof h) throw ArgError("state buffer too short");
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, kStateMagic, 8) != 0 || h.version != 2) throw ArgError("not a march state");
    if (h.U != U || h.V != V || h.W != W || h.nrhs != nrhs || h.ell != ell || h.B != B || h.B2 != B2 ||
        h.Nx != Nx || h.Ny != Ny || h.Nz != Nz || h.Hp != Hp)
        throw ArgError("state of a solver with another grid, n_rhs, ell or time blocks");
    if (h.rdepth != rdepth) throw ArgError("state of a solver with another history depth (probes differ)");
    if (bytes < state_bytes() || (size_t)h.ring_bytes + (size_t)h.far_bytes + (size_t)h.jr_bytes +
                                         (size_t)h.outer_bytes + sizeof h != state_bytes())
        throw ArgError("state buffer has the wrong size");
    if (h.n < 0 || h.n > INT32_MAX) throw ArgError("bad step count in the state");
    const char *p = (const char *)buf + sizeof h;
    drop_side();
    MJ_CHECK(hipStreamSynchronize(st));
    MJ_CHECK(hipMemcpy(ring, p, (size_t)h.ring_bytes, hipMemcpyHostToDevice));
    p += h.ring_bytes;
    if (h.far_bytes) MJ_CHECK(hipMemcpy(farbuf, p, (size_t)h.far_bytes, hipMemcpyHostToDevice));
    p += h.far_bytes;
    MJ_CHECK(hipMemcpy(Jr, p, (size_t)h.jr_bytes, hipMemcpyHostToDevice));
    p += h.jr_bytes;
    if (h.outer_bytes) MJ_CHECK(hipMemcpy(gbuf, p, (size_t)h.outer_bytes, hipMemcpyHostToDevice));
    n = (int)h.n;
    cheb_pred = std::max(0, (int)h.cheb_pred);
}

// Gradient of Phi = sum_{n=1}^{N} sum_r sum_p |E^s_{r,p}(n)|^2 with respect to eps_r of every
// voxel, by the transposed march (see mj_march.hip) with checkpointing:
//  1. forward march of all N steps, keeping the probe field of every step and, at the start
//     of every segment but the first, the real-space history J_{n0-ell-1} .. J_{n0-1} that a
//     restart at n0 needs; segments start at time-block starts, so a restart begins with a
//     far-part launch like the original march did;
//  2. segments from last to first: recompute the segment's forward steps from its checkpoint
//     (the last one is kept from step 1), storing B_n, then run the transposed march over the
//     segment's steps in reversed time, accumulating lambda_n . B_n / eps^2.
// The recomputed steps repeat the original arithmetic exactly.  Leaves the march at n = 0.
void mj_solver::adjoint_gradient(int N, int ckpt_every, double *phi, double *grad_dev, double *probe_hist)
{
    if (!waves_set) throw std::logic_error("plane waves not set (mj_set_plane_waves)");
    if (np <= 0) throw std::logic_error("the objective is the probe field: set probes first");
    if (n != 0) throw std::logic_error("the gradient run starts at n = 0 (mj_reset)");
    if (N < 1) throw ArgError("n_steps must be >= 1");
    if (rdepth < ell + 1) throw std::logic_error("probe history depth");
    // segment starts: 1, then block starts 2 + c L with L a multiple of the time block
    int L = ckpt_every > 0 ? ckpt_every : N;
    // restarts at (outer) time-block starts repeat the original arithmetic exactly
    const int period = B2 ? B2 : B;
    if (period > 1) L = ((L + period - 1) / period) * period;
    std::vector<int> starts{1};
    for (long s0 = 2 + (long)L; s0 <= N; s0 += L) starts.push_back((int)s0);
    const int C = (int)starts.size();
    auto seg_end = [&](int c) { return c + 1 < C ? starts[c + 1] - 1 : N; };
    int maxseg = 0;
    for (int c = 0; c < C; c++) maxseg = std::max(maxseg, seg_end(c) - starts[c] + 1);
    const size_t vec = (size_t)nrhs * 3 * M;
    // every step j that a restart reads (j = s0 - 1 - ell .. s0 - 1 for a segment start s0 > 1)
    // is kept once, in one pool indexed through pool_of[j], however the windows overlap
    std::vector<long> pool_of((size_t)N + 1, -1);
    long npool = 0;
    for (int c = 1; c < C; c++)
        for (int j = std::max(1, starts[c] - 1 - ell); j <= starts[c] - 1; j++)
            if (pool_of[(size_t)j] < 0) pool_of[(size_t)j] = 1;
    for (int j = 1; j <= N; j++)
        if (pool_of[(size_t)j] > 0) pool_of[(size_t)j] = npool++;
    const long sp = spec_plane();
    std::vector<void *> tmp;
    auto talloc = [&](size_t bytes, const char *what) {
        void *ptr = nullptr;
        try {
            ptr = da.get(std::max<size_t>(bytes, 8), what);
        } catch (...) {
            for (void *q : tmp) da.put(q);
            throw;
        }
        tmp.push_back(ptr);
        return ptr;
    };
    double *Ehist = (double *)talloc(sizeof(double) * (size_t)N * nrhs * np * 3, "probe history");
    double *ckpt = (double *)talloc(sizeof(double) * (size_t)std::max<long>(npool, 1) * vec, "checkpoints");
    double *Bbuf = (double *)talloc(sizeof(double) * (size_t)maxseg * vec, "gradient terms");
    double *G = (double *)talloc(sizeof(double) * vec, "adjoint source");
    double *bqb = (double *)talloc(sizeof(double) * vec, "adjoint rhs");
    double2 *ring_a = (double2 *)talloc(sizeof(double2) * (size_t)ell * nrhs * 3 * sp, "adjoint ring");
    double2 *far_a = B > 1 ? (double2 *)talloc(sizeof(double2) * (size_t)B * nrhs * 3 * sp, "adjoint blocks") : nullptr;
    double2 *g_a = B2 ? (double2 *)talloc(sizeof(double2) * (size_t)B2 * nrhs * 3 * sp, "adjoint outer blocks") : nullptr;
    double *nu_r = (double *)talloc(sizeof(double) * (size_t)rdepth * vec, "adjoint history");
    double *lam_r = (double *)talloc(sizeof(double) * (size_t)rdepth * vec, "adjoint local history");
    MJ_CHECK(hipMemsetAsync(grad_dev, 0, sizeof(double) * M, st));
    std::vector<int> pred_at((size_t)N + 2, 0);
    int adj_pred = 0;
    double2 *const ring_f = ring, *const far_f = farbuf, *const g_f = gbuf;
    double *const Jr_f = Jr;
    hipEvent_t tev[3];
    for (auto &tv : tev) MJ_CHECK(hipEventCreate(&tv));
    MJ_CHECK(hipEventRecord(tev[0], st));
    bool noconv = false;
    auto check_cg = [&] {
        for (int i = 0; i < nrhs; i++)
            if (!cgstat_h[i].done) noconv = true;
    };
    try {
        // 1. forward; the Chebyshev prediction each step starts from is kept, so that a
        // recomputed segment takes the same passes as the original steps
        const int last0 = starts[C - 1];
        for (int t = 1; t <= N; t++) {
            pred_at[(size_t)t] = cheb_pred;
            StepIO io;
            io.Pout = Ehist + (size_t)(t - 1) * nrhs * np * 3;
            io.Bout = t >= last0 ? Bbuf + (size_t)(t - last0) * vec : nullptr;
            step(io);
            check_growth();
            check_cg();
            if (pool_of[(size_t)t] >= 0)
                MJ_CHECK(hipMemcpyAsync(ckpt + (size_t)pool_of[(size_t)t] * vec, Jr + (size_t)slotR(t) * vec,
                                        sizeof(double) * vec, hipMemcpyDeviceToDevice, st));
        }
        if (probe_hist)
            MJ_CHECK(hipMemcpyAsync(probe_hist, Ehist, sizeof(double) * (size_t)N * nrhs * np * 3,
                                    hipMemcpyDeviceToDevice, st));
        std::vector<double> Eh((size_t)N * nrhs * np * 3);
        MJ_CHECK(hipMemcpyAsync(Eh.data(), Ehist, sizeof(double) * Eh.size(), hipMemcpyDeviceToHost, st));
        MJ_CHECK(hipStreamSynchronize(st));
        double ph = 0.0;
        for (double v : Eh) ph += v * v;
        if (phi) *phi = ph;
        MJ_CHECK(hipEventRecord(tev[1], st));
        // 2. backward; the transposed march has its own rings, swapped in while it runs
        int n_adj = 0;
        for (int c = C - 1; c >= 0; c--) {
            const int s0 = starts[c], s1 = seg_end(c);
            if (c < C - 1) {
                // restart the forward march at s0 from its checkpoint and recompute the segment
                drop_side();
                n = s0 - 1;
                if (c > 0) {
                    const int j0 = s0 - 1 - ell;   // first stored step
                    for (int j = std::max(1, j0); j <= s0 - 1; j++) {
                        const double *src = ckpt + (size_t)pool_of[(size_t)j] * vec;
                        MJ_CHECK(hipMemcpyAsync(Jr + (size_t)slotR(j) * vec, src, sizeof(double) * vec,
                                                hipMemcpyDeviceToDevice, st));
                        if (j <= s0 - 2)
                            mj::fft3d_forward(fft, src, ring + (size_t)slotS(j) * nrhs * 3 * sp, 3 * nrhs, st);
                    }
                }
                cheb_pred = pred_at[(size_t)s0];
                for (int t = s0; t <= s1; t++) {
                    StepIO io;
                    io.skip_probes = true;
                    io.Bout = Bbuf + (size_t)(t - s0) * vec;
                    step(io);
                    check_cg();
                }
            }
            // transposed march over j = s1 .. s0 (reversed step n' = N + 1 - j)
            drop_side();
            ring = ring_a;
            farbuf = far_a;
            gbuf = g_a;
            Jr = nu_r;
            Lr = lam_r;
            bq = bqb;
            n = n_adj;
            cheb_pred = adj_pred;
            for (int j = s1; j >= s0; j--) {
                mj::AdjArg a = adj_arg();
                a.Ehist = Ehist;
                a.N = N;
                a.j = j;
                a.G = G;
                mj::launch_adj_source(a, st);
                StepIO io;
                io.adjoint = true;
                io.G = G;
                io.Bj = Bbuf + (size_t)(j - s0) * vec;
                io.grad = grad_dev;
                step(io);
                check_cg();
            }
            n_adj = n;
            adj_pred = cheb_pred;
            drop_side();
            ring = ring_f;
            farbuf = far_f;
            gbuf = g_f;
            Jr = Jr_f;
            Lr = nullptr;
            bq = nullptr;
        }
        MJ_CHECK(hipEventRecord(tev[2], st));
        MJ_CHECK(hipStreamSynchronize(st));
    } catch (...) {
        (void)hipStreamSynchronize(st);
        if (side) (void)hipStreamSynchronize(side);
        side_pending = false;
        h_block = 0;
        ring = ring_f;
        farbuf = far_f;
        gbuf = g_f;
        Jr = Jr_f;
        Lr = nullptr;
        bq = nullptr;
        for (void *q : tmp) da.put(q);
        for (auto &tv : tev) (void)hipEventDestroy(tv);
        n = 0;
        throw;
    }
    float f_ms = 0, b_ms = 0;
    MJ_CHECK(hipEventElapsedTime(&f_ms, tev[0], tev[1]));
    MJ_CHECK(hipEventElapsedTime(&b_ms, tev[1], tev[2]));
    stat[14] = f_ms;
    stat[15] = b_ms;
    stat[16] = C;
    stat[17] = (double)npool * vec * sizeof(double);
    for (void *q : tmp) da.put(q);
    for (auto &tv : tev) (void)hipEventDestroy(tv);
    n = 0;
    if (noconv) throw std::range_error("Z_0 solve did not converge");
}

// ============================================================================ C ABI
namespace {
int fail(mj_solver *s, int code, const std::string &msg)
{
    if (s) s->err = msg;
    else g_err = msg;
    return code;
}

template <class F>
int guarded(mj_solver *s, F &&f)
{
    try {
        f();
        return MJ_OK;
    } catch (const ArgError &e) {
        return fail(s, MJ_EINVAL, e.what());
    } catch (const MemError &e) {
        return fail(s, MJ_ENOMEM, e.what());
    } catch (const HipError &e) {
        return fail(s, MJ_EHIP, e.what());
    } catch (const UnstableError &e) {
        return fail(s, MJ_EUNSTABLE, e.what());
    } catch (const std::range_error &e) {
        return fail(s, MJ_ENOCONV, e.what());
    } catch (const std::logic_error &e) {
        return fail(s, MJ_ESTATE, e.what());
    } catch (const std::exception &e) {
        return fail(s, MJ_EHIP, e.what());
    } catch (...) {
        return fail(s, MJ_EHIP, "unknown error");
    }
}
}  // namespace

extern "C" {

int mj_create(const mj_config *cfg, mj_solver **out)
{
    if (!cfg || !out) return fail(nullptr, MJ_EINVAL, "NULL argument");
    *out = nullptr;
    mj_solver *s = new (std::nothrow) mj_solver();
    if (!s) return fail(nullptr, MJ_ENOMEM, "host allocation failed");
    int rc = guarded(nullptr, [&] { s->create(*cfg); });
    if (rc != MJ_OK) {
        delete s;
        return rc;
    }
    *out = s;
    return MJ_OK;
}

void mj_destroy(mj_solver *s) { delete s; }

const char *mj_last_error(const mj_solver *s) { return s ? s->err.c_str() : g_err.c_str(); }

int mj_info(const mj_solver *s, double *out, int32_t n)
{
    if (!s || !out) return MJ_EINVAL;
    double v[24] = {(double)s->ell, (double)s->Nx, (double)s->Ny, (double)s->Nz, (double)s->B,
                    (double)s->rdepth, (double)s->nrhs, (double)s->n, (double)s->bytes, s->t_gen_ms,
                    s->t_spec_ms, (double)s->fir.size(), (double)s->np, (double)s->nw, (double)s->npairs,
                    s->t_probe_ms, (double)s->fft.Px, (double)s->fft.Py, (double)s->fft.Pz, (double)s->B2,
                    (double)s->z0_method, s->lam_lo, s->lam_hi, s->overlap ? 1.0 : 0.0};
    for (int i = 0; i < n && i < 24; i++) out[i] = v[i];
    return MJ_OK;
}

int mj_set_plane_waves(mj_solver *s, const double *khat, const double *pol, const double *width, const double *ct0,
                       const double *amp, const double *r_ref)
{
    if (!s) return MJ_EINVAL;
    return guarded(s, [&] {
        if (!khat || !pol || !width || !ct0 || !amp || !r_ref) throw ArgError("NULL wave parameter");
        std::vector<mj::WaveArg> w(s->nrhs);
        for (int i = 0; i < s->nrhs; i++) {
            double kn = 0;
            for (int c = 0; c < 3; c++) {
                w[i].k[c] = khat[3 * i + c];
                w[i].pol[c] = pol[3 * i + c];
                w[i].rref[c] = r_ref[3 * i + c];
                kn += khat[3 * i + c] * khat[3 * i + c];
            }
            if (!(std::fabs(kn - 1.0) < 1e-12)) throw ArgError("khat must be a unit vector");
            if (!(width[i] > 0.0) || !std::isfinite(width[i])) throw ArgError("width must be positive and finite");
            bool fin = std::isfinite(ct0[i]) && std::isfinite(amp[i]);
            for (int c = 0; c < 3; c++) fin = fin && std::isfinite(pol[3 * i + c]) && std::isfinite(r_ref[3 * i + c]);
            if (!fin) throw ArgError("wave parameters must be finite");
            w[i].width = width[i];
            w[i].ct0 = ct0[i];
            w[i].amp = amp[i];
            plan_wave(w[i], s->h, s->hy, s->hz);
        }
        MJ_CHECK(hipMemcpy(s->waves_d, w.data(), sizeof(mj::WaveArg) * s->nrhs, hipMemcpyHostToDevice));
        s->waves = w;
        s->waves_set = true;
    });
}

int mj_run(mj_solver *s, int32_t n_steps, double *J_hist)
{
    if (!s) return MJ_EINVAL;
    if (n_steps < 0) return fail(s, MJ_EINVAL, "n_steps < 0");
    return guarded(s, [&] { s->run(n_steps, J_hist, nullptr); });
}

int mj_march(mj_solver *s, int32_t n_steps, double *J_hist, double *probe_hist)
{
    if (!s) return MJ_EINVAL;
    if (n_steps < 0) return fail(s, MJ_EINVAL, "n_steps < 0");
    return guarded(s, [&] { s->run(n_steps, J_hist, probe_hist); });
}

int mj_step(mj_solver *s, double *J_dev, double *probe)
{
    if (!s) return MJ_EINVAL;
    return guarded(s, [&] { s->run(1, J_dev, probe); });
}

int mj_march_every(mj_solver *s, int32_t n_steps, int32_t j_every, double *J_hist, double *probe_hist)
{
    if (!s) return MJ_EINVAL;
    if (n_steps < 0) return fail(s, MJ_EINVAL, "n_steps < 0");
    if (j_every < 1) return fail(s, MJ_EINVAL, "j_every < 1");
    return guarded(s, [&] { s->run(n_steps, J_hist, probe_hist, j_every); });
}

int mj_set_eps(mj_solver *s, const double *eps_r)
{
    if (!s || !eps_r) return MJ_EINVAL;
    return guarded(s, [&] {
        if (s->n != 0) throw std::logic_error("eps is changed at n = 0 (after mj_create or mj_reset)");
        s->set_material(eps_r);
        s->restart();
        if (s->z0_method == 0) s->estimate_spectrum();
    });
}

int mj_adjoint_gradient(mj_solver *s, int32_t n_steps, int32_t ckpt_every, double *phi, double *dphi_deps,
                        double *probe_hist)
{
    if (!s || !dphi_deps) return MJ_EINVAL;
    if (n_steps < 1) return fail(s, MJ_EINVAL, "n_steps < 1");
    return guarded(s, [&] { s->adjoint_gradient(n_steps, ckpt_every, phi, dphi_deps, probe_hist); });
}

int mj_set_probes(mj_solver *s, int32_t n_probes, const double *pos)
{
    if (!s) return MJ_EINVAL;
    return guarded(s, [&] { s->set_probes(n_probes, pos); });
}

int mj_probe_kernel_values(mj_solver *s, int32_t n, const int32_t *probe, const int32_t *voxel,
                           const int32_t *lag, double *out)
{
    if (!s) return MJ_EINVAL;
    if (n < 0 || (n > 0 && (!probe || !voxel || !lag || !out))) return fail(s, MJ_EINVAL, "bad arguments");
    return guarded(s, [&] { s->offgrid_values(n, probe, voxel, lag, out); });
}

int mj_reset(mj_solver *s)
{
    if (!s) return MJ_EINVAL;
    return guarded(s, [&] { s->restart(); });
}

int mj_get_state(const mj_solver *s, void *buf, size_t *bytes)
{
    if (!s || !bytes) return MJ_EINVAL;
    mj_solver *sm = const_cast<mj_solver *>(s);
    return guarded(sm, [&] {
        const size_t need = s->state_bytes();
        if (buf) {
            if (*bytes < need) throw ArgError("state buffer too small");
            s->get_state(buf);
        }
        *bytes = need;
    });
}

int mj_set_state(mj_solver *s, const void *buf, size_t bytes)
{
    if (!s) return MJ_EINVAL;
    if (!buf) return fail(s, MJ_EINVAL, "state buffer is NULL");
    return guarded(s, [&] { s->set_state(buf, bytes); });
}

int mj_history_sum(mj_solver *s, const double *J_hist, int32_t depth, double *P)
{
    if (!s) return MJ_EINVAL;
    if (!J_hist || !P || depth < 1) return fail(s, MJ_EINVAL, "bad history arguments");
    return guarded(s, [&] { s->history_sum(J_hist, depth, P); });
}

int mj_kernel_values(mj_solver *s, int32_t n, const int32_t *lag, const int32_t *offset, double *out)
{
    if (!s) return MJ_EINVAL;
    if (n < 0 || (n > 0 && (!lag || !offset || !out))) return fail(s, MJ_EINVAL, "bad kernel value request");
    return guarded(s, [&] {
        for (int i = 0; i < n; i++) {
            if (lag[i] < 0 || lag[i] > s->ell) throw ArgError("lag out of range");
            if (std::abs(offset[3 * i]) >= s->U || std::abs(offset[3 * i + 1]) >= s->V ||
                std::abs(offset[3 * i + 2]) >= s->W)
                throw ArgError("offset out of range");
        }
        if (n == 0) return;
        mj::DevTemp tl(s->da, sizeof(int) * n, "kernel value request");
        mj::DevTemp to(s->da, sizeof(int) * 3 * n, "kernel value request");
        mj::DevTemp tv(s->da, sizeof(double) * 6 * n, "kernel values");
        int *lag_d = tl.as<int>(), *off_d = to.as<int>();
        double *out_d = tv.as<double>();
        MJ_CHECK(hipMemcpy(lag_d, lag, sizeof(int) * n, hipMemcpyHostToDevice));
        MJ_CHECK(hipMemcpy(off_d, offset, sizeof(int) * 3 * n, hipMemcpyHostToDevice));
        mj::gen_kernel_values(s->gen, n, lag_d, off_d, out_d, s->st);
        MJ_CHECK(hipMemcpyAsync(out, out_d, sizeof(double) * 6 * n, hipMemcpyDeviceToHost, s->st));
        MJ_CHECK(hipStreamSynchronize(s->st));
    });
}

int mj_kernel_values_noalloc(mj_solver *s, int32_t n, const int32_t *lag, const int32_t *offset, double *out)
{
    if (!s) return MJ_EINVAL;
    if (n < 0 || (n > 0 && (!lag || !offset || !out))) return fail(s, MJ_EINVAL, "bad kernel value request");
    if (n > kNoAllocMax)
        return fail(s, MJ_EINVAL, "at most " + std::to_string(kNoAllocMax) + " requests per call (staging array size)");
    return guarded(s, [&] {
        for (int i = 0; i < n; i++) {
            if (lag[i] < 0 || lag[i] > s->ell) throw ArgError("lag out of range");
            if (std::abs(offset[3 * i]) >= s->U || std::abs(offset[3 * i + 1]) >= s->V ||
                std::abs(offset[3 * i + 2]) >= s->W)
                throw ArgError("offset out of range");
        }
        if (n == 0) return;
        int cur = -1;
        MJ_CHECK(hipGetDevice(&cur));
        if (cur != s->dev) throw ArgError("call with the solver's device current");
        unsigned char *base = scratch_ptr(cur);
        double *out_d = (double *)base;
        int32_t *lag_d = (int32_t *)(base + (size_t)kNoAllocMax * 6 * sizeof(double));
        int32_t *off_d = lag_d + kNoAllocMax;
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        MJ_CHECK(hipMemcpyAsync(lag_d, lag, sizeof(int32_t) * n, hipMemcpyHostToDevice, s->st));
        MJ_CHECK(hipMemcpyAsync(off_d, offset, sizeof(int32_t) * 3 * n, hipMemcpyHostToDevice, s->st));
        mj::gen_kernel_values(s->gen, n, lag_d, off_d, out_d, s->st);
        MJ_CHECK(hipMemcpyAsync(out, out_d, sizeof(double) * 6 * n, hipMemcpyDeviceToHost, s->st));
        MJ_CHECK(hipStreamSynchronize(s->st));
    });
}

int mj_stats(const mj_solver *s, double *out, int32_t n)
{
    if (!s || !out) return MJ_EINVAL;
    for (int i = 0; i < n && i < 21; i++) out[i] = s->stat[i];
    return MJ_OK;
}

int mj_fft_roundtrip(mj_solver *s, const double *x, double *X, double *yout)
{
    if (!s || !x) return MJ_EINVAL;
    return guarded(s, [&] {
        // the spectrum is held with row pitch Hp; the caller's X has rows of Hx
        double2 *Xd = s->Shat;
        mj::fft3d_forward(s->fft, x, Xd, 3, s->st);
        if (X)
            MJ_CHECK(hipMemcpy2DAsync(X, sizeof(double2) * s->Hx, Xd, sizeof(double2) * s->Hp, sizeof(double2) * s->Hx,
                                      (size_t)3 * s->Nz * s->Ny, hipMemcpyDeviceToDevice, s->st));
        if (yout) mj::fft3d_inverse(s->fft, Xd, yout, 3, s->st);
        MJ_CHECK(hipStreamSynchronize(s->st));
    });
}

}  // extern "C"
