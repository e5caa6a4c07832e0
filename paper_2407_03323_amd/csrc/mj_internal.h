// Internal declarations of the MOT-JVIE HIP library (gfx950, FP64 throughout).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#define MJ_CHECK(expr)                                                                     \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw mj::HipError(std::string(#expr) + ": " + hipGetErrorString(e_));         \
    } while (0)

namespace mj {

struct HipError : std::runtime_error {
    using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
    using std::runtime_error::runtime_error;
};
struct UnstableError : std::runtime_error {
    using std::runtime_error::runtime_error;
};
struct MemError : std::runtime_error {
    using std::runtime_error::runtime_error;
};

// ---------------------------------------------------------------------------- device memory
// Every device buffer of a solver comes from here: hipMalloc/hipFree, or the caller's allocator
// (mj_config.alloc / free_, e.g. PyTorch's caching allocator) when one is given.
struct DevAlloc {
    void *(*fn_alloc)(size_t, void *) = nullptr;
    void (*fn_free)(void *, void *) = nullptr;
    void *ctx = nullptr;

    void *get(size_t bytes, const char *what) const
    {
        if (bytes == 0) bytes = 8;
        void *p = nullptr;
        if (fn_alloc) {
            p = fn_alloc(bytes, ctx);
        } else if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        if (!p)
            throw MemError(std::string("device allocation failed: ") + what + " (" + std::to_string(bytes) + " bytes)");
        return p;
    }
    void put(void *p) const
    {
        if (!p) return;
        if (fn_free) fn_free(p, ctx);
        else (void)hipFree(p);
    }
};

// A temporary device buffer released when it goes out of scope (also on an exception).
struct DevTemp {
    const DevAlloc &da;
    void *p;
    DevTemp(const DevAlloc &a, size_t bytes, const char *what) : da(a), p(a.get(bytes, what)) {}
    ~DevTemp() { da.put(p); }
    DevTemp(const DevTemp &) = delete;
    DevTemp &operator=(const DevTemp &) = delete;
    template <class T>
    T *as() const { return (T *)p; }
};

// ---------------------------------------------------------------------------- complex
__host__ __device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// ---------------------------------------------------------------------------- XCD order
// The chip hands workgroups to its 8 XCDs in turn (dispatch index b to XCD b mod 8), and every
// XCD has its own L2.  Tiles that share cache lines (the ends of unaligned rows, the planes a
// stencil reads) should meet in one L2, so kernels take their tile from
// xcd_block(b, n): XCD x works on the contiguous range of logical indices that starts at
// x q + min(x, n mod 8) (q = n / 8), in dispatch order.  A bijection of [0, n).
constexpr unsigned kXcds = 8;
__device__ inline unsigned xcd_block(unsigned b, unsigned n)
{
    const unsigned q = n / kXcds, rem = n % kXcds, x = b % kXcds, j = b / kXcds;
    return x * q + (x < rem ? x : rem) + j;
}

// ---------------------------------------------------------------------------- FFT plan
constexpr int kMaxStages = 12;
constexpr int kMaxFftN = 512;

struct FftPlan1D {
    int N = 0;
    int nst = 0;
    int radix[kMaxStages] = {};
    double2 *tw = nullptr;  // device table W_N^m = exp(-2 pi i m / N), m = 0..N-1
};

// Builds the radix plan and uploads the correctly rounded twiddle table.
void fft_plan_init(FftPlan1D &p, int N, const DevAlloc &da);
void fft_plan_free(FftPlan1D &p, const DevAlloc &da);
bool fft_size_ok(int N);
int fft_pick_size(int nmin);  // smallest even N >= nmin whose factors are all supported radices

// Geometry of one padded 3-D transform of `ncomp` real fields on a U x V x W box.
// Row pitch Hp >= Hx of the half spectra (columns Hx .. Hp-1 are never read).  Rounding the
// pitch up to whole 128-byte lines was measured on the far MAC at 104^3: it removes about a
// seventh of the line traffic but adds idle lanes, and the kernel ran 5% slower; so Hp = Hx.
inline int spectrum_pitch(int Hx) { return Hx; }

struct Fft3D {
    int U, V, W;
    int Nx, Ny, Nz, Hx, Hp;  // Hx = Nx/2 + 1, Hp = row pitch of the half spectra
    FftPlan1D px, py, pz;
    // scratch: after the x pass [ncomp][W][V][Hp], after the y pass [ncomp][W][Ny][Hp]
    double2 *bufA = nullptr, *bufB = nullptr;
    int ncomp = 0;
    int Px = 1, Py = 1, Pz = 1;  // pencils per block of the x, y and z passes
    DevAlloc da;                 // where the twiddles and scratch came from
};

void fft3d_init(Fft3D &f, int U, int V, int W, int ncomp, int Nx, int Ny, int Nz, const DevAlloc &da);
void fft3d_free(Fft3D &f);
// pencils per block of every pass: at most cap, and at most what one tile holds
void fft3d_set_pencils(Fft3D &f, int cap);
// times the candidate pencil counts of each pass on the plan's own sizes and keeps the fastest
void fft3d_autotune(Fft3D &f, hipStream_t st);
// x: [ncomp][W][V][U] real; X: [ncomp][Nz][Ny][Hp] complex (unnormalised forward DFT of the zero-padded field)
void fft3d_forward(Fft3D &f, const double *x, double2 *X, int ncomp, hipStream_t st);
// X: [ncomp][Nz][Ny][Hp]; y: [ncomp][W][V][U] = unnormalised inverse DFT restricted to the box
void fft3d_inverse(Fft3D &f, const double2 *X, double *y, int ncomp, hipStream_t st);

// ---------------------------------------------------------------------------- generator
// Shell moments per octant offset (see mj_gen.hip).  kMoments values per (offset, shell); the
// shells are c dt wide, so a voxel pair with edges h meets at most 2 |h| / (c dt) + 3 of them.
constexpr int kMoments = 19;
constexpr double kMinCdtOverH = 0.3;   // smallest c dt / max(h) the generator accepts
constexpr int kShellCap = 16;          // shells per offset at c dt = 0.3 max(h): at most 14

struct GenResult {
    double *moments = nullptr;  // [Woct][Voct][Uoct][ms][kMoments]
    int Uo = 0, Vo = 0, Wo = 0;
    int ms = 0;                 // shells stored per offset
    double r = 1.0;             // c dt, in units of the x edge
    double hv[3] = {1.0, 1.0, 1.0};   // voxel edges, in units of the x edge
};

// r = c dt and hv = voxel edges, both in units of the x edge (hv[0] = 1)
void gen_moments(GenResult &g, int U, int V, int W, double r, const double hv[3], int nquad, const DevAlloc &da,
                 hipStream_t st);
// K_k on the full periodic grid [6][Nz][Ny][Nx] (real), from the octant moments
void gen_kernel_grid(const GenResult &g, int k, int Nx, int Ny, int Nz, double *grid, hipStream_t st);
// K_k(D) for a list of (k, D): out[n][6]
// Kernels seen from test voxels centred at arbitrary points pos[p] (units of h from the grid
// corner) for source voxels pair_vox (linear index), lags pair_kmin .. pair_kmin + nw - 1
// (zero above kmax): out[nw][pair][6].
void gen_offgrid_table(const double *pos_dev, const int *pair_probe_dev, const int *pair_vox_dev,
                       const int *pair_kmin_dev, long npairs, int U, int V, double r, const double hv[3], int nw,
                       int kmax, int nquad, double *out_dev, hipStream_t st);

void gen_kernel_values(const GenResult &g, int n, const int *lag_dev, const int *off_dev, double *out_dev,
                       hipStream_t st);

}  // namespace mj
