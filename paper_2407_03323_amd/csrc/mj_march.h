// Argument blocks of the per-step march kernels.
#pragma once

#include "mj_internal.h"

namespace mj {

constexpr int kMaxLocal = 64;   // largest history depth kept in real space

struct MacArg {
    const double *Khat;      // [nk][Nz/2+1][Ny/2+1][Hp][6] real, lags 1..nk
    const double2 *ring_base;// [ring][nrhs][3][Nz][Ny][Hp]
    double2 *Shat;           // [nrhs][3][Nz][Ny][Hp]
    int Hx, Hp, Ny, Nz;      // Hx = Nx/2 + 1 frequencies in rows of pitch Hp
    int nk;                  // number of lags summed (1..nk)
    int ring;                // ring slots
    int slot_nm1;            // slot of Jhat_{n-1}
    int nrhs;
};

struct BlockMacArg {
    const double *Khat;        // [ell][Nz/2+1][Ny/2+1][Hp][6]
    const double2 *ring_base;  // [ring][nrhs][3][Nz][Ny][Hp]
    double2 *far;              // [TB][nrhs][3][Nz][Ny][Hp]
    int Hx, Hp, Ny, Nz;        // Hx = Nx/2 + 1 frequencies in rows of pitch Hp
    int nk;                    // ell (far: lags 1..nk)
    int ring;
    int nb;                    // first step of the block
    int ntarget;               // targets written by the far kernel (<= TB)
    int t;                     // near: position of the step in the block
    int nrhs;
    int jmin;                  // far: sources before step jmin count as zero (<= 1: none dropped)
    const double2 *init;       // far: partial sums the targets start from, laid out like far (NULL: zero)
    int jmax;                  // windowed far kernel: sources after step jmax count as zero (<= 0: none
                               // dropped); its lag loop then starts at nb - jmax
};

struct WaveArg {
    double k[3], pol[3], rref[3];
    double width, ct0, amp;
    // How the voxel average of a wave with two or more non-zero direction components is taken
    // (set by the host from the spreads |k_i| h_i / width): the axes by decreasing spread enter
    // as their products k_i h_i, each with the Gauss-Legendre order that bounds its error by 2^-53
    // of the amplitude, and form 0 takes the rule on all three, 1 erf on the widest and the rule
    // on the other two, 2 the two widest in closed form and the rule on the third.
    double kh[3];
    int nq[3];
    int form;
};

struct EpiArg {
    long M;
    int U, V, W;
    int nrhs;
    int n;                   // current step
    double h, hy, hz, c_dt;  // voxel edges (x, y, z) and c dt
    const double *chi, *schi, *inv_eps;
    const double *fir;       // device taps (nfir)
    int nfir;
    int nloc;                // local history depth used (>= nguess)
    int slot_of[kMaxLocal + 1];  // real-ring slot of J_{n-k}, k = 1..nloc
    int nguess;              // the solve starts from sum_{k=1}^{nguess} gx[k-1] J_{n-k} (<= nloc)
    double gx[kMaxLocal];    // extrapolation weights (the polynomial through nguess past steps)
    const double *Jring;     // [depth][nrhs][3][M]
    const double *S;         // [nrhs][3][M] convolution (normalised) or NULL at n = 1
    const WaveArg *waves;    // [nrhs]
    double glx8[8], glw8[8]; // 8-point rule on [-1/2, 1/2], weights summing to 1
    const double *gl;        // n-point rules on [-1/2, 1/2], n = 1..8: row n holds 8 nodes then 8 weights
    double *rhs, *y;         // [nrhs][3][M]
    double *uy;              // sqrt(chi) y0 in the zero-haloed layout [nrhs][3][(W+2)(V+2)(U+2)]
    // transposed march only
    const double *Lring;     // lambda history [depth][nrhs][3][M] (the local terms act on lambda)
    const double *G;         // adjoint source g_j [nrhs][3][M]
    double *bq;              // b'_j, kept for the voxels with chi = 0 [nrhs][3][M]
    const double *k0;        // the solver's K_0 stencil (the gradient term B_n)
    int oblique;             // some wave has two or more non-zero direction components
};

// Adjoint of the probe objective and the eps-gradient (see mj_march.hip).
struct AdjArg {
    long M;
    int U, V, W, nrhs;
    // adjoint source from the stored probe field
    const double *table;     // probe kernel table [nw][npairs][6]
    const int *pair_kmin;    // [npairs]
    const int *inv;          // [np][M] pair of (probe, voxel), -1 if none
    const double *table_v;   // the same table by voxel: [nw][np][M][6] (zeros where inv < 0)
    const int *kmin_v;       // [np][M] first lag of the pair's window, -1 if no pair
    const double *Ehist;     // [N][nrhs][np][3]
    int np, nw, N, j;        // j: forward step of this adjoint step
    long npairs;
    double *G;               // out [nrhs][3][M]
    // lambda from the solve
    const double *y, *schi, *c0, *bq, *nu;   // nu: [nrhs][3][M] of this step
    double *lam;             // out [nrhs][3][M]
    // gradient
    const double *Bj;        // B_j [nrhs][3][M]
    const double *inv_eps;
    double *grad;            // [M], accumulated
    const double *k0;        // the solver's K_0 stencil (the adjoint's local term)
};

struct CgScalars {
    double rz[2];            // r.z of the current and the previous iteration (alternating slots)
    double pq, rr, bb;
    int conv;                // iteration whose convergence test passed (INT_MAX: none yet)
};

// per right-hand side, read back by the host in one copy
struct CgStatus {
    int done;                // converged (set by the first iteration whose test passes)
    int iters;               // iterations taken
    double res;              // relative residual |r| / |b| at the last test
    double bb;               // |b|^2 of the solve's right-hand side (growth detector)
    double rr0;              // |r_0|^2 of the initial guess (Chebyshev solve)
};

struct CgArg {
    long M;
    int U, V, W;
    long Mp;                 // (U+2)(V+2)(W+2): vectors read by the stencil carry a zero halo
    int nrhs, nblk;          // nblk = ceil(M / 256): one voxel per thread
    double tol2;
    double d0, k0c;          // delta_0 and K_0^{xx}(0): c_0 and diag(A) follow from sqrt(chi)
    const double *schi;
    const double *rhs, *uy;  // uy, u: haloed layout [nrhs][3][Mp]
    double *y, *p, *q, *u;   // u = sqrt(chi) M^-1 r stands for the residual r
    double *part;            // [nrhs][3][nblk]
    CgScalars *scal;         // [nrhs]
    CgStatus *stat;          // [nrhs]
    // the solver's K_0(D) on its 27-point support [27][6] in device memory: entry
    // 13 + dx + 3 dy + 9 dz, components xx yy zz xy xz yz; read through the scalar cache
    const double *k0;
};

// Chebyshev iteration on the symmetrised Z_0 system with the Jacobi preconditioner M (see
// mj_march.hip): no inner products, one stencil pass per iteration.
struct ChebArg {
    CgArg cg;                // geometry, sqrt(chi), rhs, uy = s y0, y, partial sums, status, tol2
    double *r;               // residual [nrhs][3][M]
    const double *e_in;      // s d_k in the zero-haloed layout [nrhs][3][Mp]
    double *e_out;           // s d_{k+1}, same layout (the other of two buffers)
    double c1, c2;           // d_{k+1} = c1 d_k + c2 M^-1 r_{k+1}
    double inv_theta;        // d_0 = M^-1 r_0 / theta
    int want_norm;           // the pass writes partial sums of |r|^2 and the check follows it
    int passes;              // passes done when this one ends (recorded in the status)
    int rhs0, nr;            // the right-hand sides rhs0 .. rhs0 + nr - 1 only (nr = 0: all of them)
};
// r_0 = rhs - A y0, e_0 = s M^-1 r_0 / theta; reduces |r_0|^2 and |b|^2 into the status
void launch_cheb_init(const ChebArg &a, hipStream_t st);
// one iteration; with want_norm also the convergence check |r|^2 <= tol^2 |b|^2
void launch_cheb_pass(const ChebArg &a, hipStream_t st);
// pseudo-random right-hand side (zero where sqrt(chi) = 0) and zero initial guess
void launch_fill_trial(const double *schi, long M, int nrhs, double *rhs, double *y, hipStream_t st);

// Scattered field at probe points: E^s_p(n) = sum_{k=0}^{ell} sum_s K_k(r_p - r_s) J_{n-k}(s)
// over the source voxels s of the scatterer.  Pairs (p, s) are stored per probe sorted by the
// first lag kmin of their window, so the sources that lag k reaches through window slot
// k - kmin form one contiguous run: row (p, k) = pairs [row_start[p][max(0, k-nw+1)],
// row_start[p][k+1]).  The host cuts every row into chunks for the waves.
struct ProbeStepArg {
    const double *table;     // [nw][npairs][6]
    const int *pair_vox;     // [npairs]
    const int *pair_kmin;    // [npairs]
    const int *row_start;    // [np][ell + 2]
    int np, ell, nw, nrhs, n;
    // rows cut into chunks of at most kProbeChunk pairs, listed probe by probe: chunk c covers
    // pairs [ck_lo[c], ck_hi[c]) of row ck_row[c] = p (ell + 1) + k; probe p owns chunks
    // [ck_start[p], ck_start[p + 1])
    const int *ck_row, *ck_lo, *ck_hi, *ck_start;
    long nck;
    long M, npairs;
    const double *Jring;     // [rdepth][nrhs][3][M]
    int rdepth;
    double *part;            // [nrhs][nck][3]
    double *out;             // [nrhs][np][3]
};
constexpr int kProbeChunk = 1024;   // pairs of one row handled by one wave

void launch_mac(const MacArg &a, hipStream_t st);
void launch_mac_far(const BlockMacArg &a, int tb, hipStream_t st);
void launch_probes(const ProbeStepArg &a, hipStream_t st);
void launch_grad_term(const EpiArg &e, const double *Jn, const double *Jn1, double *Bout, hipStream_t st);
void launch_adj_source(const AdjArg &a, hipStream_t st);
// table_v[wl][p][m] = table[wl][inv[p][m]], kmin_v[p][m] = pair_kmin[inv[p][m]] (-1, zeros where none)
void launch_probe_table_by_voxel(const double *table, const int *pair_kmin, const int *inv, long npairs, int np,
                                 int nw, long M, double *table_v, int *kmin_v, hipStream_t st);
void launch_adj_epilogue(const EpiArg &e, hipStream_t st);
void launch_adj_lambda(const AdjArg &a, hipStream_t st);
void launch_grad_accum(const AdjArg &a, hipStream_t st);
void launch_mac_near(const BlockMacArg &a, hipStream_t st);
// far part with the rotation-free source window: tb = 4, 8, 10, 12, 14 or 16 targets
void launch_mac_win(const BlockMacArg &a, int tb, hipStream_t st, size_t lds_reserve = 0);
void launch_epilogue(const EpiArg &e, hipStream_t st);
void launch_history_local(const double *Jh, int depth, const double *S, const double *chi, const double *inv_eps,
                          const double *fir, int nfir, long M, double *P, hipStream_t st);
void launch_cg_init(const CgArg &a, hipStream_t st);
void launch_cg_a(const CgArg &a, int it, hipStream_t st);
void launch_cg_b(const CgArg &a, int it, hipStream_t st);
void launch_cg_end(const CgArg &a, int it, hipStream_t st);
void launch_cg_finish(const double *y, const double *schi, long M, int nrhs, double *J, double *Jout,
                      hipStream_t st);

}  // namespace mj
