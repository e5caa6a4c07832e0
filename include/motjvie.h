/*
 * motjvie.h -- C interface of the MI355X (gfx950) MOT-JVIE library.
 *
 * The library marches the FFT-accelerated, FIR-regularised marching-on-in-time
 * contrast-current-density volume integral equation (MOT-JVIE) of
 * van Diepen, van Beurden & Dilz, "FFT-acceleration and stabilization of the 3D
 * Marching-on-in-Time Contrast Current Density Volume Integral Equation for
 * scattering from high contrast dielectrics" (arXiv 2407.03323).
 *
 * Problem statement (Sec. 2.1): a dielectric with relative permittivity eps_r >= 1,
 * voxelised on a U x V x W box (Sec. 2.2), is illuminated by an incident field that
 * arrives after t = 0.  Unknowns are the coefficients J^a_{m,n} of the contrast
 * current (eq:J_basis) at steps t_n = n dt.  Every step solves
 *     Z_0 J_n = E_n - P_{n-1},   P_{n-1} = sum_{k=1}^{ell} Z_k J_{n-k}
 * (eq:MOTInversion, eq:PnMOT), with the history sum evaluated by zero-padded 3-D
 * FFT convolution (Sec. 3, Appendix A) and the FIR regularisation
 * Z_k -> Z_k + delta_k I (Sec. 6.1) built in.
 *
 * Conventions
 *  - Lengths in any unit; voxels are h x hy x hz (Sec. 2.2: dx, dy, dz; hy = hz = h by
 *    default).  Times enter as c*t (same unit).  c*dt may be any value in
 *    [0.3 max(h, hy, hz), min(h, hy, hz)]: the paper's choice dt = dx/c on cubic voxels
 *    (Sec. 5.2) is the largest; up to it K_0 stays on the 27 nearest offsets, which the Z_0
 *    solve assumes.  Smaller steps add lags (eq:Ell) and kernel work in proportion to h/(c dt).
 *  - Voxel index m = (w*V + v)*U + u, 0-based, x fastest (Sec. 2.2, 1-based there).
 *    Voxel (u,v,w) has its centre at ((u+1/2)h, (v+1/2)hy, (w+1/2)hz).
 *  - Vector fields are stored per component: F[a][w][v][u], a = x,y,z (the paper's
 *    eq:CurrentVector interleaves the components per voxel; same numbers).
 *  - All arithmetic is IEEE binary64.
 *  - Pointers documented "device" must point to device memory of the current HIP
 *    device (e.g. torch CUDA tensors); "host" pointers are read during the call and
 *    may be freed afterwards.  The library never takes ownership of caller memory.
 *  - Every call returns MJ_OK (0) or a negative status and never throws.  On error
 *    mj_last_error() returns a description (per handle; mj_create failures use the
 *    thread's own message, readable with mj_last_error(NULL)).
 *  - One handle must not be used by two host threads at once.  All work is enqueued
 *    on the configured stream; calls returning results to host memory synchronise it.
 */
#ifndef MOTJVIE_H
#define MOTJVIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MJ_OK = 0,
    MJ_EINVAL = -1,      /* invalid argument */
    MJ_ENOMEM = -2,      /* device allocation failed */
    MJ_EHIP = -3,        /* HIP runtime error */
    MJ_ENOCONV = -4,     /* Z_0 solve did not reach cg_rtol within cg_maxit */
    MJ_EUNSTABLE = -5,   /* the march grows without bound (right-hand side norm > 1e100 or not finite) */
    MJ_ESTATE = -6       /* call not valid in the current state */
};

typedef struct mj_solver mj_solver;

typedef struct {
    int32_t U, V, W;          /* voxels per axis (>= 1) */
    double h;                 /* voxel edge along x (> 0) */
    double c_dt;              /* c * dt, in [0.3 max edge, min edge]; MJ_EINVAL outside */
    const double *eps_r;      /* host [W][V][U], relative permittivity >= 1, finite */
    const double *fir;        /* host taps delta_0..delta_{n_fir-1} (Sec. 6.1); may be NULL if n_fir == 0 */
    int32_t n_fir;            /* 0 = no regularisation */
    int32_t n_rhs;            /* number of right-hand sides (plane waves) marched together, >= 1 */
    double cg_rtol;           /* relative residual of the Z_0 solve; <= 0 selects 1e-13 */
    int32_t cg_maxit;         /* <= 0 selects 200 */
    int32_t time_block;       /* steps per time block of the history MAC (Sec. 4.1): 1 (none), 4, 8, 10, 12,
                                 14, 16 or 32.  0 (with outer_block 0): the default, blocks of 4 inside
                                 outer blocks of 16 when ell >= 64, else blocks of 8.  < 0: chosen at
                                 mj_create by timing one period of the MAC for each of (8), (12), (16),
                                 (4 in 8), (4 in 12), (4 in 16), (8 in 16); the choices group the terms
                                 of eq:PnMOT differently, so results then vary with it at rounding level */
    void *stream;             /* hipStream_t to enqueue on; NULL = the null stream */
    int32_t quad_order;       /* Gauss-Legendre points per cell of the kernel quadrature; 0 selects 16 */
    int32_t fft_pencils;      /* pencils per block of the FFT passes: 0 = pick per pass by timing at
                                 mj_create; > 0 = at most this many (capped by what one LDS tile holds).
                                 The transforms are bit-identical for every choice. < 0: MJ_EINVAL */
    double hy, hz;            /* voxel edges along y and z; 0 selects h.  Zero-initialise a config
                                 written for cubic voxels and these keep it cubic */
    /* Optional device allocator for every buffer the solver holds or uses for a while (e.g.
       PyTorch's caching allocator, so that one pool serves the caller and the library):
       alloc(bytes, alloc_ctx) returns device memory of the current device, aligned to at
       least 256 bytes, or NULL (the call then fails with MJ_ENOMEM); free_(ptr, alloc_ctx)
       releases it.  Both or neither (else MJ_EINVAL); NULL selects hipMalloc / hipFree.  The
       buffers are used on `stream` only, and mj_destroy releases all of them. */
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free_)(void *ptr, void *ctx);
    void *alloc_ctx;
    int32_t outer_block;      /* a third level of the time division (Sec. 4.1 applied twice): steps per
                                 outer block, a multiple of time_block (which must then be 4 or 8), even,
                                 in 8 .. 16.  0 or 1: two levels (or the default, see time_block) */
    int32_t z0_solver;        /* the Z_0 solve (eq:MOTInversion) on the symmetrised Z_0 with the Jacobi
                                 preconditioner: 1 CG; 2 Chebyshev iteration on its spectrum, estimated at
                                 mj_create and mj_set_eps (one stencil pass per iteration and no inner
                                 products: fewer launches, more iterations); 0 Chebyshev up to 2^19 voxels
                                 (whatever the number of right-hand sides, which share every launch), CG
                                 above.  Both stop at cg_rtol; cg_maxit bounds their iterations */
    int32_t z0_graphs;        /* != 0: the Chebyshev passes of a solve (whose arguments depend only on the
                                 pass index) are captured once per batch shape as HIP graphs and replayed
                                 on `stream` in later steps; 0: launched one by one */
    int32_t outer_overlap;    /* three levels only: 2 forms the outer sums of each outer block over the
                                 sources before the previous block on a second stream of the library's
                                 own (non-blocking, default priority), while the previous block marches,
                                 and adds the previous block's sources at the block start on `stream`;
                                 1 forms them in one launch on `stream` at the block start; 0 the
                                 default (1).  The two group the terms of eq:PnMOT differently (results
                                 differ at rounding level); 2 holds B2 more partial sums on the device.
                                 Every entry point orders its own work after the second stream's */
} mj_config;

/*
 * mj_create -- build a solver.
 *   Computes ell (eq:Ell), generates the space-time interaction kernels K_k(D),
 *   k = 0..ell, on the device (eq:Z, Sec. 2.3), transforms them to spectra on the
 *   zero-padded grid (circulant embedding, Appendix A) and allocates the march state.  The march starts at n = 0 with J_{n'} = 0, n' <= 0.
 *   Returns MJ_EINVAL for invalid sizes/values, MJ_ENOMEM if the device memory
 *   needed (mj_info entry 8 reports what was allocated) does not fit.
 */
int mj_create(const mj_config *cfg, mj_solver **out);

/* mj_destroy -- release all device memory of the solver (NULL is ignored). */
void mj_destroy(mj_solver *s);

/* mj_last_error -- description of the last error on this handle (or thread if NULL). */
const char *mj_last_error(const mj_solver *s);

/*
 * mj_info -- sizes of the solver.  out (host, n entries used, n <= 24):
 *   [0] ell  [1] Nx [2] Ny [3] Nz (padded FFT sizes)  [4] time block B
 *   [5] history depth kept in real space  [6] n_rhs  [7] current step n
 *   [8] device bytes allocated  [9] kernel generation time (ms)  [10] spectra time (ms)
 *   [11] number of FIR taps  [12] probes  [13] lag window per probe pair
 *   [14] probe pairs  [15] probe kernel generation time (ms)
 *   [16] [17] [18] pencils per block of the x, y and z FFT passes  [19] outer time block (0: none)
 *   [20] Z_0 solver in use (0 Chebyshev, 1 CG)  [21] [22] the bounds of the eigenvalues of the
 *   Jacobi-preconditioned symmetrised Z_0 that the Chebyshev solve uses (0: not estimated)
 *   [23] 1 if the outer level runs on the second stream (outer_overlap)
 */
int mj_info(const mj_solver *s, double *out, int32_t n);

/*
 * mj_set_plane_waves -- incident Gaussian plane waves, one per right-hand side (host arrays):
 *   E^i(r,t) = amp * pol * exp(-((c t - c t0 - (r - r_ref).khat) / width)^2)
 *   khat[n_rhs][3] (unit), pol[n_rhs][3], width[n_rhs] (> 0), ct0[n_rhs], amp[n_rhs],
 *   r_ref[n_rhs][3].  The paper's pulse (eq:GaussPlaneWave) is amp = 4 E0/(sigma sqrt(pi)),
 *   width = sigma/4.  The excitation E_n (eq:E) is chi_m times the voxel average of
 *   E^i at t_n, taken with an 8-point Gauss-Legendre rule per axis.  Every value must be
 *   finite (else MJ_EINVAL and the previous waves stay).
 */
int mj_set_plane_waves(mj_solver *s, const double *khat, const double *pol, const double *width,
                       const double *ct0, const double *amp, const double *r_ref);

/*
 * mj_run -- march n_steps steps (eq:MOTInversion for n = n_cur+1 .. n_cur+n_steps).
 *   J_hist: device, nullable, [n_steps][n_rhs][3][W][V][U]; receives J_n of every step.
 *   Returns MJ_ENOCONV if a Z_0 solve missed cg_rtol (the march state stays consistent:
 *   J_n holds the last iterate).  Returns MJ_EUNSTABLE, and stops after that step, once the
 *   right-hand side of a Z_0 solve exceeds 1e100 in norm or is not finite: the unbounded
 *   growth seen in Sec. 5.2 and analysed in Sec. 6 (the alternating mode at f = 1/(2 dt)); mj_info entry 7 gives the step.
 */
int mj_run(mj_solver *s, int32_t n_steps, double *J_hist);

/*
 * mj_set_probes -- points where the scattered field is sampled during the march.
 *   pos: host [n_probes][3], same length unit as h, origin at the grid corner (voxel
 *   (u, v, w) is centred at ((u + 1/2) h, (v + 1/2) hy, (w + 1/2) hz)); copied.  0 <= n_probes
 *   <= 65536; n_probes = 0 removes the probes.  Allowed only at n = 0 (after mj_create or
 *   mj_reset), else MJ_ESTATE.
 *   The field is the scattered-field operator of the formulation (Sec. 2.1) tested, like
 *   eq:Z, on a virtual voxel of the grid's shape centred at the probe (eps_0 = 1):
 *     E^s_p(n) = sum_{k=0}^{ell} sum_{m'} K_k(r_p - r_m') J_{n-k}(m')
 *   over the voxels m' with eps_r != 1.  (K is S(J) less its local part J, and the
 *   scattered field is S(J) - J, so no local term appears, inside the scatterer or not.)
 *   The kernel values of every (probe, voxel) pair's lag window are generated on the
 *   device here, once; the march adds one pass over them per step.  Accuracy: the probe's
 *   voxel should not overlap a scatterer voxel off-centre (within one h on every axis),
 *   where the quadrature reaches only ~1e-9.
 */
int mj_set_probes(mj_solver *s, int32_t n_probes, const double *pos);

/*
 * mj_march -- mj_run with the probe output: probe_hist (device, nullable)
 *   [n_steps][n_rhs][n_probes][3] receives E^s_p(n) of every step.
 */
int mj_march(mj_solver *s, int32_t n_steps, double *J_hist, double *probe_hist);

/*
 * mj_step -- one step of eq:MOTInversion (n -> n + 1), the unit a caller's own time loop is
 *   built from.  J_dev: device, nullable, [n_rhs][3][W][V][U] receives J_{n+1}.  probe: device,
 *   nullable, [n_rhs][n_probes][3] receives E^s_p(n + 1) (probes set by mj_set_probes).  Errors as
 *   mj_run; the history sum of the step is the same as inside mj_run (a march of mj_step calls
 *   repeats mj_run bit for bit).
 */
int mj_step(mj_solver *s, double *J_dev, double *probe);

/*
 * mj_march_every -- mj_march with the current history thinned: J_hist (device, nullable)
 *   [n_steps / j_every][n_rhs][3][W][V][U] receives J_n of every j_every-th step of the call
 *   (the j_every-th, 2 j_every-th, ... step; j_every >= 1, else MJ_EINVAL).  probe_hist
 *   (device, nullable) [n_steps][n_rhs][n_probes][3] still receives every step.  For long
 *   marches at full size (2000 steps of 27 MB each at 104^3) the caller keeps a sample only.
 */
int mj_march_every(mj_solver *s, int32_t n_steps, int32_t j_every, double *J_hist, double *probe_hist);

/*
 * mj_probe_kernel_values -- K_k(r_p - r_m') as the probe path generates it, for n host
 *   requests: probe[n] (index into the probes set by mj_set_probes), voxel[n][3] (u, v, w)
 *   and lag[n] (>= 0).  out (host) [n][6]: xx, yy, zz, xy, xz, yz.
 */
int mj_probe_kernel_values(mj_solver *s, int32_t n, const int32_t *probe, const int32_t *voxel,
                           const int32_t *lag, double *out);

/*
 * mj_set_eps -- new relative permittivities (host [W][V][U], >= 1, copied) for the same
 *   grid: chi, the local coefficients c_k, Z_0 and its preconditioner are rebuilt; the
 *   interaction kernels do not depend on eps and are kept.  Only at n = 0, else MJ_ESTATE.
 *   Clears the solver's working vectors like mj_reset.
 */
int mj_set_eps(mj_solver *s, const double *eps_r);

/*
 * mj_adjoint_gradient -- objective Phi = sum_{n=1}^{n_steps} sum_rhs sum_p |E^s_p(n)|^2 over
 *   the probes set by mj_set_probes, and its gradient with respect to eps_r of every voxel,
 *   by the transposed (adjoint) march: with the march written as the block lower-triangular
 *   Toeplitz system sum_k Z_k J_{n-k} = E_n (eq:MatrixEquation), lambda solves
 *     Z_0^T lambda_j = dPhi/dJ_j - sum_{k>=1} Z_k^T lambda_{j+k},
 *     Z_k^T = diag(c_k) - K_k (*) (chi .)   (every K_k is symmetric: reciprocity of eq:Z),
 *   marched backward through the same FFT history sum, and
 *     dPhi/deps_m = sum_n lambda_n(m) . B_n(m) / eps_m^2,
 *     B_n = <E^i>(n) + sum_{k=0}^{ell} (T(k dt) J_{n-k} + K_k (*) J_{n-k}).
 *   Checkpointing: the forward march is run once, keeping the real-space history needed to
 *   restart it every ckpt_every steps (rounded up to a multiple of the time block; <= 0:
 *   one segment, nothing recomputed); the backward pass recomputes each segment from its
 *   checkpoint before marching back through it.  Memory: every current a restart reads
 *   (the ell + 1 steps before each segment start) is kept once, so at most
 *   min(n_steps, (segments - 1)(ell + 1)) currents of 3 M n_rhs values (mj_stats entry 17
 *   gives the bytes), plus one segment of gradient terms and a second set of rings for the
 *   adjoint march.
 *   phi: host, nullable.  dphi_deps: device [W][V][U] (overwritten).  probe_hist: device,
 *   nullable, [n_steps][n_rhs][n_probes][3] receives the forward probe field.  Starts at
 *   n = 0 (else MJ_ESTATE) and leaves the march at n = 0.
 */
int mj_adjoint_gradient(mj_solver *s, int32_t n_steps, int32_t ckpt_every, double *phi, double *dphi_deps,
                        double *probe_hist);

/*
 * mj_reset -- restart the march at n = 0 (all past currents zero).  Also clears the Z_0
 *   solver's working vectors, so a handle whose march ended in MJ_EUNSTABLE on non-finite
 *   values marches again from a clean state.
 */
int mj_reset(mj_solver *s);

/*
 * mj_get_state, mj_set_state -- checkpoint and resume a march.  The state is everything that a
 * later step of eq:MOTInversion reads from earlier steps:
 *   - the step count n;
 *   - the spectral history ring (the FFT of J_{n-k}, k = 1..ell, Sec. 3);
 *   - the current time block's far-part sums (Sec. 4.1);
 *   - the real-space currents that the FIR stencil, the Z_0 initial guess and the probes read.
 * The adjoint (mj_adjoint_gradient) keeps its own checkpoints and is not part of it.
 *   mj_get_state: buf host, nullable.  With buf NULL, *bytes receives the size needed.
 *   Otherwise *bytes must be at least that size (else MJ_EINVAL), and it receives the size
 *   written.  The size grows as ell x n_rhs x 48 B x the padded half-spectrum points: about
 *   40 GB at 104^3.
 *   mj_set_state: buf host.  The state must come from a solver with the same grid, n_rhs,
 *   ell, time block and real-space depth (so the same probes, if any, set before this call),
 *   else MJ_EINVAL.  The material, taps and plane waves are the caller's to match.  A march
 *   resumed this way repeats the original steps bit for bit.
 */
int mj_get_state(const mj_solver *s, void *buf, size_t *bytes);
int mj_set_state(mj_solver *s, const void *buf, size_t bytes);

/*
 * mj_history_sum -- P_{n-1} = sum_{k>=1} Z^delta_k J_{n-k} (eq:PnMOT with the FIR taps)
 *   for an explicit history, through the same FFT / spectral multiply-accumulate / inverse
 *   FFT path that the march uses (right-hand side 0).
 *   J_hist: device [depth][3][W][V][U] with J_hist[k-1] = J_{n-k}, 1 <= depth; lags beyond
 *   depth count as zero.  P: device [3][W][V][U].  Overwrites the march state (call
 *   mj_reset before marching again).
 */
int mj_history_sum(mj_solver *s, const double *J_hist, int32_t depth, double *P);

/*
 * mj_kernel_values -- interaction kernels K_k(D) as generated on the device (eq:Z without
 *   the identity and chi factors), for n requests (host arrays): lag[n] (0..ell) and
 *   offset[n][3] (integer voxel offsets, |D_i| < U_i).  out (host) [n][6] receives
 *   K^{xx}, K^{yy}, K^{zz}, K^{xy}, K^{xz}, K^{yz}.
 */
int mj_kernel_values(mj_solver *s, int32_t n, const int32_t *lag, const int32_t *offset, double *out);

/*
 * mj_kernel_values_noalloc -- mj_kernel_values for callers that cannot allocate device memory
 *   (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 *   same arguments and results, with the requests and results staged through a fixed device
 *   array built into the library (4 MiB, one per GPU, held until the process ends) instead
 *   of buffers allocated per call.  At most 65536 requests per call (else MJ_EINVAL); the
 *   solver's device must be current (else MJ_EINVAL).  The call allocates nothing.  All calls
 *   on one GPU share the array: calls from one process take turns (each synchronises its
 *   stream before it returns); calls that overlap on one GPU from outside that order race.
 */
int mj_kernel_values_noalloc(mj_solver *s, int32_t n, const int32_t *lag, const int32_t *offset, double *out);

/*
 * mj_stats -- per-phase device times of the last mj_run (HIP events on the solver's stream),
 *   in ms per step, and CG statistics.  out (host, n <= 21): [0] forward FFT  [1] history
 *   MAC  [2] inverse FFT  [3] epilogue (excitation, FIR, RHS)  [4] Z_0 solve  [5] total
 *   [6] mean CG iterations  [7] max final relative residual  [8] steps timed
 *   [9] max CG iterations  [10] mean duration of one far-part MAC launch (time-blocked,
 *   once per block)  [11] far-part launches  [12] mean duration of one near-part launch
 *   [13] probes.  [5] includes [13].  After mj_adjoint_gradient: [14] forward pass (ms,
 *   whole run)  [15] backward pass with recomputation (ms)  [16] segments  [17] checkpoint bytes.
 *   [18] mean duration of one middle-level MAC launch (three time levels).  With three levels,
 *   [10] and [11] describe the outer launches (overlapped: those on `stream`, which add the
 *   previous block's sources).  [19] mean duration of one launch on the second stream
 *   (outer_overlap = 2, events on that stream; it shares the device with the march)
 *   [20] such launches timed, those that had finished when the run returned.
 */
int mj_stats(const mj_solver *s, double *out, int32_t n);

/*
 * mj_fft_roundtrip -- diagnostic: forward 3-D FFT of x (device [3][W][V][U]) on the
 *   padded grid into X (device, [3][Nz][Ny][Nx/2+1] complex interleaved re,im), and the
 *   inverse of X restricted to the voxel box, unnormalised, into y (device [3][W][V][U]).
 *   Either output may be NULL.
 */
int mj_fft_roundtrip(mj_solver *s, const double *x, double *X, double *y);

#ifdef __cplusplus
}
#endif
#endif /* MOTJVIE_H */
