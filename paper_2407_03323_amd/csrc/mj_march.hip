// Per-step kernels of the MOT-JVIE march (FP64): spectral multiply-accumulate over the
// history lags, right-hand-side assembly (excitation, FIR taps, local terms) and the
// conjugate-gradient solve with Z_0.
#include "mj_march.h"

#include <cmath>

namespace mj {

// ---------------------------------------------------------------------------- MAC
// S^(xi) = sum_{k=1}^{nk} Khat_k(xi) Jhat_{n-k}(xi)   (eq:PnFFTMOT in the spectral domain).
// Khat_k is real and has a definite parity in every frequency axis (K^aa even, K^ab odd in
// D_a and D_b), so only the octant ky <= Ny/2, kz <= Nz/2 is stored and one load serves the
// four mirror points (ky, Ny-ky) x (kz, Nz-kz) with sign flips on the odd components.
// One thread per octant point; G right-hand sides per thread share every Khat load.
template <int G>
__global__ void __launch_bounds__(256) k_mac(MacArg a)
{
    const int Hx = a.Hx, Nyo = a.Ny / 2 + 1, Nzo = a.Nz / 2 + 1;
    const long npt = (long)Hx * Nyo * Nzo;
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= npt) return;
    const int kx = (int)(t % Hx);
    const int qy = (int)((t / Hx) % Nyo);
    const int qz = (int)(t / ((long)Hx * Nyo));
    const int r0 = blockIdx.y * G;
    // mirror points
    int ys[2] = {qy, a.Ny - qy}, zs[2] = {qz, a.Nz - qz};
    const int ny_m = (qy == 0 || 2 * qy == a.Ny) ? 1 : 2;
    const int nz_m = (qz == 0 || 2 * qz == a.Nz) ? 1 : 2;
    const long plane = (long)a.Nz * a.Ny * Hx;   // one component of one spectrum
    long off[4];
    double sy_[4], sz_[4];
    int np = 0;
    for (int iz = 0; iz < nz_m; iz++)
        for (int iy = 0; iy < ny_m; iy++) {
            off[np] = ((long)zs[iz] * a.Ny + ys[iy]) * Hx + kx;
            sy_[np] = iy ? -1.0 : 1.0;
            sz_[np] = iz ? -1.0 : 1.0;
            np++;
        }
    double2 acc[G][4][3];
#pragma unroll
    for (int g = 0; g < G; g++)
#pragma unroll
        for (int p = 0; p < 4; p++)
#pragma unroll
            for (int c = 0; c < 3; c++) acc[g][p][c] = make_double2(0.0, 0.0);

    const long koct = (long)Hx * Nyo * Nzo;
    const double *Kp = a.Khat + t;
    for (int k = 1; k <= a.nk; k++) {
        const double *Kk = Kp + (long)(k - 1) * 6 * koct;
        const double kxx = Kk[0], kyy = Kk[koct], kzz = Kk[2 * koct];
        const double kxy = Kk[3 * koct], kxz = Kk[4 * koct], kyz = Kk[5 * koct];
        int slot = a.slot_nm1 - (k - 1);
        slot %= a.ring;
        if (slot < 0) slot += a.ring;
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int r = r0 + g;
            if (r >= a.nrhs) break;
            const double2 *J = a.ring_base + ((long)slot * a.nrhs + r) * 3 * plane;
#pragma unroll
            for (int p = 0; p < 4; p++) {
                if (p >= np) break;
                const double2 jx = J[off[p]], jy = J[plane + off[p]], jz = J[2 * plane + off[p]];
                const double sxy = kxy * sy_[p], sxz = kxz * sz_[p], syz = kyz * sy_[p] * sz_[p];
                acc[g][p][0].x += kxx * jx.x + sxy * jy.x + sxz * jz.x;
                acc[g][p][0].y += kxx * jx.y + sxy * jy.y + sxz * jz.y;
                acc[g][p][1].x += sxy * jx.x + kyy * jy.x + syz * jz.x;
                acc[g][p][1].y += sxy * jx.y + kyy * jy.y + syz * jz.y;
                acc[g][p][2].x += sxz * jx.x + syz * jy.x + kzz * jz.x;
                acc[g][p][2].y += sxz * jx.y + syz * jy.y + kzz * jz.y;
            }
        }
    }
#pragma unroll
    for (int g = 0; g < G; g++) {
        const int r = r0 + g;
        if (r >= a.nrhs) break;
        double2 *S = a.Shat + (long)r * 3 * plane;
#pragma unroll
        for (int p = 0; p < 4; p++) {
            if (p >= np) break;
            S[off[p]] = acc[g][p][0];
            S[plane + off[p]] = acc[g][p][1];
            S[2 * plane + off[p]] = acc[g][p][2];
        }
    }
}

void launch_mac(const MacArg &a, hipStream_t st)
{
    const long npt = (long)a.Hx * (a.Ny / 2 + 1) * (a.Nz / 2 + 1);
    dim3 blk(256);
    if (a.nrhs == 1) {
        dim3 grd((unsigned)((npt + 255) / 256), 1);
        hipLaunchKernelGGL(k_mac<1>, grd, blk, 0, st, a);
    } else {
        dim3 grd((unsigned)((npt + 255) / 256), (a.nrhs + 1) / 2);
        hipLaunchKernelGGL(k_mac<2>, grd, blk, 0, st, a);
    }
    MJ_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------- excitation
// chi_m times the voxel average of a Gaussian plane wave at c t = n c dt (eq:E), with an
// 8-point Gauss-Legendre rule along every axis on which the wave varies (the average over an
// axis the wave does not depend on is the identity).
__device__ inline double wave_average(const WaveArg &w, const EpiArg &e, int u, int v, int z, double ct)
{
    const double tc = ct - w.ct0 - ((u + 0.5) * e.h - w.rref[0]) * w.k[0] - ((v + 0.5) * e.h - w.rref[1]) * w.k[1] -
                      ((z + 0.5) * e.h - w.rref[2]) * w.k[2];
    const double iw = 1.0 / w.width;
    const int nx = w.k[0] != 0.0 ? 8 : 1, ny = w.k[1] != 0.0 ? 8 : 1, nz = w.k[2] != 0.0 ? 8 : 1;
    double sum = 0.0;
    for (int i = 0; i < nx; i++) {
        const double ox = nx > 1 ? e.glx8[i] * e.h * w.k[0] : 0.0, wx = nx > 1 ? e.glw8[i] : 1.0;
        for (int j = 0; j < ny; j++) {
            const double oy = ny > 1 ? e.glx8[j] * e.h * w.k[1] : 0.0, wy = ny > 1 ? e.glw8[j] : 1.0;
            double sl = 0.0;
            for (int l = 0; l < nz; l++) {
                const double oz = nz > 1 ? e.glx8[l] * e.h * w.k[2] : 0.0, wz = nz > 1 ? e.glw8[l] : 1.0;
                const double x = (tc - ox - oy - oz) * iw;
                sl += wz * exp(-x * x);
            }
            sum += wx * wy * sl;
        }
    }
    return w.amp * sum;
}

// b = E_n - P_{n-1} with P_{n-1} = sum_k c_k J_{n-k} - chi (K (*) J)  (eq:MOTInversion, eq:PnMOT);
// c_1 = T(dt)/eps + delta_1, c_k = delta_k (k >= 2).  Writes the right-hand side of the
// symmetrised system (b / sqrt(chi)) and the extrapolated initial guess
// y0 = 3 y_{n-1} - 3 y_{n-2} + y_{n-3}, y = J / sqrt(chi).
__global__ void __launch_bounds__(256) k_epilogue(EpiArg e)
{
    const long M = e.M;
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= M) return;
    const double chi = e.chi[i], sc = e.schi[i];
    const int u = (int)(i % e.U), v = (int)((i / e.U) % e.V), z = (int)(i / ((long)e.U * e.V));
    double avg = 0.0;
    const WaveArg w = e.waves[r];
    if (chi != 0.0) avg = wave_average(w, e, u, v, z, e.n * e.c_dt);
    const double c1 = 0.5 * e.inv_eps[i] + (e.nfir > 1 ? e.fir[1] : 0.0);
    for (int c = 0; c < 3; c++) {
        double b = chi * (avg * w.pol[c] + (e.S ? e.S[((long)r * 3 + c) * M + i] : 0.0));
        for (int k = 1; k <= e.nloc; k++) {
            if (e.n - k < 1) break;
            const double ck = (k == 1) ? c1 : (k < e.nfir ? e.fir[k] : 0.0);
            if (ck == 0.0) continue;
            const double *Jk = e.Jring + (((long)e.slot_of[k] * e.nrhs + r) * 3 + c) * M;
            b -= ck * Jk[i];
        }
        double rhs = sc > 0.0 ? b / sc : 0.0;
        double y0 = 0.0;
        if (sc > 0.0) {
            const double inv = 1.0 / sc;
            double y1 = 0, y2 = 0, y3 = 0;
            if (e.n - 1 >= 1) y1 = e.Jring[(((long)e.slot_of[1] * e.nrhs + r) * 3 + c) * M + i] * inv;
            if (e.n - 2 >= 1) y2 = e.Jring[(((long)e.slot_of[2] * e.nrhs + r) * 3 + c) * M + i] * inv;
            if (e.n - 3 >= 1) y3 = e.Jring[(((long)e.slot_of[3] * e.nrhs + r) * 3 + c) * M + i] * inv;
            y0 = 3.0 * y1 - 3.0 * y2 + y3;
        }
        const long o = ((long)r * 3 + c) * M + i;
        e.rhs[o] = rhs;
        e.y[o] = y0;
    }
}

void launch_epilogue(const EpiArg &e, hipStream_t st)
{
    dim3 grd((unsigned)((e.M + 255) / 256), e.nrhs);
    hipLaunchKernelGGL(k_epilogue, grd, dim3(256), 0, st, e);
    MJ_CHECK(hipGetLastError());
}

// P = sum_{k=1}^{depth} c_k J_{n-k} - chi S   for an explicit history (right-hand side 0).
__global__ void k_history_local(const double *__restrict__ Jh, int depth, const double *__restrict__ S,
                                const double *__restrict__ chi, const double *__restrict__ inv_eps,
                                const double *__restrict__ fir, int nfir, long M, double *__restrict__ P)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= M) return;
    for (int c = 0; c < 3; c++) {
        double p = -chi[i] * S[c * M + i];
        for (int k = 1; k <= depth; k++) {
            double ck = (k < nfir ? fir[k] : 0.0) + (k == 1 ? 0.5 * inv_eps[i] : 0.0);
            if (ck != 0.0) p += ck * Jh[((long)(k - 1) * 3 + c) * M + i];
        }
        P[c * M + i] = p;
    }
}

void launch_history_local(const double *Jh, int depth, const double *S, const double *chi, const double *inv_eps,
                          const double *fir, int nfir, long M, double *P, hipStream_t st)
{
    hipLaunchKernelGGL(k_history_local, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, Jh, depth, S, chi,
                       inv_eps, fir, nfir, M, P);
    MJ_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------- CG
// Symmetrised Z_0:  J = D y with D = diag(sqrt(chi)),  A = C_0 - D K_0 D,
// (A y)_b(m) = c_0(m) y_b(m) - s(m) sum_{D in 27} sum_a K_0^{ba}(D) s(m-D) y_a(m-D).
// A is symmetric positive definite; Jacobi preconditioning with diag(A).
__constant__ double c_K0[27 * 6];

void upload_stencil(const double *K0_27x6)
{
    MJ_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_K0), K0_27x6, sizeof(double) * 27 * 6));
}

__device__ inline void stencil_apply(const CgArg &a, const double *__restrict__ x, long i, int u, int v, int z,
                                     double out[3])
{
    const long M = a.M;
    const double s = a.schi[i];
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    if (s != 0.0) {
        int o = 0;
        for (int dz = -1; dz <= 1; dz++) {
            const int zz = z - dz;
            for (int dy = -1; dy <= 1; dy++) {
                const int yy = v - dy;
                for (int dx = -1; dx <= 1; dx++, o++) {
                    const int xx = u - dx;
                    if (xx < 0 || xx >= a.U || yy < 0 || yy >= a.V || zz < 0 || zz >= a.W) continue;
                    const long j = ((long)zz * a.V + yy) * a.U + xx;
                    const double sj = a.schi[j];
                    if (sj == 0.0) continue;
                    const double *k = &c_K0[o * 6];
                    const double x0 = sj * x[j], x1 = sj * x[M + j], x2 = sj * x[2 * M + j];
                    acc0 += k[0] * x0 + k[3] * x1 + k[4] * x2;
                    acc1 += k[3] * x0 + k[1] * x1 + k[5] * x2;
                    acc2 += k[4] * x0 + k[5] * x1 + k[2] * x2;
                }
            }
        }
    }
    const double c0 = a.c0[i];
    out[0] = c0 * x[i] - s * acc0;
    out[1] = c0 * x[M + i] - s * acc1;
    out[2] = c0 * x[2 * M + i] - s * acc2;
}

__device__ inline double block_sum(double v, double *sm)
{
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sm[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) t += sm[w];
    return t;   // valid in thread 0
}

// every block reduces the nblk partials of one right-hand side in a fixed order
__device__ inline double reduce_partials(const double *__restrict__ part, int nblk, double *sm)
{
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) v += part[b];
    v = block_sum(v, sm);
    if (threadIdx.x == 0) sm[32] = v;
    __syncthreads();
    double out = sm[32];
    __syncthreads();
    return out;
}

// r = rhs - A y0, z = M^-1 r, p = q = 0; partials of r.z, r.r, rhs.rhs
__global__ void __launch_bounds__(256) k_cg_init(CgArg a)
{
    __shared__ double sm[40];
    const int r = blockIdx.y;
    const long M = a.M, base = (long)r * 3 * M;
    double rz = 0, rr = 0, bb = 0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < M; i += (long)gridDim.x * blockDim.x) {
        const int u = (int)(i % a.U), v = (int)((i / a.U) % a.V), z = (int)(i / ((long)a.U * a.V));
        double Ay[3];
        stencil_apply(a, a.y + base, i, u, v, z, Ay);
        const double md = a.inv_diag[i];
        for (int c = 0; c < 3; c++) {
            const long o = base + c * M + i;
            const double b = a.rhs[o];
            const double rv = a.schi[i] != 0.0 ? b - Ay[c] : 0.0;
            const double zv = md * rv;
            a.r[o] = rv;
            a.z[o] = zv;
            a.p[o] = 0.0;
            a.q[o] = 0.0;
            rz += rv * zv;
            rr += rv * rv;
            bb += b * b;
        }
    }
    const int nb = gridDim.x;
    double t = block_sum(rz, sm);
    if (threadIdx.x == 0) a.part_rz[0][r * nb + blockIdx.x] = t;
    t = block_sum(rr, sm);
    if (threadIdx.x == 0) a.part_rr[r * nb + blockIdx.x] = t;
    t = block_sum(bb, sm);
    if (threadIdx.x == 0) a.part_bb[r * nb + blockIdx.x] = t;
}

// iteration it (first half): beta = rz_it / rz_{it-1} (0 at it = 0); convergence test on
// r.r; w = A z;  p = z + beta p;  q = w + beta q;  partials of p.q
__global__ void __launch_bounds__(256) k_cg_a(CgArg a, int it)
{
    __shared__ double sm[40];
    __shared__ int skip;
    const int r = blockIdx.y;
    const int nb = gridDim.x;
    // one read of the flag per block, so the whole block takes the same branch
    if (threadIdx.x == 0) skip = a.done[r];
    __syncthreads();
    if (skip) return;
    const double rz = reduce_partials(a.part_rz[it & 1] + r * nb, nb, sm);
    const double rr = reduce_partials(a.part_rr + r * nb, nb, sm);
    const double bb = reduce_partials(a.part_bb + r * nb, nb, sm);
    const bool conv = rr <= a.tol2 * bb || bb == 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.res[r] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
        a.iters[r] = it;
    }
    if (conv) {
        // every block takes the same decision; block 0 records it for the host and later kernels
        if (blockIdx.x == 0 && threadIdx.x == 0) a.done[r] = 1;
        return;
    }
    double beta = 0.0;
    if (it > 0) {
        const double rz_old = reduce_partials(a.part_rz[(it + 1) & 1] + r * nb, nb, sm);
        beta = rz / rz_old;
    }
    const long M = a.M, base = (long)r * 3 * M;
    double pq = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < M; i += (long)gridDim.x * blockDim.x) {
        if (a.schi[i] == 0.0) continue;
        const int u = (int)(i % a.U), v = (int)((i / a.U) % a.V), z = (int)(i / ((long)a.U * a.V));
        double Az[3];
        stencil_apply(a, a.z + base, i, u, v, z, Az);
        for (int c = 0; c < 3; c++) {
            const long o = base + c * M + i;
            const double pv = a.z[o] + beta * a.p[o];
            const double qv = Az[c] + beta * a.q[o];
            a.p[o] = pv;
            a.q[o] = qv;
            pq += pv * qv;
        }
    }
    const double t = block_sum(pq, sm);
    if (threadIdx.x == 0) a.part_pq[r * nb + blockIdx.x] = t;
}

// second half: alpha = rz_it / p.q;  y += alpha p;  r -= alpha q;  z = M^-1 r;
// partials of r.z (into the other buffer) and r.r
__global__ void __launch_bounds__(256) k_cg_b(CgArg a, int it)
{
    __shared__ double sm[40];
    __shared__ int skip;
    const int r = blockIdx.y;
    const int nb = gridDim.x;
    if (threadIdx.x == 0) skip = a.done[r];
    __syncthreads();
    if (skip) return;
    const double rz = reduce_partials(a.part_rz[it & 1] + r * nb, nb, sm);
    const double pq = reduce_partials(a.part_pq + r * nb, nb, sm);
    const double alpha = rz / pq;
    const long M = a.M, base = (long)r * 3 * M;
    double rz2 = 0.0, rr = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < M; i += (long)gridDim.x * blockDim.x) {
        if (a.schi[i] == 0.0) continue;
        const double md = a.inv_diag[i];
        for (int c = 0; c < 3; c++) {
            const long o = base + c * M + i;
            a.y[o] += alpha * a.p[o];
            const double rv = a.r[o] - alpha * a.q[o];
            const double zv = md * rv;
            a.r[o] = rv;
            a.z[o] = zv;
            rz2 += rv * zv;
            rr += rv * rv;
        }
    }
    double t = block_sum(rz2, sm);
    if (threadIdx.x == 0) a.part_rz[(it + 1) & 1][r * nb + blockIdx.x] = t;
    t = block_sum(rr, sm);
    if (threadIdx.x == 0) a.part_rr[r * nb + blockIdx.x] = t;
}

// J_n = sqrt(chi) y into the real-space ring (and optionally the caller's output)
__global__ void k_cg_finish(const double *__restrict__ y, const double *__restrict__ schi, long M, int nrhs,
                            double *__restrict__ J, double *__restrict__ Jout)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= M) return;
    const double s = schi[i];
    for (int r = 0; r < nrhs; r++)
        for (int c = 0; c < 3; c++) {
            const long o = ((long)r * 3 + c) * M + i;
            const double v = s * y[o];
            J[o] = v;
            if (Jout) Jout[o] = v;
        }
}

void launch_cg_init(const CgArg &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_init, dim3(a.nblk, a.nrhs), dim3(256), 0, st, a);
    MJ_CHECK(hipGetLastError());
}
void launch_cg_a(const CgArg &a, int it, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_a, dim3(a.nblk, a.nrhs), dim3(256), 0, st, a, it);
    MJ_CHECK(hipGetLastError());
}
void launch_cg_b(const CgArg &a, int it, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_b, dim3(a.nblk, a.nrhs), dim3(256), 0, st, a, it);
    MJ_CHECK(hipGetLastError());
}
void launch_cg_finish(const double *y, const double *schi, long M, int nrhs, double *J, double *Jout,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_finish, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, y, schi, M, nrhs, J, Jout);
    MJ_CHECK(hipGetLastError());
}

}  // namespace mj
