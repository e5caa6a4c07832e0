// Per-step kernels of the MOT-JVIE march (FP64): spectral multiply-accumulate over the
// history lags, right-hand-side assembly (excitation, FIR taps, local terms) and the
// conjugate-gradient solve with Z_0.
#include "mj_march.h"

#include <climits>
#include <cmath>
#include <utility>

namespace mj {

// ---------------------------------------------------------------------------- MAC
// S^(xi) = sum_{k=1}^{nk} Khat_k(xi) Jhat_{n-k}(xi)   (eq:PnFFTMOT in the spectral domain).
// Khat_k is real and has a definite parity in every frequency axis (K^aa even, K^ab odd in
// D_a and D_b), so only the octant ky <= Ny/2, kz <= Nz/2 is stored and one load serves the
// four mirror points (ky, Ny-ky) x (kz, Nz-kz) with sign flips on the odd components.
// Layout [lag][octant point][xx, yy, zz, xy, xz, yz]: the six values of a point are one
// 48-byte record.
// One thread per octant point; G right-hand sides per thread share every Khat load.
template <int G>
__global__ void __launch_bounds__(256) k_mac(MacArg a)
{
    const int Hp = a.Hp, Nyo = a.Ny / 2 + 1, Nzo = a.Nz / 2 + 1;
    const long npt = (long)Hp * Nyo * Nzo;
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= npt) return;
    const int kx = (int)(t % Hp);
    if (kx >= a.Hx) return;   // row padding
    const int qy = (int)((t / Hp) % Nyo);
    const int qz = (int)(t / ((long)Hp * Nyo));
    const int r0 = blockIdx.y * G;
    // mirror points
    int ys[2] = {qy, a.Ny - qy}, zs[2] = {qz, a.Nz - qz};
    const int ny_m = (qy == 0 || 2 * qy == a.Ny) ? 1 : 2;
    const int nz_m = (qz == 0 || 2 * qz == a.Nz) ? 1 : 2;
    const long plane = (long)a.Nz * a.Ny * Hp;   // one component of one spectrum
    long off[4];
    double sy_[4], sz_[4];
    int np = 0;
    for (int iz = 0; iz < nz_m; iz++)
        for (int iy = 0; iy < ny_m; iy++) {
            off[np] = ((long)zs[iz] * a.Ny + ys[iy]) * Hp + kx;
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

    const long koct = (long)Hp * Nyo * Nzo;
    const double *Kp = a.Khat + 6 * t;
    for (int k = 1; k <= a.nk; k++) {
        const double *Kk = Kp + (long)(k - 1) * 6 * koct;
        const double kxx = Kk[0], kyy = Kk[1], kzz = Kk[2];
        const double kxy = Kk[3], kxz = Kk[4], kyz = Kk[5];
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
    const long npt = (long)a.Hp * (a.Ny / 2 + 1) * (a.Nz / 2 + 1);
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

// ---------------------------------------------------------------------------- time-blocked MAC
// Toeplitz time division (Sec. 4.1) in two levels.  For the block of target steps
// n_b .. n_b + TB - 1 (t = n - n_b):
//   far:  F[t] = sum_{k=t+1}^{ell} Khat_k Jhat_{n_b+t-k}   (sources before the block, all known at n_b)
//   near: S_n  = F[t] + sum_{k=1}^{t} Khat_k Jhat_{n-k}      (sources inside the block)
// The far kernel streams every lag once per block: at lag k the TB targets need the TB
// consecutive sources n_b - k .. n_b - k + TB - 1, a window that slides by one source per lag,
// so each spectrum is loaded once and reused TB times from registers.
//
// Mapping: one workgroup = 64 consecutive octant points x the 4 mirror points
// (ky, Ny-ky) x (kz, Nz-kz), one wave per mirror; the 4 waves load the same Khat values, so 3
// of the 4 loads hit in cache.  Duplicate mirrors (ky = 0 or Ny/2, kz = 0 or Nz/2) idle.
struct MirrorPoint {
    bool valid;
    long off;      // offset in one spectrum component [Nz][Ny][Hp]
    long koff;     // octant point index (its Khat record starts at 6 koff)
    double sy, sz; // parity signs of the odd components
};

__device__ inline MirrorPoint mirror_point(int Hx, int Hp, int Ny, int Nz, long group)
{
    MirrorPoint mp;
    const int Nyo = Ny / 2 + 1, Nzo = Nz / 2 + 1;
    const long nocts = (long)Hp * Nyo * Nzo;
    const long o = group * 64L + (threadIdx.x & 63);
    const int m = (threadIdx.x >> 6) & 3;
    mp.valid = o < nocts;
    if (!mp.valid) return mp;
    const int kx = (int)(o % Hp), qy = (int)((o / Hp) % Nyo), qz = (int)(o / ((long)Hp * Nyo));
    const int fy = m & 1, fz = m >> 1;
    if (kx >= Hx) mp.valid = false;   // row padding
    if (fy && (qy == 0 || 2 * qy == Ny)) mp.valid = false;
    if (fz && (qz == 0 || 2 * qz == Nz)) mp.valid = false;
    const int ky = fy ? Ny - qy : qy, kz = fz ? Nz - qz : qz;
    mp.off = ((long)kz * Ny + ky) * Hp + kx;
    mp.koff = o;
    mp.sy = fy ? -1.0 : 1.0;
    mp.sz = fz ? -1.0 : 1.0;
    return mp;
}

struct KVal {
    double xx, yy, zz, xy, xz, yz;
};

// the six values of one octant point (Kk points at its record)
__device__ inline KVal load_k(const double *__restrict__ Kk, const MirrorPoint &mp)
{
    const double2 *K2 = (const double2 *)Kk;
    const double2 a = K2[0], b = K2[1], c = K2[2];
    KVal k;
    k.xx = a.x;
    k.yy = a.y;
    k.zz = b.x;
    k.xy = b.y * mp.sy;
    k.xz = c.x * mp.sz;
    k.yz = c.y * mp.sy * mp.sz;
    return k;
}

__device__ inline void kmul_acc(const KVal &k, const double2 *j, double2 *a)
{
    a[0].x += k.xx * j[0].x + k.xy * j[1].x + k.xz * j[2].x;
    a[0].y += k.xx * j[0].y + k.xy * j[1].y + k.xz * j[2].y;
    a[1].x += k.xy * j[0].x + k.yy * j[1].x + k.yz * j[2].x;
    a[1].y += k.xy * j[0].y + k.yy * j[1].y + k.yz * j[2].y;
    a[2].x += k.xz * j[0].x + k.yz * j[1].x + k.zz * j[2].x;
    a[2].y += k.xz * j[0].y + k.yz * j[1].y + k.zz * j[2].y;
}

__device__ inline int ring_slot(int j, int ring)
{
    int s = j % ring;
    return s < 0 ? s + ring : s;
}

// Far part.  Khat is real, so the real and imaginary parts of Jhat never mix: each lane
// takes one part of one mirror point, which halves the registers per lane.  The TB = TG * G
// targets of the block are split into G groups of TG over the lanes of a wave (group g owns
// targets g TG .. g TG + TG - 1), so the registers per lane grow with TG, not TB.  For group
// g, lag k is its local lag k' = k - g TG: the lag loop is unrolled by TG so that the sliding
// source window lives in registers with compile-time slot indices; the source of local lag
// k' (J at n_b - k') goes to slot (k - 1) mod TG and local target tt at lag k reads the slot
// written at lag k - tt.  A group's sources are those of group 0 TG lags earlier, so the
// extra loads hit in cache; K_k is the same for every group.
template <int TG, int G, int PD, int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) k_mac_far(BlockMacArg a)
{
    static_assert(64 % (2 * G) == 0, "lanes split evenly into groups");
    static_assert(TG % PD == 0, "the prefetch buffers rotate with the slot window");
    constexpr int kLanesPerGroup = 64 / G;
    constexpr int kPointsPerWave = kLanesPerGroup / 2;
    const int Nyo = a.Ny / 2 + 1, Nzo = a.Nz / 2 + 1;
    const long nocts = (long)a.Hp * Nyo * Nzo;
    const int lane = threadIdx.x & 63;
    const int g = lane / kLanesPerGroup, li = lane % kLanesPerGroup;
    // the right-hand sides of one point group are adjacent blocks, so the kernel values they
    // share are read from HBM once and hit in cache for the others
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int r = lb % a.nrhs;
    const long o = (lb / a.nrhs) * (long)kPointsPerWave + (li >> 1);
    const int part = li & 1;
    const int m = threadIdx.x >> 6;
    if (o >= nocts) return;
    const int kx = (int)(o % a.Hp), qy = (int)((o / a.Hp) % Nyo), qz = (int)(o / ((long)a.Hp * Nyo));
    const int fy = m & 1, fz = m >> 1;
    if (kx >= a.Hx) return;   // row padding
    if ((fy && (qy == 0 || 2 * qy == a.Ny)) || (fz && (qz == 0 || 2 * qz == a.Nz))) return;
    const int ky = fy ? a.Ny - qy : qy, kz = fz ? a.Nz - qz : qz;
    const double sy = fy ? -1.0 : 1.0, sz = fz ? -1.0 : 1.0;
    const long off2 = 2 * (((long)kz * a.Ny + ky) * a.Hp + kx) + part;   // in doubles
    const long plane2 = 2L * a.Nz * a.Ny * a.Hp;                           // one component, in doubles
    const long koct = nocts;
    const int tg0 = g * TG;                                                // first target of the group
    constexpr int TB = TG * G;
    double acc[TG][3], jw[TG][3];
#pragma unroll
    for (int t = 0; t < TG; t++)
#pragma unroll
        for (int c = 0; c < 3; c++) acc[t][c] = jw[t][c] = 0.0;
    const unsigned joff = (unsigned)(off2 * 8), koff = (unsigned)(o * 48);
    const char *Jbase = (const char *)((const double *)a.ring_base + (long)r * 3 * plane2);
    const long slot_bytes = (long)a.nrhs * 3 * plane2 * 8, plane_bytes = plane2 * 8, koct_bytes = koct * 8;
    const char *Kbase = (const char *)a.Khat;
    // accumulate lag k with its source already in slot i: local target tt takes slot
    // (i - tt) mod TG, the source of lag k - tt
    auto accumulate = [&](int i, const double kv[6]) {
        const double kxx = kv[0], kyy = kv[1], kzz = kv[2];
        const double kxy = kv[3] * sy, kxz = kv[4] * sz, kyz = kv[5] * sy * sz;
#pragma unroll
        for (int t = 0; t < TG; t++) {
            const int sl = (i - t + TG) % TG;
            const double j0 = jw[sl][0], j1 = jw[sl][1], j2 = jw[sl][2];
            acc[t][0] = fma(kxz, j2, fma(kxy, j1, fma(kxx, j0, acc[t][0])));
            acc[t][1] = fma(kyz, j2, fma(kyy, j1, fma(kxy, j0, acc[t][1])));
            acc[t][2] = fma(kzz, j2, fma(kyz, j1, fma(kxz, j0, acc[t][2])));
        }
    };
    // loads of lag k: the lane's source sits in ring slot `slot`; ok = false (no source: the
    // lag is a near lag of the group, or the source precedes the march) gives zeros
    auto load_lag = [&](int k, int slot, bool ok, double jv[3], double kv[6]) {
        const char *J = Jbase + slot * slot_bytes;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const double v = *(const double *)(J + c * plane_bytes + joff);
            jv[c] = ok ? v : 0.0;
        }
        const double2 *K2 = (const double2 *)(Kbase + (long)(k - 1) * 6 * koct_bytes + koff);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const double2 v = K2[c];
            kv[2 * c] = v.x;
            kv[2 * c + 1] = v.y;
        }
    };
    // lags up to n_b - 1 have a source for every group (group 0's source n_b - k >= 1); later
    // lags (at most TB - 1 of them, only early in the march) still feed later targets
    const int kfull = min(a.nk, a.nb - 1);
    const int kend = min(a.nk, a.nb - 2 + TB);
    int k0 = 1;
    // full groups of TG lags, software-pipelined by one lag: the loads of lag k + 1 are in
    // flight while lag k is accumulated (the ring slot of the lane's source steps down by one
    // per lag)
    const int kgroups = kfull >= TG ? (kfull / TG) * TG : 0;
    if (kgroups > 0) {
        // PD lags in flight: buffer b = (k - 1) mod PD holds the loads of lag k
        int slot = ring_slot(a.nb - 1 + tg0, a.ring);
        double pj[PD][3], pk[PD][6];
#pragma unroll
        for (int d = 0; d < PD; d++) {
            const int kd = 1 + d <= kgroups ? 1 + d : kgroups;
            load_lag(kd, slot, kd > tg0, pj[d], pk[d]);
            if (d + 1 < PD) slot = slot == 0 ? a.ring - 1 : slot - 1;
        }
        for (; k0 + TG - 1 <= kgroups; k0 += TG) {
#pragma unroll
            for (int i = 0; i < TG; i++) {
                const int bi = i % PD;
                double kv[6];
#pragma unroll
                for (int c = 0; c < 3; c++) jw[i][c] = pj[bi][c];
#pragma unroll
                for (int c = 0; c < 6; c++) kv[c] = pk[bi][c];
                const int kn = k0 + i + PD;
                slot = slot == 0 ? a.ring - 1 : slot - 1;
                // past the last group this reloads a valid lag; the values are not used
                load_lag(kn <= kgroups ? kn : kgroups, slot, kn > tg0, pj[bi], pk[bi]);
                // keep the scheduler from sinking these loads down to their use
                __builtin_amdgcn_sched_barrier(0);
                accumulate(i, kv);
            }
        }
    }
    for (; k0 <= kend; k0 += TG) {
#pragma unroll
        for (int i = 0; i < TG; i++) {
            const int k = k0 + i;
            if (k > kend) break;
            const int j = a.nb - k + tg0;
            double kv[6];
            load_lag(k, ring_slot(j, a.ring), k > tg0 && j >= 1, jw[i], kv);
            accumulate(i, kv);
        }
    }
    double *Fd = (double *)a.far;
#pragma unroll
    for (int tt = 0; tt < TG; tt++) {
        const int t = tg0 + tt;
        if (t >= a.ntarget) break;
        double *F = Fd + ((long)t * a.nrhs + r) * 3 * plane2 + off2;
        F[0] = acc[tt][0];
        F[plane2] = acc[tt][1];
        F[2 * plane2] = acc[tt][2];
    }
}

// Far part with a rotation-free source window.  Targets t = 0 .. TG - 1 are steps n_b + t; each
// sums F[t] = init[t] + sum_k Khat_k Jhat_{n_b + t - k} over the lags k >= t + 1 whose source
// n_b + t - k is at least jmin (and at least 1) and, if jmax > 0, at most jmax.  One lane = one
// part (real or imaginary) of one mirror point, as in k_mac_far with one target group.  The lane
// loads, at lag k, the source s_k = n_b - k of target 0; target t at lag k takes s_{k - t},
// loaded t lags earlier.  Sources sit in W = TG + PD register slots, s_k in slot
// (k - klo + 1) mod W, klo being the first lag: the load of lag k + PD (issued before lag k is
// accumulated) overwrites the slot of s_{k - TG}, which no target needs at lag k or later, so no
// value ever moves between registers.  Kernel values of lag k sit in slot (k - klo + 1) mod
// (PD + 1).  The lag loop is unrolled by UF, a multiple of both slot counts, so that every slot
// index is a compile-time constant.
constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

template <int TG, int PD, int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) k_mac_win(BlockMacArg a)
{
    constexpr int W = TG + PD, KS = PD + 1;
    constexpr int UF = W / gcd_c(W, KS) * KS;
    const int Nyo = a.Ny / 2 + 1, Nzo = a.Nz / 2 + 1;
    const long nocts = (long)a.Hp * Nyo * Nzo;
    const int lane = threadIdx.x & 63;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int r = lb % a.nrhs;
    const long o = (lb / a.nrhs) * 32L + (lane >> 1);
    const int part = lane & 1;
    const int m = threadIdx.x >> 6;
    if (o >= nocts) return;
    const int kx = (int)(o % a.Hp), qy = (int)((o / a.Hp) % Nyo), qz = (int)(o / ((long)a.Hp * Nyo));
    const int fy = m & 1, fz = m >> 1;
    if (kx >= a.Hx) return;   // row padding
    if ((fy && (qy == 0 || 2 * qy == a.Ny)) || (fz && (qz == 0 || 2 * qz == a.Nz))) return;
    const int ky = fy ? a.Ny - qy : qy, kz = fz ? a.Nz - qz : qz;
    const double sy = fy ? -1.0 : 1.0, sz = fz ? -1.0 : 1.0;
    const long plane2 = 2L * a.Nz * a.Ny * a.Hp;                           // one component, in doubles
    const unsigned joff = (unsigned)(2 * (((long)kz * a.Ny + ky) * a.Hp + kx) + part) * 8u;
    const unsigned koff = (unsigned)(o * 48);
    const long slot_bytes = (long)a.nrhs * 3 * plane2 * 8, plane_bytes = plane2 * 8;
    const char *Jbase = (const char *)a.ring_base + (long)r * 3 * plane_bytes;
    const char *Kbase = (const char *)a.Khat;
    const long klag_bytes = 6 * nocts * 8;
    const int nb = a.nb, jlo = max(1, a.jmin);
    // the largest lag with a term: target TG - 1 reaches source jlo at lag nb + TG - 1 - jlo
    const int kmax = min(a.nk, nb - jlo + TG - 1);
    // the smallest: target 0 reaches source jmax at lag nb - jmax, and no target has a source
    // after jmax below that lag
    const int klo = a.jmax > 0 ? max(1, nb - a.jmax) : 1;

    // accumulators and source slots per component: arrays of at most TG + PD doubles each, which
    // the compiler keeps in registers
    double ax[TG], ay[TG], az[TG];
#pragma unroll
    for (int t = 0; t < TG; t++) ax[t] = ay[t] = az[t] = 0.0;
    if (a.init) {
        const double *I = (const double *)a.init + (long)r * 3 * plane2 + joff / 8;
        [&]<int... T>(std::integer_sequence<int, T...>) __attribute__((always_inline)) {
            ((T < a.ntarget ? (ax[T] = I[(long)T * a.nrhs * 3 * plane2],
                               ay[T] = I[(long)T * a.nrhs * 3 * plane2 + plane2],
                               az[T] = I[(long)T * a.nrhs * 3 * plane2 + 2 * plane2], 0)
                            : 0),
             ...);
        }(std::make_integer_sequence<int, TG>{});
    }
    double jx[W], jy[W], jz[W];
    double k0s[KS], k1s[KS], k2s[KS], k3s[KS], k4s[KS], k5s[KS];   // xx yy zz xy xz yz
#pragma unroll
    for (int s = 0; s < W; s++) jx[s] = jy[s] = jz[s] = 0.0;   // sources before the first lag are zero
    // the loads of lag k into a source slot and a kernel slot.  With many lags (UL: 10 targets or
    // more) every call issues the same six loads, so that the wait before each lag's arithmetic
    // counts only the loads issued after its own (a load skipped on some path makes the compiler
    // wait for all of them): lags beyond kmax reload lag kmax, whose values no target uses, and a
    // source before jlo reads a valid slot and is replaced by zero.  The middle level's short
    // launches (4 targets, at most 15 lags, 3 of them without a source) skip those loads instead.
    constexpr bool UL = TG >= 10;
    auto load = [&](int k, double &vx, double &vy, double &vz, double &c0, double &c1, double &c2, double &c3,
                    double &c4, double &c5) __attribute__((always_inline)) {
        if (!UL && k > kmax) return;
        const int kk = UL ? min(k, kmax) : k;
        const int j = nb - kk;
        const bool ok = j >= jlo;
        if (UL) {
            const char *J = Jbase + ring_slot(ok ? j : jlo, a.ring) * slot_bytes + joff;
            const double x = *(const double *)J;
            const double y = *(const double *)(J + plane_bytes);
            const double z = *(const double *)(J + 2 * plane_bytes);
            vx = ok ? x : 0.0;
            vy = ok ? y : 0.0;
            vz = ok ? z : 0.0;
        } else if (ok) {
            const char *J = Jbase + ring_slot(j, a.ring) * slot_bytes + joff;
            vx = *(const double *)J;
            vy = *(const double *)(J + plane_bytes);
            vz = *(const double *)(J + 2 * plane_bytes);
        } else {
            vx = vy = vz = 0.0;
        }
        const double2 *K2 = (const double2 *)(Kbase + (long)(kk - 1) * klag_bytes + koff);
        const double2 v0 = K2[0], v1 = K2[1], v2 = K2[2];
        c0 = v0.x;
        c1 = v0.y;
        c2 = v1.x;
        c3 = v1.y;
        c4 = v2.x;
        c5 = v2.y;
    };
    // lag k = k0 + i, k0 = klo mod UF: source slot of s_{k - t} is (1 + i - t) mod W.  Slots of
    // sources before lag klo are never loaded and stay zero, which is their value: they lie
    // after jmax.  The UF steps are expanded from a compile-time index sequence, so every slot
    // index is a constant.
    auto step = [&](auto ic, int k0, bool guard) __attribute__((always_inline)) {
        constexpr int i = decltype(ic)::value;
        const int k = k0 + i;
        constexpr int ls = (1 + i + PD) % W, lk = (1 + i + PD) % KS, ck = (1 + i) % KS;
        if (!UL && guard && k > kmax) return;
        load(k + PD, jx[ls], jy[ls], jz[ls], k0s[lk], k1s[lk], k2s[lk], k3s[lk], k4s[lk], k5s[lk]);
        __builtin_amdgcn_sched_barrier(0);
        if (UL && guard && k > kmax) return;
        const double kxx = k0s[ck], kyy = k1s[ck], kzz = k2s[ck];
        const double kxy = k3s[ck] * sy, kxz = k4s[ck] * sz, kyz = k5s[ck] * sy * sz;
        [&]<int... T>(std::integer_sequence<int, T...>) __attribute__((always_inline)) {
            ((ax[T] = fma(kxz, jz[(1 + i - T + 4 * W) % W],
                          fma(kxy, jy[(1 + i - T + 4 * W) % W], fma(kxx, jx[(1 + i - T + 4 * W) % W], ax[T]))),
              ay[T] = fma(kyz, jz[(1 + i - T + 4 * W) % W],
                          fma(kyy, jy[(1 + i - T + 4 * W) % W], fma(kxy, jx[(1 + i - T + 4 * W) % W], ay[T]))),
              az[T] = fma(kzz, jz[(1 + i - T + 4 * W) % W],
                          fma(kyz, jy[(1 + i - T + 4 * W) % W], fma(kxz, jx[(1 + i - T + 4 * W) % W], az[T])))),
             ...);
        }(std::make_integer_sequence<int, TG>{});
    };
    auto body = [&](int k0, bool guard) __attribute__((always_inline)) {
        [&]<int... I>(std::integer_sequence<int, I...>) __attribute__((always_inline)) {
            (step(std::integral_constant<int, I>{}, k0, guard), ...);
        }(std::make_integer_sequence<int, UF>{});
    };
    (void)body;
#pragma unroll
    for (int d = 0; d < PD; d++) {
        const int ls = (1 + d) % W, lk = (1 + d) % KS;
        load(klo + d, jx[ls], jy[ls], jz[ls], k0s[lk], k1s[lk], k2s[lk], k3s[lk], k4s[lk], k5s[lk]);
    }
    int k0 = klo;
    for (; k0 <= kmax; k0 += UF) body(k0, true);
    double *Fd = (double *)a.far + (long)r * 3 * plane2 + joff / 8;
    [&]<int... T>(std::integer_sequence<int, T...>) __attribute__((always_inline)) {
        ((T < a.ntarget ? (Fd[(long)T * a.nrhs * 3 * plane2] = ax[T],
                           Fd[(long)T * a.nrhs * 3 * plane2 + plane2] = ay[T],
                           Fd[(long)T * a.nrhs * 3 * plane2 + 2 * plane2] = az[T], 0)
                        : 0),
         ...);
    }(std::make_integer_sequence<int, TG>{});
}

// near part of step n = n_b + t, accumulated in place into F[t]
__global__ void __launch_bounds__(256) k_mac_near(BlockMacArg a)
{
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const MirrorPoint mp = mirror_point(a.Hx, a.Hp, a.Ny, a.Nz, lb / a.nrhs);
    if (!mp.valid) return;
    const int r = lb % a.nrhs;
    const long plane = (long)a.Nz * a.Ny * a.Hp;
    const long koct = (long)a.Hp * (a.Ny / 2 + 1) * (a.Nz / 2 + 1);
    const int t = a.t;
    double2 *F = a.far + ((long)t * a.nrhs + r) * 3 * plane + mp.off;
    double2 acc[3] = {F[0], F[plane], F[2 * plane]};
    const double *Kp = a.Khat + 6 * mp.koff;
    const int n = a.nb + t;
    // lags beyond the kernel's support (k > nk) contribute nothing; sources before the
    // march started (j < 1) are zero.  Two lags per pass so their loads overlap.
    const int kmax = min(t, a.nk);
    for (int k = 1; k <= kmax; k += 2) {
        const bool two = k + 1 <= kmax;
        const int j0 = n - k, j1 = n - k - 1;
        const double2 *J0 = a.ring_base + ((long)ring_slot(j0, a.ring) * a.nrhs + r) * 3 * plane + mp.off;
        const double2 *J1 = a.ring_base + ((long)ring_slot(two ? j1 : j0, a.ring) * a.nrhs + r) * 3 * plane + mp.off;
        double2 jv0[3] = {J0[0], J0[plane], J0[2 * plane]};
        double2 jv1[3] = {J1[0], J1[plane], J1[2 * plane]};
        const KVal kv0 = load_k(Kp + (long)(k - 1) * 6 * koct, mp);
        const KVal kv1 = load_k(Kp + (long)(two ? k : k - 1) * 6 * koct, mp);
        if (j0 >= 1) kmul_acc(kv0, jv0, acc);
        if (two && j1 >= 1) kmul_acc(kv1, jv1, acc);
    }
    F[0] = acc[0];
    F[plane] = acc[1];
    F[2 * plane] = acc[2];
}

void launch_mac_far(const BlockMacArg &a, int tb, hipStream_t st)
{
    // 10 to 16 targets: the windowed kernel; 4, 8 and 32: the grouped one (at 8 targets it ran
    // 12.10 against 11.61 ms per launch at 104^3).  Neither takes jmin or init here.
    if (tb >= 10 && tb <= 16 && tb % 2 == 0) {
        launch_mac_win(a, tb, st);
        return;
    }
    const long nocts = (long)a.Hp * (a.Ny / 2 + 1) * (a.Nz / 2 + 1);
    // the grouped kernel for 4 and 32 targets: TB = TG * G targets per launch; points per block = 32 / G
    auto grid = [&](int G) { return dim3((unsigned)((nocts + 32 / G - 1) / (32 / G) * a.nrhs)); };
    const dim3 blk(256);
    switch (tb) {
    // last argument: waves per SIMD the register budget is held to.  At TB = 8, three waves
    // (168 VGPRs, one lag in flight) measured slower than two waves with two lags in flight.
    case 4: hipLaunchKernelGGL((k_mac_far<4, 1, 2, 3>), grid(1), blk, 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_mac_far<8, 1, 2, 2>), grid(1), blk, 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_mac_far<8, 4, 2, 2>), grid(4), blk, 0, st, a); break;
    default: throw ArgError("unsupported time block (4, 8, 10, 12, 14, 16 or 32)");
    }
    MJ_CHECK(hipGetLastError());
}

// lds_reserve: LDS bytes each block claims without using them, which caps the blocks a CU
// holds at once (and so leaves room on every CU for other kernels running beside this one)
void launch_mac_win(const BlockMacArg &a, int tb, hipStream_t st, size_t lds_reserve)
{
    const long nocts = (long)a.Hp * (a.Ny / 2 + 1) * (a.Nz / 2 + 1);
    const dim3 grid((unsigned)((nocts + 31) / 32 * a.nrhs)), blk(256);
    if (lds_reserve > 0 && tb == 16) {
        MJ_CHECK(hipFuncSetAttribute((const void *)k_mac_win<16, 1, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds_reserve));
        hipLaunchKernelGGL((k_mac_win<16, 1, 2>), grid, blk, lds_reserve, st, a);
        MJ_CHECK(hipGetLastError());
        return;
    }
    // second argument: lags in flight; the register file holds two at 8 targets, one above
    // (166 to 238 VGPRs, two waves per SIMD).  At 16 targets two lags in flight also fit (256
    // VGPRs) but ran 16.3 against 15.5 ms per launch at 104^3
    switch (tb) {
    case 4: hipLaunchKernelGGL((k_mac_win<4, 2, 3>), grid, blk, 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_mac_win<8, 2, 2>), grid, blk, 0, st, a); break;
    case 10: hipLaunchKernelGGL((k_mac_win<10, 1, 2>), grid, blk, 0, st, a); break;
    case 12: hipLaunchKernelGGL((k_mac_win<12, 1, 2>), grid, blk, 0, st, a); break;
    case 14: hipLaunchKernelGGL((k_mac_win<14, 1, 2>), grid, blk, 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_mac_win<16, 1, 2>), grid, blk, 0, st, a); break;
    default: throw ArgError("unsupported target count of the windowed far kernel (4, 8, 10, 12, 14 or 16)");
    }
    MJ_CHECK(hipGetLastError());
}

void launch_mac_near(const BlockMacArg &a, hipStream_t st)
{
    const long nocts = (long)a.Hp * (a.Ny / 2 + 1) * (a.Nz / 2 + 1);
    dim3 grd((unsigned)((nocts + 63) / 64 * a.nrhs)), blk(256);
    hipLaunchKernelGGL(k_mac_near, grd, blk, 0, st, a);
    MJ_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------- excitation
// Coefficients every lane reads alike (the K_0 stencil, the FIR taps, the quadrature rules)
// through the scalar cache: a pointer into the constant address space makes them scalar loads
typedef __attribute__((address_space(4))) const double kconst_t;
__device__ inline kconst_t *kconst(const double *p) { return (kconst_t *)p; }

// chi_m times the voxel average of a Gaussian plane wave at c t = n c dt (eq:E).  The average
// over an axis the wave does not depend on is the identity.  A wave along one axis takes the
// 8-point Gauss-Legendre rule on it.  A wave with two or three non-zero components follows the
// plan the host made from its spreads s_i = |k_i| h_i / w (w the pulse width):
//  * form 0: on each axis the n-point rule with the least n whose remainder bound
//    (n!)^4 / ((2n + 1) ((2n)!)^3) s^2n max|d^2n/dx^2n exp(-x^2)| (the Gauss-Legendre remainder,
//    the derivative bounded by Cramer's inequality) stays below 2^-53; at 64^3 with a width of
//    8.5 voxels that is 4 or 5 points an axis where the oracle's rule takes 8;
//  * form 1, once the widest axis would need 6 points or more: that axis in closed form,
//    (w sqrt(pi) / (2 k_a h_a)) (erf((T + k_a h_a / 2) / w) - erf((T - k_a h_a / 2) / w)), through
//    erfc where both arguments lie in one tail, and the rule on the other two;
//  * form 2, once the second widest spread is beyond what the 8-point rule integrates to 2^-53
//    (pulses narrower than about 1.4 voxels): the two widest axes in closed form.  With
//    c_a = k_a h_a / (2w), c_b likewise and t = T / w, their average is (sqrt(pi) / (8 c_a c_b))
//    times the second difference G(t + c_b + c_a) - G(t + c_b - c_a) - G(t - c_b + c_a)
//    + G(t - c_b - c_a) of G(z) = z erf(z) + exp(-z^2) / sqrt(pi) = |z| + ierfc(|z|), the
//    antiderivative of erf, where ierfc(x) = exp(-x^2) / sqrt(pi) - x erfc(x).
// Each form is within a few units in the last place of the exact average wherever the oracle's
// 8-point rule is too, and more exact where the rule is not.  CF = false leaves the plan out of
// the kernel (its registers slow the right-hand side when every wave runs along an axis); a
// launch takes CF = true whenever one of its waves does not, and a wave along an axis takes the
// same 8-point rule either way.
template <bool CF>
__device__ inline double wave_average(const WaveArg &w, const EpiArg &e, int u, int v, int z, double ct)
{
    const double tc = ct - w.ct0 - ((u + 0.5) * e.h - w.rref[0]) * w.k[0] - ((v + 0.5) * e.hy - w.rref[1]) * w.k[1] -
                      ((z + 0.5) * e.hz - w.rref[2]) * w.k[2];
    const double iw = 1.0 / w.width;
    if (CF && (w.k[0] != 0.0) + (w.k[1] != 0.0) + (w.k[2] != 0.0) >= 2) {
        kconst_t *ga = kconst(e.gl) + 16 * w.nq[0], *gb = kconst(e.gl) + 16 * w.nq[1];
        kconst_t *gc = kconst(e.gl) + 16 * w.nq[2];
        const int na = w.nq[0], nb = w.nq[1], nc = w.nq[2];
        if (w.form == 2) {
            const double ca = 0.5 * w.kh[0] * iw, cb = 0.5 * w.kh[1] * iw;
            double sum = 0.0;
            for (int l = 0; l < nc; l++) {
                const double t = (tc - gc[l] * w.kh[2]) * iw;
                const double z[4] = {fabs(t + cb + ca), fabs(t + cb - ca), fabs(t - cb + ca), fabs(t - cb - ca)};
                // the |z| terms cancel exactly once all four arguments share a sign
                double g = fabs(t) >= fabs(ca) + fabs(cb) ? 0.0 : (z[0] - z[1]) - (z[2] - z[3]);
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const double ie = 0.5641895835477563 * exp(-z[q] * z[q]) - z[q] * erfc(z[q]);
                    g += (q == 0 || q == 3) ? ie : -ie;
                }
                sum += gc[8 + l] * g;
            }
            return w.amp * sum * (0.2215567313631895 / (ca * cb));   // sqrt(pi) / 8
        }
        if (w.form == 1) {
            const double half = 0.5 * w.kh[0];
            double sum = 0.0;
            for (int i = 0; i < nb; i++) {
                const double o1 = gb[i] * w.kh[1];
                double sl = 0.0;
                for (int j = 0; j < nc; j++) {
                    const double T = tc - o1 - gc[j] * w.kh[2];
                    const double u1 = (T + half) * iw, u2 = (T - half) * iw;
                    // erf(u1) - erf(u2), through erfc where both lie in one tail
                    const double d = (u1 > 0.0 && u2 > 0.0)   ? erfc(u2) - erfc(u1)
                                     : (u1 < 0.0 && u2 < 0.0) ? erfc(-u1) - erfc(-u2)
                                                              : erf(u1) - erf(u2);
                    sl += gc[8 + j] * d;
                }
                sum += gb[8 + i] * sl;
            }
            return w.amp * sum * (0.8862269254527580 * w.width / w.kh[0]);   // sqrt(pi) / 2
        }
        double sum = 0.0;
        for (int i = 0; i < na; i++) {
            const double o0 = ga[i] * w.kh[0];
            for (int j = 0; j < nb; j++) {
                const double o1 = o0 + gb[j] * w.kh[1];
                double sl = 0.0;
                for (int l = 0; l < nc; l++) {
                    const double x = (tc - o1 - gc[l] * w.kh[2]) * iw;
                    sl += gc[8 + l] * exp(-x * x);
                }
                sum += ga[8 + i] * gb[8 + j] * sl;
            }
        }
        return w.amp * sum;
    }
    const int nx = w.k[0] != 0.0 ? 8 : 1, ny = w.k[1] != 0.0 ? 8 : 1, nz = w.k[2] != 0.0 ? 8 : 1;
    double sum = 0.0;
    for (int i = 0; i < nx; i++) {
        const double ox = nx > 1 ? e.glx8[i] * e.h * w.k[0] : 0.0, wx = nx > 1 ? e.glw8[i] : 1.0;
        for (int j = 0; j < ny; j++) {
            const double oy = ny > 1 ? e.glx8[j] * e.hy * w.k[1] : 0.0, wy = ny > 1 ? e.glw8[j] : 1.0;
            double sl = 0.0;
            for (int l = 0; l < nz; l++) {
                const double oz = nz > 1 ? e.glx8[l] * e.hz * w.k[2] : 0.0, wz = nz > 1 ? e.glw8[l] : 1.0;
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
// y0 = sum_{k=1}^{nguess} gx_k y_{n-k}, y = J / sqrt(chi).
template <bool CF>
__global__ void __launch_bounds__(256) k_epilogue(EpiArg e)
{
    const long M = e.M;
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= M) return;
    const double chi = e.chi[i], sc = e.schi[i];
    const int u = (int)(i % e.U), v = (int)((i / e.U) % e.V), z = (int)(i / ((long)e.U * e.V));
    const long Mp = (long)(e.U + 2) * (e.V + 2) * (e.W + 2);
    const long ip = ((long)(z + 1) * (e.V + 2) + (v + 1)) * (e.U + 2) + (u + 1);
    if (sc == 0.0) {
        // vacuum voxel: its current and every term of its row vanish
        for (int c = 0; c < 3; c++) {
            const long o = ((long)r * 3 + c) * M + i;
            e.rhs[o] = 0.0;
            e.y[o] = 0.0;
            e.uy[((long)r * 3 + c) * Mp + ip] = 0.0;
        }
        return;
    }
    const WaveArg w = e.waves[r];
    const double avg = wave_average<CF>(w, e, u, v, z, e.n * e.c_dt);
    const double c1 = 0.5 * e.inv_eps[i] + (e.nfir > 1 ? e.fir[1] : 0.0);
    const int kmax = min(e.nloc, e.n - 1);   // lags with a past current
    // initial guess of the Z_0 solve: the polynomial through the last nguess solutions,
    // evaluated at step n (the current is smooth in time, so this lands close to y_n).  The
    // three components of a past current are read together, eight lags at a time, and the
    // taps come through the scalar cache; each component still sums its lags in order.
    double b[3], g[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const long o = ((long)r * 3 + c) * M + i;
        b[c] = chi * (avg * w.pol[c] + (e.S ? e.S[o] : 0.0));
    }
    kconst_t *fir = kconst(e.fir);
#pragma unroll 8
    for (int k = 1; k <= kmax; k++) {
        const double *J = e.Jring + ((long)e.slot_of[k] * e.nrhs + r) * 3 * M + i;
        const double j0 = J[0], j1 = J[M], j2 = J[2 * M];
        const double ck = (k == 1) ? c1 : (k < e.nfir ? fir[k] : 0.0);
        b[0] -= ck * j0;
        b[1] -= ck * j1;
        b[2] -= ck * j2;
        if (k <= e.nguess) {
            const double gk = e.gx[k - 1];
            g[0] += gk * j0;
            g[1] += gk * j1;
            g[2] += gk * j2;
        }
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const long o = ((long)r * 3 + c) * M + i;
        const double y0 = g[c] / sc;
        e.rhs[o] = b[c] / sc;
        e.y[o] = y0;
        e.uy[((long)r * 3 + c) * Mp + ip] = sc * y0;
    }
}

void launch_epilogue(const EpiArg &e, hipStream_t st)
{
    dim3 grd((unsigned)((e.M + 255) / 256), e.nrhs);
    if (e.oblique) hipLaunchKernelGGL(k_epilogue<true>, grd, dim3(256), 0, st, e);
    else hipLaunchKernelGGL(k_epilogue<false>, grd, dim3(256), 0, st, e);
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
// (A z)_b(m) = c_0(m) z_b(m) - s(m) sum_{D in 27} sum_a K_0^{ba}(D) u_a(m-D),   u = s z.
// K_0(D) = K_0(-D) for every component, so the 26 neighbours are summed in 13 pairs.
// A is symmetric positive definite; Jacobi preconditioning with diag(A), z = M^-1 r = md r.
//
// Stored vectors: y, p, q = A p (kept by recurrence) and u = s z in the zero-haloed layout the
// stencil reads.  The residual is not stored: where s != 0, r = u / (s md) and z = u / s.
// The update y += alpha_it p_it is applied by the next iteration's first kernel, which reads
// p_it anyway; the solve ends with one more such pass.
//
// Reductions: every block writes its partial sums; a one-block kernel per right-hand side adds
// them in block order and stores the scalars, so the results do not depend on scheduling.  The
// same kernel takes the convergence test and keeps the status record, and the iteration kernels
// read its outcome (CgScalars::conv) from the previous launch.

// sum_{D} K_0(D) u(m - D) at haloed index ip (the halo of u is zero, so no bounds tests);
// ctr receives u(m) itself
__device__ inline void stencil_apply(const CgArg &a, const double *__restrict__ u, long ip, double out[3],
                                     double ctr[3])
{
    const long Mp = a.Mp;
    const long sy = a.U + 2, sz = (long)(a.U + 2) * (a.V + 2);
    double acc0, acc1, acc2;
    {
        kconst_t *k = kconst(a.k0) + 13 * 6;
        const double u0 = u[ip], u1 = u[Mp + ip], u2 = u[2 * Mp + ip];
        ctr[0] = u0;
        ctr[1] = u1;
        ctr[2] = u2;
        acc0 = k[0] * u0 + k[3] * u1 + k[4] * u2;
        acc1 = k[3] * u0 + k[1] * u1 + k[5] * u2;
        acc2 = k[4] * u0 + k[5] * u1 + k[2] * u2;
    }
#pragma unroll
    for (int o = 14; o < 27; o++) {
        // entry o = 13 + dx + 3 dy + 9 dz holds K_0(D); its pair is -D
        const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
        const long off = dx + dy * sy + dz * sz;
        const double s0 = u[ip - off] + u[ip + off];
        const double s1 = u[Mp + ip - off] + u[Mp + ip + off];
        const double s2 = u[2 * Mp + ip - off] + u[2 * Mp + ip + off];
        kconst_t *k = kconst(a.k0) + o * 6;
        acc0 += k[0] * s0 + k[3] * s1 + k[4] * s2;
        acc1 += k[3] * s0 + k[1] * s1 + k[5] * s2;
        acc2 += k[4] * s0 + k[5] * s1 + k[2] * s2;
    }
    out[0] = acc0;
    out[1] = acc1;
    out[2] = acc2;
}

// c_0 = T(0)/eps + delta_0 with T(0) = 1/2 and 1/eps = 1 - chi, and the Jacobi weight
// 1 / (c_0 - chi K_0^{xx}(0)), both from s = sqrt(chi): two coefficient streams fewer per pass.
// The diagonal of K_0 at D = 0 is isotropic for cubic voxels; for unequal edges the x entry
// stands in for all three, which keeps the preconditioner symmetric positive definite (the
// solve still converges to the same tolerance)
__device__ inline double cg_c0(const CgArg &a, double s) { return 0.5 * (1.0 - s * s) + a.d0; }
__device__ inline double cg_md(const CgArg &a, double s, double c0) { return 1.0 / (c0 - s * s * a.k0c); }

__device__ inline long haloed(const CgArg &a, long i)
{
    const int x = (int)(i % a.U), y = (int)((i / a.U) % a.V), z = (int)(i / ((long)a.U * a.V));
    return ((long)(z + 1) * (a.V + 2) + (y + 1)) * (a.U + 2) + (x + 1);
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

// Stores the NV partial sums of logical block bx (every thread calls it).
template <int NV>
__device__ inline void block_partials(const double (&v)[NV], double *part, int nb, int bx)
{
    __shared__ double sm[8];
#pragma unroll
    for (int q = 0; q < NV; q++) {
        const double t = block_sum(v[q], sm);
        if (threadIdx.x == 0) part[(size_t)q * nb + bx] = t;
    }
}

// Logical (block, right-hand side) of a CG kernel on the grid (nblk, nrhs), in XCD order over
// the linear dispatch index, so that the blocks holding neighbouring planes of the stencil
// input share an L2.
struct CgBlock {
    int bx, r;
};
__device__ inline CgBlock cg_block()
{
    const unsigned lb = xcd_block(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    return CgBlock{(int)(lb % gridDim.x), (int)(lb / gridDim.x)};
}

// One block per right-hand side adds the partials of one CG kernel in block order; the number
// of sums tells which kernel wrote them:
//   NV = 3 (k_cg_init): rz_0, r.r, b.b and the test at iteration 0
//   NV = 1 (k_cg_a):    p.q
//   NV = 2 (k_cg_b):    rz_{it+1}, r.r and the test at iteration it + 1
// The test |r|^2 <= tol^2 |b|^2 (or b = 0) sets conv to the iteration that passed it.  The
// host enqueues iterations in batches, so launches past the end of a solve are routine.
template <int NV>
__global__ void __launch_bounds__(1024) k_cg_reduce(CgArg a, int it)
{
    constexpr int kUnroll = 8;
    __shared__ double sm[16];
    const int r = blockIdx.x, nb = a.nblk;
    // k_cg_a and k_cg_b of iteration it wrote no partials once the solve ended at conv <= it;
    // the scalars and the status stay as the end left them
    if (NV != 3 && a.scal[r].conv <= it) return;
    const double *pr = a.part + (size_t)r * 3 * nb;
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) acc[q] = 0.0;
    for (int b0 = threadIdx.x; b0 < nb; b0 += kUnroll * 1024) {
        double v[kUnroll][NV];
#pragma unroll
        for (int j = 0; j < kUnroll; j++) {
            const int b = b0 + j * 1024;
#pragma unroll
            for (int q = 0; q < NV; q++) v[j][q] = b < nb ? pr[(size_t)q * nb + b] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kUnroll; j++)
#pragma unroll
            for (int q = 0; q < NV; q++) acc[q] += v[j][q];
    }
#pragma unroll
    for (int q = 0; q < NV; q++) acc[q] = block_sum(acc[q], sm);
    if (threadIdx.x != 0) return;
    CgScalars *sc = a.scal + r;
    int iter;
    if constexpr (NV == 1) {
        sc->pq = acc[0];
        return;
    } else if constexpr (NV == 3) {
        iter = 0;
        sc->rz[0] = acc[0];
        sc->rr = acc[1];
        sc->bb = acc[2];
    } else {
        iter = it + 1;
        sc->rz[iter & 1] = acc[0];
        sc->rr = acc[1];
    }
    const double rr = sc->rr, bb = sc->bb;
    const bool pass = rr <= a.tol2 * bb || bb == 0.0;
    sc->conv = pass ? iter : INT_MAX;
    a.stat[r] = CgStatus{pass ? 1 : 0, iter, bb > 0.0 ? sqrt(rr / bb) : 0.0, bb, 0.0};
}

// r = rhs - A y0 (uy = s y0), u = s M^-1 r; partials rz, rr, bb
__global__ void __launch_bounds__(256) k_cg_init(CgArg a)
{
    const CgBlock cb = cg_block();
    const int r = cb.r;
    const long M = a.M, base = (long)r * 3 * M;
    const long i = cb.bx * (long)blockDim.x + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};   // rz, rr, bb
    if (i < M) {
        const double s = a.schi[i];
        const double c0 = cg_c0(a, s);
        const double md = s != 0.0 ? cg_md(a, s, c0) : 0.0;
        double Ay[3] = {0.0, 0.0, 0.0};
        const long ip = haloed(a, i), bp = (long)r * 3 * a.Mp;
        if (s != 0.0) {
            double Ku[3], ctr[3];
            stencil_apply(a, a.uy + bp, ip, Ku, ctr);
            for (int c = 0; c < 3; c++) Ay[c] = c0 * a.y[base + c * M + i] - s * Ku[c];
        }
        for (int c = 0; c < 3; c++) {
            const long o = base + c * M + i;
            const double b = a.rhs[o];
            const double rv = s != 0.0 ? b - Ay[c] : 0.0;
            const double zv = md * rv;
            a.u[bp + c * a.Mp + ip] = s * zv;
            v[0] += rv * zv;
            v[1] += rv * rv;
            v[2] += b * b;
        }
    }
    block_partials<3>(v, a.part + (size_t)r * 3 * gridDim.x, gridDim.x, cb.bx);
}

// Iteration it, first half: y += alpha_{it-1} p_{it-1};  then, unless the solve ends here,
// beta = rz_it / rz_{it-1} (0 at it = 0);  w = A z;  p = z + beta p;  q = w + beta q;  partial p.q.
// The solve ends here when the test passed at iteration it, or when finish is set (the host's
// last pass); launches after that return at once.
__global__ void __launch_bounds__(256) k_cg_a(CgArg a, int it, int finish)
{
    const CgBlock cb = cg_block();
    const int r = cb.r;
    const CgScalars *sc = a.scal + r;
    const int conv = sc->conv;
    if (conv < it) return;
    const bool last = conv == it || finish;
    if (last && it == 0) return;
    // at it > 0: slot (it + 1) & 1 holds rz_{it-1}, pq holds p_{it-1}.q_{it-1}
    const double alpha = it > 0 ? sc->rz[(it + 1) & 1] / sc->pq : 0.0;
    const double beta = it > 0 ? sc->rz[it & 1] / sc->rz[(it + 1) & 1] : 0.0;
    const long M = a.M, base = (long)r * 3 * M;
    const long i = cb.bx * (long)blockDim.x + threadIdx.x;
    if (last) {
        if (i < M && a.schi[i] != 0.0)
            for (int c = 0; c < 3; c++) a.y[base + c * M + i] += alpha * a.p[base + c * M + i];
        return;
    }
    double v[1] = {0.0};
    if (i < M) {
        const double s = a.schi[i];
        if (s != 0.0) {
            double Ku[3], uc[3];
            stencil_apply(a, a.u + (long)r * 3 * a.Mp, haloed(a, i), Ku, uc);
            const double c0 = cg_c0(a, s), inv_s = 1.0 / s;
            for (int c = 0; c < 3; c++) {
                const long o = base + c * M + i;
                const double zv = uc[c] * inv_s;
                // at it = 0, alpha = beta = 0 and p, q hold finite values of the previous solve
                // (the update stays unconditional: a branch here makes the compiler duplicate
                // the loop body)
                const double po = a.p[o];
                a.y[o] += alpha * po;
                const double pv = zv + beta * po;
                const double qv = (c0 * zv - s * Ku[c]) + beta * a.q[o];
                a.p[o] = pv;
                a.q[o] = qv;
                v[0] += pv * qv;
            }
        }
    }
    block_partials<1>(v, a.part + (size_t)r * 3 * gridDim.x, gridDim.x, cb.bx);
}

// second half: alpha = rz_it / p.q;  r -= alpha q, kept as u -= alpha s md q;  partials
// rz_{it+1} and r.r
__global__ void __launch_bounds__(256) k_cg_b(CgArg a, int it)
{
    const CgBlock cb = cg_block();
    const int r = cb.r;
    const CgScalars *sc = a.scal + r;
    if (sc->conv <= it) return;
    const double alpha = sc->rz[it & 1] / sc->pq;
    const long M = a.M, base = (long)r * 3 * M;
    const long i = cb.bx * (long)blockDim.x + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (i < M) {
        const double s = a.schi[i];
        if (s != 0.0) {
            const double md = cg_md(a, s, cg_c0(a, s));
            const double f = s * md, inv_f = 1.0 / f;
            const long up = (long)r * 3 * a.Mp + haloed(a, i);
            for (int c = 0; c < 3; c++) {
                const double un = a.u[up + c * a.Mp] - alpha * f * a.q[base + c * M + i];
                a.u[up + c * a.Mp] = un;
                const double rv = un * inv_f;
                v[0] += md * rv * rv;
                v[1] += rv * rv;
            }
        }
    }
    block_partials<2>(v, a.part + (size_t)r * 3 * gridDim.x, gridDim.x, cb.bx);
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

template <int NV>
static void launch_reduce(const CgArg &a, int it, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_reduce<NV>, dim3(a.nrhs), dim3(1024), 0, st, a, it);
    MJ_CHECK(hipGetLastError());
}
void launch_cg_init(const CgArg &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_init, dim3(a.nblk, a.nrhs), dim3(256), 0, st, a);
    MJ_CHECK(hipGetLastError());
    launch_reduce<3>(a, 0, st);
}
void launch_cg_a(const CgArg &a, int it, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_a, dim3(a.nblk, a.nrhs), dim3(256), 0, st, a, it, 0);
    MJ_CHECK(hipGetLastError());
    launch_reduce<1>(a, it, st);
}
void launch_cg_b(const CgArg &a, int it, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_b, dim3(a.nblk, a.nrhs), dim3(256), 0, st, a, it);
    MJ_CHECK(hipGetLastError());
    launch_reduce<2>(a, it, st);
}
void launch_cg_end(const CgArg &a, int it, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_a, dim3(a.nblk, a.nrhs), dim3(256), 0, st, a, it, 1);
    MJ_CHECK(hipGetLastError());
}
void launch_cg_finish(const double *y, const double *schi, long M, int nrhs, double *J, double *Jout,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_finish, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, y, schi, M, nrhs, J, Jout);
    MJ_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------- Chebyshev
// Chebyshev iteration (the three-term recurrence of Saad, "Iterative Methods for Sparse Linear
// Systems", Alg. 12.1, with the Jacobi preconditioner) on A y = rhs, for the eigenvalues of
// M^-1 A in [theta - delta, theta + delta]:
//   r_0 = rhs - A y_0,  d_0 = M^-1 r_0 / theta,
//   y_{k+1} = y_k + d_k,  r_{k+1} = r_k - A d_k,  d_{k+1} = c1_k d_k + c2_k M^-1 r_{k+1},
// with c1_k = rho_{k+1} rho_k, c2_k = 2 rho_{k+1} / delta, rho_0 = delta / theta,
// rho_{k+1} = 1 / (2 theta / delta - rho_k): scalars that do not depend on the data, so the
// iteration needs no inner products.  One pass per iteration: A d_k needs d_k at the 26
// neighbours, so d is kept as e = s d in the zero-haloed stencil layout, in two buffers that
// the passes alternate.  Voxels with s = 0 stay out (their e is zero and y is zero).

// Both Chebyshev kernels come in two builds.  OCC holds the registers to 7 waves per SIMD
// (68 VGPRs against 141), which hides more latency once the launch fills the chip (104^3:
// 1.12 against 1.23 ms per solve; 16 right-hand sides at 64^3: 5.98-6.07 against 6.12-6.36 ms).
// On small grids, whose few blocks cannot use the waves, the loads each thread keeps in flight
// matter more (32^3: 0.240 against 0.192 ms, 48^3: 0.272 against 0.258 ms).  The arithmetic is
// the same.
constexpr long kChebOccBlocks = 2048;   // blocks per launch from which OCC is used

// r_0, e_0 and the partial sums of |r_0|^2 and |b|^2
template <bool OCC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC ? 6 : 1))) k_cheb_init(ChebArg a)
{
    const CgArg &g = a.cg;
    const CgBlock cb = cg_block();
    const int r = cb.r + a.rhs0;
    const long M = g.M, base = (long)r * 3 * M;
    const long i = cb.bx * (long)blockDim.x + threadIdx.x;
    double v[2] = {0.0, 0.0};   // rr, bb
    if (i < M) {
        const double s = g.schi[i];
        const long ip = haloed(g, i), bp = (long)r * 3 * g.Mp;
        if (s != 0.0) {
            const double c0 = cg_c0(g, s), md = cg_md(g, s, c0);
            double Ku[3], ctr[3];
            stencil_apply(g, g.uy + bp, ip, Ku, ctr);
            for (int c = 0; c < 3; c++) {
                const long o = base + c * M + i;
                const double b = g.rhs[o];
                const double rv = b - (c0 * g.y[o] - s * Ku[c]);
                a.r[o] = rv;
                a.e_out[bp + c * g.Mp + ip] = s * md * rv * a.inv_theta;
                v[0] += rv * rv;
                v[1] += b * b;
            }
        } else {
            for (int c = 0; c < 3; c++) {
                a.r[base + c * M + i] = 0.0;
                a.e_out[bp + c * g.Mp + ip] = 0.0;
            }
        }
    }
    block_partials<2>(v, g.part + (size_t)r * 3 * gridDim.x, gridDim.x, cb.bx);
}

// one iteration: y += d, r -= A d, d' = c1 d + c2 M^-1 r (partial |r|^2 when asked)
template <bool OCC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC ? 6 : 1))) k_cheb_pass(ChebArg a)
{
    const CgArg &g = a.cg;
    const CgBlock cb = cg_block();
    const int r = cb.r + a.rhs0;
    const long M = g.M, base = (long)r * 3 * M;
    const long i = cb.bx * (long)blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (i < M) {
        const double s = g.schi[i];
        if (s != 0.0) {
            const long ip = haloed(g, i), bp = (long)r * 3 * g.Mp;
            double Ke[3], ectr[3];
            stencil_apply(g, a.e_in + bp, ip, Ke, ectr);
            const double c0 = cg_c0(g, s), md = cg_md(g, s, c0), inv_s = 1.0 / s;
            for (int c = 0; c < 3; c++) {
                const long o = base + c * M + i;
                const double d = ectr[c] * inv_s;
                g.y[o] += d;
                const double rv = a.r[o] - (c0 * d - s * Ke[c]);
                a.r[o] = rv;
                a.e_out[bp + c * g.Mp + ip] = s * (a.c1 * d + a.c2 * md * rv);
                v[0] += rv * rv;
            }
        }
    }
    if (a.want_norm) block_partials<1>(v, g.part + (size_t)r * 3 * gridDim.x, gridDim.x, cb.bx);
}

// One block per right-hand side adds the partials in block order.  NV = 2 after the init pass
// (|r_0|^2, |b|^2), NV = 1 after a pass with want_norm (|r|^2): the status records the test.
template <int NV>
__global__ void __launch_bounds__(1024) k_cheb_reduce(ChebArg a)
{
    __shared__ double sm[16];
    const CgArg &g = a.cg;
    const int r = blockIdx.x + a.rhs0, nb = g.nblk;
    const double *pr = g.part + (size_t)r * 3 * nb;
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) acc[q] = 0.0;
    for (int b = threadIdx.x; b < nb; b += 1024)
#pragma unroll
        for (int q = 0; q < NV; q++) acc[q] += pr[(size_t)q * nb + b];
#pragma unroll
    for (int q = 0; q < NV; q++) acc[q] = block_sum(acc[q], sm);
    if (threadIdx.x != 0) return;
    CgScalars *sc = g.scal + r;
    if constexpr (NV == 2) {
        sc->rr = acc[0];
        sc->bb = acc[1];
        sc->rz[0] = acc[0];   // |r_0|^2, kept for the status of the check
    } else {
        sc->rr = acc[0];
    }
    const double rr = sc->rr, bb = sc->bb;
    const bool pass = rr <= g.tol2 * bb || bb == 0.0;
    g.stat[r] = CgStatus{pass ? 1 : 0, a.passes, bb > 0.0 ? sqrt(rr / bb) : 0.0, bb, sc->rz[0]};
}

// A deterministic pseudo-random right-hand side (values in [-1, 1), zero where s = 0) and a
// zero initial guess, for the spectral estimate of M^-1 A.
__global__ void k_fill_trial(const double *__restrict__ schi, long M, int nrhs, double *__restrict__ rhs,
                             double *__restrict__ y)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= M) return;
    const bool in = schi[i] != 0.0;
    for (int r = 0; r < nrhs; r++)
        for (int c = 0; c < 3; c++) {
            const long o = ((long)r * 3 + c) * M + i;
            unsigned long long x = (unsigned long long)o * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
            x ^= x >> 31;
            x *= 0xBF58476D1CE4E5B9ull;
            x ^= x >> 29;
            rhs[o] = in ? (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0 : 0.0;
            y[o] = 0.0;
        }
}

void launch_fill_trial(const double *schi, long M, int nrhs, double *rhs, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_trial, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, schi, M, nrhs, rhs, y);
    MJ_CHECK(hipGetLastError());
}

void launch_cheb_init(const ChebArg &a, hipStream_t st)
{
    const int nr = a.nr > 0 ? a.nr : a.cg.nrhs;
    if (a.rhs0 < 0 || a.rhs0 + nr > a.cg.nrhs) throw ArgError("Chebyshev launch: right-hand sides out of range");
    if ((long)a.cg.nblk * nr >= kChebOccBlocks)
        hipLaunchKernelGGL(k_cheb_init<true>, dim3(a.cg.nblk, nr), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_cheb_init<false>, dim3(a.cg.nblk, nr), dim3(256), 0, st, a);
    MJ_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_cheb_reduce<2>, dim3(nr), dim3(1024), 0, st, a);
    MJ_CHECK(hipGetLastError());
}
void launch_cheb_pass(const ChebArg &a, hipStream_t st)
{
    const int nr = a.nr > 0 ? a.nr : a.cg.nrhs;
    if (a.rhs0 < 0 || a.rhs0 + nr > a.cg.nrhs) throw ArgError("Chebyshev launch: right-hand sides out of range");
    if ((long)a.cg.nblk * nr >= kChebOccBlocks)
        hipLaunchKernelGGL(k_cheb_pass<true>, dim3(a.cg.nblk, nr), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_cheb_pass<false>, dim3(a.cg.nblk, nr), dim3(256), 0, st, a);
    MJ_CHECK(hipGetLastError());
    if (a.want_norm) {
        hipLaunchKernelGGL(k_cheb_reduce<1>, dim3(nr), dim3(1024), 0, st, a);
        MJ_CHECK(hipGetLastError());
    }
}

// ---------------------------------------------------------------------------- probes
// One wave per chunk (at most kProbeChunk pairs of one row (p, k)): the sources whose lag window
// holds k, each through its window slot k - kmin, against J_{n-k}; lanes take pairs q and q + 64
// together (two independent gathers in flight), and the wave sums in fixed order.
__global__ void __launch_bounds__(256) k_probe_rows(ProbeStepArg a)
{
    const int lane = threadIdx.x & 63;
    const long c = blockIdx.x * 4L + (threadIdx.x >> 6);
    const int r = blockIdx.y;
    if (c >= a.nck) return;
    const int L1 = a.ell + 1;
    const int k = a.ck_row[c] % L1;
    double acc[3] = {0.0, 0.0, 0.0};
    const int j = a.n - k;
    if (j >= 1) {
        const int lo = a.ck_lo[c], hi = a.ck_hi[c];
        const double *J = a.Jring + ((long)(j % a.rdepth) * a.nrhs + r) * 3 * a.M;
        for (int q0 = lo + lane; q0 < hi; q0 += 128) {
            const int q1 = q0 + 64;
            const bool two = q1 < hi;
            const int qb = two ? q1 : q0;
            const int wl0 = k - a.pair_kmin[q0], wl1 = k - a.pair_kmin[qb];
            const long m0 = a.pair_vox[q0], m1 = a.pair_vox[qb];
            const double *K0 = a.table + ((long)wl0 * a.npairs + q0) * 6;
            const double *K1 = a.table + ((long)wl1 * a.npairs + qb) * 6;
            const double x0 = J[m0], y0 = J[a.M + m0], z0 = J[2 * a.M + m0];
            const double x1 = J[m1], y1 = J[a.M + m1], z1 = J[2 * a.M + m1];
            const double f = two ? 1.0 : 0.0;
            acc[0] += K0[0] * x0 + K0[3] * y0 + K0[4] * z0;
            acc[1] += K0[3] * x0 + K0[1] * y0 + K0[5] * z0;
            acc[2] += K0[4] * x0 + K0[5] * y0 + K0[2] * z0;
            acc[0] += f * (K1[0] * x1 + K1[3] * y1 + K1[4] * z1);
            acc[1] += f * (K1[3] * x1 + K1[1] * y1 + K1[5] * z1);
            acc[2] += f * (K1[4] * x1 + K1[5] * y1 + K1[2] * z1);
        }
    }
#pragma unroll
    for (int cc = 0; cc < 3; cc++)
        for (int off = 32; off >= 1; off >>= 1) acc[cc] += __shfl_xor(acc[cc], off);
    if (lane == 0) {
        double *o = a.part + ((long)r * a.nck + c) * 3;
        o[0] = acc[0];
        o[1] = acc[1];
        o[2] = acc[2];
    }
}

// E^s_p(n) = sum over the chunks of probe p (rows k = 0 .. ell in order): one wave per
// (rhs, probe), lane l adds chunks l, l + 64, ... in order, then a fixed butterfly.
__global__ void __launch_bounds__(64) k_probe_sum(ProbeStepArg a)
{
    const int r = blockIdx.x / a.np, p = blockIdx.x % a.np;
    const int lane = threadIdx.x;
    const double *src = a.part + (long)r * a.nck * 3;
    double s[3] = {0.0, 0.0, 0.0};
    for (long i = a.ck_start[p] + lane; i < a.ck_start[p + 1]; i += 64)
#pragma unroll
        for (int cc = 0; cc < 3; cc++) s[cc] += src[3 * i + cc];
#pragma unroll
    for (int cc = 0; cc < 3; cc++)
        for (int off = 32; off >= 1; off >>= 1) s[cc] += __shfl_xor(s[cc], off);
    if (lane == 0)
        for (int cc = 0; cc < 3; cc++) a.out[((long)r * a.np + p) * 3 + cc] = s[cc];
}

void launch_probes(const ProbeStepArg &a, hipStream_t st)
{
    if (a.nck > 0) {
        hipLaunchKernelGGL(k_probe_rows, dim3((unsigned)((a.nck + 3) / 4), a.nrhs), dim3(256), 0, st, a);
        MJ_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_probe_sum, dim3((unsigned)((long)a.nrhs * a.np)), dim3(64), 0, st, a);
    MJ_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------- adjoint
// The march is the block lower-triangular Toeplitz system sum_k Z_k J_{n-k} = E_n
// (eq:MatrixEquation, eq:MOTInversion); its transpose runs backward in time,
//   Z_0^T lambda_j = g_j - sum_{k>=1} Z_k^T lambda_{j+k},  Z_k^T = diag(c_k) - K_k (*) (chi .),
// since every K_k is a symmetric operator (K^ab(D) = K^ba(D) = K^ab(-D)).  With nu = chi lambda
// the sum over k >= 1 is the same spectral history sum as the forward one, in reversed time.
// For the objective Phi = sum_n sum_p |E^s_p(n)|^2 and dc_k/deps = -T(k dt)/eps^2,
// dchi/deps = 1/eps^2, dE_n/deps = <E^i>/eps^2:
//   dPhi/deps_m = sum_n lambda_n(m) . B_n(m) / eps_m^2,
//   B_n = <E^i>(n) + sum_{k=0}^{ell} (T(k dt) J_{n-k} + K_k (*) J_{n-k}).

// (K_0 (*) x)(m) on the plain (non-haloed) layout, with bounds tests
__device__ inline void stencil_plain(const double *K0, const double *__restrict__ x, long M, int U, int V, int W,
                                     int u, int v, int w, double out[3])
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int o = 0; o < 27; o++) {
        const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
        const int su = u - dx, sv = v - dy, sw = w - dz;
        if (su < 0 || su >= U || sv < 0 || sv >= V || sw < 0 || sw >= W) continue;
        const long j = ((long)sw * V + sv) * U + su;
        const double x0 = x[j], x1 = x[M + j], x2 = x[2 * M + j];
        kconst_t *k = kconst(K0) + o * 6;
        a0 += k[0] * x0 + k[3] * x1 + k[4] * x2;
        a1 += k[3] * x0 + k[1] * x1 + k[5] * x2;
        a2 += k[4] * x0 + k[5] * x1 + k[2] * x2;
    }
    out[0] = a0;
    out[1] = a1;
    out[2] = a2;
}

// B_n for every voxel (forward steps of the gradient run).  Jn, Jn1: J_n and J_{n-1}
// ([nrhs][3][M], Jn1 NULL at n = 1); e.S holds sum_{k>=1} K_k (*) J_{n-k} of this step.
__global__ void __launch_bounds__(256) k_grad_term(EpiArg e, const double *__restrict__ Jn,
                                                   const double *__restrict__ Jn1, double *__restrict__ Bout)
{
    const long M = e.M;
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= M) return;
    const int u = (int)(i % e.U), v = (int)((i / e.U) % e.V), w = (int)(i / ((long)e.U * e.V));
    const WaveArg wa = e.waves[r];
    const double avg = wave_average<true>(wa, e, u, v, w, e.n * e.c_dt);
    double k0[3];
    stencil_plain(e.k0, Jn + (long)r * 3 * M, M, e.U, e.V, e.W, u, v, w, k0);
    for (int c = 0; c < 3; c++) {
        const long o = ((long)r * 3 + c) * M + i;
        double b = avg * wa.pol[c] + 0.5 * Jn[o] + k0[c];   // T(0) = T(dt) = 1/2, T(k dt) = 0 for k >= 2
        if (Jn1) b += 0.5 * Jn1[o];
        if (e.S) b += e.S[o];
        Bout[o] = b;
    }
}

// g_j(m) = dPhi/dJ_j(m) = 2 sum_p sum_{k=0}^{ell} K_k(r_p - r_m) E^s_p(j + k), E^s_p(n) = 0 for n > N
__global__ void __launch_bounds__(256) k_adj_source(AdjArg a)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= a.M) return;
    double acc[3] = {0.0, 0.0, 0.0};
    // the voxel-ordered copy of the table: neighbouring lanes read neighbouring records
    for (int p = 0; p < a.np; p++) {
        const int kmin = a.kmin_v[(long)p * a.M + i];
        if (kmin < 0) continue;
        for (int wl = 0; wl < a.nw; wl++) {
            const int jj = a.j + kmin + wl;
            if (jj > a.N) break;
            const double *K = a.table_v + (((long)wl * a.np + p) * a.M + i) * 6;
            const double *E = a.Ehist + (((long)(jj - 1) * a.nrhs + r) * a.np + p) * 3;
            acc[0] += K[0] * E[0] + K[3] * E[1] + K[4] * E[2];
            acc[1] += K[3] * E[0] + K[1] * E[1] + K[5] * E[2];
            acc[2] += K[4] * E[0] + K[5] * E[1] + K[2] * E[2];
        }
    }
    for (int c = 0; c < 3; c++) a.G[((long)r * 3 + c) * a.M + i] = 2.0 * acc[c];
}

__global__ void k_probe_table_by_voxel(const double *__restrict__ table, const int *__restrict__ pair_kmin,
                                       const int *__restrict__ inv, long npairs, int np, int nw, long M,
                                       double *__restrict__ table_v, int *__restrict__ kmin_v)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;   // (wl, p, m)
    if (t >= (long)nw * np * M) return;
    const long pm = t % ((long)np * M);
    const int wl = (int)(t / ((long)np * M));
    const int q = inv[pm];
    double *dst = table_v + t * 6;
    if (q < 0) {
        for (int c = 0; c < 6; c++) dst[c] = 0.0;
        if (wl == 0) kmin_v[pm] = -1;
        return;
    }
    const double *src = table + ((long)wl * npairs + q) * 6;
    for (int c = 0; c < 6; c++) dst[c] = src[c];
    if (wl == 0) kmin_v[pm] = pair_kmin[q];
}

// b'_j = g_j - sum_{k=1}^{nloc} c_k lambda_{j+k} + sum_{k>=1} K_k (*) nu_{j+k}; the solve takes
// A mu = sqrt(chi) b' (Z_0^T = D^-1 A D), started from the extrapolation (weights gx) of mu = nu / sqrt(chi).
// The ring slots count the reversed step n' = N + 1 - j, so "n' - k" is step j + k.
__global__ void __launch_bounds__(256) k_adj_epilogue(EpiArg e)
{
    const long M = e.M;
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= M) return;
    const double sc = e.schi[i];
    const int u = (int)(i % e.U), v = (int)((i / e.U) % e.V), z = (int)(i / ((long)e.U * e.V));
    const double c1 = 0.5 * e.inv_eps[i] + (e.nfir > 1 ? e.fir[1] : 0.0);
    const long Mp = (long)(e.U + 2) * (e.V + 2) * (e.W + 2);
    const long ip = ((long)(z + 1) * (e.V + 2) + (v + 1)) * (e.U + 2) + (u + 1);
    for (int c = 0; c < 3; c++) {
        const long o = ((long)r * 3 + c) * M + i;
        double b = e.G[o] + (e.S ? e.S[o] : 0.0);
        for (int k = 1; k <= e.nloc; k++) {
            if (e.n - k < 1) break;
            const double ck = (k == 1) ? c1 : (k < e.nfir ? e.fir[k] : 0.0);
            if (ck == 0.0) continue;
            b -= ck * e.Lring[(((long)e.slot_of[k] * e.nrhs + r) * 3 + c) * M + i];
        }
        e.bq[o] = b;
        double y0 = 0.0;
        if (sc > 0.0) {
            double g = 0.0;
            for (int k = 1; k <= e.nguess; k++)
                if (e.n - k >= 1) g += e.gx[k - 1] * e.Jring[(((long)e.slot_of[k] * e.nrhs + r) * 3 + c) * M + i];
            y0 = g / sc;
        }
        e.rhs[o] = sc * b;
        e.y[o] = y0;
        e.uy[((long)r * 3 + c) * Mp + ip] = sc * y0;
    }
}

// lambda_j = mu / sqrt(chi) where chi > 0; where chi = 0 the row of Z_0^T reads
// c_0 lambda - K_0 (*) nu = b', so lambda = (b' + K_0 (*) nu) / c_0 there.
__global__ void __launch_bounds__(256) k_adj_lambda(AdjArg a)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= a.M) return;
    const double sc = a.schi[i];
    const long M = a.M;
    if (sc > 0.0) {
        for (int c = 0; c < 3; c++) {
            const long o = ((long)r * 3 + c) * M + i;
            a.lam[o] = a.y[o] / sc;
        }
        return;
    }
    const int u = (int)(i % a.U), v = (int)((i / a.U) % a.V), w = (int)(i / ((long)a.U * a.V));
    double kn[3];
    stencil_plain(a.k0, a.nu + (long)r * 3 * M, M, a.U, a.V, a.W, u, v, w, kn);
    for (int c = 0; c < 3; c++) {
        const long o = ((long)r * 3 + c) * M + i;
        a.lam[o] = (a.bq[o] + kn[c]) / a.c0[i];
    }
}

// grad(m) += sum_r lambda_j(m) . B_j(m) / eps_m^2
__global__ void __launch_bounds__(256) k_grad_accum(AdjArg a)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= a.M) return;
    double s = 0.0;
    for (int r = 0; r < a.nrhs; r++)
        for (int c = 0; c < 3; c++) {
            const long o = ((long)r * 3 + c) * a.M + i;
            s += a.lam[o] * a.Bj[o];
        }
    const double ie = a.inv_eps[i];
    a.grad[i] += s * ie * ie;
}

static dim3 voxel_grid(long M, int nrhs) { return dim3((unsigned)((M + 255) / 256), nrhs); }

void launch_grad_term(const EpiArg &e, const double *Jn, const double *Jn1, double *Bout, hipStream_t st)
{
    hipLaunchKernelGGL(k_grad_term, voxel_grid(e.M, e.nrhs), dim3(256), 0, st, e, Jn, Jn1, Bout);
    MJ_CHECK(hipGetLastError());
}
void launch_probe_table_by_voxel(const double *table, const int *pair_kmin, const int *inv, long npairs, int np,
                                 int nw, long M, double *table_v, int *kmin_v, hipStream_t st)
{
    const long n = (long)nw * np * M;
    hipLaunchKernelGGL(k_probe_table_by_voxel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, table, pair_kmin,
                       inv, npairs, np, nw, M, table_v, kmin_v);
    MJ_CHECK(hipGetLastError());
}

void launch_adj_source(const AdjArg &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_source, voxel_grid(a.M, a.nrhs), dim3(256), 0, st, a);
    MJ_CHECK(hipGetLastError());
}
void launch_adj_epilogue(const EpiArg &e, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_epilogue, voxel_grid(e.M, e.nrhs), dim3(256), 0, st, e);
    MJ_CHECK(hipGetLastError());
}
void launch_adj_lambda(const AdjArg &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_lambda, voxel_grid(a.M, a.nrhs), dim3(256), 0, st, a);
    MJ_CHECK(hipGetLastError());
}
void launch_grad_accum(const AdjArg &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_grad_accum, dim3((unsigned)((a.M + 255) / 256)), dim3(256), 0, st, a);
    MJ_CHECK(hipGetLastError());
}

}  // namespace mj
