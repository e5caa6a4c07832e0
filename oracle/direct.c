/*
 * ORACLE -- test infrastructure, not product code.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load,
 * call or link this file.  It shares no code with the HIP library.
 *
 * Direct (O(M^2) per lag) evaluation of the spatial convolution part of the
 * history sum of eq:PnMOT (Sec. 2.4):
 *
 *   out^b(m) = sum_{k=1}^{nlag} sum_{m'} sum_a K^{ba}_k(m - m') J^a_{n-k}(m')
 *
 * for target voxels m (all of them, or a list).  No FFT, no blocking, no reordering
 * beyond the plain triple sum.
 *
 * Layouts (all row-major, x fastest):
 *   K   [nlag][6][2W-1][2V-1][2U-1]  lags 1..nlag, components xx,yy,zz,xy,xz,yz,
 *                                     offset D stored at index D + (U-1, V-1, W-1)
 *   Jh  [nlag][3][W][V][U]            Jh[k-1] = J_{n-k}
 *   out [3][ntarget]  (or [3][W][V][U] when targets == NULL)
 */
#include <stddef.h>

static const int comp_of[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};

void or_conv(int U, int V, int W, int nlag, const double *K, const double *Jh,
             const long *targets, long ntargets, double *out)
{
    long M = (long)U * V * W;
    long nx = 2L * U - 1, ny = 2L * V - 1, nz = 2L * W - 1;
    long noff = nx * ny * nz;
    long nt = targets ? ntargets : M;
#pragma omp parallel for schedule(dynamic, 1)
    for (long it = 0; it < nt; it++) {
        long m = targets ? targets[it] : it;
        long u = m % U, v = (m / U) % V, w = m / ((long)U * V);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int k = 1; k <= nlag; k++) {
            const double *Kk = K + (size_t)(k - 1) * 6 * noff;
            const double *Jk = Jh + (size_t)(k - 1) * 3 * M;
            for (long w2 = 0; w2 < W; w2++)
                for (long v2 = 0; v2 < V; v2++)
                    for (long u2 = 0; u2 < U; u2++) {
                        long m2 = (w2 * V + v2) * U + u2;
                        long off = ((w - w2 + W - 1) * ny + (v - v2 + V - 1)) * nx + (u - u2 + U - 1);
                        for (int b = 0; b < 3; b++)
                            for (int a = 0; a < 3; a++)
                                acc[b] += Kk[comp_of[b][a] * noff + off] * Jk[a * M + m2];
                    }
        }
        for (int b = 0; b < 3; b++) out[b * nt + it] = acc[b];
    }
}
