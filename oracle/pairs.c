/*
 * ORACLE -- test infrastructure, not product code.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load,
 * call or link this file.  It shares no code with the HIP library.
 *
 * Direct history convolution for a sparse set of source voxels and a list of target
 * voxels, with every kernel value computed on the spot (eq:PnMOT restricted to the
 * given sources; used where a full kernel table is too large to build):
 *
 *   out^b(t) = sum_{k=1}^{nlag} sum_{s} sum_a K^{ba}_k(r_t - r_s) J^a_{n-k}(s)
 *
 *   tgt [nt][3], src [ns][3]  integer voxel coordinates (u, v, w)
 *   Js  [nlag][3][ns]         Js[k-1] = J_{n-k} at the sources
 *   out [3][nt]
 */
#include <math.h>
#include <stdlib.h>

void or_kernel_entry(double r, int k, double Dx, double Dy, double Dz, int ngl, double *out);

static const int comp_of[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};

void or_conv_pairs(double r, int nlag, const int *tgt, long nt, const int *src, long ns,
                   const double *Js, int ngl, double *out)
{
    for (long i = 0; i < 3 * nt; i++) out[i] = 0.0;
#pragma omp parallel for schedule(dynamic, 1)
    for (long it = 0; it < nt; it++) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (long is = 0; is < ns; is++) {
            double D[3];
            double a2 = 0.0, b2 = 0.0;
            for (int i = 0; i < 3; i++) {
                D[i] = (double)(tgt[3 * it + i] - src[3 * is + i]);
                double d = fabs(D[i]);
                double m = d - 1.0 > 0.0 ? d - 1.0 : 0.0;
                a2 += m * m;
                b2 += (d + 1.0) * (d + 1.0);
            }
            double rmin = sqrt(a2), rmax = sqrt(b2);
            for (int k = 1; k <= nlag; k++) {
                /* the lag's support (r(k-2), r(k+1)) must meet the pair's distances */
                if (!(r * (k + 1) > rmin && r * (k - 2) < rmax)) continue;
                double K[6];
                or_kernel_entry(r, k, D[0], D[1], D[2], ngl, K);
                const double *J = Js + (long)(k - 1) * 3 * ns;
                for (int b = 0; b < 3; b++)
                    for (int a = 0; a < 3; a++)
                        acc[b] += K[comp_of[b][a]] * J[a * ns + is];
            }
        }
        for (int b = 0; b < 3; b++) out[b * nt + it] = acc[b];
    }
}
