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

void or_kernel_entry_h(double r, const double *h, int k, double Dx, double Dy, double Dz, int ngl, double *out);

static const int comp_of[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};

void or_conv_pairs(double r, const double *h, int nlag, const int *tgt, long nt, const int *src, long ns,
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
                double m = d - 1.0 > 0.0 ? (d - 1.0) * h[i] : 0.0;
                a2 += m * m;
                b2 += (d + 1.0) * (d + 1.0) * h[i] * h[i];
            }
            double rmin = sqrt(a2), rmax = sqrt(b2);
            for (int k = 1; k <= nlag; k++) {
                /* the lag's support (r(k-2), r(k+1)) must meet the pair's distances */
                if (!(r * (k + 1) > rmin && r * (k - 2) < rmax)) continue;
                double K[6];
                or_kernel_entry_h(r, h, k, D[0], D[1], D[2], ngl, K);
                const double *J = Js + (long)(k - 1) * 3 * ns;
                for (int b = 0; b < 3; b++)
                    for (int a = 0; a < 3; a++)
                        acc[b] += K[comp_of[b][a]] * J[a * ns + is];
            }
        }
        for (int b = 0; b < 3; b++) out[b * nt + it] = acc[b];
    }
}

/*
 * Kernel values seen from virtual test voxels (side h, centred at arbitrary points: the
 * probes) for a list of source voxels, every lag k = 0..kmax computed on the spot:
 *
 *   out[p][s][k][6] = K_k(r_p - r_s),   r_s = source centre (u + 1/2, v + 1/2, w + 1/2)
 *
 * with zeros outside the lag support of the pair.  The scattered field at the probe is then
 * E^s_p(n) = sum_k sum_s K_k(r_p - r_s) J_{n-k}(s): the scattered-field operator of the
 * formulation (Sec. 2.1) tested like eq:Z on a voxel that is not part of the grid.
 *
 *   probe [np][3]  points in voxel steps per axis from the grid corner
 *   src   [ns][3]  integer voxel coordinates (u, v, w)
 */
void or_probe_kernels(double r, const double *h, int kmax, const double *probe, long np, const int *src, long ns,
                      int ngl, double *out)
{
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (long ip = 0; ip < np; ip++)
        for (long is = 0; is < ns; is++) {
            double D[3], a2 = 0.0, b2 = 0.0;
            for (int i = 0; i < 3; i++) {
                D[i] = probe[3 * ip + i] - ((double)src[3 * is + i] + 0.5);
                double d = fabs(D[i]);
                double m = d - 1.0 > 0.0 ? (d - 1.0) * h[i] : 0.0;
                a2 += m * m;
                b2 += (d + 1.0) * (d + 1.0) * h[i] * h[i];
            }
            double rmin = sqrt(a2), rmax = sqrt(b2);
            double *o = out + ((ip * ns + is) * (long)(kmax + 1)) * 6;
            for (int k = 0; k <= kmax; k++) {
                double *K = o + 6 * k;
                if (!(r * (k + 1) > rmin && r * (k - 2) < rmax)) {
                    for (int c = 0; c < 6; c++) K[c] = 0.0;
                    continue;
                }
                or_kernel_entry_h(r, h, k, D[0], D[1], D[2], ngl, K);
            }
        }
}
