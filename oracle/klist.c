/*
 * ORACLE -- test infrastructure, not product code.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load,
 * call or link this file.  It shares no code with the HIP library.
 *
 * K_k(D) (eq:Z, kquad.c) for a list of (lag, offset) requests, in parallel, with the
 * Huygens support test of the dense table: K_k(D) vanishes unless the lag window
 * (c dt (k - 2), c dt (k + 1)) of the temporal basis meets the range of distances
 * [R_min(D), R_max(D)] between points of the two voxels.
 */
#include <math.h>

void or_kernel_entry_h(double r, const double *h, int k, double Dx, double Dy, double Dz, int ngl, double *out);

/* Distances between points of two voxels at offset D (voxel steps), edges h. */
static void pair_radii(const double D[3], const double h[3], double *rmin, double *rmax)
{
    double a = 0.0, b = 0.0;
    for (int i = 0; i < 3; i++) {
        double d = fabs(D[i]);
        double m = d > 1.0 ? (d - 1.0) * h[i] : 0.0;
        a += m * m;
        b += (d + 1.0) * (d + 1.0) * h[i] * h[i];
    }
    *rmin = sqrt(a);
    *rmax = sqrt(b);
}

/* k[n], D[n][3] -> out[n][6] = {xx, yy, zz, xy, xz, yz}; skip_outside != 0 sets the entries
 * outside the support to exactly 0 without evaluating them. */
void or_kernel_list_h(double r, const double *h, long n, const int *k, const double *D, int ngl, int skip_outside,
                      double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < n; i++) {
        const double *d = D + 3 * i;
        double *o = out + 6 * i;
        for (int c = 0; c < 6; c++) o[c] = 0.0;
        if (skip_outside) {
            double rmin, rmax;
            pair_radii(d, h, &rmin, &rmax);
            if (!(r * (k[i] + 1) > rmin && r * (k[i] - 2) < rmax)) continue;
        }
        or_kernel_entry_h(r, h, k[i], d[0], d[1], d[2], ngl, o);
    }
}
