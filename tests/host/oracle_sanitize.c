/* Test harness: every entry point of the CPU oracle on small inputs, built with AddressSanitizer
 * and UndefinedBehaviorSanitizer by tests/test_sanitizers.py.  Prints a checksum; any invalid
 * access or undefined operation aborts the run. */
#include <stdio.h>
#include <stdlib.h>

void or_kernel_entry_h(double r, const double *h, int k, double Dx, double Dy, double Dz, int ngl, double *out);
void or_kernel_table_h(double r, const double *h, int U, int V, int W, int kmax, int ngl, int skip_outside,
                       double *K);
void or_conv(int U, int V, int W, int nlag, const double *K, const double *Jh, const long *targets, long ntargets,
             double *out);
void or_conv_pairs(double r, const double *h, int nlag, const int *tgt, long nt, const int *src, long ns,
                   const double *Js, int ngl, double *out);
void or_probe_kernels(double r, const double *h, int kmax, const double *probe, long np, const int *src, long ns,
                      int ngl, double *out);

int main(void)
{
    const int U = 3, V = 2, W = 2, kmax = 6, ngl = 8;
    const double hs[2][3] = {{1.0, 1.0, 1.0}, {1.0, 0.7, 1.3}};
    const double rs[2] = {1.0, 0.6};
    double sum = 0.0;
    for (int g = 0; g < 2; g++) {
        const double *h = hs[g];
        const double r = rs[g];
        double K6[6];
        or_kernel_entry_h(r, h, 2, 1.3, -0.7, 0.45, ngl, K6);
        for (int c = 0; c < 6; c++) sum += K6[c];
        const long noff = (2L * U - 1) * (2L * V - 1) * (2L * W - 1);
        double *K = calloc((size_t)(kmax + 1) * 6 * noff, sizeof(double));
        or_kernel_table_h(r, h, U, V, W, kmax, ngl, 1, K);
        const long M = (long)U * V * W;
        double *Jh = malloc(sizeof(double) * (size_t)kmax * 3 * M);
        for (long i = 0; i < (long)kmax * 3 * M; i++) Jh[i] = (double)((i * 7919) % 101) / 101.0 - 0.5;
        double *out = calloc((size_t)3 * M, sizeof(double));
        or_conv(U, V, W, kmax, K + 6 * noff, Jh, NULL, 0, out);
        for (long i = 0; i < 3 * M; i++) sum += out[i];
        int tgt[6] = {0, 0, 0, 2, 1, 1}, src[9] = {1, 0, 0, 0, 1, 1, 2, 1, 0};
        double Js[3 * 3 * 3], outp[3 * 2];
        for (int i = 0; i < 27; i++) Js[i] = 0.1 * i - 1.0;
        or_conv_pairs(r, h, 3, tgt, 2, src, 3, Js, ngl, outp);
        for (int i = 0; i < 6; i++) sum += outp[i];
        double probe[6] = {4.2, 1.0, 1.0, -1.5, 0.5, 2.5};
        double *pk = calloc((size_t)2 * 3 * (kmax + 1) * 6, sizeof(double));
        or_probe_kernels(r, h, kmax, probe, 2, src, 3, ngl, pk);
        for (int i = 0; i < 2 * 3 * (kmax + 1) * 6; i++) sum += pk[i];
        free(K);
        free(Jh);
        free(out);
        free(pk);
    }
    printf("checksum %.17g\n", sum);
    return 0;
}
