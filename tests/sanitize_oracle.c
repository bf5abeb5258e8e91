/* The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (gcc):
 * 1-D transforms of every length 1..130, a sphere count, and one application
 * of the operator with a constant potential (out = v0 c).  Exits non-zero on a
 * failed check; the sanitizers abort on their own findings. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_fft1d(const double *in, double *out, long L, int sign);
long oracle_sphere(const double cell[9], double ecut, const double kpt[3], int *hkl, long cap);
int oracle_apply(const int grid[3], const double cell[9], double ecut, const double kpt[3],
                 int sign, const double *c, long nb, const double *V, double *out, int nthreads);

int main(void)
{
    int fail = 0;
    for (long L = 1; L <= 130; ++L) {
        double *x = malloc(sizeof(double) * 2 * L), *y = malloc(sizeof(double) * 2 * L);
        for (long i = 0; i < 2 * L; ++i) x[i] = (i == 2) ? 1.0 : 0.0; /* delta at n = 1 */
        if (oracle_fft1d(x, y, L, -1) != 0) fail = 1;
        if (L > 1) {
            /* DFT of a delta at n = 1 is exp(-2 pi i k / L) */
            for (long k = 0; k < L; ++k) {
                double a = 6.283185307179586 * (double)k / (double)L;
                if (fabs(y[2 * k] - cos(a)) > 1e-13 || fabs(y[2 * k + 1] + sin(a)) > 1e-13) fail = 1;
            }
        }
        free(x);
        free(y);
    }
    const double tp = 6.283185307179586476925286766559;
    double cell[9] = {tp, 0, 0, 0, tp, 0, 0, 0, tp}, k[3] = {0, 0, 0};
    long npw = oracle_sphere(cell, 18.0, k, NULL, 0);
    if (npw != 925) fail = 1;
    int *hkl = malloc(sizeof(int) * 3 * (size_t)npw);
    oracle_sphere(cell, 18.0, k, hkl, npw);
    int grid[3] = {24, 24, 24};
    long N = 24L * 24 * 24, nb = 2;
    double *c = malloc(sizeof(double) * 2 * (size_t)(npw * nb));
    double *out = malloc(sizeof(double) * 2 * (size_t)(npw * nb));
    double *V = malloc(sizeof(double) * (size_t)N);
    for (long i = 0; i < 2 * npw * nb; ++i) c[i] = sin(0.37 * (double)i);
    for (long i = 0; i < N; ++i) V[i] = 2.5;
    if (oracle_apply(grid, cell, 18.0, k, -1, c, nb, V, out, 1) != 0) fail = 1;
    for (long i = 0; i < 2 * npw * nb; ++i)
        if (fabs(out[i] - 2.5 * c[i]) > 1e-13) fail = 1;
    free(hkl);
    free(c);
    free(out);
    free(V);
    printf("%s\n", fail ? "FAILED" : "OK");
    return fail;
}
