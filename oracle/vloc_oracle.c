/*
 * vloc_oracle.c -- plain, slow, obviously-correct FP64 CPU oracle for the
 * action of a local potential on plane-wave wave functions.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * constant with the GPU path.
 *
 * What it computes (Gao, Mo, Fang, Wang, "Parallel 3-dim FFTs with load
 * balancing of the plane waves"):
 *   - the cutoff sphere S = { g in Z^3 : |k+G|^2 <= 2 Ecut (1 + 1e-12) }
 *     with G = h b1 + k b2 + l b3 and b = 2 pi A^{-T}   (Sec. 2, eq. 3;
 *     the non-strict inequality plus relative slack is this library's reading
 *     of the boundary, see the design notes);
 *   - the plane-wave expansion onto the grid (Sec. 2, eq. 2):
 *       psi(j) = sum_{g in S} c(g) exp(-2 pi i (h j1/N1 + k j2/N2 + l j3/N3));
 *     the factor exp(-i k.r) cancels between the two transforms because V is
 *     lattice periodic, so only the periodic part is transformed;
 *   - the local-potential action (Sec. 2, the paragraph after eq. 3: transform
 *     to real space, multiply by the diagonal V, transform back):
 *       out(g) = (1/N) sum_j exp(+2 pi i (h j1/N1 + k j2/N2 + l j3/N3)) V(j) psi(j).
 *   Real-space arrays are stored [N3][N2][N1] with x (j1) fastest.
 *
 * The 3-D transform is done the textbook way: the full cube is zeroed, the
 * sphere is scattered to (h mod N1, k mod N2, l mod N3), and three unpruned
 * passes of 1-D DFTs run along x, y and z (Sec. 3.2: a 3-D FFT is three sets of
 * 1-D FFTs).  The 1-D DFT is a recursive decimation-in-time mixed-radix
 * transform that splits off the smallest prime factor and falls back to the
 * O(L^2) definition for any prime.  Twiddles are cos/sin of the angle whose
 * integer numerator is reduced modulo L first.  No pruning, no fusion.
 *
 * `sign` selects the transform convention: sign = -1 is the paper's (eq. 2,
 * exp(-i ...) from G to r); sign = +1 flips both exponents (used only to check
 * the reflection identity).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cplx;

static const double TWO_PI = 6.283185307179586476925286766559;

/* exp(sign * 2 pi i * num / L), num reduced exactly modulo L first. */
static cplx twiddle(long num, long L, int sign)
{
    long j = num % L;
    if (j < 0) j += L;
    double a = TWO_PI * (double)j / (double)L;
    cplx w = { cos(a), (double)sign * sin(a) };
    return w;
}

static long smallest_factor(long L)
{
    if (L % 2 == 0) return 2;
    if (L % 3 == 0) return 3;
    if (L % 5 == 0) return 5;
    for (long p = 7; p * p <= L; p += 2)
        if (L % p == 0) return p;
    return L; /* prime: the combine step below is then the plain DFT */
}

/* out[k'] = sum_n in[n*is] exp(sign 2 pi i n k'/L), k' in [0, L).
 * Decimation in time: n = p n' + r, X[k + q m] = sum_r W^{r(k+qm)} Y_r[k]. */
static void fft_rec(const cplx *in, long is, cplx *out, long L, int sign)
{
    if (L == 1) { out[0] = in[0]; return; }
    long p = smallest_factor(L);
    long m = L / p;
    for (long r = 0; r < p; r++)
        fft_rec(in + r * is, is * p, out + r * m, m, sign);
    cplx *y = (cplx *)malloc(sizeof(cplx) * (size_t)p);
    for (long k = 0; k < m; k++) {
        for (long r = 0; r < p; r++) y[r] = out[r * m + k];
        for (long q = 0; q < p; q++) {
            double sr = 0.0, si = 0.0;
            for (long r = 0; r < p; r++) {
                cplx w = twiddle(r * (k + q * m), L, sign);
                sr += w.re * y[r].re - w.im * y[r].im;
                si += w.re * y[r].im + w.im * y[r].re;
            }
            out[k + q * m].re = sr;
            out[k + q * m].im = si;
        }
    }
    free(y);
}

/* One 1-D transform, exported so tests can pin it directly. */
int oracle_fft1d(const double *in, double *out, long L, int sign)
{
    if (!in || !out || L < 1 || (sign != 1 && sign != -1)) return -1;
    fft_rec((const cplx *)in, 1, (cplx *)out, L, sign);
    return 0;
}

/* ---------------------------------------------------------------- sphere */

/* B rows b_j with a_i . b_j = 2 pi delta_ij, i.e. B = 2 pi (A^{-1})^T. */
static int reciprocal(const double A[9], double B[9], double *det_out)
{
    double det = A[0] * (A[4] * A[8] - A[5] * A[7])
               - A[1] * (A[3] * A[8] - A[5] * A[6])
               + A[2] * (A[3] * A[7] - A[4] * A[6]);
    *det_out = det;
    if (!(det > 0.0) || !isfinite(det)) return -1;
    /* inverse via cofactors: inv[i][j] = cof[j][i] / det; B[j][i] = 2pi inv[i][j] */
    double cof[9];
    cof[0] =  (A[4] * A[8] - A[5] * A[7]);
    cof[1] = -(A[3] * A[8] - A[5] * A[6]);
    cof[2] =  (A[3] * A[7] - A[4] * A[6]);
    cof[3] = -(A[1] * A[8] - A[2] * A[7]);
    cof[4] =  (A[0] * A[8] - A[2] * A[6]);
    cof[5] = -(A[0] * A[7] - A[1] * A[6]);
    cof[6] =  (A[1] * A[5] - A[2] * A[4]);
    cof[7] = -(A[0] * A[5] - A[2] * A[3]);
    cof[8] =  (A[0] * A[4] - A[1] * A[3]);
    /* (A^{-1})^T = cof / det */
    for (int i = 0; i < 9; i++) B[i] = TWO_PI * cof[i] / det;
    return 0;
}

/* Enumerate S in lexicographic (h, k, l) order.  Returns the count, or -1 on a
 * bad cell / cutoff.  hkl (3 ints per point) may be NULL to only count; at
 * most `cap` points are written. */
long oracle_sphere(const double cell[9], double ecut, const double kpt[3],
                   int32_t *hkl, long cap)
{
    double B[9], det;
    if (!cell || !kpt || !(ecut >= 0.0) || !isfinite(ecut)) return -1;
    if (reciprocal(cell, B, &det) != 0) return -1;
    double gcut2 = 2.0 * ecut;
    double lim2 = gcut2 * (1.0 + 1e-12);
    double gcut = sqrt(gcut2);
    long lo[3], hi[3];
    for (int i = 0; i < 3; i++) {
        double alen = sqrt(cell[3 * i] * cell[3 * i] + cell[3 * i + 1] * cell[3 * i + 1]
                           + cell[3 * i + 2] * cell[3 * i + 2]);
        double ext = gcut * alen / TWO_PI * (1.0 + 1e-9) + 1e-9;
        lo[i] = (long)floor(-ext - kpt[i]) - 1;
        hi[i] = (long)ceil(ext - kpt[i]) + 1;
    }
    long n = 0;
    for (long h = lo[0]; h <= hi[0]; h++)
        for (long k = lo[1]; k <= hi[1]; k++)
            for (long l = lo[2]; l <= hi[2]; l++) {
                double f0 = (double)h + kpt[0], f1 = (double)k + kpt[1], f2 = (double)l + kpt[2];
                double gx = f0 * B[0] + f1 * B[3] + f2 * B[6];
                double gy = f0 * B[1] + f1 * B[4] + f2 * B[7];
                double gz = f0 * B[2] + f1 * B[5] + f2 * B[8];
                double g2 = gx * gx + gy * gy + gz * gz;
                if (g2 <= lim2) {
                    if (hkl && n < cap) {
                        hkl[3 * n] = (int32_t)h;
                        hkl[3 * n + 1] = (int32_t)k;
                        hkl[3 * n + 2] = (int32_t)l;
                    }
                    n++;
                }
            }
    return n;
}

/* ------------------------------------------------------------ transforms */

static long wrap(long v, long n) { long r = v % n; return r < 0 ? r + n : r; }

/* In-place 3-D transform of a [N3][N2][N1] cube: x lines, then y, then z. */
static void fft3d(cplx *cube, const int grid[3], int sign)
{
    long N1 = grid[0], N2 = grid[1], N3 = grid[2];
    long Lmax = N1 > N2 ? N1 : N2;
    if (N3 > Lmax) Lmax = N3;
    cplx *a = (cplx *)malloc(sizeof(cplx) * (size_t)Lmax);
    cplx *b = (cplx *)malloc(sizeof(cplx) * (size_t)Lmax);
    for (long z = 0; z < N3; z++)
        for (long y = 0; y < N2; y++) {
            cplx *line = cube + (z * N2 + y) * N1;
            memcpy(a, line, sizeof(cplx) * (size_t)N1);
            fft_rec(a, 1, b, N1, sign);
            memcpy(line, b, sizeof(cplx) * (size_t)N1);
        }
    for (long z = 0; z < N3; z++)
        for (long x = 0; x < N1; x++) {
            for (long y = 0; y < N2; y++) a[y] = cube[(z * N2 + y) * N1 + x];
            fft_rec(a, 1, b, N2, sign);
            for (long y = 0; y < N2; y++) cube[(z * N2 + y) * N1 + x] = b[y];
        }
    for (long y = 0; y < N2; y++)
        for (long x = 0; x < N1; x++) {
            for (long z = 0; z < N3; z++) a[z] = cube[(z * N2 + y) * N1 + x];
            fft_rec(a, 1, b, N3, sign);
            for (long z = 0; z < N3; z++) cube[(z * N2 + y) * N1 + x] = b[z];
        }
    free(a);
    free(b);
}

typedef struct {
    long npw;
    int32_t *hkl;
    long *pos; /* flat grid index of each sphere point */
} sphere_t;

/* Own sphere plus the grid position of each point; fails when two points of
 * the sphere land on the same grid point (the grid is too small). */
static int sphere_on_grid(const int grid[3], const double cell[9], double ecut,
                          const double kpt[3], sphere_t *s)
{
    if (!grid || grid[0] < 1 || grid[1] < 1 || grid[2] < 1) return -1;
    long n = oracle_sphere(cell, ecut, kpt, NULL, 0);
    if (n < 0) return -1;
    s->npw = n;
    s->hkl = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(n > 0 ? n : 1));
    s->pos = (long *)malloc(sizeof(long) * (size_t)(n > 0 ? n : 1));
    oracle_sphere(cell, ecut, kpt, s->hkl, n);
    long N = (long)grid[0] * grid[1] * grid[2];
    unsigned char *seen = (unsigned char *)calloc((size_t)N, 1);
    int ok = 0;
    for (long i = 0; i < n; i++) {
        long x = wrap(s->hkl[3 * i], grid[0]);
        long y = wrap(s->hkl[3 * i + 1], grid[1]);
        long z = wrap(s->hkl[3 * i + 2], grid[2]);
        long p = (z * grid[1] + y) * grid[0] + x;
        if (seen[p]) ok = -2;
        seen[p] = 1;
        s->pos[i] = p;
    }
    free(seen);
    if (ok != 0) { free(s->hkl); free(s->pos); }
    return ok;
}

static void sphere_free(sphere_t *s) { free(s->hkl); free(s->pos); }

static int threads_or_default(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* psi[b] = full grid of band b (N complex per band), G -> r with `sign`. */
int oracle_g2r(const int grid[3], const double cell[9], double ecut, const double kpt[3],
               int sign, const double *c, long nbands, double *psi, int nthreads)
{
    sphere_t s;
    if (sign != 1 && sign != -1) return -1;
    int rc = sphere_on_grid(grid, cell, ecut, kpt, &s);
    if (rc) return rc;
    long N = (long)grid[0] * grid[1] * grid[2];
    int nt = threads_or_default(nthreads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (long b = 0; b < nbands; b++) {
        cplx *cube = (cplx *)psi + b * N;
        const cplx *cb = (const cplx *)c + b * s.npw;
        memset(cube, 0, sizeof(cplx) * (size_t)N);
        for (long i = 0; i < s.npw; i++) cube[s.pos[i]] = cb[i];
        fft3d(cube, grid, sign);
    }
    sphere_free(&s);
    return 0;
}

/* c_out[b][g] = (1/N) sum_j exp(-sign ...) psi[b](j), gathered on the sphere. */
int oracle_r2g(const int grid[3], const double cell[9], double ecut, const double kpt[3],
               int sign, const double *psi, long nbands, double *c_out, int nthreads)
{
    sphere_t s;
    if (sign != 1 && sign != -1) return -1;
    int rc = sphere_on_grid(grid, cell, ecut, kpt, &s);
    if (rc) return rc;
    long N = (long)grid[0] * grid[1] * grid[2];
    int nt = threads_or_default(nthreads);
#pragma omp parallel num_threads(nt)
    {
        cplx *cube = (cplx *)malloc(sizeof(cplx) * (size_t)N);
#pragma omp for schedule(dynamic, 1)
        for (long b = 0; b < nbands; b++) {
            memcpy(cube, (const cplx *)psi + b * N, sizeof(cplx) * (size_t)N);
            fft3d(cube, grid, -sign);
            cplx *ob = (cplx *)c_out + b * s.npw;
            for (long i = 0; i < s.npw; i++) {
                ob[i].re = cube[s.pos[i]].re / (double)N;
                ob[i].im = cube[s.pos[i]].im / (double)N;
            }
        }
        free(cube);
    }
    sphere_free(&s);
    return 0;
}

/* out[b] = gather( (1/N) FFT_{-sign}( V * FFT_{sign}( scatter(c[b]) ) ) ). */
int oracle_apply(const int grid[3], const double cell[9], double ecut, const double kpt[3],
                 int sign, const double *c, long nbands, const double *V, double *out,
                 int nthreads)
{
    sphere_t s;
    if (sign != 1 && sign != -1) return -1;
    int rc = sphere_on_grid(grid, cell, ecut, kpt, &s);
    if (rc) return rc;
    long N = (long)grid[0] * grid[1] * grid[2];
    int nt = threads_or_default(nthreads);
#pragma omp parallel num_threads(nt)
    {
        cplx *cube = (cplx *)malloc(sizeof(cplx) * (size_t)N);
#pragma omp for schedule(dynamic, 1)
        for (long b = 0; b < nbands; b++) {
            const cplx *cb = (const cplx *)c + b * s.npw;
            memset(cube, 0, sizeof(cplx) * (size_t)N);
            for (long i = 0; i < s.npw; i++) cube[s.pos[i]] = cb[i];
            fft3d(cube, grid, sign);
            for (long j = 0; j < N; j++) {
                cube[j].re *= V[j];
                cube[j].im *= V[j];
            }
            fft3d(cube, grid, -sign);
            cplx *ob = (cplx *)out + b * s.npw;
            for (long i = 0; i < s.npw; i++) {
                ob[i].re = cube[s.pos[i]].re / (double)N;
                ob[i].im = cube[s.pos[i]].im / (double)N;
            }
        }
        free(cube);
    }
    sphere_free(&s);
    return 0;
}

int oracle_max_threads(void) { return threads_or_default(0); }
