// reduce.hip -- FP64 reductions and band scaling around the V_loc path.
//
// For E = sum_n w_n Re <c_n | V c_n> (the local-potential energy of weighted
// bands):
//   e_n    = Re sum_g conj(c_n(g)) out_n(g)              (band_dot, FP64)
//   E      = sum_n w_n e_n                               (weighted_sum, FP64)
//   dE/dV  = (1/N) sum_n w_n |psi_n(j)|^2                (density_reduce of the
//            partial planes the plane kernel accumulates in FP64)
//   dE/dc_n = 2 w_n (V c_n)(g)                           (scale_bands)
// All sums run in a fixed order (no atomics), so results are reproducible.
#include "kernels.hpp"

namespace vloc {

template <typename T>
struct Cplx;
template <>
struct Cplx<double> {
    using type = double2;
};
template <>
struct Cplx<float> {
    using type = float2;
};

__global__ void k_fill_f64(double *x, long long n, double v)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ void k_scale_real(const double *__restrict__ x, long long n,
                             const double *__restrict__ scale, double factor,
                             double *__restrict__ y)
{
    const double f = factor * (scale ? scale[0] : 1.0);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = f * x[i];
}

// rho[j] += scale * inv_n * sum_{s < nsub} partial[s][j'], s ascending, where
// j = (z, y, x) and j' is j itself, or with full != 0 the full-plane kernel's
// index (z, x, yp), yp = L2y (y mod L1y) + y / L1y.
__global__ void k_density_reduce(const double *__restrict__ partial, int nsub, int N1, int N2,
                                 int N3, int full, int L1y, int L2y, double inv_n,
                                 const double *__restrict__ scale, double *__restrict__ rho)
{
    const double f = inv_n * (scale ? scale[0] : 1.0);
    const long long n = (long long)N1 * N2 * N3;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        long long src = i;
        if (full) {
            const long long zy = i / N1;
            const int x = (int)(i - zy * N1);
            const long long z = zy / N2;
            const int y = (int)(zy - z * N2);
            const int yp = L2y * (y % L1y) + y / L1y;
            src = (z * N1 + x) * N2 + yp;
        }
        double acc = 0.0;
        for (int s = 0; s < nsub; ++s) acc += partial[(long long)s * n + src];
        rho[i] += f * acc;
    }
}

// Fixed-order tree sum of one value per thread over a 256-thread block.
__device__ double block_sum_256(double v, double *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    return sh[0];
}

// out[n] = Re sum_g conj(a[n][g]) b[n][g]: one block per band, FP64.  Each
// thread keeps four partial sums (coefficients g, g + 256, g + 512, g + 768 of
// each 1024-wide step), so that eight loads are in flight per thread instead of
// one dependent chain; the partial sums and the block tree combine in a fixed
// order (the result does not depend on timing).
template <typename T>
__global__ __launch_bounds__(256) void k_band_dot(const typename Cplx<T>::type *__restrict__ a,
                                                  const typename Cplx<T>::type *__restrict__ b,
                                                  long long npw, double *__restrict__ out)
{
    __shared__ double sh[256];
    const long long base = (long long)blockIdx.x * npw;
    const auto *pa = a + base;
    const auto *pb = b + base;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    long long g = threadIdx.x;
    for (; g + 768 < npw; g += 1024) {
        typename Cplx<T>::type x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            x[u] = pa[g + 256 * u];
            y[u] = pb[g + 256 * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            acc[u] += (double)x[u].x * (double)y[u].x + (double)x[u].y * (double)y[u].y;
    }
    // at most three coefficients remain
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        const long long gu = g + 256 * u;
        if (gu < npw) {
            const auto x = pa[gu];
            const auto y = pb[gu];
            acc[u] += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
        }
    }
    const double s = block_sum_256((acc[0] + acc[1]) + (acc[2] + acc[3]), sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// out[0] = sum_n w[n] x[n], one block, fixed order.
__global__ __launch_bounds__(256) void k_weighted_sum(const double *__restrict__ x,
                                                      const double *__restrict__ w, long long n,
                                                      double *__restrict__ out)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) acc += w[i] * x[i];
    const double s = block_sum_256(acc, sh);
    if (threadIdx.x == 0) out[0] = s;
}

// y[n][g] = factor * scale * w[n] * x[n][g] (w, scale may be NULL = 1).  Block
// b covers 1024 coefficients of band b / bpb (bpb blocks per band): the band
// and its factor are uniform per block, and each thread moves four elements.
template <typename T>
__global__ __launch_bounds__(256) void k_scale_bands(const typename Cplx<T>::type *__restrict__ x,
                                                     long long npw, unsigned bpb,
                                                     const double *__restrict__ w,
                                                     const double *__restrict__ scale,
                                                     double factor,
                                                     typename Cplx<T>::type *__restrict__ y)
{
    const unsigned n = blockIdx.x / bpb, part = blockIdx.x - n * bpb;
    const T f = (T)(factor * (scale ? scale[0] : 1.0) * (w ? w[n] : 1.0));
    const long long base = (long long)n * npw;
    const long long g0 = (long long)part * 1024 + threadIdx.x;
    typename Cplx<T>::type v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (g0 + 256 * u < npw) v[u] = x[base + g0 + 256 * u];
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (g0 + 256 * u < npw) {
            v[u].x *= f;
            v[u].y *= f;
            y[base + g0 + 256 * u] = v[u];
        }
}

static unsigned grid_for(long long n, unsigned cap = 4096)
{
    long long b = (n + 255) / 256;
    if (b < 1) b = 1;
    return (unsigned)(b < cap ? b : cap);
}

hipError_t launch_fill_f64(double *x, int64_t n, double v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(256), 0, st, x, (long long)n, v);
    return hipGetLastError();
}

hipError_t launch_scale_real(const double *x, int64_t n, const double *scale, double factor,
                             double *y, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_real, dim3(grid_for(n)), dim3(256), 0, st, x, (long long)n, scale,
                       factor, y);
    return hipGetLastError();
}

hipError_t launch_density_reduce(const Geometry &g, const double *partial, int nsub,
                                 const double *scale, double *rho, hipStream_t st)
{
    const int64_t n = (int64_t)g.N1 * g.N2 * g.N3;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_density_reduce, dim3(grid_for(n)), dim3(256), 0, st, partial, nsub,
                       g.N1, g.N2, g.N3, g.full, g.L1y, g.L2y, g.inv_n, scale, rho);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_band_dot(const void *a, const void *b, int64_t npw, int64_t nb, double *out,
                           hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    using C = typename Cplx<T>::type;
    hipLaunchKernelGGL(k_band_dot<T>, dim3((unsigned)nb), dim3(256), 0, st,
                       reinterpret_cast<const C *>(a), reinterpret_cast<const C *>(b),
                       (long long)npw, out);
    return hipGetLastError();
}

hipError_t launch_weighted_sum(const double *x, const double *w, int64_t n, double *out,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_weighted_sum, dim3(1), dim3(256), 0, st, x, w, (long long)n, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_bands(const void *x, int64_t npw, int64_t nb, const double *w,
                              const double *scale, double factor, void *y, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    using C = typename Cplx<T>::type;
    if (npw <= 0) return hipSuccess;
    const int64_t bpb = (npw + 1023) / 1024;
    if (bpb * nb > 0x7FFFFFFFLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scale_bands<T>, dim3((unsigned)(bpb * nb)), dim3(256), 0, st,
                       reinterpret_cast<const C *>(x), (long long)npw, (unsigned)bpb, w, scale,
                       factor, reinterpret_cast<C *>(y));
    return hipGetLastError();
}

template hipError_t launch_band_dot<double>(const void *, const void *, int64_t, int64_t,
                                            double *, hipStream_t);
template hipError_t launch_band_dot<float>(const void *, const void *, int64_t, int64_t,
                                           double *, hipStream_t);
template hipError_t launch_scale_bands<double>(const void *, int64_t, int64_t, const double *,
                                               const double *, double, void *, hipStream_t);
template hipError_t launch_scale_bands<float>(const void *, int64_t, int64_t, const double *,
                                              const double *, double, void *, hipStream_t);

} // namespace vloc
