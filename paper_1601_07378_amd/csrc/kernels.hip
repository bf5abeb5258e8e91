// kernels.hip -- the compact 3-D transform pair around the local potential,
// written for gfx950 (64-wide wavefronts, 160 KiB LDS per CU).
//
// Paper mapping (Gao, Mo, Fang, Wang, arXiv:1601.07378):
//   - eq. 2 fixes the sign: G -> r uses exp(-2 pi i ...), unnormalised;
//     r -> G uses exp(+2 pi i ...) and 1/N;
//   - Sec. 2 (after eq. 3): transform, multiply by the diagonal V, transform back;
//   - Sec. 4.3 (compact 3-D FFT): the first 1-D pass runs only on the columns
//     meeting the sphere (here z-sticks, kernel K1), the second only on the
//     columns meeting that cylinder (here the occupied x-planes of each
//     z-plane, kernel K2), the third on the whole plane (K2's x pass).  The
//     reverse transform mirrors it and only the needed outputs are kept.
//   - Sec. 3.2 (greedy): sticks are dealt to workgroups by descending
//     plane-wave count; the deal is made on the host (plan.cpp).
//
// Every 1-D transform of length L = L1*L2 is done in two register stages:
//   forward  A : task n2 takes x[n2 + L2 n1] (n1 < L1), runs an L1-point DFT,
//                multiplies output k1 by W_L^{n2 k1} and stores it at n2 + L2 k1;
//            B : task k1 takes the L2 contiguous values at L2 k1 + n2, runs an
//                L2-point DFT; output k2 is frequency k1 + L1 k2, kept at
//                position L2 k1 + k2 ("transposed order");
//   reverse  B': the same L2-point step on transposed input;
//            A': task n2 takes positions n2 + L2 k1, multiplies by W_L^{n2 k1},
//                runs the L1-point DFT and stores x[n2 + L2 n1] in natural order.
// Between A and B (and B' and A') values cross threads through LDS.
#include <type_traits>

#include "dft_codelets.h"
#include "kernels.hpp"

namespace vloc {

template <typename T>
struct Cx;
template <>
struct Cx<double> {
    using type = double2;
};
template <>
struct Cx<float> {
    using type = float2;
};
template <typename T>
using cx = typename Cx<T>::type;

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b)
{
    cx<T> v;
    v.x = a;
    v.y = b;
    return v;
}

// Calls f with a compile-time codelet size equal to the runtime r.
template <typename F>
__device__ __forceinline__ void with_codelet(int r, F &&f)
{
    switch (r) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 10: f(std::integral_constant<int, 10>{}); break;
    case 12: f(std::integral_constant<int, 12>{}); break;
    case 15: f(std::integral_constant<int, 15>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: break;
    }
}

// x[k1] *= W_L^{S n2 k1}; the table holds exp(-2 pi i j / L) and n2 k1 < L.
template <int R, int S, typename T>
__device__ __forceinline__ void twiddle(T *xr, T *xi, int n2, const cx<T> *__restrict__ tw)
{
#pragma unroll
    for (int k1 = 1; k1 < R; ++k1) {
        cx<T> w = tw[n2 * k1];
        T wr = w.x, wi = (S < 0) ? w.y : -w.y;
        T a = xr[k1], b = xi[k1];
        xr[k1] = a * wr - b * wi;
        xi[k1] = a * wi + b * wr;
    }
}

// ------------------------------------------------------------------ K1
// One workgroup per (stick group, band).  Stage A loads c straight from HBM
// (only the stick's own run is non-zero), stage B writes the z-transformed
// stick to S[band][z][slot]; lanes of consecutive sticks write consecutive
// slots.
template <typename T>
__global__ __launch_bounds__(256) void k_stick_fwd(Geometry g, DevTables t,
                                                   const cx<T> *__restrict__ c,
                                                   cx<T> *__restrict__ S, long long band0)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *lines = reinterpret_cast<cx<T> *>(smem_raw);
    const int2 gi = t.groups[blockIdx.x];
    const int s0 = gi.x, ns = gi.y, bl = blockIdx.y;
    const cx<T> *cb = c + (band0 + bl) * (long long)g.npw;
    const cx<T> *tw = reinterpret_cast<const cx<T> *>(t.twz);
    const int L1 = g.L1z, L2 = g.L2z, N3 = g.N3, ldz = g.ldz;

    with_codelet(L1, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        for (int task = threadIdx.x; task < ns * L2; task += blockDim.x) {
            const int j = task / L2, n2 = task - j * L2;
            const int4 si = t.slot_info[s0 + j];
            T xr[R], xi[R];
#pragma unroll
            for (int n1 = 0; n1 < R; ++n1) {
                int i = n2 + L2 * n1 - si.z;
                if (i < 0) i += N3;
                cx<T> v = mk<T>(T(0), T(0));
                if (i < si.y) v = cb[si.x + i];
                xr[n1] = v.x;
                xi[n1] = v.y;
            }
            Dft<R, -1, T>::run(xr, xi);
            twiddle<R, -1, T>(xr, xi, n2, tw);
            cx<T> *line = lines + j * ldz + n2;
#pragma unroll
            for (int k1 = 0; k1 < R; ++k1) line[L2 * k1] = mk<T>(xr[k1], xi[k1]);
        }
    });
    __syncthreads();
    with_codelet(L2, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        for (int task = threadIdx.x; task < ns * L1; task += blockDim.x) {
            const int k1 = task / ns, j = task - k1 * ns;
            const cx<T> *line = lines + j * ldz + L2 * k1;
            T xr[R], xi[R];
#pragma unroll
            for (int n2 = 0; n2 < R; ++n2) {
                cx<T> v = line[n2];
                xr[n2] = v.x;
                xi[n2] = v.y;
            }
            Dft<R, -1, T>::run(xr, xi);
            cx<T> *Sb = S + (long long)bl * N3 * g.nst + s0 + j;
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2)
                Sb[(long long)(k1 + L1 * k2) * g.nst] = mk<T>(xr[k2], xi[k2]);
        }
    });
}

// ------------------------------------------------------------------ K3
// Mirror of K1: stage B' reads S[band][z][slot] (coalesced over sticks), stage
// A' keeps only the stick's own run, scales by 1/N and writes out.
template <typename T>
__global__ __launch_bounds__(256) void k_stick_bwd(Geometry g, DevTables t,
                                                   const cx<T> *__restrict__ S,
                                                   cx<T> *__restrict__ out, long long band0)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *lines = reinterpret_cast<cx<T> *>(smem_raw);
    const int2 gi = t.groups[blockIdx.x];
    const int s0 = gi.x, ns = gi.y, bl = blockIdx.y;
    cx<T> *ob = out + (band0 + bl) * (long long)g.npw;
    const cx<T> *tw = reinterpret_cast<const cx<T> *>(t.twz);
    const int L1 = g.L1z, L2 = g.L2z, N3 = g.N3, ldz = g.ldz;
    const T inv_n = T(g.inv_n);

    with_codelet(L2, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        for (int task = threadIdx.x; task < ns * L1; task += blockDim.x) {
            const int k1 = task / ns, j = task - k1 * ns;
            const cx<T> *Sb = S + (long long)bl * N3 * g.nst + s0 + j;
            T xr[R], xi[R];
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) {
                cx<T> v = Sb[(long long)(k1 + L1 * k2) * g.nst];
                xr[k2] = v.x;
                xi[k2] = v.y;
            }
            Dft<R, +1, T>::run(xr, xi);
            cx<T> *line = lines + j * ldz + L2 * k1;
#pragma unroll
            for (int n2 = 0; n2 < R; ++n2) line[n2] = mk<T>(xr[n2], xi[n2]);
        }
    });
    __syncthreads();
    with_codelet(L1, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        for (int task = threadIdx.x; task < ns * L2; task += blockDim.x) {
            const int j = task / L2, n2 = task - j * L2;
            const cx<T> *line = lines + j * ldz + n2;
            T xr[R], xi[R];
#pragma unroll
            for (int k1 = 0; k1 < R; ++k1) {
                cx<T> v = line[L2 * k1];
                xr[k1] = v.x;
                xi[k1] = v.y;
            }
            twiddle<R, +1, T>(xr, xi, n2, tw);
            Dft<R, +1, T>::run(xr, xi);
            const int4 si = t.slot_info[s0 + j];
#pragma unroll
            for (int n1 = 0; n1 < R; ++n1) {
                int i = n2 + L2 * n1 - si.z;
                if (i < 0) i += N3;
                if (i < si.y) ob[si.x + i] = mk<T>(xr[n1] * inv_n, xi[n1] * inv_n);
            }
        }
    });
}

// ------------------------------------------------------------------ K2
// One workgroup per (band, z-plane).  LDS holds the occupied part of the plane,
// P[h - hmin][y] (nxo columns of N2), plus a batch of full x rows.
//   1. S[band][z][*] -> P (zero elsewhere);
//   2. y transforms (-i) on the nxo columns: the cylinder -> cuboid step;
//   3. per batch of rows: full x transform (-i), times V[z][y][x], x transform
//      (+i), keeping only the nxo occupied outputs;
//   4. y transforms (+i) on the nxo columns;
//   5. P -> S[band][z][*] at the sticks' positions.
// Real-space psi for the plane never leaves registers/LDS.  After step 2 the
// columns are in transposed order: row y sits at L2y (y mod L1y) + y / L1y.
template <typename T, int MODE>
__global__ __launch_bounds__(512) void k_plane(Geometry g, DevTables t, cx<T> *__restrict__ S,
                                               const T *__restrict__ V,
                                               cx<T> *__restrict__ psi, long long band0, int nb)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *plane = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *rowbuf = plane + g.nxo * g.ldy;
    const int tid = threadIdx.x, nthr = blockDim.x;

    // XCD-aware order: consecutive workgroups go to different XCDs, so give
    // each XCD a contiguous run of (z, band) pairs; the bands of one z then
    // share that XCD's L2 copy of the V plane.
    const int nblk = gridDim.x;
    int jb = blockIdx.x;
    if ((nblk & 7) == 0) jb = (blockIdx.x & 7) * (nblk >> 3) + (blockIdx.x >> 3);
    const int z = jb / nb, bl = jb - z * nb;

    const int N1 = g.N1, N2 = g.N2, nxo = g.nxo, ldy = g.ldy, ldx = g.ldx;
    const int L1x = g.L1x, L2x = g.L2x, L1y = g.L1y, L2y = g.L2y;
    const cx<T> *twx = reinterpret_cast<const cx<T> *>(t.twx);
    const cx<T> *twy = reinterpret_cast<const cx<T> *>(t.twy);
    cx<T> *Sz = S + ((long long)bl * g.N3 + z) * g.nst;
    cx<T> *psiz = psi ? psi + (((band0 + bl) * (long long)g.N3 + z) * N2) * N1 : nullptr;
    const T *Vz = V ? V + (long long)z * N2 * N1 : nullptr;

    if (MODE != MODE_R2G) {
        for (int e = tid; e < nxo * ldy; e += nthr) plane[e] = mk<T>(T(0), T(0));
        __syncthreads();
        for (int s = tid; s < g.nst; s += nthr) plane[t.slot_info[s].w] = Sz[s];
        __syncthreads();
        // y forward, stage A
        with_codelet(L1y, [&](auto RC) {
            constexpr int R = decltype(RC)::value;
            for (int task = tid; task < nxo * L2y; task += nthr) {
                const int hc = task / L2y, n2 = task - hc * L2y;
                cx<T> *col = plane + hc * ldy + n2;
                T xr[R], xi[R];
#pragma unroll
                for (int n1 = 0; n1 < R; ++n1) {
                    cx<T> v = col[L2y * n1];
                    xr[n1] = v.x;
                    xi[n1] = v.y;
                }
                Dft<R, -1, T>::run(xr, xi);
                twiddle<R, -1, T>(xr, xi, n2, twy);
#pragma unroll
                for (int k1 = 0; k1 < R; ++k1) col[L2y * k1] = mk<T>(xr[k1], xi[k1]);
            }
        });
        __syncthreads();
        // y forward, stage B
        with_codelet(L2y, [&](auto RC) {
            constexpr int R = decltype(RC)::value;
            for (int task = tid; task < nxo * L1y; task += nthr) {
                const int hc = task / L1y, k1 = task - hc * L1y;
                cx<T> *col = plane + hc * ldy + L2y * k1;
                T xr[R], xi[R];
#pragma unroll
                for (int n2 = 0; n2 < R; ++n2) {
                    cx<T> v = col[n2];
                    xr[n2] = v.x;
                    xi[n2] = v.y;
                }
                Dft<R, -1, T>::run(xr, xi);
#pragma unroll
                for (int k2 = 0; k2 < R; ++k2) col[k2] = mk<T>(xr[k2], xi[k2]);
            }
        });
        __syncthreads();
    }

    // x pass, in batches of rows
    for (int y0 = 0; y0 < N2; y0 += g.rows) {
        const int nr = min(g.rows, N2 - y0);
        if (MODE != MODE_R2G) {
            with_codelet(L1x, [&](auto RC) {
                constexpr int R = decltype(RC)::value;
                for (int task = tid; task < nr * L2x; task += nthr) {
                    const int r = task / L2x, n2 = task - r * L2x;
                    const int y = y0 + r;
                    const int yp = L2y * (y % L1y) + y / L1y;
                    T xr[R], xi[R];
#pragma unroll
                    for (int n1 = 0; n1 < R; ++n1) {
                        int hc = n2 + L2x * n1 - g.hmin_mod;
                        if (hc < 0) hc += N1;
                        cx<T> v = mk<T>(T(0), T(0));
                        if (hc < nxo) v = plane[hc * ldy + yp];
                        xr[n1] = v.x;
                        xi[n1] = v.y;
                    }
                    Dft<R, -1, T>::run(xr, xi);
                    twiddle<R, -1, T>(xr, xi, n2, twx);
                    cx<T> *row = rowbuf + r * ldx + n2;
#pragma unroll
                    for (int k1 = 0; k1 < R; ++k1) row[L2x * k1] = mk<T>(xr[k1], xi[k1]);
                }
            });
            __syncthreads();
        }
        with_codelet(L2x, [&](auto RC) {
            constexpr int R = decltype(RC)::value;
            for (int task = tid; task < nr * L1x; task += nthr) {
                const int r = task / L1x, k1 = task - r * L1x;
                const int y = y0 + r;
                cx<T> *row = rowbuf + r * ldx + L2x * k1;
                T xr[R], xi[R];
                if (MODE == MODE_R2G) {
                    const cx<T> *src = psiz + (long long)y * N1 + k1;
#pragma unroll
                    for (int k2 = 0; k2 < R; ++k2) {
                        cx<T> v = src[L1x * k2];
                        xr[k2] = v.x;
                        xi[k2] = v.y;
                    }
                } else {
#pragma unroll
                    for (int n2 = 0; n2 < R; ++n2) {
                        cx<T> v = row[n2];
                        xr[n2] = v.x;
                        xi[n2] = v.y;
                    }
                    Dft<R, -1, T>::run(xr, xi);
                }
                if (MODE == MODE_G2R) {
                    cx<T> *dst = psiz + (long long)y * N1 + k1;
#pragma unroll
                    for (int k2 = 0; k2 < R; ++k2) dst[L1x * k2] = mk<T>(xr[k2], xi[k2]);
                } else {
                    if (MODE == MODE_APPLY) {
                        const T *vrow = Vz + (long long)y * N1 + k1;
#pragma unroll
                        for (int k2 = 0; k2 < R; ++k2) {
                            T v = vrow[L1x * k2];
                            xr[k2] *= v;
                            xi[k2] *= v;
                        }
                    }
                    Dft<R, +1, T>::run(xr, xi);
#pragma unroll
                    for (int n2 = 0; n2 < R; ++n2) row[n2] = mk<T>(xr[n2], xi[n2]);
                }
            }
        });
        __syncthreads();
        if (MODE != MODE_G2R) {
            with_codelet(L1x, [&](auto RC) {
                constexpr int R = decltype(RC)::value;
                for (int task = tid; task < nr * L2x; task += nthr) {
                    const int r = task / L2x, n2 = task - r * L2x;
                    const int y = y0 + r;
                    const int yp = L2y * (y % L1y) + y / L1y;
                    const cx<T> *row = rowbuf + r * ldx + n2;
                    T xr[R], xi[R];
#pragma unroll
                    for (int k1 = 0; k1 < R; ++k1) {
                        cx<T> v = row[L2x * k1];
                        xr[k1] = v.x;
                        xi[k1] = v.y;
                    }
                    twiddle<R, +1, T>(xr, xi, n2, twx);
                    Dft<R, +1, T>::run(xr, xi);
#pragma unroll
                    for (int n1 = 0; n1 < R; ++n1) {
                        int hc = n2 + L2x * n1 - g.hmin_mod;
                        if (hc < 0) hc += N1;
                        if (hc < nxo) plane[hc * ldy + yp] = mk<T>(xr[n1], xi[n1]);
                    }
                }
            });
            __syncthreads();
        }
    }
    if (MODE == MODE_G2R) return;

    // y reverse, stage B'
    with_codelet(L2y, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        for (int task = tid; task < nxo * L1y; task += nthr) {
            const int hc = task / L1y, k1 = task - hc * L1y;
            cx<T> *col = plane + hc * ldy + L2y * k1;
            T xr[R], xi[R];
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) {
                cx<T> v = col[k2];
                xr[k2] = v.x;
                xi[k2] = v.y;
            }
            Dft<R, +1, T>::run(xr, xi);
#pragma unroll
            for (int n2 = 0; n2 < R; ++n2) col[n2] = mk<T>(xr[n2], xi[n2]);
        }
    });
    __syncthreads();
    // y reverse, stage A'
    with_codelet(L1y, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        for (int task = tid; task < nxo * L2y; task += nthr) {
            const int hc = task / L2y, n2 = task - hc * L2y;
            cx<T> *col = plane + hc * ldy + n2;
            T xr[R], xi[R];
#pragma unroll
            for (int k1 = 0; k1 < R; ++k1) {
                cx<T> v = col[L2y * k1];
                xr[k1] = v.x;
                xi[k1] = v.y;
            }
            twiddle<R, +1, T>(xr, xi, n2, twy);
            Dft<R, +1, T>::run(xr, xi);
#pragma unroll
            for (int n1 = 0; n1 < R; ++n1) col[L2y * n1] = mk<T>(xr[n1], xi[n1]);
        }
    });
    __syncthreads();
    for (int s = tid; s < g.nst; s += nthr) Sz[s] = plane[t.slot_info[s].w];
}

// ------------------------------------------------------------ launchers

template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T>
hipError_t launch_stick_fwd(const Geometry &g, const DevTables &t, const void *c, int64_t band0,
                            int nb, void *S, int threads, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    size_t lds = (size_t)g.group_cap * g.ldz * sizeof(cx<T>);
    hipError_t e = allow_lds(k_stick_fwd<T>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stick_fwd<T>, dim3(g.ngroups, nb), dim3(threads), lds, st, g, t,
                       reinterpret_cast<const cx<T> *>(c), reinterpret_cast<cx<T> *>(S),
                       (long long)band0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stick_bwd(const Geometry &g, const DevTables &t, const void *S, void *out,
                            int64_t band0, int nb, int threads, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    size_t lds = (size_t)g.group_cap * g.ldz * sizeof(cx<T>);
    hipError_t e = allow_lds(k_stick_bwd<T>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stick_bwd<T>, dim3(g.ngroups, nb), dim3(threads), lds, st, g, t,
                       reinterpret_cast<const cx<T> *>(S), reinterpret_cast<cx<T> *>(out),
                       (long long)band0);
    return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t launch_plane_mode(const Geometry &g, const DevTables &t, void *S, const void *V,
                                    void *psi, int64_t band0, int nb, int threads, int lds,
                                    hipStream_t st)
{
    hipError_t e = allow_lds(k_plane<T, MODE>, (size_t)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_plane<T, MODE>), dim3((unsigned)nb * g.N3), dim3(threads), (size_t)lds,
                       st, g, t, reinterpret_cast<cx<T> *>(S), reinterpret_cast<const T *>(V),
                       reinterpret_cast<cx<T> *>(psi), (long long)band0, nb);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_plane(const Geometry &g, const DevTables &t, int mode, void *S, const void *V,
                        void *psi, int64_t band0, int nb, int threads, int lds_bytes,
                        hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    switch (mode) {
    case MODE_APPLY:
        return launch_plane_mode<T, MODE_APPLY>(g, t, S, V, psi, band0, nb, threads, lds_bytes, st);
    case MODE_G2R:
        return launch_plane_mode<T, MODE_G2R>(g, t, S, V, psi, band0, nb, threads, lds_bytes, st);
    case MODE_R2G:
        return launch_plane_mode<T, MODE_R2G>(g, t, S, V, psi, band0, nb, threads, lds_bytes, st);
    default: return hipErrorInvalidValue;
    }
}

#define VLOC_INSTANTIATE(T)                                                                       \
    template hipError_t launch_stick_fwd<T>(const Geometry &, const DevTables &, const void *,   \
                                            int64_t, int, void *, int, hipStream_t);             \
    template hipError_t launch_stick_bwd<T>(const Geometry &, const DevTables &, const void *,   \
                                            void *, int64_t, int, int, hipStream_t);             \
    template hipError_t launch_plane<T>(const Geometry &, const DevTables &, int, void *,         \
                                        const void *, void *, int64_t, int, int, int,            \
                                        hipStream_t);
VLOC_INSTANTIATE(double)
VLOC_INSTANTIATE(float)

} // namespace vloc
