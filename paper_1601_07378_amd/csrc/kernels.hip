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
#include <algorithm>
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

// Calls f with a compile-time codelet size equal to the runtime r.  Sizes
// above MAXR are not compiled (workgroups of more than 512 threads have too
// few registers for them, and a kernel that holds the paths of larger sizes
// carries their register pressure into every other size); the launchers never
// run such a kernel with them.
template <int MAXR = 32, typename F>
__device__ __forceinline__ void with_codelet(int r, F &&f)
{
    if constexpr (MAXR > 16) {
        switch (r) {
        case 18: f(std::integral_constant<int, 18>{}); return;
        case 20: f(std::integral_constant<int, 20>{}); return;
        case 24: f(std::integral_constant<int, 24>{}); return;
        case 25: f(std::integral_constant<int, 25>{}); return;
        case 27: f(std::integral_constant<int, 27>{}); return;
        case 30: f(std::integral_constant<int, 30>{}); return;
        case 32: f(std::integral_constant<int, 32>{}); return;
        default: break;
        }
    }
    switch (r) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 10:
        if constexpr (MAXR >= 10) f(std::integral_constant<int, 10>{});
        break;
    case 12:
        if constexpr (MAXR >= 12) f(std::integral_constant<int, 12>{});
        break;
    case 15:
        if constexpr (MAXR >= 15) f(std::integral_constant<int, 15>{});
        break;
    case 16:
        if constexpr (MAXR >= 16) f(std::integral_constant<int, 16>{});
        break;
    default: break;
    }
}

// Compile-time size CT if non-zero, else the runtime r through the switch.
template <int CT, int MAXR = 32, typename F>
__device__ __forceinline__ void with_size(int r, F &&f)
{
    if constexpr (CT > 0)
        f(std::integral_constant<int, CT>{});
    else
        with_codelet<MAXR>(r, f);
}

// Bit n1 of a zero mask ZM is set when every input x[n2 + L2 n1] of stage A
// is zero for every task (positions that no sphere point reaches); stage A
// then skips those loads, the codelet folds the zeros, and the reverse stage
// A' skips computing and storing those outputs, which nothing reads.
template <int ZM>
__device__ __forceinline__ constexpr bool masked(int n1)
{
    return ZM != 0 && ((ZM >> n1) & 1);
}

// x[k1] *= W_L^{S n2 k1}, L = R L2; the table holds W_L^{n2 k1} =
// exp(-2 pi i n2 k1 / L) at [n2][k1] (R entries per n2), so a task's
// twiddles are one contiguous run.
template <int R, int S, typename T>
__device__ __forceinline__ void twiddle(T *xr, T *xi, int n2, const cx<T> *__restrict__ tw)
{
    const cx<T> *w_n2 = tw + n2 * R;
#pragma unroll
    for (int k1 = 1; k1 < R; ++k1) {
        cx<T> w = w_n2[k1];
        T wr = w.x, wi = (S < 0) ? w.y : -w.y;
        T a = xr[k1], b = xi[k1];
        xr[k1] = a * wr - b * wi;
        xi[k1] = a * wi + b * wr;
    }
}

// The same with fewer table reads.  For an 8-point first stage only w^1, w^2
// and w^4 are read; w^3, w^5, w^6 and w^7 are their products (one or two
// roundings from the tabulated values): four complex multiplies instead of four
// reads; a 16-point stage (FP64) also reads w^8 and forms the rest likewise.  Used where reads are the scarcer resource: the FP64 whole-plane
// kernel (its LDS traffic is as long as its arithmetic) and, with ANY, the
// forward stick kernel in both precisions (its twiddle loads were a third of
// its vector-memory instructions).
template <int R, int S, typename T, bool ANY = false>
__device__ __forceinline__ void twiddle_pw(T *xr, T *xi, int n2, const cx<T> *__restrict__ tw)
{
    if constexpr (R == 8 && (ANY || std::is_same<T, double>::value)) {
        const cx<T> *w_n2 = tw + n2 * R;
        const cx<T> a = w_n2[1], b = w_n2[2], d = w_n2[4];
        auto mul = [](cx<T> u, cx<T> v) {
            return mk<T>(u.x * v.x - u.y * v.y, u.x * v.y + u.y * v.x);
        };
        cx<T> w[R];
        w[1] = a;
        w[2] = b;
        w[3] = mul(a, b);
        w[4] = d;
        w[5] = mul(a, d);
        w[6] = mul(b, d);
        w[7] = mul(w[3], d);
#pragma unroll
        for (int k1 = 1; k1 < R; ++k1) {
            T wr = w[k1].x, wi = (S < 0) ? w[k1].y : -w[k1].y;
            T u = xr[k1], v = xi[k1];
            xr[k1] = u * wr - v * wi;
            xi[k1] = u * wi + v * wr;
        }
        return;
    }
    if constexpr (R == 16 && (ANY || std::is_same<T, double>::value)) {
        // w^1, w^2, w^4, w^8 read; w^3 and w^5..w^7 products of them (at most
        // two roundings), w^9..w^15 = w^(k - 8) w^8 (at most three): 4 reads
        // and 11 complex multiplies instead of 15 reads, and 8 twiddles live
        const cx<T> *w_n2 = tw + n2 * R;
        const cx<T> w1 = w_n2[1], w2 = w_n2[2], w4 = w_n2[4], w8 = w_n2[8];
        auto mul = [](cx<T> u, cx<T> v) {
            return mk<T>(u.x * v.x - u.y * v.y, u.x * v.y + u.y * v.x);
        };
        auto app = [&](int k1, cx<T> w) {
            T wr = w.x, wi = (S < 0) ? w.y : -w.y;
            T u = xr[k1], v = xi[k1];
            xr[k1] = u * wr - v * wi;
            xi[k1] = u * wi + v * wr;
        };
        cx<T> lo[8];
        lo[0] = mk<T>(T(1), T(0));
        lo[1] = w1;
        lo[2] = w2;
        lo[3] = mul(w1, w2);
        lo[4] = w4;
        lo[5] = mul(w1, w4);
        lo[6] = mul(w2, w4);
        lo[7] = mul(lo[3], w4);
#pragma unroll
        for (int k = 1; k < 8; ++k) app(k, lo[k]);
        app(8, w8);
#pragma unroll
        for (int k = 1; k < 8; ++k) app(8 + k, mul(lo[k], w8));
        return;
    }
    twiddle<R, S, T>(xr, xi, n2, tw);
}

// Segment of a launch by a uniform key (stick-kernel block or launch band):
// the last segment whose first key is <= v.  The descriptor is read from the
// kernel-argument segment with a uniform index (scalar loads), not held in
// registers across the kernel.
__device__ __forceinline__ Seg seg_by_block(const Launch &L, int v)
{
    int s = 0;
    for (int i = 1; i < L.nseg; ++i)
        if (v >= L.seg[i].blk_lo) s = i;
    return L.seg[s];
}
// Block numbering of K3: consecutive workgroups go to the eight XCDs in turn,
// so renumber them to give each XCD one contiguous range of (band, group)
// items; the output cache lines shared by neighbouring groups (the ends of
// their coefficient runs) then meet in one L2 instead of being written back
// partially from two.  A bijection on [0, nblk) for any nblk.  (K1 keeps the
// hardware order, measured faster for its S writes.)
__device__ __forceinline__ int xcd_block(int nblk)
{
    const int b = blockIdx.x, x = b & 7, q = nblk >> 3, r = nblk & 7;
    return x * q + min(x, r) + (b >> 3);
}
__device__ __forceinline__ int seg_index_by_band(const Launch &L, int v)
{
    int s = 0;
    for (int i = 1; i < L.nseg; ++i)
        if (v >= L.seg[i].band_lo) s = i;
    return s;
}
__device__ __forceinline__ Seg seg_at(const Launch &L, int s)
{
    return L.seg[s];
}

// Real mode: the value at position i of a stick's run for the band pair
// (a, b), d = A + i B, where A, B are the coefficients of bands a, b at that
// g; a mirror stick (-h, -k) reads the half-sphere run of its partner in
// reverse, conjugated (c(-g) = conj c(g)); the (0, 0) stick reads l >= 0
// directly and l < 0 mirrored, with Im c(0) taken as 0.
template <typename T>
__device__ __forceinline__ cx<T> gamma_pair(const cx<T> *__restrict__ ca,
                                            const cx<T> *__restrict__ cb, int4 gm, int i)
{
    int idx;
    bool mir, zero = false;
    if (gm.y == 0) {
        idx = gm.x + i;
        mir = false;
    } else if (gm.y == 1) {
        idx = gm.x - i;
        mir = true;
    } else {
        const int l = i - gm.z;
        mir = l < 0;
        zero = l == 0;
        idx = gm.x + (mir ? -l : l);
    }
    cx<T> a = ca[idx];
    cx<T> b = cb ? cb[idx] : mk<T>(T(0), T(0));
    T ai = mir ? -a.y : a.y, bi = mir ? -b.y : b.y;
    if (zero) ai = bi = T(0);
    return mk<T>(a.x - bi, ai + b.x);
}

// ------------------------------------------------------------------ K1
// One workgroup per (stick group, band) of a segment.  Stage A loads c
// straight from HBM (only the stick's own run is non-zero), stage B writes the
// z-transformed stick to S[band][z][slot]; lanes of consecutive sticks write
// consecutive slots.
template <typename T, int CZ1, int CZ2, int ZZ, bool GAM>
__global__ __launch_bounds__(512) void k_stick_fwd(Geometry g, DevTables t, Launch L,
                                                   cx<T> *__restrict__ S)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *lines = reinterpret_cast<cx<T> *>(smem_raw);
    const Seg sg = seg_by_block(L, blockIdx.x);
    const int rb = blockIdx.x - sg.blk_lo;
    const int bl = rb / sg.ngroups, gr = rb - bl * sg.ngroups;
    const int2 gi = t.groups[sg.group_off + gr];
    const int s0 = gi.x, ns = gi.y;
    const int4 *slot_info = t.slot_info + sg.slot_off;
    // real mode: launch band bl is the pair of real bands 2 bl, 2 bl + 1
    const cx<T> *cb = reinterpret_cast<const cx<T> *>(sg.in) +
                      (GAM ? 2 * bl : bl) * (long long)sg.npw;
    const cx<T> *cb2 = (GAM && 2 * bl + 1 < sg.nbr) ? cb + sg.npw : nullptr;
    const cx<T> *tw = reinterpret_cast<const cx<T> *>(t.twz);
    const int L1 = CZ1 ? CZ1 : g.L1z, L2 = CZ2 ? CZ2 : g.L2z;
    const int N3 = CZ1 ? CZ1 * CZ2 : g.N3, ldz = CZ1 ? CZ1 * CZ2 + 1 : g.ldz;

    with_size<CZ1>(L1, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        for (int task = threadIdx.x; task < ns * L2; task += blockDim.x) {
            const int j = task / L2, n2 = task - j * L2;
            const int4 si = slot_info[s0 + j];
            int4 gm = make_int4(0, 0, 0, 0);
            if (GAM) gm = t.gam[sg.slot_off + s0 + j];
            T xr[R], xi[R];
#pragma unroll
            for (int n1 = 0; n1 < R; ++n1) {
                cx<T> v = mk<T>(T(0), T(0));
                if (!masked<ZZ>(n1)) {
                    int i = n2 + L2 * n1 - si.z;
                    if (i < 0) i += N3;
                    if (i < si.y) v = GAM ? gamma_pair<T>(cb, cb2, gm, i) : cb[si.x + i];
                }
                xr[n1] = v.x;
                xi[n1] = v.y;
            }
            Dft<R, -1, T>::run(xr, xi);
            twiddle_pw<R, -1, T, true>(xr, xi, n2, tw);
            cx<T> *line = lines + j * ldz + n2;
#pragma unroll
            for (int k1 = 0; k1 < R; ++k1) line[L2 * k1] = mk<T>(xr[k1], xi[k1]);
        }
    });
    __syncthreads();
    with_size<CZ2>(L2, [&](auto RC) {
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
            cx<T> *Sb = S + sg.s_off + (long long)bl * N3 * sg.nst + s0 + j;
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2)
                Sb[(long long)(k1 + L1 * k2) * sg.nst] = mk<T>(xr[k2], xi[k2]);
        }
    });
}

// ------------------------------------------------------------------ K3
// Mirror of K1: stage B' reads S[band][z][slot] (coalesced over sticks), stage
// A' keeps only the stick's own run, scales by 1/N and writes out.
template <typename T, int CZ1, int CZ2, int ZZ, bool GAM>
__global__ __launch_bounds__(512) void k_stick_bwd(Geometry g, DevTables t, Launch L,
                                                   const cx<T> *__restrict__ S)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *lines = reinterpret_cast<cx<T> *>(smem_raw);
    const int vb = xcd_block(L.nblk);
    const Seg sg = seg_by_block(L, vb);
    const int rb = vb - sg.blk_lo;
    const int bl = rb / sg.ngroups, gr = rb - bl * sg.ngroups;
    const int2 gi = t.groups[sg.group_off + gr];
    const int s0 = gi.x, ns = gi.y;
    const int4 *slot_info = t.slot_info + sg.slot_off;
    cx<T> *ob = reinterpret_cast<cx<T> *>(sg.out) + (GAM ? 2 * bl : bl) * (long long)sg.npw;
    const int L1 = CZ1 ? CZ1 : g.L1z, L2 = CZ2 ? CZ2 : g.L2z;
    const int N3 = CZ1 ? CZ1 * CZ2 : g.N3, ldz = CZ1 ? CZ1 * CZ2 + 1 : g.ldz;
    const T inv_n = T(g.inv_n);
    // stage twiddles into LDS after the stick lines (read after the barrier
    // between stages B' and A')
    cx<T> *tw = lines + g.group_cap * ldz;
    const cx<T> *twg = reinterpret_cast<const cx<T> *>(t.twz);
    for (int i = threadIdx.x; i < N3; i += blockDim.x) tw[i] = twg[i];

    with_size<CZ2>(L2, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        for (int task = threadIdx.x; task < ns * L1; task += blockDim.x) {
            const int k1 = task / ns, j = task - k1 * ns;
            const cx<T> *Sb = S + sg.s_off + (long long)bl * N3 * sg.nst + s0 + j;
            T xr[R], xi[R];
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) {
                cx<T> v = Sb[(long long)(k1 + L1 * k2) * sg.nst];
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
    with_size<CZ1>(L1, [&](auto RC) {
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
            if constexpr (GAM) {
                // back into the line in natural z order (the task's own positions)
                cx<T> *ln = lines + j * ldz + n2;
#pragma unroll
                for (int n1 = 0; n1 < R; ++n1)
                    if (!masked<ZZ>(n1)) ln[L2 * n1] = mk<T>(xr[n1], xi[n1]);
            } else {
                const int4 si = slot_info[s0 + j];
#pragma unroll
                for (int n1 = 0; n1 < R; ++n1) {
                    if (masked<ZZ>(n1)) continue;
                    int i = n2 + L2 * n1 - si.z;
                    if (i < 0) i += N3;
                    if (i < si.y) ob[si.x + i] = mk<T>(xr[n1] * inv_n, xi[n1] * inv_n);
                }
            }
        }
    });
    if constexpr (GAM) {
        // Split the pair: with e = transform of d = A + i B at g and f at -g,
        // A(g) = (e + conj f) / 2 and B(g) = (e - conj f) / (2 i); only the
        // half sphere is written (sticks of H and l >= 0 of the (0, 0) stick).
        __syncthreads();
        cx<T> *ob2 = (2 * bl + 1 < sg.nbr) ? ob + sg.npw : nullptr;
        const T h = T(0.5 * g.inv_n);
        for (int task = threadIdx.x; task < ns * N3; task += blockDim.x) {
            const int j = task / N3, z = task - j * N3;
            const int4 gm = t.gam[sg.slot_off + s0 + j];
            if (gm.y == 1) continue;
            const int4 si = slot_info[s0 + j];
            int i = z - si.z;
            if (i < 0) i += N3;
            if (i >= si.y) continue;
            int oi = gm.x + i;
            if (gm.y == 2) {
                if (i < gm.z) continue;
                oi = gm.x + (i - gm.z);
            }
            const cx<T> e = lines[j * ldz + z];
            const cx<T> f = lines[gm.w * ldz + (z == 0 ? 0 : N3 - z)];
            ob[oi] = mk<T>((e.x + f.x) * h, (e.y - f.y) * h);
            if (ob2) ob2[oi] = mk<T>((e.y + f.y) * h, (f.x - e.x) * h);
        }
    }
}

// ------------------------------------------------------------------ K2
// One workgroup per (band, z-plane).  LDS holds the occupied part of the plane,
// P[h - hmin][y] (nxo columns of N2, column stride ldy), plus one private batch
// of full x rows for each wavefront that takes part in the x pass.
//   1. S[band][z][*] -> P at the sticks' positions;
//   2. y transforms (-i) on the nxo columns (the cylinder -> cuboid step); a
//      column's input is non-zero only on its own k range, so P needs no
//      zero fill;
//   3. x pass, wavefront-local: each wave takes a contiguous block of rows and
//      runs, per batch of rows, the full x transform (-i), the multiply by
//      V[z][y][x] and the x transform (+i), keeping only the nxo occupied
//      outputs; only wave-level ordering is needed inside the pass;
//   4. y transforms (+i) on the nxo columns, storing only the stick positions;
//   5. P -> S[band][z][*].
// Real-space psi of the plane never leaves registers/LDS.  After step 2 the
// columns are in transposed order: row y sits at L2y (y mod L1y) + y / L1y.
// Row buffers keep position p at p + p / L2x so that the strided stage-B
// accesses hit distinct LDS banks; y stages map consecutive lanes to
// consecutive columns (stride ldy, odd) for the same reason.


// Orders LDS accesses of one wavefront (LDS executes a wave's operations in
// issue order; this keeps the compiler from moving accesses across).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// DPP quad permutations: lane i reads lane i^1 / i^2 of its quad.
constexpr int kQuadXor1 = 0xB1; // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E; // quad_perm [2,3,0,1]

template <int CTRL>
__device__ __forceinline__ double quad_swap(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float quad_swap(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Radix-4 step across the four lanes of a quad, for each of the Q values a
// lane holds.  Forward (S = -1): lane q holds Y_q[k] and ends with
// X[k + Q p(q)] = sum_q' Y_q'[k] W_4^{S q' p}, p(q) = {0, 2, 1, 3}[q]:
//   stage 1 (lanes q, q^2): u = s1 own + partner, s1 = -1 for q >= 2;
//   lane 3 multiplies by W_4^S (= S i);
//   stage 2 (lanes q, q^1): X = s2 own + partner, s2 = -1 for odd q.
// Reverse (S = +1) runs the same steps in the opposite order so that lane q
// ends with Z_q[k] = sum_p X[k + Q p] W_4^{S q p}.
template <int Q, int S, typename T>
__device__ __forceinline__ void quad_radix4(T *xr, T *xi, int q)
{
    const T s1 = (q & 2) ? T(-1) : T(1);
    const T s2 = (q & 1) ? T(-1) : T(1);
    // twist on lane 3: (re, im) -> (-S im, S re), as t = c0 (re, im) + c1 (-im, re)
    const T c0 = (q == 3) ? T(0) : T(1);
    const T c1 = (q == 3) ? T(S) : T(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        T ar = xr[k], ai = xi[k];
        if constexpr (S < 0) {
            T pr = quad_swap<kQuadXor2>(ar), pi = quad_swap<kQuadXor2>(ai);
            ar = s1 * ar + pr;
            ai = s1 * ai + pi;
        } else {
            T pr = quad_swap<kQuadXor1>(ar), pi = quad_swap<kQuadXor1>(ai);
            ar = s2 * ar + pr;
            ai = s2 * ai + pi;
        }
        T tr = c0 * ar - c1 * ai;
        T ti = c0 * ai + c1 * ar;
        if constexpr (S < 0) {
            T pr = quad_swap<kQuadXor1>(tr), pi = quad_swap<kQuadXor1>(ti);
            xr[k] = s2 * tr + pr;
            xi[k] = s2 * ti + pi;
        } else {
            T pr = quad_swap<kQuadXor2>(tr), pi = quad_swap<kQuadXor2>(ti);
            xr[k] = s1 * tr + pr;
            xi[k] = s1 * ti + pi;
        }
    }
}

// Per k: forward radix-4 across the quad, multiply by V at the lane's own
// frequency k + Q p(q), reverse radix-4; V is read one value at a time.
template <typename T>
__device__ __forceinline__ void quad_radix4_v_one(T &xr, T &xi, T v, T s1, T s2, T c0, T c1)
{
    T ar = xr, ai = xi;
    T pr = quad_swap<kQuadXor2>(ar), pi = quad_swap<kQuadXor2>(ai);
    ar = s1 * ar + pr;
    ai = s1 * ai + pi;
    T tr = c0 * ar + c1 * ai; // lane 3: -i (ar + i ai) = (ai, -ar)
    T ti = c0 * ai - c1 * ar;
    pr = quad_swap<kQuadXor1>(tr);
    pi = quad_swap<kQuadXor1>(ti);
    ar = (s2 * tr + pr) * v;
    ai = (s2 * ti + pi) * v;
    pr = quad_swap<kQuadXor1>(ar);
    pi = quad_swap<kQuadXor1>(ai);
    ar = s2 * ar + pr;
    ai = s2 * ai + pi;
    tr = c0 * ar - c1 * ai; // lane 3: +i (ar + i ai) = (-ai, ar)
    ti = c0 * ai + c1 * ar;
    pr = quad_swap<kQuadXor2>(tr);
    pi = quad_swap<kQuadXor2>(ti);
    xr = s1 * tr + pr;
    xi = s1 * ti + pi;
}

// Per k: forward radix-4 across the quad, multiply by V at the lane's own
// frequency k + Q p(q), reverse radix-4.  V is read in groups of G values,
// one group ahead of its use (the memory barrier keeps the compiler from
// hoisting every load to the top, which would cost 2 Q registers).
template <int Q, typename T>
__device__ __forceinline__ void quad_radix4_v(T *xr, T *xi, int q, const T *__restrict__ vrow)
{
    constexpr int G = (Q % 6 == 0) ? 6 : ((Q % 4 == 0) ? 4 : ((Q % 5 == 0) ? 5 : Q));
    const T s1 = (q & 2) ? T(-1) : T(1);
    const T s2 = (q & 1) ? T(-1) : T(1);
    const T c0 = (q == 3) ? T(0) : T(1);
    const T c1 = (q == 3) ? T(1) : T(0);
    T vb[G];
#pragma unroll
    for (int j = 0; j < G; ++j) vb[j] = vrow[j];
#pragma unroll
    for (int g0 = 0; g0 < Q; g0 += G) {
        T vn[G];
        if (g0 + G < Q) {
#pragma unroll
            for (int j = 0; j < G; ++j) vn[j] = vrow[g0 + G + j];
        }
#pragma unroll
        for (int j = 0; j < G; ++j) quad_radix4_v_one(xr[g0 + j], xi[g0 + j], vb[j], s1, s2, c0, c1);
        asm volatile("" ::: "memory");
        if (g0 + G < Q) {
#pragma unroll
            for (int j = 0; j < G; ++j) vb[j] = vn[j];
        }
    }
}

// x[k] *= W_L^{S q k} for k < Q, twiddles built in FP64 by a recurrence from
// exp(-2 pi i q / L), re-anchored from the exact table every 8 steps.
template <int Q, int S, typename T>
__device__ __forceinline__ void quad_twiddle(T *xr, T *xi, int q, int L,
                                             const double2 *__restrict__ tw64)
{
    const double2 b = tw64[q];
    const double br = b.x, bi = (S < 0) ? b.y : -b.y;
    double wr = 1.0, wi = 0.0;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
        if (k % 8 == 0) {
            const double2 a = tw64[(q * k) % L];
            wr = a.x;
            wi = (S < 0) ? a.y : -a.y;
        } else {
            double nr = wr * br - wi * bi;
            wi = wr * bi + wi * br;
            wr = nr;
        }
        T a = xr[k], c = xi[k];
        T twr = T(wr), twi = T(wi);
        xr[k] = a * twr - c * twi;
        xi[k] = a * twi + c * twr;
    }
}

template <typename T, int MODE, int CX1, int CX2, int CY1, int CY2, int ZX, int ZY, int XQ,
          int PF, int MR>
__device__ __forceinline__ void plane_body(const Geometry &g, const DevTables &t, const Launch &L,
                                           cx<T> *__restrict__ S, const T *__restrict__ V,
                                           cx<T> *__restrict__ psi, long long band0)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *plane = reinterpret_cast<cx<T> *>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
    const int L1x = CX1 ? CX1 : g.L1x, L2x = CX2 ? CX2 : g.L2x;
    const int L1y = CY1 ? CY1 : g.L1y, L2y = CY2 ? CY2 : g.L2y;
    // specialised splits make the line lengths and LDS strides compile-time
    const int N1 = CX1 ? CX1 * CX2 : (XQ ? 4 * XQ : g.N1);
    const int N2 = CY1 ? CY1 * CY2 : g.N2;
    const int ldy = CY1 ? CY1 * CY2 + 1 : g.ldy;
    const int nxo = g.nxo;
    // task / nxo by a 64-bit multiply and shift (exact for tasks < 2^16)
    auto div_nxo = [&](int v) {
        return (int)(((unsigned long long)(unsigned)v * g.nxo_magic) >> 40);
    };
    // row buffer length: L1x (L2x + 1) padded to L2x mod 16 (bank spread of
    // the stage-A writes across two rows); the host uses the same rule
    const int RB = g.rb;
    const int RL = CX1 ? CX1 * (CX2 + 1) + (((CX2 - CX1 * (CX2 + 1)) % 16 + 16) % 16) : g.rl;
    cx<T> *rows = plane + nxo * ldy + wave * RB * RL;

    const cx<T> *twx = reinterpret_cast<const cx<T> *>(t.twx);
    const cx<T> *twy = reinterpret_cast<const cx<T> *>(t.twy);
    const int nb = L.nbt;

    // Work items: a plane (z, band) for the transforms; for the density a
    // (z, band subset) pair whose bands this workgroup runs one after another,
    // so that it alone updates the subset's partial density plane.
    // Persistent schedule: workgroup i runs on XCD i mod 8, so each XCD takes a
    // contiguous eighth of the items in z-major order (the bands of one z
    // share that XCD's L2 copy of the V plane).  Every workgroup reaches the
    // end of its range.
    // density scheduling (items = (z, band subset)) and accumulation; the
    // multiply by the potential
    constexpr bool DENS = (MODE == MODE_DENSITY || MODE == MODE_APPLY_DENSITY);
    constexpr bool POT = (MODE == MODE_APPLY || MODE == MODE_APPLY_DENSITY);
    const int nsub = DENS ? g.nsub : 1;
    const int bps = DENS ? (nb + nsub - 1) / nsub : 1;
    const int total = DENS ? g.N3 * nsub : nb * g.N3;
    int j0 = blockIdx.x, jstep = gridDim.x, jend = total;
    if ((gridDim.x & 7) == 0 && (total & 7) == 0) {
        const int share = total >> 3, xcd = blockIdx.x & 7;
        j0 = xcd * share + (blockIdx.x >> 3);
        jstep = gridDim.x >> 3;
        jend = (xcd + 1) * share;
    }
    auto plane_of = [&](int j, int k, int &zz, int &bb) {
        if (DENS) {
            zz = j / nsub;
            bb = (j - zz * nsub) * bps + k;
        } else {
            zz = j / nb;
            bb = j - zz * nb;
        }
    };
    // next non-empty plane of this workgroup's sequence; false at the end
    auto advance = [&](int &j, int &k) -> bool {
        for (;;) {
            if (DENS && k + 1 < bps)
                ++k;
            else {
                j += jstep;
                k = 0;
            }
            if (j >= jend) return false;
            int zz, bb;
            plane_of(j, k, zz, bb);
            if (bb < nb) return true;
            k = bps; // rest of this subset is empty: go to the next item
        }
    };
    // Segment of a launch band (the density runs one segment).
    auto seg_of = [&](int bb) { return DENS ? 0 : seg_index_by_band(L, bb); };
    // The first PF slots of this thread keep their plane positions in
    // registers while consecutive planes belong to one segment, and their
    // values for the next plane are loaded while the current plane is
    // transformed.
    int spos[PF];
    cx<T> sval[PF];
    int spos_seg = -1;
    auto load_pos = [&](int si) {
        const Seg sg = seg_at(L, si);
        const int4 *sl_info = t.slot_info + sg.slot_off;
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int sl = tid + i * nthr;
            spos[i] = sl < sg.nst ? sl_info[sl].w : 0;
        }
        spos_seg = si;
    };
#pragma unroll
    for (int i = 0; i < PF; ++i) sval[i] = mk<T>(T(0), T(0));
    load_pos(0);
    auto prefetch = [&](int zz, int bb) {
        const Seg sg = seg_at(L, seg_of(bb));
        const cx<T> *Sj = S + sg.s_off + ((long long)(bb - sg.band_lo) * g.N3 + zz) * sg.nst;
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int sl = tid + i * nthr;
            if (sl < sg.nst) sval[i] = Sj[sl];
        }
    };
    int jc = j0, kc = 0;
    bool have = jc < jend;
    if (have) {
        int zz, bb;
        plane_of(jc, kc, zz, bb);
        if (bb >= nb) have = advance(jc, kc);
    }
    if (MODE != MODE_R2G && have) {
        int zz, bb;
        plane_of(jc, kc, zz, bb);
        prefetch(zz, bb);
    }

    for (; have; have = advance(jc, kc)) {
    int z, bl;
    plane_of(jc, kc, z, bl);
    const int si = seg_of(bl);
    const Seg sg = seg_at(L, si);
    const int nst = sg.nst;
    const int4 *slots = t.slot_info + sg.slot_off;
    const int2 *cols = t.cols + sg.col_off;
    cx<T> *Sz = S + sg.s_off + ((long long)(bl - sg.band_lo) * g.N3 + z) * nst;
    if (si != spos_seg) load_pos(si);
    cx<T> *psiz = psi ? psi + (((band0 + bl) * (long long)g.N3 + z) * N2) * N1 : nullptr;
    const T *Vz = V ? V + (long long)z * N2 * N1 : nullptr;
    double *accz = DENS ? t.partial + ((long long)(bl / bps) * g.N3 + z) * N2 * N1 : nullptr;

    if (MODE != MODE_R2G) {
#pragma unroll
        for (int i = 0; i < PF; ++i)
            if (tid + i * nthr < nst) plane[spos[i]] = sval[i];
        for (int sl = tid + PF * nthr; sl < nst; sl += nthr) plane[slots[sl].w] = Sz[sl];
        for (int i = tid; i < sg.nholes; i += nthr)
            plane[t.holes[sg.hole_off + i]] = mk<T>(T(0), T(0));
        __syncthreads();
        {
            int jn = jc, kn = kc, zz, bb;
            if (advance(jn, kn)) {
                plane_of(jn, kn, zz, bb);
                prefetch(zz, bb);
            }
        }
        // y forward, stage A (lanes along columns)
        with_size<CY1, MR>(L1y, [&](auto RC) {
            constexpr int R = decltype(RC)::value;
            for (int task = tid; task < nxo * L2y; task += nthr) {
                const int n2 = div_nxo(task), hc = task - n2 * nxo;
                const int2 ci = cols[hc];
                cx<T> *col = plane + hc * ldy + n2;
                T xr[R], xi[R];
#pragma unroll
                for (int n1 = 0; n1 < R; ++n1) {
                    cx<T> v = mk<T>(T(0), T(0));
                    if (!masked<ZY>(n1)) {
                        // in-plane read, then select: no divergent branch
                        int rel = n2 + L2y * n1 - ci.x;
                        if (rel < 0) rel += N2;
                        const cx<T> u = col[L2y * n1];
                        if (rel < ci.y) v = u;
                    }
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
        // y forward, stage B (lanes along columns)
        with_size<CY2, MR>(L2y, [&](auto RC) {
            constexpr int R = decltype(RC)::value;
            for (int task = tid; task < nxo * L1y; task += nthr) {
                const int k1 = div_nxo(task), hc = task - k1 * nxo;
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

    if constexpr (XQ > 0) {
        // x pass, one quad of lanes per row: N1 = 4 XQ, lane q of the quad
        // holds x[q + 4 m]; an XQ-point register DFT, twiddles, and the
        // radix-4 step across the quad give X[k + XQ p(q)] on lane q; after
        // the potential the steps run in reverse.
        const int q = tid & 3, y = tid >> 2;
        const double2 *tw64 = t.twx64;
        if (y < N2) {
            const int yp = L2y * (y % L1y) + y / L1y;
            T xr[XQ], xi[XQ];
            if (MODE != MODE_R2G) {
#pragma unroll
                for (int m = 0; m < XQ; ++m) {
                    int hc = q + 4 * m - g.hmin_mod;
                    if (hc < 0) hc += N1;
                    cx<T> v = mk<T>(T(0), T(0));
                    if (hc < nxo) v = plane[hc * ldy + yp];
                    xr[m] = v.x;
                    xi[m] = v.y;
                }
                Dft<XQ, -1, T>::run(xr, xi);
                quad_twiddle<XQ, -1, T>(xr, xi, q, N1, tw64);
                if (MODE == MODE_G2R) quad_radix4<XQ, -1, T>(xr, xi, q);
            }
            const int pq = ((q & 1) << 1) | (q >> 1); // p(q) = {0, 2, 1, 3}
            if (MODE == MODE_G2R) {
                cx<T> *dst = psiz + (long long)y * N1 + XQ * pq;
#pragma unroll
                for (int k = 0; k < XQ; ++k) dst[k] = mk<T>(xr[k], xi[k]);
            } else {
                if (MODE == MODE_APPLY) {
                    quad_radix4_v<XQ, T>(xr, xi, q, Vz + (long long)y * N1 + XQ * pq);
                } else {
                    const cx<T> *src = psiz + (long long)y * N1 + XQ * pq;
#pragma unroll
                    for (int k = 0; k < XQ; ++k) {
                        cx<T> v = src[k];
                        xr[k] = v.x;
                        xi[k] = v.y;
                    }
                    quad_radix4<XQ, +1, T>(xr, xi, q);
                }
                quad_twiddle<XQ, +1, T>(xr, xi, q, N1, tw64);
                Dft<XQ, +1, T>::run(xr, xi);
#pragma unroll
                for (int m = 0; m < XQ; ++m) {
                    int hc = q + 4 * m - g.hmin_mod;
                    if (hc < 0) hc += N1;
                    if (hc < nxo) plane[hc * ldy + yp] = mk<T>(xr[m], xi[m]);
                }
            }
        }
    } else if (wave < g.xw) {
    // x pass: waves 0 .. xw-1 each own a contiguous block of rows and a private
    // row buffer of rb rows; a stage needing more than 64 tasks loops
        const int rpw = (N2 + g.xw - 1) / g.xw;
        const int ybeg = wave * rpw, yend = min(N2, ybeg + rpw);
        for (int y0 = ybeg; y0 < yend; y0 += RB) {
            const int nr = min(RB, yend - y0);
            if (MODE != MODE_R2G) {
                with_size<CX1, MR>(L1x, [&](auto RC) {
                    constexpr int R = decltype(RC)::value;
                    for (int task = lane; task < nr * L2x; task += 64) {
                        const int r = task / L2x, n2 = task - r * L2x;
                        const int y = y0 + r;
                        const int yp = L2y * (y % L1y) + y / L1y;
                        T xr[R], xi[R];
#pragma unroll
                        for (int n1 = 0; n1 < R; ++n1) {
                            cx<T> v = mk<T>(T(0), T(0));
                            if (!masked<ZX>(n1)) {
                                int hc = n2 + L2x * n1 - g.hmin_mod;
                                if (hc < 0) hc += N1;
                                if (hc < nxo) v = plane[hc * ldy + yp];
                            }
                            xr[n1] = v.x;
                            xi[n1] = v.y;
                        }
                        Dft<R, -1, T>::run(xr, xi);
                        twiddle<R, -1, T>(xr, xi, n2, twx);
                        cx<T> *row = rows + r * RL + n2;
#pragma unroll
                        for (int k1 = 0; k1 < R; ++k1) row[(L2x + 1) * k1] = mk<T>(xr[k1], xi[k1]);
                    }
                });
                wave_sync();
            }
            with_size<CX2, MR>(L2x, [&](auto RC) {
                constexpr int R = decltype(RC)::value;
                for (int task = lane; task < nr * L1x; task += 64) {
                    const int r = task / L1x, k1 = task - r * L1x;
                    const int y = y0 + r;
                    cx<T> *row = rows + r * RL + (L2x + 1) * k1;
                    T xr[R], xi[R];
                    T vv[R];
                    if (POT) {
                        const T *vrow = Vz + (long long)y * N1 + k1;
#pragma unroll
                        for (int k2 = 0; k2 < R; ++k2) vv[k2] = vrow[L1x * k2];
                    }
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
                    } else if (MODE == MODE_DENSITY) {
                        // w_b |psi_b(x, y, z)|^2 into this subset's partial plane;
                        // the lane owns these points for every band of the subset
                        const double wb = t.wts[band0 + bl];
                        double *acc = accz + (long long)y * N1 + k1;
#pragma unroll
                        for (int k2 = 0; k2 < R; ++k2) {
                            const double a = (double)xr[k2], b = (double)xi[k2];
                            acc[L1x * k2] += wb * (a * a + b * b);
                        }
                    } else {
                        if (MODE == MODE_APPLY_DENSITY) {
                            const double wb = t.wts[band0 + bl];
                            double *acc = accz + (long long)y * N1 + k1;
#pragma unroll
                            for (int k2 = 0; k2 < R; ++k2) {
                                const double a = (double)xr[k2], b = (double)xi[k2];
                                acc[L1x * k2] += wb * (a * a + b * b);
                            }
                        }
                        if (POT) {
#pragma unroll
                            for (int k2 = 0; k2 < R; ++k2) {
                                xr[k2] *= vv[k2];
                                xi[k2] *= vv[k2];
                            }
                        }
                        Dft<R, +1, T>::run(xr, xi);
#pragma unroll
                        for (int n2 = 0; n2 < R; ++n2) row[n2] = mk<T>(xr[n2], xi[n2]);
                    }
                }
            });
            wave_sync();
            if (MODE != MODE_G2R && MODE != MODE_DENSITY) {
                with_size<CX1, MR>(L1x, [&](auto RC) {
                    constexpr int R = decltype(RC)::value;
                    for (int task = lane; task < nr * L2x; task += 64) {
                        const int r = task / L2x, n2 = task - r * L2x;
                        const int y = y0 + r;
                        const int yp = L2y * (y % L1y) + y / L1y;
                        const cx<T> *row = rows + r * RL + n2;
                        T xr[R], xi[R];
#pragma unroll
                        for (int k1 = 0; k1 < R; ++k1) {
                            cx<T> v = row[(L2x + 1) * k1];
                            xr[k1] = v.x;
                            xi[k1] = v.y;
                        }
                        twiddle<R, +1, T>(xr, xi, n2, twx);
                        Dft<R, +1, T>::run(xr, xi);
#pragma unroll
                        for (int n1 = 0; n1 < R; ++n1) {
                            if (masked<ZX>(n1)) continue;
                            int hc = n2 + L2x * n1 - g.hmin_mod;
                            if (hc < 0) hc += N1;
                            if (hc < nxo) plane[hc * ldy + yp] = mk<T>(xr[n1], xi[n1]);
                        }
                    }
                });
                wave_sync();
            }
        }
    }
    __syncthreads();
    if (MODE == MODE_G2R || MODE == MODE_DENSITY) continue;

    // y reverse, stage B' (lanes along columns)
    with_size<CY2, MR>(L2y, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        for (int task = tid; task < nxo * L1y; task += nthr) {
            const int k1 = div_nxo(task), hc = task - k1 * nxo;
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
    // y reverse, stage A' (lanes along columns): only stick positions are kept
    with_size<CY1, MR>(L1y, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        for (int task = tid; task < nxo * L2y; task += nthr) {
            const int n2 = div_nxo(task), hc = task - n2 * nxo;
            const int2 ci = cols[hc];
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
            for (int n1 = 0; n1 < R; ++n1) {
                if (masked<ZY>(n1)) continue;
                int rel = n2 + L2y * n1 - ci.x;
                if (rel < 0) rel += N2;
                if (rel < ci.y) col[L2y * n1] = mk<T>(xr[n1], xi[n1]);
            }
        }
    });
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PF; ++i)
        if (tid + i * nthr < nst) Sz[tid + i * nthr] = plane[spos[i]];
    for (int sl = tid + PF * nthr; sl < nst; sl += nthr) Sz[sl] = plane[slots[sl].w];
    __syncthreads(); // the next plane's scatter overwrites P
    }
}

// LDS row-buffer variant (any split), up to 512 threads.  The first 4
// slots of each thread are prefetched for the next plane (2048 slots).
template <typename T, int MODE, int CX1, int CX2, int CY1, int CY2, int ZX, int ZY>
__global__ __launch_bounds__(512) void k_plane(Geometry g, DevTables t, Launch L,
                                               cx<T> *__restrict__ S, const T *__restrict__ V,
                                               cx<T> *__restrict__ psi, long long band0)
{
    plane_body<T, MODE, CX1, CX2, CY1, CY2, ZX, ZY, 0, 4, 32>(g, t, L, S, V, psi, band0);
}

// The same with up to 1024 threads (16 waves: more latency hiding for FP64,
// whose plane and row buffers fill the LDS of a CU); 2 prefetched slots per
// thread, 128 registers per lane.
template <typename T, int MODE, int CX1, int CX2, int CY1, int CY2, int ZX, int ZY>
__global__ __launch_bounds__(1024) void k_plane_wide(Geometry g, DevTables t, Launch L,
                                                     cx<T> *__restrict__ S,
                                                     const T *__restrict__ V,
                                                     cx<T> *__restrict__ psi, long long band0)
{
    plane_body<T, MODE, CX1, CX2, CY1, CY2, ZX, ZY, 0, 2, 16>(g, t, L, S, V, psi, band0);
}

// ------------------------------------------------------- K2, full plane
// Full-plane variant of the plane kernel: LDS holds the whole plane P[x][y]
// (N1 columns of N2, column stride ldy), so the x pass runs in place on every
// row and needs no row buffers; its three stages spread over all threads of
// the workgroup with lanes along the (transposed-order) row index, which keeps
// LDS accesses contiguous.  The y pass runs on the occupied columns only.
// Zero masks of the x stage-A groups: ZX = no occupied x (never read, never
// written back), FX = every x occupied (read and written unconditionally);
// other groups check occupancy per position.  Non-occupied positions of a row
// may hold stale values: they are never read as input.  The potential comes
// pre-arranged as VT[z][x][yp] (yp = position of row y after the y pass).
template <typename T, int MODE, int CX1, int CX2, int CY1, int CY2, int ZX, int FX, int ZY, int PF,
          bool WPR, int YT, int MR, int DA = 0>
__device__ __forceinline__ void plane_full_body(const Geometry &g, const DevTables &t,
                                                const Launch &L, cx<T> *__restrict__ S,
                                                const T *__restrict__ VT,
                                                cx<T> *__restrict__ psi, long long band0)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *plane = reinterpret_cast<cx<T> *>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int L1x = CX1 ? CX1 : g.L1x, L2x = CX2 ? CX2 : g.L2x;
    const int L1y = CY1 ? CY1 : g.L1y, L2y = CY2 ? CY2 : g.L2y;
    const int N1 = CX1 ? CX1 * CX2 : g.N1;
    const int N2 = CY1 ? CY1 * CY2 : g.N2;
    const int ldy = CY1 ? CY1 * CY2 + 1 : g.ldy;
    // occupied x-planes of the current segment (set again when a plane of
    // another segment comes up)
    int nxo = L.seg[0].nxo, hx = L.seg[0].hmin_mod;
    unsigned long long nxo_magic = L.seg[0].nxo_magic;
    // task / nxo by a 64-bit multiply and shift (exact for tasks < 2^16)
    auto div_nxo = [&](int v) {
        return (int)(((unsigned long long)(unsigned)v * nxo_magic) >> 40);
    };
    // LDS after the plane: the y and x stage twiddles and the occupied columns'
    // k ranges, so that the transform stages issue no vector-memory loads other
    // than the potential (a wait on one would also wait for the stick-buffer
    // prefetch and stores still in flight)
    cx<T> *twy = plane + N1 * ldy;
    cx<T> *twx = twy + N2;
    int2 *cols = reinterpret_cast<int2 *>(twx + N1);
    for (int i = tid; i < N2; i += nthr) twy[i] = reinterpret_cast<const cx<T> *>(t.twy)[i];
    for (int i = tid; i < N1; i += nthr) twx[i] = reinterpret_cast<const cx<T> *>(t.twx)[i];
    const int nb = L.nbt;
    // column of occupied x-plane hc
    auto col_of = [&](int hc) {
        int x = hx + hc;
        return x >= N1 ? x - N1 : x;
    };
    // x occupied?
    auto occupied = [&](int x) {
        int r = x - hx;
        if (r < 0) r += N1;
        return r < nxo;
    };

    // work items and persistent XCD-aware schedule as in plane_body
    // density scheduling (items = (z, band subset)) and accumulation; the
    // multiply by the potential
    constexpr bool DENS = (MODE == MODE_DENSITY || MODE == MODE_APPLY_DENSITY);
    constexpr bool POT = (MODE == MODE_APPLY || MODE == MODE_APPLY_DENSITY);
    const int nsub = DENS ? g.nsub : 1;
    const int bps = DENS ? (nb + nsub - 1) / nsub : 1;
    const int total = DENS ? g.N3 * nsub : nb * g.N3;
    int j0 = blockIdx.x, jstep = gridDim.x, jend = total;
    if ((gridDim.x & 7) == 0 && (total & 7) == 0) {
        const int share = total >> 3, xcd = blockIdx.x & 7;
        j0 = xcd * share + (blockIdx.x >> 3);
        jstep = gridDim.x >> 3;
        jend = (xcd + 1) * share;
    }
    auto plane_of = [&](int j, int k, int &zz, int &bb) {
        if (DENS) {
            zz = j / nsub;
            bb = (j - zz * nsub) * bps + k;
        } else {
            zz = j / nb;
            bb = j - zz * nb;
        }
    };
    auto advance = [&](int &j, int &k) -> bool {
        for (;;) {
            if (DENS && k + 1 < bps)
                ++k;
            else {
                j += jstep;
                k = 0;
            }
            if (j >= jend) return false;
            int zz, bb;
            plane_of(j, k, zz, bb);
            if (bb < nb) return true;
            k = bps;
        }
    };
    auto seg_of = [&](int bb) { return DENS ? 0 : seg_index_by_band(L, bb); };
    // DA > 0 (density modes, compiled x split, at most DA x stage-B tasks per
    // thread): a thread's stage-B tasks are the same (k1, yp) on every plane,
    // so it sums w_b |psi_b|^2 over the bands of a work item in registers and
    // adds the sums to the item's partial plane once, when the item ends,
    // instead of a read-modify-write of the partial plane per band
    constexpr bool DAC = DA > 0 && DENS && !WPR && CX2 > 0;
    constexpr int NDA = DAC ? DA : 1;
    constexpr int RDA = DAC ? CX2 : 1;
    double dacc[NDA][RDA];
#pragma unroll
    for (int u = 0; u < NDA; ++u)
#pragma unroll
        for (int k2 = 0; k2 < RDA; ++k2) dacc[u][k2] = 0.0;
    // Direct y stage A (launches of one segment, at most YT y tasks per
    // thread): the forward pass takes its stage-A inputs straight from the
    // prefetched stick values and the reverse pass stores its stage-A' outputs
    // straight to S, so the plane needs no scatter and no gather.  A thread's
    // tasks (yhc, yn2) = tid + u nthr and the slots of their positions stay the
    // same for every plane.
    constexpr bool DYC = YT > 0 && CY1 > 0 &&
                         (MODE == MODE_APPLY || MODE == MODE_DENSITY || MODE == MODE_APPLY_DENSITY);
    constexpr int RY = CY1 > 0 ? CY1 : 1;
    constexpr int NU = YT > 0 ? YT : 1;
    const bool dy = DYC && L.nseg == 1 && nxo * L2y <= NU * nthr;
    bool ymine[NU];
    int yn2[NU], yhc[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int task = tid + u * nthr;
        ymine[u] = task < nxo * L2y;
        yn2[u] = div_nxo(task);
        yhc[u] = task - yn2[u] * nxo;
    }
    // Prefetch registers, shared by the two forms: plane positions and values
    // of the slots tid + i nthr (scatter form), or slots and values of the
    // thread's y-task positions (direct form)
    constexpr int NP = (DYC && NU * RY > PF) ? NU * RY : PF;
    int pos[NP];
    cx<T> pre[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        pos[i] = -1;
        pre[i] = mk<T>(T(0), T(0));
    }
    int spos_seg = -1;
    auto load_pos = [&](int si) {
        const Seg sg = seg_at(L, si);
        const int4 *sl_info = t.slot_info + sg.slot_off;
        if (DYC && dy) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int *ys = t.yslot + (long long)(sg.col_off + yhc[u]) * N2 + yn2[u];
#pragma unroll
                for (int n1 = 0; n1 < RY; ++n1)
                    pos[u * RY + n1] = (ymine[u] && !masked<ZY>(n1)) ? ys[L2y * n1] : -1;
            }
        } else {
#pragma unroll
            for (int i = 0; i < PF; ++i) {
                const int sl = tid + i * nthr;
                pos[i] = sl < sg.nst ? sl_info[sl].w : 0;
            }
        }
        // the segment's occupied range and column ranges into LDS (read after
        // the next barrier)
        nxo = sg.nxo;
        hx = sg.hmin_mod;
        nxo_magic = sg.nxo_magic;
        for (int i = tid; i < nxo; i += nthr) cols[i] = t.cols[sg.col_off + i];
        spos_seg = si;
    };
    load_pos(0);
    __syncthreads(); // twiddles and column ranges in LDS
    auto prefetch = [&](int zz, int bb) {
        const Seg sg = seg_at(L, seg_of(bb));
        const cx<T> *Sj = S + sg.s_off + ((long long)(bb - sg.band_lo) * g.N3 + zz) * sg.nst;
        if (DYC && dy) {
#pragma unroll
            for (int i = 0; i < NU * RY; ++i)
                if (!masked<ZY>(i % RY))
                    pre[i] = pos[i] >= 0 ? Sj[pos[i]] : mk<T>(T(0), T(0));
            return;
        }
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int sl = tid + i * nthr;
            if (sl < sg.nst) pre[i] = Sj[sl];
        }
    };
    int jc = j0, kc = 0;
    bool have = jc < jend;
    if (have) {
        int zz, bb;
        plane_of(jc, kc, zz, bb);
        if (bb >= nb) have = advance(jc, kc);
    }
    if (MODE != MODE_R2G && have) {
        int zz, bb;
        plane_of(jc, kc, zz, bb);
        prefetch(zz, bb);
    }

    for (; have; have = advance(jc, kc)) {
    int z, bl;
    plane_of(jc, kc, z, bl);
    const int si = seg_of(bl);
    const Seg sg = seg_at(L, si);
    const int nst = sg.nst;
    const int4 *slots = t.slot_info + sg.slot_off;
    cx<T> *Sz = S + sg.s_off + ((long long)(bl - sg.band_lo) * g.N3 + z) * nst;
    if (si != spos_seg) load_pos(si);
    cx<T> *psiz = psi ? psi + (((band0 + bl) * (long long)g.N3 + z) * N2) * N1 : nullptr;
    const T *VTz = VT ? VT + (long long)z * N1 * N2 : nullptr;
    // density partial plane in [x][yp] order
    double *accz = DENS ? t.partial + ((long long)(bl / bps) * g.N3 + z) * N1 * N2 : nullptr;

    if (MODE != MODE_R2G) {
        if (DYC && dy) {
            // y forward, stage A, from the prefetched stick values (zero where no
            // stick); the thread's positions are the ones it read back last plane
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                if (!ymine[u]) continue;
                cx<T> *col = plane + col_of(yhc[u]) * ldy + yn2[u];
                T xr[RY], xi[RY];
#pragma unroll
                for (int n1 = 0; n1 < RY; ++n1) {
                    xr[n1] = pre[u * RY + n1].x;
                    xi[n1] = pre[u * RY + n1].y;
                }
                Dft<RY, -1, T>::run(xr, xi);
                twiddle_pw<RY, -1, T>(xr, xi, yn2[u], twy);
#pragma unroll
                for (int k1 = 0; k1 < RY; ++k1) col[L2y * k1] = mk<T>(xr[k1], xi[k1]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < PF; ++i)
                if (tid + i * nthr < nst) plane[pos[i]] = pre[i];
            for (int sl = tid + PF * nthr; sl < nst; sl += nthr) plane[slots[sl].w] = Sz[sl];
            for (int i = tid; i < sg.nholes; i += nthr)
                plane[t.holes[sg.hole_off + i]] = mk<T>(T(0), T(0));
            __syncthreads();
            // y forward, stage A (lanes along occupied columns)
            with_size<CY1, MR>(L1y, [&](auto RC) {
                constexpr int R = decltype(RC)::value;
                for (int task = tid; task < nxo * L2y; task += nthr) {
                    const int n2 = div_nxo(task), hc = task - n2 * nxo;
                    const int2 ci = cols[hc];
                    cx<T> *col = plane + col_of(hc) * ldy + n2;
                    T xr[R], xi[R];
#pragma unroll
                    for (int n1 = 0; n1 < R; ++n1) {
                        cx<T> v = mk<T>(T(0), T(0));
                        if (!masked<ZY>(n1)) {
                            // in-plane read, then select: no divergent branch
                            int rel = n2 + L2y * n1 - ci.x;
                            if (rel < 0) rel += N2;
                            const cx<T> u = col[L2y * n1];
                            if (rel < ci.y) v = u;
                        }
                        xr[n1] = v.x;
                        xi[n1] = v.y;
                    }
                    Dft<R, -1, T>::run(xr, xi);
                    twiddle_pw<R, -1, T>(xr, xi, n2, twy);
#pragma unroll
                    for (int k1 = 0; k1 < R; ++k1) col[L2y * k1] = mk<T>(xr[k1], xi[k1]);
                }
            });
        }
        __syncthreads();
        // y forward, stage B
        with_size<CY2, MR>(L2y, [&](auto RC) {
            constexpr int R = decltype(RC)::value;
            for (int task = tid; task < nxo * L1y; task += nthr) {
                const int k1 = div_nxo(task), hc = task - k1 * nxo;
                cx<T> *col = plane + col_of(hc) * ldy + L2y * k1;
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

    // x pass.  stage_a: forward x stage A of row yp for n2 (inputs x = n2 + L2x n1);
    // stage_b: stage B of row yp for k1 (frequencies x = k1 + L1x k2) with the
    // potential, the density or the real-space values; stage_a2: reverse stage
    // A', occupied outputs only.  All in place in P.
    auto stage_a = [&](int n2, int yp) {
        with_size<CX1, MR>(L1x, [&](auto RC) {
            constexpr int R = decltype(RC)::value;
            cx<T> *row = plane + n2 * ldy + yp;
            T xr[R], xi[R];
#pragma unroll
            for (int n1 = 0; n1 < R; ++n1) {
                cx<T> v = mk<T>(T(0), T(0));
                if (!masked<ZX>(n1)) {
                    const cx<T> u = row[L2x * n1 * ldy];
                    if (masked<FX>(n1) || occupied(n2 + L2x * n1)) v = u;
                }
                xr[n1] = v.x;
                xi[n1] = v.y;
            }
            Dft<R, -1, T>::run(xr, xi);
            twiddle_pw<R, -1, T>(xr, xi, n2, twx);
#pragma unroll
            for (int k1 = 0; k1 < R; ++k1) row[L2x * k1 * ldy] = mk<T>(xr[k1], xi[k1]);
        });
    };
    // w_b |psi_b|^2 of one stage-B task (x = k1 + L1x k2, row yp) into the
    // registers of the thread's task u, or straight into the partial plane
    auto add_density = [&](auto RC, const T *xr, const T *xi, int k1, int yp, int u) {
        constexpr int R = decltype(RC)::value;
        const double wb = t.wts[band0 + bl];
        if constexpr (DAC) {
#pragma unroll
            for (int k2 = 0; k2 < RDA; ++k2) {
                const double a = (double)xr[k2], b = (double)xi[k2];
                dacc[u][k2] += wb * (a * a + b * b);
            }
        } else {
            double *acc = accz + (long long)k1 * N2 + yp;
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) {
                const double a = (double)xr[k2], b = (double)xi[k2];
                acc[(long long)L1x * k2 * N2] += wb * (a * a + b * b);
            }
        }
    };
    auto stage_b = [&](int k1, int yp, int u) {
        with_size<CX2, MR>(L2x, [&](auto RC) {
            constexpr int R = decltype(RC)::value;
            cx<T> *row = plane + L2x * k1 * ldy + yp;
            T xr[R], xi[R];
            T vv[R];
            if (POT) {
                // the task's R values of the potential are contiguous
                const T *vrun = VTz + ((long long)k1 * N2 + yp) * R;
#pragma unroll
                for (int k2 = 0; k2 < R; ++k2) vv[k2] = vrun[k2];
            }
            // natural row index of position yp (psi is [z][y][x])
            const int y = (yp % L2y) * L1y + yp / L2y;
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
                    cx<T> v = row[n2 * ldy];
                    xr[n2] = v.x;
                    xi[n2] = v.y;
                }
                Dft<R, -1, T>::run(xr, xi);
            }
            if (MODE == MODE_G2R) {
                cx<T> *dst = psiz + (long long)y * N1 + k1;
#pragma unroll
                for (int k2 = 0; k2 < R; ++k2) dst[L1x * k2] = mk<T>(xr[k2], xi[k2]);
            } else if (MODE == MODE_DENSITY) {
                add_density(RC, xr, xi, k1, yp, u);
            } else {
                if (MODE == MODE_APPLY_DENSITY) add_density(RC, xr, xi, k1, yp, u);
                if (POT) {
#pragma unroll
                    for (int k2 = 0; k2 < R; ++k2) {
                        xr[k2] *= vv[k2];
                        xi[k2] *= vv[k2];
                    }
                }
                Dft<R, +1, T>::run(xr, xi);
#pragma unroll
                for (int n2 = 0; n2 < R; ++n2) row[n2 * ldy] = mk<T>(xr[n2], xi[n2]);
            }
        });
    };
    auto stage_a2 = [&](int n2, int yp) {
        with_size<CX1, MR>(L1x, [&](auto RC) {
            constexpr int R = decltype(RC)::value;
            cx<T> *row = plane + n2 * ldy + yp;
            T xr[R], xi[R];
#pragma unroll
            for (int k1 = 0; k1 < R; ++k1) {
                cx<T> v = row[L2x * k1 * ldy];
                xr[k1] = v.x;
                xi[k1] = v.y;
            }
            twiddle_pw<R, +1, T>(xr, xi, n2, twx);
            Dft<R, +1, T>::run(xr, xi);
#pragma unroll
            for (int n1 = 0; n1 < R; ++n1) {
                if (masked<ZX>(n1)) continue;
                if (masked<FX>(n1) || occupied(n2 + L2x * n1))
                    row[L2x * n1 * ldy] = mk<T>(xr[n1], xi[n1]);
            }
        });
    };
    constexpr bool XPASS_ONLY_FWD = (MODE == MODE_G2R || MODE == MODE_DENSITY);
    auto prefetch_next = [&]() {
        if (MODE == MODE_R2G) return;
        int jn = jc, kn = kc, zz, bb;
        if (advance(jn, kn)) {
            plane_of(jn, kn, zz, bb);
            prefetch(zz, bb);
        }
    };
    if constexpr (WPR) {
        // each wavefront owns a block of rows (in yp order), in batches whose
        // stage-A tasks fill at most one wavefront; only wavefront ordering
        const int lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
        const int rpw = (N2 + nwaves - 1) / nwaves;
        const int ybeg = min(N2, wave * rpw), yend = min(N2, ybeg + rpw);
        const int rbx = L2x >= 64 ? 1 : 64 / L2x;
        for (int y0 = ybeg; y0 < yend; y0 += rbx) {
            const int nr = min(rbx, yend - y0);
            if (MODE != MODE_R2G) {
                for (int task = lane; task < nr * L2x; task += 64)
                    stage_a(task / nr, y0 + task % nr);
                wave_sync();
            }
            for (int task = lane; task < nr * L1x; task += 64)
                stage_b(task / nr, y0 + task % nr, 0);
            wave_sync();
            if (!XPASS_ONLY_FWD) {
                for (int task = lane; task < nr * L2x; task += 64)
                    stage_a2(task / nr, y0 + task % nr);
                wave_sync();
            }
        }
        prefetch_next();
        __syncthreads();
        if (XPASS_ONLY_FWD) continue;
    } else {
        // the three stages spread over the whole workgroup, lanes along yp
        if (MODE != MODE_R2G) {
            for (int task = tid; task < L2x * N2; task += nthr) stage_a(task / N2, task % N2);
            __syncthreads();
        }
        if constexpr (DAC) {
            // the thread's tasks u (at most NDA, checked by the launcher); the
            // sums go to the partial plane when the next plane is another item's
#pragma unroll
            for (int u = 0; u < NDA; ++u) {
                const int task = tid + u * nthr;
                if (task < L1x * N2) stage_b(task / N2, task % N2, u);
            }
            int jn = jc, kn = kc;
            if (!advance(jn, kn) || jn != jc) {
#pragma unroll
                for (int u = 0; u < NDA; ++u) {
                    const int task = tid + u * nthr;
                    if (task >= L1x * N2) continue;
                    double *acc = accz + (long long)(task / N2) * N2 + task % N2;
#pragma unroll
                    for (int k2 = 0; k2 < RDA; ++k2) {
                        acc[(long long)L1x * k2 * N2] += dacc[u][k2];
                        dacc[u][k2] = 0.0;
                    }
                }
            }
        } else {
            for (int task = tid; task < L1x * N2; task += nthr) stage_b(task / N2, task % N2, 0);
        }
        // the next plane's stick values: issued after the potential's loads, so
        // their latency hides behind the reverse stages
        prefetch_next();
        __syncthreads();
        if (XPASS_ONLY_FWD) continue;
        for (int task = tid; task < L2x * N2; task += nthr) stage_a2(task / N2, task % N2);
        __syncthreads();
    }
    // y reverse, stage B'
    with_size<CY2, MR>(L2y, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        for (int task = tid; task < nxo * L1y; task += nthr) {
            const int k1 = div_nxo(task), hc = task - k1 * nxo;
            cx<T> *col = plane + col_of(hc) * ldy + L2y * k1;
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
    if (DYC && dy) {
        // y reverse, stage A', stick positions stored straight to S; the next
        // plane's stage A writes only this thread's positions, so no barrier
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            if (!ymine[u]) continue;
            cx<T> *col = plane + col_of(yhc[u]) * ldy + yn2[u];
            T xr[RY], xi[RY];
#pragma unroll
            for (int k1 = 0; k1 < RY; ++k1) {
                cx<T> v = col[L2y * k1];
                xr[k1] = v.x;
                xi[k1] = v.y;
            }
            twiddle_pw<RY, +1, T>(xr, xi, yn2[u], twy);
            Dft<RY, +1, T>::run(xr, xi);
#pragma unroll
            for (int n1 = 0; n1 < RY; ++n1) {
                if (masked<ZY>(n1)) continue;
                if (pos[u * RY + n1] >= 0) Sz[pos[u * RY + n1]] = mk<T>(xr[n1], xi[n1]);
            }
        }
        continue;
    }
    // y reverse, stage A': only stick positions are kept
    with_size<CY1, MR>(L1y, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        for (int task = tid; task < nxo * L2y; task += nthr) {
            const int n2 = div_nxo(task), hc = task - n2 * nxo;
            const int2 ci = cols[hc];
            cx<T> *col = plane + col_of(hc) * ldy + n2;
            T xr[R], xi[R];
#pragma unroll
            for (int k1 = 0; k1 < R; ++k1) {
                cx<T> v = col[L2y * k1];
                xr[k1] = v.x;
                xi[k1] = v.y;
            }
            twiddle_pw<R, +1, T>(xr, xi, n2, twy);
            Dft<R, +1, T>::run(xr, xi);
#pragma unroll
            for (int n1 = 0; n1 < R; ++n1) {
                if (masked<ZY>(n1)) continue;
                int rel = n2 + L2y * n1 - ci.x;
                if (rel < 0) rel += N2;
                if (rel < ci.y) col[L2y * n1] = mk<T>(xr[n1], xi[n1]);
            }
        }
    });
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PF; ++i)
        if (tid + i * nthr < nst) Sz[tid + i * nthr] = plane[pos[i]];
    for (int sl = tid + PF * nthr; sl < nst; sl += nthr) Sz[sl] = plane[slots[sl].w];
    __syncthreads(); // the next plane's scatter overwrites P
    }
}

// YT > 0: the direct y form with up to YT y tasks per thread (chosen by the
// launcher when the geometry allows it; a separate instantiation, so that the
// scatter form does not carry its registers)
// GMR > 0: the runtime-sized kernel compiled for line codelets of at most
// GMR points only
// DA > 0: density sums in registers over the x stage-B tasks of a thread (at
// most DA of them)
template <typename T, int MODE, int CX1, int CX2, int CY1, int CY2, int ZX, int FX, int ZY,
          int MAXT, bool WPR, int YT, int GMR = 0, int DA = 0>
__global__ __launch_bounds__(MAXT) void k_plane_full(Geometry g, DevTables t, Launch L,
                                                     cx<T> *__restrict__ S,
                                                     const T *__restrict__ VT,
                                                     cx<T> *__restrict__ psi, long long band0)
{
    // prefetched slots per thread cover 2048 slots
    plane_full_body<T, MODE, CX1, CX2, CY1, CY2, ZX, FX, ZY, (2048 + MAXT - 1) / MAXT, WPR, YT,
                    (GMR ? GMR : (MAXT > 512 ? 16 : 32)), DA>(g, t, L, S, VT, psi, band0);
}

// ------------------------------------------------------- K2, parted plane
// For planes that do not fit in LDS whole.  The y passes run on the occupied
// columns C (nxo x N2, stride ldy, indexed by occupied column hc); the x pass
// runs in P parts of rpp = N2 / P rows (positions yp of the transposed row
// order) through one row buffer R (N1 x (rpp + 1), column stride rpp + 1) that
// shares the LDS with C.  The rows of the parts that are not in R wait in a
// per-workgroup device scratch G (nxo x N2 values, [hc][yp], small enough to
// stay mostly in L2):
//   y stage B      writes part 0 into R and the other parts into G;
//   x stage A      of part p > 0 reads its occupied inputs from G;
//   x stage A'     of part p < P - 1 writes its occupied outputs into G, the
//                  last part keeps them in R;
//   y stage B'     reads part P - 1 from R and the others from G, then rebuilds C.
// rpp is a multiple of L2y, so that the rows of one y stage-B line (positions
// [L2y k1, L2y k1 + L2y)) lie in one part.  Because R overlaps C, the y stage-B
// lines that write R (part 0) and the y stage-B' lines that read it (part
// P - 1) hold their values across a barrier, in one round (nxo L1y / P <=
// threads, checked by the planner).  The y passes use the scatter form (sticks
// scattered into C and gathered back).  The stage arithmetic is that of the
// whole-plane kernel.
template <typename T, int MODE, int CX1, int CX2, int CY1, int CY2, int ZX, int FX, int ZY, int PF,
          int MR, int DA = 0>
__device__ __forceinline__ void plane_parts_body(const Geometry &g, const DevTables &t,
                                                 const Launch &L, cx<T> *__restrict__ S,
                                                 const T *__restrict__ VT,
                                                 cx<T> *__restrict__ psi, long long band0)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int L1x = CX1 ? CX1 : g.L1x, L2x = CX2 ? CX2 : g.L2x;
    const int L1y = CY1 ? CY1 : g.L1y, L2y = CY2 ? CY2 : g.L2y;
    const int N1 = CX1 ? CX1 * CX2 : g.N1;
    const int N2 = CY1 ? CY1 * CY2 : g.N2;
    const int ldy = CY1 ? CY1 * CY2 + 1 : g.ldy;
    const int P = g.parts, rpp = N2 / P, ldr = rpp + 1;
    const int nxo = g.nxo, hx = g.hmin_mod;
    auto div_nxo = [&](int v) {
        return (int)(((unsigned long long)(unsigned)v * g.nxo_magic) >> 40);
    };
    cx<T> *twy = buf + g.parts_elems;
    cx<T> *twx = twy + N2;
    int2 *cols = reinterpret_cast<int2 *>(twx + N1);
    for (int i = tid; i < N2; i += nthr) twy[i] = reinterpret_cast<const cx<T> *>(t.twy)[i];
    for (int i = tid; i < N1; i += nthr) twx[i] = reinterpret_cast<const cx<T> *>(t.twx)[i];
    // this workgroup's scratch rows
    cx<T> *G = reinterpret_cast<cx<T> *>(t.parts) + (long long)blockIdx.x * nxo * N2;
    const int nb = L.nbt;
    auto col_of = [&](int hc) {
        int x = hx + hc;
        return x >= N1 ? x - N1 : x;
    };
    // occupied column of x, or a value >= nxo
    auto hc_of = [&](int x) {
        int r = x - hx;
        return r < 0 ? r + N1 : r;
    };

    // persistent XCD-aware schedule and density items as in the whole-plane kernel
    constexpr bool DENS = (MODE == MODE_DENSITY || MODE == MODE_APPLY_DENSITY);
    constexpr bool POT = (MODE == MODE_APPLY || MODE == MODE_APPLY_DENSITY);
    const int nsub = DENS ? g.nsub : 1;
    const int bps = DENS ? (nb + nsub - 1) / nsub : 1;
    const int total = DENS ? g.N3 * nsub : nb * g.N3;
    int j0 = blockIdx.x, jstep = gridDim.x, jend = total;
    if ((gridDim.x & 7) == 0 && (total & 7) == 0) {
        const int share = total >> 3, xcd = blockIdx.x & 7;
        j0 = xcd * share + (blockIdx.x >> 3);
        jstep = gridDim.x >> 3;
        jend = (xcd + 1) * share;
    }
    auto plane_of = [&](int j, int k, int &zz, int &bb) {
        if (DENS) {
            zz = j / nsub;
            bb = (j - zz * nsub) * bps + k;
        } else {
            zz = j / nb;
            bb = j - zz * nb;
        }
    };
    auto advance = [&](int &j, int &k) -> bool {
        for (;;) {
            if (DENS && k + 1 < bps)
                ++k;
            else {
                j += jstep;
                k = 0;
            }
            if (j >= jend) return false;
            int zz, bb;
            plane_of(j, k, zz, bb);
            if (bb < nb) return true;
            k = bps;
        }
    };
    auto seg_of = [&](int bb) { return DENS ? 0 : seg_index_by_band(L, bb); };
    // prefetched stick values of slots tid + i nthr and their positions in C
    int pos[PF];
    cx<T> pre[PF];
#pragma unroll
    for (int i = 0; i < PF; ++i) {
        pos[i] = 0;
        pre[i] = mk<T>(T(0), T(0));
    }
    int spos_seg = -1;
    auto load_pos = [&](int si) {
        const Seg sg = seg_at(L, si);
        const int4 *sl_info = t.slot_info + sg.slot_off;
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int sl = tid + i * nthr;
            pos[i] = sl < sg.nst ? sl_info[sl].w : 0;
        }
        for (int i = tid; i < nxo; i += nthr) cols[i] = t.cols[sg.col_off + i];
        spos_seg = si;
    };
    load_pos(0);
    __syncthreads(); // twiddles and column ranges in LDS
    auto prefetch = [&](int zz, int bb) {
        const Seg sg = seg_at(L, seg_of(bb));
        const cx<T> *Sj = S + sg.s_off + ((long long)(bb - sg.band_lo) * g.N3 + zz) * sg.nst;
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int sl = tid + i * nthr;
            if (sl < sg.nst) pre[i] = Sj[sl];
        }
    };
    int jc = j0, kc = 0;
    bool have = jc < jend;
    if (have) {
        int zz, bb;
        plane_of(jc, kc, zz, bb);
        if (bb >= nb) have = advance(jc, kc);
    }
    if (MODE != MODE_R2G && have) {
        int zz, bb;
        plane_of(jc, kc, zz, bb);
        prefetch(zz, bb);
    }
    constexpr bool XPASS_ONLY_FWD = (MODE == MODE_G2R || MODE == MODE_DENSITY);
    // DA > 0 (density modes, compiled splits, P = DA parts of at most one x
    // stage-B task per thread): the thread's stage-B task of each part is the
    // same on every plane, so the density sums of a work item stay in
    // registers, the part in progress in dacc[0] (the array rotates by one
    // after each part) and go to the partial plane when the item ends.  These
    // kernels run 512 threads (256 registers each), so the y stage-B lines
    // held across a barrier may take a second round (TWO).
    constexpr bool DAC = DA > 0 && DENS && CX2 > 0;
    constexpr bool TWO = DAC;
    constexpr int NDA = DAC ? DA : 1;
    constexpr int RDA = DAC ? CX2 : 1;
    double dacc[NDA][RDA];
#pragma unroll
    for (int u = 0; u < NDA; ++u)
#pragma unroll
        for (int k2 = 0; k2 < RDA; ++k2) dacc[u][k2] = 0.0;

    for (; have; have = advance(jc, kc)) {
    int z, bl;
    plane_of(jc, kc, z, bl);
    const int si = seg_of(bl);
    const Seg sg = seg_at(L, si);
    const int nst = sg.nst;
    const int4 *slots = t.slot_info + sg.slot_off;
    cx<T> *Sz = S + sg.s_off + ((long long)(bl - sg.band_lo) * g.N3 + z) * nst;
    if (si != spos_seg) load_pos(si);
    cx<T> *psiz = psi ? psi + (((band0 + bl) * (long long)g.N3 + z) * N2) * N1 : nullptr;
    const T *VTz = VT ? VT + (long long)z * N1 * N2 : nullptr;
    double *accz = DENS ? t.partial + ((long long)(bl / bps) * g.N3 + z) * N1 * N2 : nullptr;

    if (MODE != MODE_R2G) {
        // sticks into C, zeros at the holes of the columns' k spans
#pragma unroll
        for (int i = 0; i < PF; ++i)
            if (tid + i * nthr < nst) buf[pos[i]] = pre[i];
        for (int sl = tid + PF * nthr; sl < nst; sl += nthr) buf[slots[sl].w] = Sz[sl];
        for (int i = tid; i < sg.nholes; i += nthr)
            buf[t.holes[sg.hole_off + i]] = mk<T>(T(0), T(0));
        __syncthreads();
        // y forward, stage A (lanes along occupied columns)
        with_size<CY1, MR>(L1y, [&](auto RC) {
            constexpr int R = decltype(RC)::value;
            for (int task = tid; task < nxo * L2y; task += nthr) {
                const int n2 = div_nxo(task), hc = task - n2 * nxo;
                const int2 ci = cols[hc];
                cx<T> *col = buf + hc * ldy + n2;
                T xr[R], xi[R];
#pragma unroll
                for (int n1 = 0; n1 < R; ++n1) {
                    cx<T> v = mk<T>(T(0), T(0));
                    if (!masked<ZY>(n1)) {
                        int rel = n2 + L2y * n1 - ci.x;
                        if (rel < 0) rel += N2;
                        const cx<T> u = col[L2y * n1];
                        if (rel < ci.y) v = u;
                    }
                    xr[n1] = v.x;
                    xi[n1] = v.y;
                }
                Dft<R, -1, T>::run(xr, xi);
                twiddle_pw<R, -1, T>(xr, xi, n2, twy);
#pragma unroll
                for (int k1 = 0; k1 < R; ++k1) col[L2y * k1] = mk<T>(xr[k1], xi[k1]);
            }
        });
        __syncthreads();
        // y forward, stage B.  Lines of parts 1.. go to G with no wait; the
        // lines of part 0 go to R, which overlaps C: they read every input
        // before a barrier and write after it (one round, nxo L1y / P tasks)
        with_size<CY2, MR>(L2y, [&](auto RC) {
            constexpr int R = decltype(RC)::value;
            const int k1r = L1y / P; // lines k1 < k1r hold the rows of part 0
            auto line = [&](int hc, int k1, T *xr, T *xi) {
                const cx<T> *col = buf + hc * ldy + L2y * k1;
#pragma unroll
                for (int n2 = 0; n2 < R; ++n2) {
                    cx<T> v = col[n2];
                    xr[n2] = v.x;
                    xi[n2] = v.y;
                }
                Dft<R, -1, T>::run(xr, xi);
            };
            for (int task = tid; task < nxo * (L1y - k1r); task += nthr) {
                const int k1 = k1r + div_nxo(task), hc = task - (k1 - k1r) * nxo;
                T xr[R], xi[R];
                line(hc, k1, xr, xi);
                cx<T> *dst = G + (long long)hc * N2 + L2y * k1;
#pragma unroll
                for (int k2 = 0; k2 < R; ++k2) dst[k2] = mk<T>(xr[k2], xi[k2]);
            }
            const int task = tid;
            const bool act = task < nxo * k1r;
            const int k1 = div_nxo(task), hc = task - k1 * nxo;
            T xr[R], xi[R];
            if (act) line(hc, k1, xr, xi);
            // second round (TWO): line tid + nthr
            constexpr int R2 = TWO ? R : 1;
            const int tb = tid + nthr;
            const bool actb = TWO && tb < nxo * k1r;
            const int k1b = div_nxo(tb), hcb = tb - k1b * nxo;
            T yr[R2], yi[R2];
            if constexpr (TWO)
                if (actb) line(hcb, k1b, yr, yi);
            __syncthreads();
            if (act) {
                cx<T> *dst = buf + col_of(hc) * ldr + L2y * k1;
#pragma unroll
                for (int k2 = 0; k2 < R; ++k2) dst[k2] = mk<T>(xr[k2], xi[k2]);
            }
            if constexpr (TWO)
                if (actb) {
                    cx<T> *dst = buf + col_of(hcb) * ldr + L2y * k1b;
#pragma unroll
                    for (int k2 = 0; k2 < R; ++k2) dst[k2] = mk<T>(yr[k2], yi[k2]);
                }
        });
        __syncthreads();
    }

    // x pass, part by part: stage_a forward stage A of row yp (= yb + r) for
    // n2; stage_b stage B for k1 with the potential, the density or the
    // real-space values; stage_a2 reverse stage A', occupied outputs only
    // w_b |psi_b|^2 of one stage-B task into the registers of the part in
    // progress, or straight into the partial plane
    auto add_density = [&](auto RC, const T *xr, const T *xi, int k1, int yp) {
        constexpr int R = decltype(RC)::value;
        const double wb = t.wts[band0 + bl];
        if constexpr (DAC) {
#pragma unroll
            for (int k2 = 0; k2 < RDA; ++k2) {
                const double a = (double)xr[k2], b = (double)xi[k2];
                dacc[0][k2] += wb * (a * a + b * b);
            }
        } else {
            double *acc = accz + (long long)k1 * N2 + yp;
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) {
                const double a = (double)xr[k2], b = (double)xi[k2];
                acc[(long long)L1x * k2 * N2] += wb * (a * a + b * b);
            }
        }
    };
    for (int part = 0; part < P; ++part) {
        const int yb = part * rpp;
        const bool first = part == 0, last = part == P - 1;
        if (MODE != MODE_R2G) {
            with_size<CX1, MR>(L1x, [&](auto RC) {
                constexpr int R = decltype(RC)::value;
                for (int task = tid; task < L2x * rpp; task += nthr) {
                    const int n2 = task / rpp, r = task - n2 * rpp;
                    cx<T> *row = buf + n2 * ldr + r;
                    T xr[R], xi[R];
#pragma unroll
                    for (int n1 = 0; n1 < R; ++n1) {
                        cx<T> v = mk<T>(T(0), T(0));
                        if (!masked<ZX>(n1)) {
                            const int x = n2 + L2x * n1;
                            const int hc = hc_of(x);
                            const bool occ = masked<FX>(n1) || hc < nxo;
                            if (first) {
                                const cx<T> u = row[L2x * n1 * ldr];
                                if (occ) v = u;
                            } else if (occ) {
                                v = G[(long long)hc * N2 + yb + r];
                            }
                        }
                        xr[n1] = v.x;
                        xi[n1] = v.y;
                    }
                    Dft<R, -1, T>::run(xr, xi);
                    twiddle_pw<R, -1, T>(xr, xi, n2, twx);
#pragma unroll
                    for (int k1 = 0; k1 < R; ++k1) row[L2x * k1 * ldr] = mk<T>(xr[k1], xi[k1]);
                }
            });
            __syncthreads();
        }
        with_size<CX2, MR>(L2x, [&](auto RC) {
            constexpr int R = decltype(RC)::value;
            for (int task = tid; task < L1x * rpp; task += nthr) {
                const int k1 = task / rpp, r = task - k1 * rpp, yp = yb + r;
                cx<T> *row = buf + L2x * k1 * ldr + r;
                T xr[R], xi[R];
                T vv[R];
                if (POT) {
                    const T *vrun = VTz + ((long long)k1 * N2 + yp) * R;
#pragma unroll
                    for (int k2 = 0; k2 < R; ++k2) vv[k2] = vrun[k2];
                }
                const int y = (yp % L2y) * L1y + yp / L2y;
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
                        cx<T> v = row[n2 * ldr];
                        xr[n2] = v.x;
                        xi[n2] = v.y;
                    }
                    Dft<R, -1, T>::run(xr, xi);
                }
                if (MODE == MODE_G2R) {
                    cx<T> *dst = psiz + (long long)y * N1 + k1;
#pragma unroll
                    for (int k2 = 0; k2 < R; ++k2) dst[L1x * k2] = mk<T>(xr[k2], xi[k2]);
                } else if (MODE == MODE_DENSITY) {
                    add_density(RC, xr, xi, k1, yp);
                } else {
                    if (MODE == MODE_APPLY_DENSITY) add_density(RC, xr, xi, k1, yp);
                    if (POT) {
#pragma unroll
                        for (int k2 = 0; k2 < R; ++k2) {
                            xr[k2] *= vv[k2];
                            xi[k2] *= vv[k2];
                        }
                    }
                    Dft<R, +1, T>::run(xr, xi);
#pragma unroll
                    for (int n2 = 0; n2 < R; ++n2) row[n2 * ldr] = mk<T>(xr[n2], xi[n2]);
                }
            }
        });
        if constexpr (DAC && NDA > 1) {
#pragma unroll
            for (int k2 = 0; k2 < RDA; ++k2) {
                const double d0 = dacc[0][k2];
#pragma unroll
                for (int u = 0; u + 1 < NDA; ++u) dacc[u][k2] = dacc[u + 1][k2];
                dacc[NDA - 1][k2] = d0;
            }
        }
        if (last && MODE != MODE_R2G) {
            // the next plane's stick values, issued after the potential's loads
            int jn = jc, kn = kc, zz, bb;
            if (advance(jn, kn)) {
                plane_of(jn, kn, zz, bb);
                prefetch(zz, bb);
            }
        }
        __syncthreads();
        if (XPASS_ONLY_FWD) continue;
        with_size<CX1, MR>(L1x, [&](auto RC) {
            constexpr int R = decltype(RC)::value;
            for (int task = tid; task < L2x * rpp; task += nthr) {
                const int n2 = task / rpp, r = task - n2 * rpp;
                cx<T> *row = buf + n2 * ldr + r;
                T xr[R], xi[R];
#pragma unroll
                for (int k1 = 0; k1 < R; ++k1) {
                    cx<T> v = row[L2x * k1 * ldr];
                    xr[k1] = v.x;
                    xi[k1] = v.y;
                }
                twiddle_pw<R, +1, T>(xr, xi, n2, twx);
                Dft<R, +1, T>::run(xr, xi);
#pragma unroll
                for (int n1 = 0; n1 < R; ++n1) {
                    if (masked<ZX>(n1)) continue;
                    const int x = n2 + L2x * n1;
                    const int hc = hc_of(x);
                    if (!masked<FX>(n1) && hc >= nxo) continue;
                    if (last)
                        row[L2x * n1 * ldr] = mk<T>(xr[n1], xi[n1]);
                    else
                        G[(long long)hc * N2 + yb + r] = mk<T>(xr[n1], xi[n1]);
                }
            }
        });
        __syncthreads();
    }
    if constexpr (DAC) {
        // the item's sums to its partial plane when the next plane is another item's
        int jn = jc, kn = kc;
        if ((!advance(jn, kn) || jn != jc) && tid < L1x * rpp) {
            const int k1 = tid / rpp, r = tid - k1 * rpp;
#pragma unroll
            for (int u = 0; u < NDA; ++u) {
                double *acc = accz + (long long)k1 * N2 + u * rpp + r;
#pragma unroll
                for (int k2 = 0; k2 < RDA; ++k2) {
                    acc[(long long)L1x * k2 * N2] += dacc[u][k2];
                    dacc[u][k2] = 0.0;
                }
            }
        }
    }
    if (XPASS_ONLY_FWD) continue;
    // y reverse, stage B', then C rebuilt (it overlaps R): the lines of the
    // last part read R before a barrier (one round, nxo L1y / P tasks), the
    // lines of the other parts read G after it
    with_size<CY2, MR>(L2y, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        const int k1l = L1y - L1y / P; // lines k1 >= k1l hold the rows of the last part
        auto put = [&](int hc, int k1, T *xr, T *xi) {
            Dft<R, +1, T>::run(xr, xi);
            cx<T> *col = buf + hc * ldy + L2y * k1;
#pragma unroll
            for (int n2 = 0; n2 < R; ++n2) col[n2] = mk<T>(xr[n2], xi[n2]);
        };
        const int task = tid;
        const bool act = task < nxo * (L1y - k1l);
        const int k1 = k1l + div_nxo(task), hc = task - (k1 - k1l) * nxo;
        T xr[R], xi[R];
        if (act) {
            const cx<T> *src = buf + col_of(hc) * ldr + (L2y * k1 - (P - 1) * rpp);
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) {
                cx<T> v = src[k2];
                xr[k2] = v.x;
                xi[k2] = v.y;
            }
        }
        // second round (TWO): line tid + nthr
        constexpr int R2 = TWO ? R : 1;
        const int tb = tid + nthr;
        const bool actb = TWO && tb < nxo * (L1y - k1l);
        const int k1b = k1l + div_nxo(tb), hcb = tb - (k1b - k1l) * nxo;
        T yr2[R2], yi2[R2];
        if constexpr (TWO)
            if (actb) {
                const cx<T> *src = buf + col_of(hcb) * ldr + (L2y * k1b - (P - 1) * rpp);
#pragma unroll
                for (int k2 = 0; k2 < R; ++k2) {
                    cx<T> v = src[k2];
                    yr2[k2] = v.x;
                    yi2[k2] = v.y;
                }
            }
        __syncthreads();
        if (act) put(hc, k1, xr, xi);
        if constexpr (TWO)
            if (actb) put(hcb, k1b, yr2, yi2);
        for (int tg = tid; tg < nxo * k1l; tg += nthr) {
            const int k1g = div_nxo(tg), hcg = tg - k1g * nxo;
            const cx<T> *src = G + (long long)hcg * N2 + L2y * k1g;
            T yr[R], yi[R];
#pragma unroll
            for (int k2 = 0; k2 < R; ++k2) {
                cx<T> v = src[k2];
                yr[k2] = v.x;
                yi[k2] = v.y;
            }
            put(hcg, k1g, yr, yi);
        }
    });
    __syncthreads();
    // y reverse, stage A': only stick positions are kept
    with_size<CY1, MR>(L1y, [&](auto RC) {
        constexpr int R = decltype(RC)::value;
        for (int task = tid; task < nxo * L2y; task += nthr) {
            const int n2 = div_nxo(task), hc = task - n2 * nxo;
            const int2 ci = cols[hc];
            cx<T> *col = buf + hc * ldy + n2;
            T xr[R], xi[R];
#pragma unroll
            for (int k1 = 0; k1 < R; ++k1) {
                cx<T> v = col[L2y * k1];
                xr[k1] = v.x;
                xi[k1] = v.y;
            }
            twiddle_pw<R, +1, T>(xr, xi, n2, twy);
            Dft<R, +1, T>::run(xr, xi);
#pragma unroll
            for (int n1 = 0; n1 < R; ++n1) {
                if (masked<ZY>(n1)) continue;
                int rel = n2 + L2y * n1 - ci.x;
                if (rel < 0) rel += N2;
                if (rel < ci.y) col[L2y * n1] = mk<T>(xr[n1], xi[n1]);
            }
        }
    });
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PF; ++i)
        if (tid + i * nthr < nst) Sz[tid + i * nthr] = buf[pos[i]];
    for (int sl = tid + PF * nthr; sl < nst; sl += nthr) Sz[sl] = buf[slots[sl].w];
    __syncthreads(); // the next plane's scatter overwrites C
    }
}

// DA > 0: density sums in registers over DA parts (one x stage-B task per
// thread and part)
template <typename T, int MODE, int CX1, int CX2, int CY1, int CY2, int ZX, int FX, int ZY,
          int MAXT, int GMR = 0, int DA = 0>
__global__ __launch_bounds__(MAXT) void k_plane_parts(Geometry g, DevTables t, Launch L,
                                                      cx<T> *__restrict__ S,
                                                      const T *__restrict__ VT,
                                                      cx<T> *__restrict__ psi, long long band0)
{
    // prefetched slots per thread cover 2048 slots
    plane_parts_body<T, MODE, CX1, CX2, CY1, CY2, ZX, FX, ZY, (2048 + MAXT - 1) / MAXT,
                     (GMR ? GMR : (MAXT > 512 ? 16 : 32)), DA>(g, t, L, S, VT, psi, band0);
}

// ------------------------------------------------------- K2, row blocks
// Row-block form of the whole-plane kernel (application, launches of one
// segment, y pass in the direct form).  After y stage A, the L2y-point stage-B
// transforms of index k1 touch only the rows at positions [L2y k1, L2y k1 + L2y)
// of the transposed row order, and so do the x transforms of those rows, the
// potential, the reverse x transforms and the reverse y stage B'.  One
// wavefront runs that whole chain for one such block of rows, with wavefront
// ordering only between its stages; the workgroup synchronises twice per
// plane, after y stage A (which writes every block) and before y stage A'
// (which reads every block).  The wavefronts of a plane then no longer move
// through the stages in step, so the LDS traffic of one overlaps the
// arithmetic of another.
// The column stride is N2 + 7 complex values (7 mod 16): lanes along columns
// (y stages) and lanes along eight rows of two neighbouring columns (x stages)
// then fall on distinct LDS banks but for one pair.
constexpr int kRowBlockPad = 7;

template <int N1, int N2>
__host__ __device__ constexpr int rowblock_lds_elems()
{
    return N1 * (N2 + kRowBlockPad) + N1 + N2;
}

template <typename T, int CX1, int CX2, int CY1, int CY2, int ZX, int FX, int ZY, int MAXT>
__global__ __launch_bounds__(MAXT) void k_plane_rowblock(Geometry g, DevTables t, Launch L,
                                                         cx<T> *__restrict__ S,
                                                         const T *__restrict__ VT)
{
    constexpr int L1x = CX1, L2x = CX2, L1y = CY1, L2y = CY2;
    constexpr int N1 = L1x * L2x, N2 = L1y * L2y, ldy = N2 + kRowBlockPad;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *plane = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *twy = plane + N1 * ldy; // stage twiddles of y and x, [n2][k1]
    cx<T> *twx = twy + N2;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
    const int nxo = g.nxo, hx = g.hmin_mod;
    for (int i = tid; i < N2; i += nthr) twy[i] = reinterpret_cast<const cx<T> *>(t.twy)[i];
    for (int i = tid; i < N1; i += nthr) twx[i] = reinterpret_cast<const cx<T> *>(t.twx)[i];
    const Seg sg = L.seg[0];
    const int nb = L.nbt;
    auto col_of = [&](int hc) {
        int x = hx + hc;
        return x >= N1 ? x - N1 : x;
    };
    auto occupied = [&](int x) {
        int r = x - hx;
        if (r < 0) r += N1;
        return r < nxo;
    };
    // persistent XCD-aware schedule over the planes j = z nb + band (as in the
    // other plane kernels)
    const int total = nb * g.N3;
    int j0 = blockIdx.x, jstep = gridDim.x, jend = total;
    if ((gridDim.x & 7) == 0 && (total & 7) == 0) {
        const int share = total >> 3, xcd = blockIdx.x & 7;
        j0 = xcd * share + (blockIdx.x >> 3);
        jstep = gridDim.x >> 3;
        jend = (xcd + 1) * share;
    }
    // The thread's y stage-A task (occupied column yhc, n2 = yn2; the launcher
    // guarantees nxo L2y <= threads) and the slots of its inputs in S, the same
    // for every plane
    const bool ymine = tid < nxo * L2y;
    const int yn2 = (int)(((unsigned long long)(unsigned)tid * g.nxo_magic) >> 40);
    const int yhc = tid - yn2 * nxo;
    int pos[L1y];
    cx<T> pre[L1y];
#pragma unroll
    for (int n1 = 0; n1 < L1y; ++n1) {
        pos[n1] = -1;
        pre[n1] = mk<T>(T(0), T(0));
    }
    if (ymine) {
        const int *ys = t.yslot + (long long)(sg.col_off + yhc) * N2 + yn2;
#pragma unroll
        for (int n1 = 0; n1 < L1y; ++n1)
            if (!masked<ZY>(n1)) pos[n1] = ys[L2y * n1];
    }
    auto prefetch = [&](int jj) {
        const int zz = jj / nb, bb = jj - zz * nb;
        const cx<T> *Sj = S + sg.s_off + ((long long)bb * g.N3 + zz) * sg.nst;
#pragma unroll
        for (int n1 = 0; n1 < L1y; ++n1)
            if (!masked<ZY>(n1)) pre[n1] = pos[n1] >= 0 ? Sj[pos[n1]] : mk<T>(T(0), T(0));
    };
    // y stage A from the prefetched stick values (zero where no stick)
    auto y_stage_a = [&]() {
        cx<T> *col = plane + col_of(yhc) * ldy + yn2;
        T xr[L1y], xi[L1y];
#pragma unroll
        for (int n1 = 0; n1 < L1y; ++n1) {
            xr[n1] = pre[n1].x;
            xi[n1] = pre[n1].y;
        }
        Dft<L1y, -1, T>::run(xr, xi);
        twiddle_pw<L1y, -1, T>(xr, xi, yn2, twy);
#pragma unroll
        for (int k1 = 0; k1 < L1y; ++k1) col[L2y * k1] = mk<T>(xr[k1], xi[k1]);
    };
    // y stage A', stick positions stored straight to the plane's slice of S
    auto y_stage_a2 = [&](cx<T> *Sd) {
        cx<T> *col = plane + col_of(yhc) * ldy + yn2;
        T xr[L1y], xi[L1y];
#pragma unroll
        for (int k1 = 0; k1 < L1y; ++k1) {
            cx<T> v = col[L2y * k1];
            xr[k1] = v.x;
            xi[k1] = v.y;
        }
        twiddle_pw<L1y, +1, T>(xr, xi, yn2, twy);
        Dft<L1y, +1, T>::run(xr, xi);
#pragma unroll
        for (int n1 = 0; n1 < L1y; ++n1)
            if (!masked<ZY>(n1) && pos[n1] >= 0) Sd[pos[n1]] = mk<T>(xr[n1], xi[n1]);
    };
    __syncthreads(); // twiddles in LDS
    if (ymine && j0 < jend) prefetch(j0);
    cx<T> *Sprev = nullptr;
    for (int jc = j0; jc < jend; jc += jstep) {
        const int z = jc / nb, bl = jc - z * nb;
        cx<T> *Sz = S + sg.s_off + ((long long)bl * g.N3 + z) * sg.nst;
        const T *VTz = VT + (long long)z * N1 * N2;
        // y stage A' of the previous plane and y stage A of this one: the
        // thread's own positions of its column
        if (ymine) {
            if (Sprev) y_stage_a2(Sprev);
            y_stage_a();
        }
        __syncthreads();
        const bool more = jc + jstep < jend;
        bool fetched = false;
        for (int jb = wave; jb < L1y; jb += nwaves) {
            const int yp0 = L2y * jb;
            constexpr int NBT = L2y * L1x; // x stage-B tasks of the block
            constexpr int RB = (NBT + 63) / 64;
            // y stage B (lanes along occupied columns)
            for (int hc = lane; hc < nxo; hc += 64) {
                cx<T> *col = plane + col_of(hc) * ldy + yp0;
                T xr[L2y], xi[L2y];
#pragma unroll
                for (int n2 = 0; n2 < L2y; ++n2) {
                    cx<T> v = col[n2];
                    xr[n2] = v.x;
                    xi[n2] = v.y;
                }
                Dft<L2y, -1, T>::run(xr, xi);
#pragma unroll
                for (int k2 = 0; k2 < L2y; ++k2) col[k2] = mk<T>(xr[k2], xi[k2]);
            }
            wave_sync();
            // x stage A of the block's rows (r = u mod L2y, n2 = u / L2y)
            for (int u = lane; u < L2y * L2x; u += 64) {
                const int r = u % L2y, n2 = u / L2y;
                cx<T> *row = plane + n2 * ldy + yp0 + r;
                T xr[L1x], xi[L1x];
#pragma unroll
                for (int n1 = 0; n1 < L1x; ++n1) {
                    cx<T> v = mk<T>(T(0), T(0));
                    if (!masked<ZX>(n1)) {
                        const cx<T> w = row[L2x * n1 * ldy];
                        if (masked<FX>(n1) || occupied(n2 + L2x * n1)) v = w;
                    }
                    xr[n1] = v.x;
                    xi[n1] = v.y;
                }
                Dft<L1x, -1, T>::run(xr, xi);
                twiddle_pw<L1x, -1, T>(xr, xi, n2, twx);
#pragma unroll
                for (int k1 = 0; k1 < L1x; ++k1) row[L2x * k1 * ldy] = mk<T>(xr[k1], xi[k1]);
            }
            wave_sync();
            // x stage B, the potential, reverse stage B (tasks r = u mod L2y, k1 = u /
            // L2y); the potential of every round is loaded first
            T vv[RB][L2x];
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
                const int u = lane + 64 * rr;
                if (u < NBT) {
                    const int r = u % L2y, k1 = u / L2y;
                    const T *vrun = VTz + ((long long)k1 * N2 + yp0 + r) * L2x;
#pragma unroll
                    for (int k2 = 0; k2 < L2x; ++k2) vv[rr][k2] = vrun[k2];
                }
            }
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
                const int u = lane + 64 * rr;
                if (u < NBT) {
                    const int r = u % L2y, k1 = u / L2y;
                    cx<T> *row = plane + L2x * k1 * ldy + yp0 + r;
                    T xr[L2x], xi[L2x];
#pragma unroll
                    for (int n2 = 0; n2 < L2x; ++n2) {
                        cx<T> v = row[n2 * ldy];
                        xr[n2] = v.x;
                        xi[n2] = v.y;
                    }
                    Dft<L2x, -1, T>::run(xr, xi);
#pragma unroll
                    for (int k2 = 0; k2 < L2x; ++k2) {
                        xr[k2] *= vv[rr][k2];
                        xi[k2] *= vv[rr][k2];
                    }
                    Dft<L2x, +1, T>::run(xr, xi);
#pragma unroll
                    for (int n2 = 0; n2 < L2x; ++n2) row[n2 * ldy] = mk<T>(xr[n2], xi[n2]);
                }
            }
            wave_sync();
            // the next plane's stick values: issued after the potential's loads,
            // they complete behind the rest of the plane
            if (!fetched) {
                fetched = true;
                if (ymine && more) prefetch(jc + jstep);
            }
            // x stage A', occupied outputs only
            for (int u = lane; u < L2y * L2x; u += 64) {
                const int r = u % L2y, n2 = u / L2y;
                cx<T> *row = plane + n2 * ldy + yp0 + r;
                T xr[L1x], xi[L1x];
#pragma unroll
                for (int k1 = 0; k1 < L1x; ++k1) {
                    cx<T> v = row[L2x * k1 * ldy];
                    xr[k1] = v.x;
                    xi[k1] = v.y;
                }
                twiddle_pw<L1x, +1, T>(xr, xi, n2, twx);
                Dft<L1x, +1, T>::run(xr, xi);
#pragma unroll
                for (int n1 = 0; n1 < L1x; ++n1) {
                    if (masked<ZX>(n1)) continue;
                    if (masked<FX>(n1) || occupied(n2 + L2x * n1))
                        row[L2x * n1 * ldy] = mk<T>(xr[n1], xi[n1]);
                }
            }
            wave_sync();
            // y stage B' (lanes along occupied columns)
            for (int hc = lane; hc < nxo; hc += 64) {
                cx<T> *col = plane + col_of(hc) * ldy + yp0;
                T xr[L2y], xi[L2y];
#pragma unroll
                for (int k2 = 0; k2 < L2y; ++k2) {
                    cx<T> v = col[k2];
                    xr[k2] = v.x;
                    xi[k2] = v.y;
                }
                Dft<L2y, +1, T>::run(xr, xi);
#pragma unroll
                for (int n2 = 0; n2 < L2y; ++n2) col[n2] = mk<T>(xr[n2], xi[n2]);
            }
            wave_sync();
        }
        if (!fetched && ymine && more) prefetch(jc + jstep);
        __syncthreads();
        Sprev = Sz;
    }
    if (ymine && Sprev) y_stage_a2(Sprev);
}

// VT[z][k1][yp][k2] = V[z][y][x] with x = k1 + L1x k2 and yp = L2y (y mod L1y)
// + y / L1y: the potential in the order the full-plane kernel's x stage B
// reads it (each task's L2x values contiguous, tasks along yp adjacent).
// One workgroup per (z, block of kArrangeRows consecutive yp): the rows are
// read whole (coalesced) into LDS, then every (k1, yp, k2) run of the block,
// kArrangeRows * L2x contiguous values per k1, is written out.
constexpr int kArrangeRows = 8;
template <typename T>
__global__ void k_arrange_v(const T *__restrict__ V, T *__restrict__ VT, int N1, int N2, int N3,
                            int L1x, int L2x, int L1y, int L2y)
{
    extern __shared__ unsigned char smem_raw[];
    T *rows = reinterpret_cast<T *>(smem_raw); // [kArrangeRows][N1]
    const int nyb = (N2 + kArrangeRows - 1) / kArrangeRows;
    const int z = blockIdx.x / nyb, yp0 = (blockIdx.x - z * nyb) * kArrangeRows;
    const int nr = min(kArrangeRows, N2 - yp0);
    for (int t = threadIdx.x; t < nr * N1; t += blockDim.x) {
        const int r = t / N1, x = t - r * N1;
        const int yp = yp0 + r, y = (yp % L2y) * L1y + yp / L2y;
        rows[t] = V[((long long)z * N2 + y) * N1 + x];
    }
    __syncthreads();
    const int run = nr * L2x;
    for (int t = threadIdx.x; t < L1x * run; t += blockDim.x) {
        const int k1 = t / run, u = t - k1 * run;
        const int r = u / L2x, k2 = u - r * L2x;
        VT[(((long long)z * L1x + k1) * N2 + yp0 + r) * L2x + k2] = rows[r * N1 + k1 + L1x * k2];
    }
}

// Quad variant: no row buffer, so the occupied plane is the only LDS and two
// workgroups fit on a CU even in FP64; 3 waves per SIMD bound the registers.
template <typename T, int MODE, int XQ, int CY1, int CY2>
__global__ __attribute__((amdgpu_flat_work_group_size(64, 512), amdgpu_waves_per_eu(3)))
void k_plane_quad(Geometry g, DevTables t, Launch L, cx<T> *__restrict__ S,
                  const T *__restrict__ V, cx<T> *__restrict__ psi, long long band0)
{
    plane_body<T, MODE, 0, 0, CY1, CY2, 0, 0, XQ, 4, 16>(g, t, L, S, V, psi, band0);
}

// ------------------------------------------------------------ launchers
//
// The launchers are compiled in parts, each part once per precision, so that
// the build runs them in parallel: VLOC_PART_STICK (stick kernels, potential
// arrangement and the plane-kernel dispatch), VLOC_PART_FULL_APPLY and
// VLOC_PART_FULL_AUX (whole-plane kernels of the application, and of the
// diagnostic transforms and the density) and VLOC_PART_ROWS (row-buffer and
// lane-quad kernels).  Without a part macro everything but the tuner's
// specialisations is compiled.
#if !defined(VLOC_PART_STICK) && !defined(VLOC_PART_FULL_APPLY) &&                               \
    !defined(VLOC_PART_FULL_AUX) && !defined(VLOC_PART_ROWS) && !defined(VLOC_PART_TUNE)
#define VLOC_PART_STICK
#define VLOC_PART_FULL_APPLY
#define VLOC_PART_FULL_AUX
#define VLOC_PART_ROWS
#endif
// VLOC_PART_TUNE (the tuner's specialisations) is compiled once per precision
// with VLOC_TUNE_T naming it.
#if defined(VLOC_PART_FULL_APPLY) || defined(VLOC_PART_FULL_AUX)
#define VLOC_PART_FULL
#endif

// Persistent plane grid: the workgroups that are resident at once (a
// multiple of 8 so that the XCD schedule applies), never more than the planes.
[[maybe_unused]] static unsigned plane_blocks(const Geometry &g, int nb)
{
    long long total = (long long)nb * g.N3;
    long long res = (long long)g.resident_plane_wgs;
    if (res >= 8) res &= ~7LL;
    if (res < 1) res = 1;
    return (unsigned)(total < res ? total : res);
}

template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Largest codelet of the plane kernel's x and y splits: kernels of more than
// 512 threads are compiled for codelets of at most 16 points.
[[maybe_unused]] static int plane_codelet_max(const Geometry &g)
{
    return std::max(std::max(g.L1x, g.L2x), std::max(g.L1y, g.L2y));
}

// Class of the runtime-sized plane kernels for this plan: codelets of at most
// 10 or 12 points, else every size (0).  With the 15- and 16-point paths an
// FP64 kernel of 1024 threads spills 130 registers; limited to 10 points it
// spills none.
[[maybe_unused]] static int plane_codelet_class(const Geometry &g)
{
    const int m = plane_codelet_max(g);
    return m <= 10 ? 10 : (m <= 12 ? 12 : 0);
}

#if defined(VLOC_PART_STICK)
// Line splits and zero masks compiled as specialisations of the stick
// kernels; any other plan runs the same kernels with runtime sizes.  A
// specialisation serves every plan whose zero mask contains its own (it then
// skips fewer of the zero groups), so for each split the larger masks come
// first.
#define VLOC_STICK_SPECS(X)                                                                       \
    X(8, 12, 0x38) X(8, 12, 0) X(4, 6, 0x4) X(4, 6, 0) X(8, 16, 0x3C) X(8, 16, 0x38)            \
    X(8, 16, 0) X(8, 10, 0x38) X(8, 10, 0)

template <typename T>
hipError_t launch_stick_fwd(const Geometry &g, const DevTables &t, const Launch &L, void *S,
                            int threads, hipStream_t st)
{
    if (L.nblk <= 0) return hipSuccess;
    size_t lds = (size_t)g.group_cap * g.ldz * sizeof(cx<T>);
    auto go = [&](auto kern) {
        hipError_t e = allow_lds(kern, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(L.nblk), dim3(threads), lds, st, g, t, L,
                           reinterpret_cast<cx<T> *>(S));
        return hipGetLastError();
    };
#define VLOC_K1(A, B, Z)                                                                           \
    if (g.L1z == A && g.L2z == B && (g.zz & Z) == Z)                                              \
        return g.gamma ? go(k_stick_fwd<T, A, B, Z, true>) : go(k_stick_fwd<T, A, B, Z, false>);
    VLOC_STICK_SPECS(VLOC_K1)
#undef VLOC_K1
    return g.gamma ? go(k_stick_fwd<T, 0, 0, 0, true>) : go(k_stick_fwd<T, 0, 0, 0, false>);
}

template <typename T>
hipError_t launch_stick_bwd(const Geometry &g, const DevTables &t, const Launch &L, const void *S,
                            int threads, hipStream_t st)
{
    if (L.nblk <= 0) return hipSuccess;
    size_t lds = ((size_t)g.group_cap * g.ldz + g.N3) * sizeof(cx<T>);
    auto go = [&](auto kern) {
        hipError_t e = allow_lds(kern, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(L.nblk), dim3(threads), lds, st, g, t, L,
                           reinterpret_cast<const cx<T> *>(S));
        return hipGetLastError();
    };
#define VLOC_K3(A, B, Z)                                                                           \
    if (g.L1z == A && g.L2z == B && (g.zz & Z) == Z)                                              \
        return g.gamma ? go(k_stick_bwd<T, A, B, Z, true>) : go(k_stick_bwd<T, A, B, Z, false>);
    VLOC_STICK_SPECS(VLOC_K3)
#undef VLOC_K3
    return g.gamma ? go(k_stick_bwd<T, 0, 0, 0, true>) : go(k_stick_bwd<T, 0, 0, 0, false>);
}
#endif // VLOC_PART_STICK

#if defined(VLOC_PART_ROWS)
template <typename T, int MODE, int X1, int X2, int Y1, int Y2, int ZX, int ZY>
static hipError_t launch_plane_sized(const Geometry &g, const DevTables &t, const Launch &L,
                                     void *S, const void *V, void *psi, int64_t band0,
                                     int threads, int lds, hipStream_t st)
{
    auto go = [&](auto kern) {
        hipError_t e = allow_lds(kern, (size_t)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(plane_blocks(g, L.nbt)), dim3(threads), (size_t)lds, st, g,
                           t, L, reinterpret_cast<cx<T> *>(S), reinterpret_cast<const T *>(V),
                           reinterpret_cast<cx<T> *>(psi), (long long)band0);
        return hipGetLastError();
    };
    if (threads <= 512) return go(k_plane<T, MODE, X1, X2, Y1, Y2, ZX, ZY>);
    // wide workgroups: compiled for FP64 application and density only, with
    // codelets of at most 16 points
    if constexpr (std::is_same<T, double>::value &&
                  (MODE == MODE_APPLY || MODE == MODE_DENSITY || MODE == MODE_APPLY_DENSITY))
        if (plane_codelet_max(g) <= 16) return go(k_plane_wide<T, MODE, X1, X2, Y1, Y2, ZX, ZY>);
    return hipErrorInvalidValue;
}

template <typename T, int MODE, int XQ, int Y1, int Y2>
static hipError_t launch_plane_quad(const Geometry &g, const DevTables &t, const Launch &L,
                                    void *S, const void *V, void *psi, int64_t band0,
                                    int threads, int lds, hipStream_t st)
{
    auto kern = k_plane_quad<T, MODE, XQ, Y1, Y2>;
    hipError_t e = allow_lds(kern, (size_t)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(plane_blocks(g, L.nbt)), dim3(threads), (size_t)lds, st, g, t,
                       L, reinterpret_cast<cx<T> *>(S), reinterpret_cast<const T *>(V),
                       reinterpret_cast<cx<T> *>(psi), (long long)band0);
    return hipGetLastError();
}

// Row-buffer and lane-quad layouts.  Specialised line splits for the common
// grids; any other split runs the same kernel with runtime sizes.  A
// specialisation serves every plan whose zero masks contain its own.
template <typename T, int MODE>
hipError_t launch_plane_rows_mode(const Geometry &g, const DevTables &t, const Launch &L, void *S,
                                  const void *V, void *psi, int64_t band0, int threads, int lds,
                                  hipStream_t st)
{
    if constexpr (MODE != MODE_DENSITY && MODE != MODE_APPLY_DENSITY) if (g.xq) {
#define VLOC_QUAD_CASE(XQ, Y1, Y2)                                                                 \
        if (g.xq == XQ && g.L1y == Y1 && g.L2y == Y2)                                             \
            return launch_plane_quad<T, MODE, XQ, Y1, Y2>(g, t, L, S, V, psi, band0, threads,     \
                                                           lds, st);
        VLOC_QUAD_CASE(24, 8, 12)
        VLOC_QUAD_CASE(6, 4, 6)
        VLOC_QUAD_CASE(18, 8, 12)
        VLOC_QUAD_CASE(20, 8, 10)
#undef VLOC_QUAD_CASE
        return hipErrorInvalidValue;
    }
#define VLOC_PLANE_CASE(X1, X2, Y1, Y2, ZX, ZY)                                                    \
    if (g.L1x == X1 && g.L2x == X2 && g.L1y == Y1 && g.L2y == Y2 && (g.zx & ZX) == ZX &&          \
        (g.zy & ZY) == ZY)                                                                        \
        return launch_plane_sized<T, MODE, X1, X2, Y1, Y2, ZX, ZY>(g, t, L, S, V, psi, band0,     \
                                                                   threads, lds, st);
    VLOC_PLANE_CASE(8, 12, 8, 12, 0x38, 0x38)
    VLOC_PLANE_CASE(8, 12, 8, 12, 0, 0)
    VLOC_PLANE_CASE(4, 6, 4, 6, 0x4, 0x4)
    VLOC_PLANE_CASE(4, 6, 4, 6, 0, 0)
    VLOC_PLANE_CASE(8, 16, 8, 16, 0x38, 0x38)
    VLOC_PLANE_CASE(8, 16, 8, 16, 0, 0)
    VLOC_PLANE_CASE(8, 10, 8, 10, 0x38, 0x38)
    VLOC_PLANE_CASE(8, 10, 8, 10, 0, 0)
    VLOC_PLANE_CASE(8, 9, 8, 12, 0x38, 0x3C)
    VLOC_PLANE_CASE(8, 9, 8, 12, 0, 0)
#undef VLOC_PLANE_CASE
    return launch_plane_sized<T, MODE, 0, 0, 0, 0, 0, 0>(g, t, L, S, V, psi, band0, threads, lds,
                                                         st);
}
#endif // VLOC_PART_ROWS

#if defined(VLOC_PART_FULL)
// GMR: class of the runtime-sized kernel (plane_codelet_class; 0 otherwise)
template <typename T, int MODE, int X1, int X2, int Y1, int Y2, int ZX, int FX, int ZY,
          int GMR = 0>
static hipError_t launch_plane_full(const Geometry &g, const DevTables &t, const Launch &L,
                                    void *S, const void *VT, void *psi, int64_t band0,
                                    int threads, int lds, hipStream_t st)
{
    auto go = [&](auto kern, int nthr) {
        hipError_t e = allow_lds(kern, (size_t)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(plane_blocks(g, L.nbt)), dim3(nthr), (size_t)lds, st, g, t,
                           L, reinterpret_cast<cx<T> *>(S), reinterpret_cast<const T *>(VT),
                           reinterpret_cast<cx<T> *>(psi), (long long)band0);
        return hipGetLastError();
    };
    // direct y form: one segment, a specialised y split, apply (and FP32
    // density; the FP64 density kernel would spill with it)
    constexpr bool DYK = Y1 > 0 && (MODE == MODE_APPLY ||
                                    ((MODE == MODE_DENSITY || MODE == MODE_APPLY_DENSITY) &&
                                     std::is_same<T, float>::value));
    const bool dyok = DYK && L.nseg == 1;
    auto pick = [&](auto wpr) {
        constexpr bool W = decltype(wpr)::value;
        constexpr int G = W ? 0 : GMR;
        // more than 512 threads: compiled for FP64 application and density with
        // codelets of at most 16 points; the diagnostic transforms run the same
        // body on 512 threads
        if constexpr (std::is_same<T, double>::value &&
                      (MODE == MODE_APPLY || MODE == MODE_DENSITY ||
                       MODE == MODE_APPLY_DENSITY)) {
            const bool dy1 = !W && dyok && L.seg[0].nxo * g.L2y <= threads;
            if (threads > 512 && plane_codelet_max(g) > 16) return hipErrorInvalidValue;
            if (threads > 768) {
                if constexpr (DYK && !W)
                    if (dy1)
                        return go(k_plane_full<T, MODE, X1, X2, Y1, Y2, ZX, FX, ZY, 1024, W, 1, G>,
                                  threads);
                return go(k_plane_full<T, MODE, X1, X2, Y1, Y2, ZX, FX, ZY, 1024, W, 0, G>, threads);
            }
            if (threads > 512) {
                if constexpr (DYK && !W)
                    if (dy1)
                        return go(k_plane_full<T, MODE, X1, X2, Y1, Y2, ZX, FX, ZY, 768, W, 1, G>,
                                  threads);
                return go(k_plane_full<T, MODE, X1, X2, Y1, Y2, ZX, FX, ZY, 768, W, 0, G>, threads);
            }
        }
        const int nt = threads < 512 ? threads : 512;
        // FP32 density with a plane that leaves one workgroup per CU: 1024
        // threads (128 registers each), one x stage-B task per thread, and the
        // density sums of a work item held in registers; the y passes in the
        // scatter form (the direct form's prefetch registers would spill)
        constexpr bool DAK = std::is_same<T, float>::value &&
                             (MODE == MODE_DENSITY || MODE == MODE_APPLY_DENSITY) && X1 > 0 &&
                             Y1 > 0 && 8LL * X1 * X2 * Y1 * Y2 > 80 * 1024 && X1 * Y1 * Y2 <= 1024;
        if constexpr (DAK && !W)
            if (2LL * lds > 160 * 1024 && threads >= 512)
                return go(k_plane_full<T, MODE, X1, X2, Y1, Y2, ZX, FX, ZY, 1024, W, 0, G, 1>, 1024);
        // FP32 application on such planes: 1024 threads as well (128 registers
        // each, no spill in the direct y form)
        constexpr bool A1K = std::is_same<T, float>::value && MODE == MODE_APPLY && X1 > 0 &&
                             Y1 > 0 && 8LL * X1 * X2 * Y1 * Y2 > 80 * 1024;
        if constexpr (A1K && !W)
            if (2LL * lds > 160 * 1024 && threads >= 512 && dyok &&
                L.seg[0].nxo * g.L2y <= 1024)
                return go(k_plane_full<T, MODE, X1, X2, Y1, Y2, ZX, FX, ZY, 1024, W, 1, G>, 1024);
        // the same for the runtime-sized FP32 application (codelets of at most
        // 16 points, scatter y form)
        if constexpr (std::is_same<T, float>::value && MODE == MODE_APPLY && X1 == 0 && !W)
            if (2LL * lds > 160 * 1024 && threads >= 512 && plane_codelet_max(g) <= 16)
                return go(k_plane_full<T, MODE, 0, 0, 0, 0, 0, 0, 0, 1024, W, 0, G ? G : 16>,
                          1024);
        if constexpr (DYK && !W && std::is_same<T, float>::value)
            if (dyok && L.seg[0].nxo * g.L2y <= 2 * nt)
                return go(k_plane_full<T, MODE, X1, X2, Y1, Y2, ZX, FX, ZY, 512, W, 2, G>, nt);
        return go(k_plane_full<T, MODE, X1, X2, Y1, Y2, ZX, FX, ZY, 512, W, 0, G>, nt);
    };
    if (g.full == 2) return pick(std::true_type{});
    return pick(std::false_type{});
}

// Row-block kernel: compiled splits and zero masks (a specialisation serves
// every plan whose masks contain its own); false where none applies.
template <typename T>
static bool launch_plane_rowblock(const Geometry &g, const DevTables &t, const Launch &L, void *S,
                                  const void *VT, int threads, hipStream_t st, hipError_t &err)
{
    if (L.nseg != 1 || threads != 768 || g.nxo * g.L2y > threads) return false;
    auto go = [&](auto kern, int elems) {
        const size_t lds = (size_t)elems * sizeof(cx<T>);
        err = allow_lds(kern, lds);
        if (err != hipSuccess) return true;
        hipLaunchKernelGGL(kern, dim3(plane_blocks(g, L.nbt)), dim3(threads), lds, st, g, t, L,
                           reinterpret_cast<cx<T> *>(S), reinterpret_cast<const T *>(VT));
        err = hipGetLastError();
        return true;
    };
#define VLOC_ROWBLOCK_CASE(X1, X2, Y1, Y2, ZX, FX, ZY)                                             \
    if (g.L1x == X1 && g.L2x == X2 && g.L1y == Y1 && g.L2y == Y2 && (g.zx & ZX) == ZX &&          \
        (g.fx & FX) == FX && (g.zy & ZY) == ZY)                                                   \
        return go(k_plane_rowblock<T, X1, X2, Y1, Y2, ZX, FX, ZY, 768>,                            \
                  rowblock_lds_elems<X1 * X2, Y1 * Y2>());
    if constexpr (std::is_same<T, double>::value) {
        VLOC_ROWBLOCK_CASE(12, 8, 12, 8, 0x1F0, 0xE07, 0x1F0)
        VLOC_ROWBLOCK_CASE(12, 8, 12, 8, 0, 0, 0)
    }
#undef VLOC_ROWBLOCK_CASE
    return false;
}

// Parted-plane layout: compiled splits for the 128 x 128 planes of the
// |G| <= 32 sphere (y split 16 x 8, both x splits); any other split runs the
// same kernel with runtime sizes.
template <typename T, int MODE>
static hipError_t launch_plane_parts(const Geometry &g, const DevTables &t, const Launch &L,
                                     void *S, const void *V, void *psi, int64_t band0,
                                     int threads, int lds, hipStream_t st)
{
    if (!t.parts || g.parts < 1 || threads > 1024 || (threads > 512 && plane_codelet_max(g) > 16))
        return hipErrorInvalidValue;
    auto go = [&](auto kern) {
        hipError_t e = allow_lds(kern, (size_t)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(plane_blocks(g, L.nbt)), dim3(threads), (size_t)lds, st, g,
                           t, L, reinterpret_cast<cx<T> *>(S), reinterpret_cast<const T *>(V),
                           reinterpret_cast<cx<T> *>(psi), (long long)band0);
        return hipGetLastError();
    };
    // FP64 density, x split 8 x 16, y split 16 x 8, two parts: the density sums
    // stay in registers over a work item (512 threads, so 256 registers per
    // thread; one x stage-B task per thread and part, the held y stage-B lines
    // in at most two rounds)
    if constexpr (std::is_same<T, double>::value &&
                  (MODE == MODE_DENSITY || MODE == MODE_APPLY_DENSITY)) {
        if (g.L1x == 8 && g.L2x == 16 && g.L1y == 16 && g.L2y == 8 && (g.zx & 0x38) == 0x38 &&
            (g.fx & 0xC3) == 0xC3 && (g.zy & 0xFE0) == 0xFE0 && g.parts == 2 && threads >= 512 &&
            8 * (g.N2 / 2) <= 512 && g.nxo * (16 / 2) <= 2 * 512) {
            auto kern = k_plane_parts<T, MODE, 8, 16, 16, 8, 0x38, 0xC3, 0xFE0, 512, 0, 2>;
            hipError_t e = allow_lds(kern, (size_t)lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kern, dim3(plane_blocks(g, L.nbt)), dim3(512), (size_t)lds, st, g,
                               t, L, reinterpret_cast<cx<T> *>(S), reinterpret_cast<const T *>(V),
                               reinterpret_cast<cx<T> *>(psi), (long long)band0);
            return hipGetLastError();
        }
    }
#define VLOC_PARTS_CASE(X1, X2, Y1, Y2, ZX, FX, ZY)                                                \
    if (g.L1x == X1 && g.L2x == X2 && g.L1y == Y1 && g.L2y == Y2 && (g.zx & ZX) == ZX &&          \
        (g.fx & FX) == FX && (g.zy & ZY) == ZY)                                                   \
        return threads > 768   ? go(k_plane_parts<T, MODE, X1, X2, Y1, Y2, ZX, FX, ZY, 1024>)      \
               : threads > 512 ? go(k_plane_parts<T, MODE, X1, X2, Y1, Y2, ZX, FX, ZY, 768>)       \
                               : go(k_plane_parts<T, MODE, X1, X2, Y1, Y2, ZX, FX, ZY, 512>);
    VLOC_PARTS_CASE(16, 8, 16, 8, 0xFE0, 0xF00F, 0xFE0)
    VLOC_PARTS_CASE(8, 16, 16, 8, 0x38, 0xC3, 0xFE0)
#undef VLOC_PARTS_CASE
    auto generic = [&](auto cls) {
        constexpr int C = decltype(cls)::value;
        return threads > 768   ? go(k_plane_parts<T, MODE, 0, 0, 0, 0, 0, 0, 0, 1024, C>)
               : threads > 512 ? go(k_plane_parts<T, MODE, 0, 0, 0, 0, 0, 0, 0, 768, C>)
                               : go(k_plane_parts<T, MODE, 0, 0, 0, 0, 0, 0, 0, 512, C>);
    };
    switch (plane_codelet_class(g)) {
    case 10: return generic(std::integral_constant<int, 10>{});
    case 12: return generic(std::integral_constant<int, 12>{});
    default: return generic(std::integral_constant<int, 0>{});
    }
}

// Whole-plane layout.  Specialised line splits for the common grids; any
// other split runs the same kernel with runtime sizes.
template <typename T, int MODE>
hipError_t launch_plane_full_mode(const Geometry &g, const DevTables &t, const Launch &L, void *S,
                                  const void *V, void *psi, int64_t band0, int threads, int lds,
                                  hipStream_t st)
{
    if (g.full == 4)
        return launch_plane_parts<T, MODE>(g, t, L, S, V, psi, band0, threads, lds, st);
    if constexpr (MODE == MODE_APPLY) {
        hipError_t err = hipSuccess;
        if (g.full == 3 && launch_plane_rowblock<T>(g, t, L, S, V, threads, st, err)) return err;
    }
#define VLOC_FULL_CASE(X1, X2, Y1, Y2, ZX, FX, ZY)                                                 \
    if (g.L1x == X1 && g.L2x == X2 && g.L1y == Y1 && g.L2y == Y2 && (g.zx & ZX) == ZX &&          \
        (g.fx & FX) == FX && (g.zy & ZY) == ZY)                                                   \
        return launch_plane_full<T, MODE, X1, X2, Y1, Y2, ZX, FX, ZY>(g, t, L, S, V, psi, band0,   \
                                                                     threads, lds, st);
    VLOC_FULL_CASE(8, 12, 8, 12, 0x38, 0xC3, 0x38)
    VLOC_FULL_CASE(12, 8, 8, 12, 0x1F0, 0xE07, 0x38)
    VLOC_FULL_CASE(8, 9, 8, 12, 0x38, 0xC3, 0x3C)
    VLOC_FULL_CASE(8, 16, 8, 16, 0x38, 0xC3, 0x38)
    VLOC_FULL_CASE(8, 16, 16, 8, 0x38, 0xC3, 0xFE0)
    VLOC_FULL_CASE(8, 10, 8, 10, 0x38, 0xC3, 0x38)
    VLOC_FULL_CASE(4, 6, 4, 6, 0x4, 0x9, 0x4)
#undef VLOC_FULL_CASE
    if constexpr (MODE == MODE_APPLY) {
        bool hit = false;
        hipError_t err = launch_plane_full_tuned<T>(g, t, L, S, V, threads, lds, st, hit);
        if (hit) return err;
    }
    switch (plane_codelet_class(g)) {
    case 10:
        return launch_plane_full<T, MODE, 0, 0, 0, 0, 0, 0, 0, 10>(g, t, L, S, V, psi, band0,
                                                                   threads, lds, st);
    case 12:
        return launch_plane_full<T, MODE, 0, 0, 0, 0, 0, 0, 0, 12>(g, t, L, S, V, psi, band0,
                                                                   threads, lds, st);
    default:
        return launch_plane_full<T, MODE, 0, 0, 0, 0, 0, 0, 0>(g, t, L, S, V, psi, band0, threads,
                                                               lds, st);
    }
}
#endif // VLOC_PART_FULL

#if defined(VLOC_PART_TUNE)
// Compiled specialisations for the schedule tuner: every split of the x and y
// lines into two codelets of at most 16 points, for the plane sizes and
// occupied ranges of the workloads below, so that a split the tuner tries runs
// compiled code with its zero masks rather than the run-time-sized kernel.
// The list is generated at compile time from the workloads (no hand-kept
// table): N1 x N2 with occupied x-planes [hlo, hhi] and rows [klo, khi].
struct TuneGeom {
    int N1, N2, hlo, hhi, klo, khi;
};
constexpr TuneGeom kTuneGeoms[] = {
    {96, 96, -24, 24, -24, 24},  // 96^3 grid, |G| <= 24
    {72, 96, -18, 18, -18, 18},  // 72 x 96 x 128 grid, |g + k| <= 18 (union over k)
    {128, 128, -32, 32, -32, 32} // 128^3 grid, |G| <= 32
};
constexpr int kNumTuneGeoms = (int)(sizeof kTuneGeoms / sizeof kTuneGeoms[0]);
constexpr int kTuneCodelets[] = {2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16};
constexpr int kNumTuneCodelets = (int)(sizeof kTuneCodelets / sizeof kTuneCodelets[0]);

constexpr bool tune_codelet(int r)
{
    for (int c : kTuneCodelets)
        if (c == r) return true;
    return false;
}
// i-th first factor L1 of a split L = L1 L2 with both factors codelets (0 if none)
constexpr int tune_split(int L, int i)
{
    for (int c : kTuneCodelets)
        if (L % c == 0 && tune_codelet(L / c) && i-- == 0) return c;
    return 0;
}
// Zero and full masks of the stage-A input groups {n2 + L2 n1} for occupied
// positions [lo, hi] taken mod L (the planner's rule).
constexpr int tune_mask(int L1, int L2, int lo, int hi, bool full)
{
    const int L = L1 * L2;
    int m = 0;
    for (int n1 = 0; n1 < L1; ++n1) {
        bool any = false, all = true;
        for (int n2 = 0; n2 < L2; ++n2) {
            const int pos = n2 + L2 * n1;
            const int r = ((pos - lo) % L + L) % L;
            const bool occ = lo + r <= hi;
            any = any || occ;
            all = all && occ;
        }
        if (full ? all : !any) m |= 1 << n1;
    }
    return m;
}

// The variants the planner's thread counts use: FP64 1024 and 768 threads,
// FP32 512, each in the direct y form where the y tasks fit, else the scatter
// form.
template <typename T, int X1, int X2, int Y1, int Y2, int ZX, int FX, int ZY>
static hipError_t launch_plane_full_lean(const Geometry &g, const DevTables &t, const Launch &L,
                                         void *S, const void *VT, int threads, int lds,
                                         hipStream_t st, bool &hit)
{
    auto go = [&](auto kern) {
        hit = true;
        hipError_t e = allow_lds(kern, (size_t)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(plane_blocks(g, L.nbt)), dim3(threads), (size_t)lds, st, g,
                           t, L, reinterpret_cast<cx<T> *>(S), reinterpret_cast<const T *>(VT),
                           (cx<T> *)nullptr, 0LL);
        return hipGetLastError();
    };
    if (g.full != 1) return hipSuccess;
    const bool one = L.nseg == 1;
    if constexpr (std::is_same<T, double>::value) {
        const bool dy = one && L.seg[0].nxo * Y2 <= threads;
        if (threads == 1024)
            return dy ? go(k_plane_full<T, MODE_APPLY, X1, X2, Y1, Y2, ZX, FX, ZY, 1024, false, 1>)
                      : go(k_plane_full<T, MODE_APPLY, X1, X2, Y1, Y2, ZX, FX, ZY, 1024, false, 0>);
        if (threads == 768)
            return dy ? go(k_plane_full<T, MODE_APPLY, X1, X2, Y1, Y2, ZX, FX, ZY, 768, false, 1>)
                      : go(k_plane_full<T, MODE_APPLY, X1, X2, Y1, Y2, ZX, FX, ZY, 768, false, 0>);
    } else {
        const bool dy = one && L.seg[0].nxo * Y2 <= 2 * threads;
        if (threads == 512)
            return dy ? go(k_plane_full<T, MODE_APPLY, X1, X2, Y1, Y2, ZX, FX, ZY, 512, false, 2>)
                      : go(k_plane_full<T, MODE_APPLY, X1, X2, Y1, Y2, ZX, FX, ZY, 512, false, 0>);
    }
    return hipSuccess;
}

template <typename T, int G, int IX, int IY>
static hipError_t try_tuned(const Geometry &g, const DevTables &t, const Launch &L, void *S,
                            const void *VT, int threads, int lds, hipStream_t st, bool &hit)
{
    if (g.N1 != kTuneGeoms[G].N1 || g.N2 != kTuneGeoms[G].N2) return hipSuccess;
    constexpr TuneGeom tg = kTuneGeoms[G];
    constexpr int X1 = tune_split(tg.N1, IX), Y1 = tune_split(tg.N2, IY);
    if constexpr (X1 > 0 && Y1 > 0) {
        constexpr int X2 = tg.N1 / X1, Y2 = tg.N2 / Y1;
        constexpr int ZX = tune_mask(X1, X2, tg.hlo, tg.hhi, false);
        constexpr int FX = tune_mask(X1, X2, tg.hlo, tg.hhi, true);
        constexpr int ZY = tune_mask(Y1, Y2, tg.klo, tg.khi, false);
        if (g.N1 == tg.N1 && g.N2 == tg.N2 && g.L1x == X1 && g.L1y == Y1 && (g.zx & ZX) == ZX &&
            (g.fx & FX) == FX && (g.zy & ZY) == ZY) {
            hipError_t e =
                launch_plane_full_lean<T, X1, X2, Y1, Y2, ZX, FX, ZY>(g, t, L, S, VT, threads, lds,
                                                                      st, hit);
            if (hit) return e;
        }
    }
    if constexpr (IY + 1 < kNumTuneCodelets)
        return try_tuned<T, G, IX, IY + 1>(g, t, L, S, VT, threads, lds, st, hit);
    else if constexpr (IX + 1 < kNumTuneCodelets)
        return try_tuned<T, G, IX + 1, 0>(g, t, L, S, VT, threads, lds, st, hit);
    return hipSuccess;
}

// One part per workload geometry (VLOC_TUNE_G), compiled in parallel.
template <typename T, int G>
hipError_t launch_plane_full_tuned_g(const Geometry &g, const DevTables &t, const Launch &L,
                                     void *S, const void *VT, int threads, int lds,
                                     hipStream_t st, bool &hit)
{
    return try_tuned<T, G, 0, 0>(g, t, L, S, VT, threads, lds, st, hit);
}
template hipError_t launch_plane_full_tuned_g<VLOC_TUNE_T, VLOC_TUNE_G>(
    const Geometry &, const DevTables &, const Launch &, void *, const void *, int, int,
    hipStream_t, bool &);
#endif // VLOC_PART_TUNE

#if defined(VLOC_PART_FULL_APPLY)
template <typename T>
hipError_t launch_plane_full_tuned(const Geometry &g, const DevTables &t, const Launch &L,
                                   void *S, const void *VT, int threads, int lds, hipStream_t st,
                                   bool &hit)
{
    hit = false;
    hipError_t e = launch_plane_full_tuned_g<T, 0>(g, t, L, S, VT, threads, lds, st, hit);
    if (!hit) e = launch_plane_full_tuned_g<T, 1>(g, t, L, S, VT, threads, lds, st, hit);
    if (!hit) e = launch_plane_full_tuned_g<T, 2>(g, t, L, S, VT, threads, lds, st, hit);
    return e;
}
#endif

#if defined(VLOC_PART_STICK)
template <typename T>
hipError_t launch_plane(const Geometry &g, const DevTables &t, const Launch &L, int mode, void *S,
                        const void *V, void *psi, int64_t band0, int threads, int lds_bytes,
                        hipStream_t st)
{
    if (L.nbt <= 0) return hipSuccess;
    if (mode != MODE_APPLY && L.nseg != 1) return hipErrorInvalidValue;
    if ((mode == MODE_DENSITY || mode == MODE_APPLY_DENSITY) && g.xq)
        return hipErrorInvalidValue; // no density in the lane-quad x pass
    auto run = [&](auto m) {
        constexpr int M = decltype(m)::value;
        return g.full ? launch_plane_full_mode<T, M>(g, t, L, S, V, psi, band0, threads,
                                                     lds_bytes, st)
                      : launch_plane_rows_mode<T, M>(g, t, L, S, V, psi, band0, threads,
                                                     lds_bytes, st);
    };
    switch (mode) {
    case MODE_APPLY: return run(std::integral_constant<int, MODE_APPLY>{});
    case MODE_G2R: return run(std::integral_constant<int, MODE_G2R>{});
    case MODE_R2G: return run(std::integral_constant<int, MODE_R2G>{});
    case MODE_DENSITY: return run(std::integral_constant<int, MODE_DENSITY>{});
    case MODE_APPLY_DENSITY: return run(std::integral_constant<int, MODE_APPLY_DENSITY>{});
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_arrange_v(const Geometry &g, const void *V, void *VT, hipStream_t st)
{
    const int nyb = (g.N2 + kArrangeRows - 1) / kArrangeRows;
    const size_t lds = (size_t)kArrangeRows * g.N1 * sizeof(T);
    hipLaunchKernelGGL(k_arrange_v<T>, dim3((unsigned)(g.N3 * nyb)), dim3(256), lds, st,
                       reinterpret_cast<const T *>(V), reinterpret_cast<T *>(VT), g.N1, g.N2,
                       g.N3, g.L1x, g.L2x, g.L1y, g.L2y);
    return hipGetLastError();
}
#endif // VLOC_PART_STICK

// The build compiles this file once per precision and part (in parallel).
#define VLOC_PLANE_APPLY(T, F)                                                                    \
    template hipError_t F<T, MODE_APPLY>(const Geometry &, const DevTables &, const Launch &,    \
                                         void *, const void *, void *, int64_t, int, int,        \
                                         hipStream_t);
#define VLOC_PLANE_AUX(T, F)                                                                      \
    template hipError_t F<T, MODE_G2R>(const Geometry &, const DevTables &, const Launch &,      \
                                       void *, const void *, void *, int64_t, int, int,          \
                                       hipStream_t);                                             \
    template hipError_t F<T, MODE_R2G>(const Geometry &, const DevTables &, const Launch &,      \
                                       void *, const void *, void *, int64_t, int, int,          \
                                       hipStream_t);                                             \
    template hipError_t F<T, MODE_DENSITY>(const Geometry &, const DevTables &, const Launch &,  \
                                           void *, const void *, void *, int64_t, int, int,      \
                                           hipStream_t);                                         \
    template hipError_t F<T, MODE_APPLY_DENSITY>(const Geometry &, const DevTables &,             \
                                                 const Launch &, void *, const void *, void *,   \
                                                 int64_t, int, int, hipStream_t);
#if defined(VLOC_PART_STICK)
#define VLOC_INSTANTIATE_STICK(T)                                                                 \
    template hipError_t launch_stick_fwd<T>(const Geometry &, const DevTables &, const Launch &, \
                                            void *, int, hipStream_t);                           \
    template hipError_t launch_stick_bwd<T>(const Geometry &, const DevTables &, const Launch &, \
                                            const void *, int, hipStream_t);                     \
    template hipError_t launch_plane<T>(const Geometry &, const DevTables &, const Launch &, int, \
                                        void *, const void *, void *, int64_t, int, int,         \
                                        hipStream_t);                                            \
    template hipError_t launch_arrange_v<T>(const Geometry &, const void *, void *, hipStream_t);
#else
#define VLOC_INSTANTIATE_STICK(T)
#endif
#if defined(VLOC_PART_FULL_APPLY)
#define VLOC_INSTANTIATE_FULL_APPLY(T) VLOC_PLANE_APPLY(T, launch_plane_full_mode)
#else
#define VLOC_INSTANTIATE_FULL_APPLY(T)
#endif
#if defined(VLOC_PART_FULL_AUX)
#define VLOC_INSTANTIATE_FULL_AUX(T) VLOC_PLANE_AUX(T, launch_plane_full_mode)
#else
#define VLOC_INSTANTIATE_FULL_AUX(T)
#endif
#if defined(VLOC_PART_ROWS)
#define VLOC_INSTANTIATE_ROWS(T)                                                                  \
    VLOC_PLANE_APPLY(T, launch_plane_rows_mode) VLOC_PLANE_AUX(T, launch_plane_rows_mode)
#else
#define VLOC_INSTANTIATE_ROWS(T)
#endif
#define VLOC_INSTANTIATE(T)                                                                       \
    VLOC_INSTANTIATE_STICK(T) VLOC_INSTANTIATE_FULL_APPLY(T) VLOC_INSTANTIATE_FULL_AUX(T)        \
    VLOC_INSTANTIATE_ROWS(T)
#if !defined(VLOC_ONLY_F32)
VLOC_INSTANTIATE(double)
#endif
#if !defined(VLOC_ONLY_F64)
VLOC_INSTANTIATE(float)
#endif

} // namespace vloc
