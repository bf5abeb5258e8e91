// kernels.hpp -- launch interface of the three transform kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace vloc {

// APPLY_DENSITY: the application and, from the same real-space values, the
// weighted density of the launch's bands (one pass instead of two).
enum PlaneMode {
    MODE_APPLY = 0,
    MODE_G2R = 1,
    MODE_R2G = 2,
    MODE_DENSITY = 3,
    MODE_APPLY_DENSITY = 4
};

// Tables and sizes shared by the kernels of one plan (device pointers).
struct DevTables {
    const int4 *slot_info;  // per slot: {offset, count, lmin mod N3, plane position}
    const int2 *groups;     // per group: {first slot, number of sticks}
    const int2 *cols;       // per occupied x-plane: {first k mod N2, number of k}
    const void *twx, *twy, *twz; // exp(-2 pi i n2 k1 / L) at [n2][k1] (L = L1 L2, k1 < L1),
                                 // complex of the plan precision
    const double2 *twx64;        // exp(-2 pi i j / N1) in FP64 (quad x pass)
    double *partial;             // density: [nsub][N3][N2][N1] partial sums (FP64)
    const double *wts;           // density: band weights (FP64)
    // real mode, per slot: {source offset in the half-sphere arrays, kind
    // (0 = stick of the half sphere, 1 = its mirror, 2 = the (0, 0) stick),
    // -lmin of the (0, 0) stick, index in the group of the mirror stick}
    const int4 *gam;
    // whole-plane layout, per occupied x-plane hc and row y (hc-major, N2 per
    // hc): the slot of stick (hmin + hc, y), or -1
    const int *yslot;
    // plane positions that lie inside an occupied x-plane's k span but hold no
    // stick (zero in the y pass's input); rows [hole_off, hole_off + nholes)
    // of a segment
    const int *holes;
    // parted plane: per workgroup of the plane grid, nxo x N2 values [hc][yp]
    // (rows of the parts not in the row buffer)
    void *parts;
};

struct Geometry {
    int N1, N2, N3;
    int L1x, L2x, L1y, L2y, L1z, L2z;
    int nxo;        // occupied x-planes
    unsigned long long nxo_magic; // ceil(2^40 / nxo): v / nxo = (v nxo_magic) >> 40, v < 2^16
    int hmin_mod;   // hmin mod N1
    int ldy, ldx, ldz;
    int rb, rl;     // x rows per wavefront batch, padded row length in the plane kernel
    int xw;         // wavefronts taking part in the x pass
    int xq;         // > 0: quad x pass with N1 = 4 xq (no row buffer)
    int zx, zy, zz; // zero masks of the first-stage input groups per axis (0 = none)
    int fx;         // x stage-A groups whose every position is occupied
    int full;       // plane kernel holds the whole plane, x pass in place: 1 = spread
                    // over the workgroup, 2 = rows owned by wavefronts, 3 = row blocks;
                    // 4 = parted plane (0 = row buffers or lane quads)
    int parts;      // parted plane: x-pass parts of N2 / parts rows
    int parts_elems; // parted plane: LDS elements of the columns / row buffer region
    int resident_plane_wgs; // plane workgroups resident at once on the device
    int nsub;       // density: band subsets per launch
    int group_cap;  // most sticks in one group (over all segments)
    int gamma;      // real mode: a launch band is a pair of real bands
    double inv_n;   // 1 / (N1 N2 N3)
};

// One launch covers the bands of up to kMaxSeg k-points ("segments") that
// share the grid and the occupied-plane geometry.  Segment s owns launch bands
// [band_lo, band_lo + nb), its stick buffer at S + s_off ([band][z][slot],
// nst slots), its rows of the device tables, and blocks
// [blk_lo, blk_lo + nb * ngroups) of the stick kernels (group fastest).
constexpr int kMaxSeg = 8;
struct Seg {
    const void *in;   // stick forward input: c of the segment's first band
    void *out;        // stick backward output: out of the segment's first band
    long long s_off;  // element offset of the segment's stick buffer in S
    int nst, npw, ngroups;
    int slot_off, group_off, col_off; // first row in slot_info, groups, cols
    int band_lo, nb, blk_lo;
    int nbr;          // real mode: real bands from `in` / `out` (2 nb or 2 nb - 1)
    int hole_off, nholes; // rows of the segment in the hole table
    // the segment's occupied x-planes (a batch with a whole-plane layout plans
    // each k-point on its own occupied range): count, ceil(2^40 / count) and
    // first x-plane mod N1
    int nxo, hmin_mod;
    unsigned long long nxo_magic;
};
struct Launch {
    int nseg;  // segments in use (1 .. kMaxSeg)
    int nbt;   // bands of all segments
    int nblk;  // stick-kernel blocks of all segments
    Seg seg[kMaxSeg];
};

// K1: stick z-transforms (G -> r direction) from each segment's c into the
// stick buffer S.
template <typename T>
hipError_t launch_stick_fwd(const Geometry &g, const DevTables &t, const Launch &L, void *S,
                            int threads, hipStream_t st);
// K2: plane kernel over the planes of every segment.  APPLY: S -> S in place.
// G2R: S -> psi rows; R2G: psi -> S; DENSITY: weighted |psi|^2 into the
// partial planes; APPLY_DENSITY: both APPLY and DENSITY.  The last three take one segment; psi and the weights are
// indexed from band band0 (the launch's first band in the caller's arrays).
template <typename T>
hipError_t launch_plane(const Geometry &g, const DevTables &t, const Launch &L, int mode, void *S,
                        const void *V, void *psi, int64_t band0, int threads, int lds_bytes,
                        hipStream_t st);
// The plane-kernel launchers of the two layouts (whole plane in LDS; occupied
// x-planes with row buffers or lane quads), called by launch_plane.
template <typename T, int MODE>
hipError_t launch_plane_full_mode(const Geometry &g, const DevTables &t, const Launch &L, void *S,
                                  const void *V, void *psi, int64_t band0, int threads, int lds,
                                  hipStream_t st);
template <typename T, int MODE>
hipError_t launch_plane_rows_mode(const Geometry &g, const DevTables &t, const Launch &L, void *S,
                                  const void *V, void *psi, int64_t band0, int threads, int lds,
                                  hipStream_t st);
// Compiled specialisations of the whole-plane application kernel for the
// splits the schedule tuner tries; hit = false where none applies.
template <typename T>
hipError_t launch_plane_full_tuned(const Geometry &g, const DevTables &t, const Launch &L,
                                   void *S, const void *VT, int threads, int lds, hipStream_t st,
                                   bool &hit);
// ... those of workload geometry G (one compiled part each)
template <typename T, int G>
hipError_t launch_plane_full_tuned_g(const Geometry &g, const DevTables &t, const Launch &L,
                                     void *S, const void *VT, int threads, int lds,
                                     hipStream_t st, bool &hit);
// Density helpers (reduce.hip): FP64 reductions and band scaling.
hipError_t launch_fill_f64(double *x, int64_t n, double v, hipStream_t st);
// y[i] = factor * s * x[i], s = scale[0] (or 1 if scale is NULL); y may equal x.
hipError_t launch_scale_real(const double *x, int64_t n, const double *scale, double factor,
                             double *y, hipStream_t st);
// partial planes in [z][y][x] order, or with full != 0 in the full-plane
// kernel's [z][x][yp] order
hipError_t launch_density_reduce(const Geometry &g, const double *partial, int nsub,
                                 const double *scale, double *rho, hipStream_t st);
template <typename T>
hipError_t launch_band_dot(const void *a, const void *b, int64_t npw, int64_t nb, double *out,
                           hipStream_t st);
hipError_t launch_weighted_sum(const double *x, const double *w, int64_t n, double *out,
                               hipStream_t st);
template <typename T>
hipError_t launch_scale_bands(const void *x, int64_t npw, int64_t nb, const double *w,
                              const double *scale, double factor, void *y, hipStream_t st);

// VT[z][k1][yp][k2] = V[z][y][k1 + L1x k2] with yp the row's position after the
// y pass (the full-plane kernel's order of the potential).
template <typename T>
hipError_t launch_arrange_v(const Geometry &g, const void *V, void *VT, hipStream_t st);
// K3: stick z-transforms (r -> G direction) with 1/N, gathering into each
// segment's out.
template <typename T>
hipError_t launch_stick_bwd(const Geometry &g, const DevTables &t, const Launch &L, const void *S,
                            int threads, hipStream_t st);

} // namespace vloc
