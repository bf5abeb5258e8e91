// plan.hpp -- host-side plan of the compact local-potential application.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/vloc.h"

namespace vloc {

// One z-stick: the sphere points sharing (h, k); a contiguous run of c.
struct Stick {
    int32_t h, k, offset, count, lmin;
};

// How a line of length L is split into two register codelets, L = L1 * L2.
struct Split {
    int L = 0, L1 = 0, L2 = 0;
};

// Occupied index ranges a plan must cover at least: the k-points of a batch
// share one plane layout, so each member covers the union of their ranges.
struct Occupied {
    int32_t hmin, hmax, kmin, kmax, lmin, lmax;
};

struct HostPlan {
    int32_t grid[3] = {0, 0, 0};
    double cell[9] = {};
    double ecut = 0.0;
    double kpt[3] = {};
    vloc_options opt{};

    std::vector<int32_t> hkl;      // npw * 3, canonical order
    std::vector<Stick> sticks;     // canonical (h, k) order
    int32_t hmin = 0, hmax = 0, kmin = 0, kmax = 0, nxo = 0;
    int32_t lmin = 0, lmax = 0;
    int32_t zx = 0, zy = 0, zz = 0; // stage-A input groups that are zero on every line
    int32_t fx = 0;                 // x stage-A groups whose every position is occupied
    int32_t plane_full = 0;         // whole plane in LDS, x pass in place: 1 = spread
                                    // over the workgroup, 2 = rows per wavefront, 3 = row
                                    // blocks; 4 = parted plane (see plane_parts)
    int32_t plane_parts = 0;        // parted plane: x pass in this many parts of N2 / parts
                                    // rows, the others in a per-workgroup device scratch

    // deal of sticks to groups; slots are numbered so that each group's
    // sticks are contiguous
    int32_t ngroups = 0, group_cap = 0;
    std::vector<int32_t> group_of_stick;   // canonical stick -> group
    std::vector<int32_t> stick_of_slot;    // slot -> canonical stick
    std::vector<int32_t> group_start, group_size;

    Split sx, sy, sz;
    int32_t band_chunk = 0;   // bands per internal chunk
    int32_t density_chunk = 0; // bands per chunk of the density passes
    int32_t plane_rows = 0;   // x-pass rows per batch in the plane kernel
    int32_t plane_threads = 0;
    int32_t plane_lds = 0;    // bytes of LDS per plane workgroup
    int32_t stick_threads = 0;
    int32_t ldy = 0, ldx = 0, ldz = 0; // LDS line strides (complex elements)
    int32_t plane_rb = 0, plane_rl = 0; // x rows per wave batch, padded row length
    int32_t plane_xw = 0;               // wavefronts running the x pass
    int32_t plane_xq = 0;               // > 0: quad x pass, N1 = 4 plane_xq
    std::vector<int32_t> col_kmin, col_kcnt; // per occupied x-plane: first k, span of k
    std::vector<int32_t> holes;   // (h, k) pairs inside an x-plane's k span with no stick

    // real (gamma) mode: coefficients of the half sphere only, two bands per
    // complex transform
    bool gamma = false;
    std::vector<int32_t> half_hkl;  // half sphere, canonical order
    std::vector<int32_t> mirror;    // stick -> stick (-h, -k)
    std::vector<int32_t> half_off;  // stick -> offset of its half-sphere run (or -1)

    int64_t npw() const { return (int64_t)hkl.size() / 3; }
    // coefficients per band in the caller's arrays
    int64_t npw_io() const { return gamma ? (int64_t)half_hkl.size() / 3 : npw(); }
    int64_t nst() const { return (int64_t)sticks.size(); }
    int elem_bytes() const { return opt.precision == VLOC_F32 ? 8 : 16; }
};

// Builds everything host-side; returns VLOC_OK or an error with a message.
// With cover != NULL the occupied ranges are widened to include *cover.
vloc_status build_host_plan(HostPlan &p, const int32_t grid[3], const double cell[9], double ecut,
                            const double k[3], const vloc_options *opt, std::string &err,
                            const Occupied *cover = nullptr);

bool split_length(int L, Split &s);
bool is_codelet(int r); // r is a compiled codelet length

// exp(-2 pi i j / L) for j < L, FP64, angle numerator reduced exactly.
std::vector<double> twiddle_table(int L);

} // namespace vloc
