// plan.cpp -- host planner: cutoff sphere, z-stick table, occupied ranges,
// greedy stick-to-group deal, line splits and LDS sizing.
//
// Sphere (Sec. 2, eq. 3): |k+G|^2 <= 2 Ecut (1 + 1e-12), G = h b1 + k b2 + l b3.
// Compact FFT regions (Sec. 4.3): the first pass runs only on z-sticks that meet
// the sphere; the second only on the x-planes those sticks occupy; the last on
// the whole plane.  Deal (Sec. 3.2): columns sorted by descending plane-wave
// count, dealt to groups in turn.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>

namespace vloc {

static const double kTwoPi = 6.283185307179586476925286766559;

bool split_length(int L, Split &s)
{
    static const int codelets[] = {1, 2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16};
    int best1 = 0, best2 = 0;
    for (int a : codelets) {
        if (L % a) continue;
        int b = L / a;
        bool ok = false;
        for (int c : codelets) ok |= (c == b);
        if (!ok || a > b) continue;
        if (best1 == 0 || (b - a) < (best2 - best1)) {
            best1 = a;
            best2 = b;
        }
    }
    if (best1 == 0) return false;
    s.L = L;
    s.L1 = best1;
    s.L2 = best2;
    return true;
}

std::vector<double> twiddle_table(int L)
{
    std::vector<double> t(2 * (size_t)L);
    for (int j = 0; j < L; ++j) {
        // angle 2 pi j / L with j already in [0, L); use symmetry so that the
        // argument of cos/sin stays in [0, pi/4]
        long n8 = 8L * j;
        long oct = n8 / L;
        double c, s;
        // reduce to quadrant q and residue r: angle = pi/2 (q + r/L)
        long q = (4L * j) / L, r = 4L * j - q * L;
        if (2 * r <= L) {
            double b = (kTwoPi / 4) * (double)r / (double)L;
            c = std::cos(b);
            s = std::sin(b);
        } else {
            double b = (kTwoPi / 4) * (double)(L - r) / (double)L;
            c = std::sin(b);
            s = std::cos(b);
        }
        (void)oct;
        double cr, sr;
        switch (q) {
        case 0: cr = c; sr = s; break;
        case 1: cr = -s; sr = c; break;
        case 2: cr = -c; sr = -s; break;
        default: cr = s; sr = -c; break;
        }
        t[2 * j] = cr;
        t[2 * j + 1] = -sr; // exp(-i angle)
    }
    return t;
}

static bool reciprocal_rows(const double A[9], double B[9])
{
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                 A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!std::isfinite(det) || !(det > 0.0)) return false;
    // b_j = 2 pi (a_k x a_l) / det for cyclic (j, k, l)
    const double *a1 = A, *a2 = A + 3, *a3 = A + 6;
    auto cross = [](const double *u, const double *v, double *w) {
        w[0] = u[1] * v[2] - u[2] * v[1];
        w[1] = u[2] * v[0] - u[0] * v[2];
        w[2] = u[0] * v[1] - u[1] * v[0];
    };
    cross(a2, a3, B);
    cross(a3, a1, B + 3);
    cross(a1, a2, B + 6);
    for (int i = 0; i < 9; ++i) B[i] *= kTwoPi / det;
    return true;
}

vloc_status build_host_plan(HostPlan &p, const int32_t grid[3], const double cell[9], double ecut,
                            const double k[3], const vloc_options *opt, std::string &err)
{
    if (!grid || !cell || !k) {
        err = "NULL grid, cell or k";
        return VLOC_E_INVALID;
    }
    p.opt = opt ? *opt : vloc_options{};
    if (p.opt.precision != VLOC_F64 && p.opt.precision != VLOC_F32) {
        err = "precision must be VLOC_F64 or VLOC_F32";
        return VLOC_E_INVALID;
    }
    if (p.opt.deal < 0 || p.opt.deal > 2) {
        err = "unknown deal mode";
        return VLOC_E_INVALID;
    }
    if (p.opt.sticks_per_group < 0 || p.opt.sticks_per_group > 64 || p.opt.band_chunk < 0 ||
        p.opt.plane_rows < 0 || p.opt.plane_threads < 0 || p.opt.plane_threads > 512 ||
        (p.opt.plane_threads % 64) != 0) {
        err = "option out of range (sticks_per_group 0..64, plane_threads 0 or 64..512 step 64)";
        return VLOC_E_INVALID;
    }
    for (int i = 0; i < 3; ++i) {
        p.grid[i] = grid[i];
        p.kpt[i] = k[i];
        if (grid[i] < 1 || grid[i] > 256) {
            err = "grid dimension outside [1, 256]";
            return VLOC_E_GRID;
        }
    }
    if (!split_length(grid[0], p.sx) || !split_length(grid[1], p.sy) ||
        !split_length(grid[2], p.sz)) {
        err = "grid dimension is not a product of two codelet sizes {1..6,8,9,10,12,15,16}";
        return VLOC_E_GRID;
    }
    for (int i = 0; i < 9; ++i) {
        p.cell[i] = cell[i];
        if (!std::isfinite(cell[i])) {
            err = "non-finite cell";
            return VLOC_E_CELL;
        }
    }
    double B[9];
    if (!reciprocal_rows(cell, B)) {
        err = "cell determinant must be positive";
        return VLOC_E_CELL;
    }
    if (!std::isfinite(ecut) || !(ecut > 0.0) || !std::isfinite(k[0]) || !std::isfinite(k[1]) ||
        !std::isfinite(k[2])) {
        err = "ecut must be positive and k finite";
        return VLOC_E_SPHERE;
    }
    p.ecut = ecut;

    // ---- sphere: box |g_i + k_i| <= Gcut |a_i| / (2 pi), then the exact test
    const double g2max = 2.0 * ecut * (1.0 + 1e-12);
    const double gcut = std::sqrt(2.0 * ecut);
    long lo[3], hi[3];
    for (int i = 0; i < 3; ++i) {
        double alen = std::sqrt(cell[3 * i] * cell[3 * i] + cell[3 * i + 1] * cell[3 * i + 1] +
                                cell[3 * i + 2] * cell[3 * i + 2]);
        double ext = gcut * alen / kTwoPi;
        lo[i] = (long)std::floor(-ext - k[i]) - 1;
        hi[i] = (long)std::ceil(ext - k[i]) + 1;
        if (hi[i] - lo[i] > 4096) {
            err = "cutoff sphere too large";
            return VLOC_E_SPHERE;
        }
    }
    p.hkl.clear();
    p.sticks.clear();
    for (long h = lo[0]; h <= hi[0]; ++h)
        for (long kk = lo[1]; kk <= hi[1]; ++kk) {
            int32_t first = -1, cnt = 0;
            for (long l = lo[2]; l <= hi[2]; ++l) {
                double f0 = h + k[0], f1 = kk + k[1], f2 = l + k[2];
                double gx = f0 * B[0] + f1 * B[3] + f2 * B[6];
                double gy = f0 * B[1] + f1 * B[4] + f2 * B[7];
                double gz = f0 * B[2] + f1 * B[5] + f2 * B[8];
                if (gx * gx + gy * gy + gz * gz <= g2max) {
                    if (cnt > 0 && l != first + cnt) {
                        err = "internal: stick is not contiguous";
                        return VLOC_E_SPHERE;
                    }
                    if (cnt == 0) first = (int32_t)l;
                    p.hkl.push_back((int32_t)h);
                    p.hkl.push_back((int32_t)kk);
                    p.hkl.push_back((int32_t)l);
                    ++cnt;
                }
            }
            if (cnt > 0) {
                int32_t off = (int32_t)(p.hkl.size() / 3) - cnt;
                p.sticks.push_back(Stick{(int32_t)h, (int32_t)kk, off, cnt, first});
            }
        }
    if (p.sticks.empty()) {
        err = "empty cutoff sphere";
        return VLOC_E_SPHERE;
    }
    // ---- occupied ranges and aliasing
    p.hmin = p.hmax = p.sticks[0].h;
    p.kmin = p.kmax = p.sticks[0].k;
    int32_t lmin = p.sticks[0].lmin, lmax = lmin;
    for (const Stick &s : p.sticks) {
        p.hmin = std::min(p.hmin, s.h);
        p.hmax = std::max(p.hmax, s.h);
        p.kmin = std::min(p.kmin, s.k);
        p.kmax = std::max(p.kmax, s.k);
        lmin = std::min(lmin, s.lmin);
        lmax = std::max(lmax, s.lmin + s.count - 1);
    }
    if (p.hmax - p.hmin >= grid[0] || p.kmax - p.kmin >= grid[1] || lmax - lmin >= grid[2]) {
        char buf[160];
        std::snprintf(buf, sizeof buf,
                      "sphere extent (%d, %d, %d) does not fit the grid (%d, %d, %d): aliasing",
                      p.hmax - p.hmin + 1, p.kmax - p.kmin + 1, lmax - lmin + 1, grid[0], grid[1],
                      grid[2]);
        err = buf;
        return VLOC_E_SPHERE;
    }
    p.nxo = p.hmax - p.hmin + 1;

    // ---- launch geometry
    const int es = p.elem_bytes();
    const int Lz = grid[2];
    p.stick_threads = 256;
    int tasks_per_stick = std::max(p.sz.L1, p.sz.L2);
    p.group_cap = p.opt.sticks_per_group ? p.opt.sticks_per_group
                                         : std::max(1, p.stick_threads / tasks_per_stick);
    p.group_cap = std::min<int32_t>(p.group_cap, (int32_t)p.sticks.size());
    p.ldz = Lz + 1;
    const int64_t nst = p.nst();
    p.ngroups = (int32_t)((nst + p.group_cap - 1) / p.group_cap);

    // ---- deal (Sec. 3.2): sort by descending count, ties in canonical order
    std::vector<int32_t> order(nst);
    std::iota(order.begin(), order.end(), 0);
    if (p.opt.deal != VLOC_DEAL_CONTIGUOUS)
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return p.sticks[a].count > p.sticks[b].count;
        });
    p.group_of_stick.assign(nst, 0);
    std::vector<std::vector<int32_t>> members(p.ngroups);
    for (int64_t r = 0; r < nst; ++r) {
        int32_t g;
        if (p.opt.deal == VLOC_DEAL_CONTIGUOUS) {
            g = (int32_t)(r / p.group_cap);
        } else {
            g = (int32_t)(r % p.ngroups);
            if (p.opt.deal == VLOC_DEAL_SNAKE && ((r / p.ngroups) & 1)) g = p.ngroups - 1 - g;
        }
        p.group_of_stick[order[r]] = g;
        members[g].push_back(order[r]);
    }
    p.stick_of_slot.clear();
    p.group_start.assign(p.ngroups, 0);
    p.group_size.assign(p.ngroups, 0);
    for (int32_t g = 0; g < p.ngroups; ++g) {
        p.group_start[g] = (int32_t)p.stick_of_slot.size();
        p.group_size[g] = (int32_t)members[g].size();
        for (int32_t s : members[g]) p.stick_of_slot.push_back(s);
    }

    // ---- plane kernel sizing: plane (nxo x N2) plus a batch of full x rows
    p.ldy = grid[1] + 1;
    p.ldx = grid[0] + 1;
    const int64_t plane_bytes = (int64_t)p.nxo * p.ldy * es;
    const int64_t row_bytes = (int64_t)p.ldx * es;
    const int64_t lds_max = 160 * 1024;
    p.plane_threads = p.opt.plane_threads ? p.opt.plane_threads : 512;
    int xtasks = std::max(p.sx.L1, p.sx.L2);
    int rows = p.opt.plane_rows;
    if (rows == 0) {
        rows = std::max(1, p.plane_threads / xtasks);
        // a smaller batch that leaves room for two workgroups per CU wins if it
        // still keeps half the threads busy
        int64_t two = (lds_max / 2 - plane_bytes) / row_bytes;
        if (two * xtasks >= p.plane_threads / 2) rows = (int)std::min<int64_t>(rows, two);
    }
    rows = std::min(rows, grid[1]);
    if (plane_bytes + rows * row_bytes > lds_max) {
        rows = (int)((lds_max - plane_bytes) / row_bytes);
        if (rows < 1) {
            err = "occupied plane does not fit in LDS";
            return VLOC_E_GRID;
        }
    }
    p.plane_rows = rows;
    p.plane_lds = (int32_t)(plane_bytes + rows * row_bytes);

    // ---- band chunk: stick buffer of one chunk <= 128 MiB (stays in the 256 MB
    // memory-side cache between the three kernels)
    int64_t per_band = (int64_t)Lz * nst * es;
    int64_t chunk = std::max<int64_t>(1, (128LL << 20) / per_band);
    if (p.opt.band_chunk) chunk = p.opt.band_chunk;
    p.band_chunk = (int32_t)std::min<int64_t>(chunk, 1 << 20);
    return VLOC_OK;
}

} // namespace vloc
