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
#include <climits>
#include <cmath>
#include <cstdio>
#include <numeric>

namespace vloc {

static const double kTwoPi = 6.283185307179586476925286766559;

// Register DFT codelets compiled in the kernels (dft_codelets.h).  Every
// 2,3,5-smooth length up to kMaxLine is a product of two of them.
static const int kCodelets[] = {1, 2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16, 18, 20, 24, 25, 27, 30, 32};
static const int kNumCodelets = (int)(sizeof kCodelets / sizeof kCodelets[0]);
static const int kMaxLine = 960;

bool is_codelet(int r)
{
    for (int c : kCodelets)
        if (c == r) return true;
    return false;
}

bool split_length(int L, Split &s)
{
    const int *codelets = kCodelets;
    int best1 = 0, best2 = 0;
    for (int i = 0; i < kNumCodelets; ++i) {
        const int a = codelets[i];
        if (L % a) continue;
        int b = L / a;
        if (!is_codelet(b) || a > b) continue;
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

// Bit n1 is set when no occupied position v in [lo, hi] (taken mod L) falls in
// the stage-A input group {n2 + L2 n1 : n2 < L2}.
static int32_t zero_mask(const Split &s, long lo, long hi)
{
    int32_t m = 0;
    for (int n1 = 0; n1 < s.L1; ++n1) {
        bool any = false;
        for (int n2 = 0; n2 < s.L2 && !any; ++n2) {
            long pos = n2 + (long)s.L2 * n1;
            long r = ((pos - lo) % s.L + s.L) % s.L;
            any = lo + r <= hi;
        }
        if (!any) m |= 1 << n1;
    }
    return m;
}

// Bit n1 is set when every position of the stage-A group {n2 + L2 n1} is
// occupied (lies in [lo, hi] taken mod L).
static int32_t full_mask(const Split &s, long lo, long hi)
{
    int32_t m = 0;
    for (int n1 = 0; n1 < s.L1; ++n1) {
        bool all = true;
        for (int n2 = 0; n2 < s.L2 && all; ++n2) {
            long pos = n2 + (long)s.L2 * n1;
            long r = ((pos - lo) % s.L + s.L) % s.L;
            all = lo + r <= hi;
        }
        if (all) m |= 1 << n1;
    }
    return m;
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

// Real (gamma) mode: psi real <=> c(-g) = conj(c(g)), so only the half sphere
// H = {h > 0} u {h = 0, k > 0} u {h = k = 0, l >= 0} is stored (canonical order
// restricted to H).  Per stick: its mirror stick (-h, -k) and the offset of
// its part of H in the half storage (for the (0, 0) stick: of l = 0).
static vloc_status build_gamma_tables(HostPlan &p, std::string &err)
{
    const int64_t nst = p.nst();
    const int32_t kspan = p.kmax - p.kmin + 1;
    std::vector<int32_t> at((size_t)(p.hmax - p.hmin + 1) * kspan, -1);
    for (int64_t i = 0; i < nst; ++i)
        at[(size_t)(p.sticks[i].h - p.hmin) * kspan + (p.sticks[i].k - p.kmin)] = (int32_t)i;
    p.mirror.assign(nst, -1);
    p.half_off.assign(nst, -1);
    p.half_hkl.clear();
    for (int64_t i = 0; i < nst; ++i) {
        const Stick &s = p.sticks[i];
        const int32_t mh = -s.h, mk = -s.k;
        int32_t m = -1;
        if (mh >= p.hmin && mh <= p.hmax && mk >= p.kmin && mk <= p.kmax)
            m = at[(size_t)(mh - p.hmin) * kspan + (mk - p.kmin)];
        if (m < 0 || p.sticks[m].count != s.count ||
            p.sticks[m].lmin != -(s.lmin + s.count - 1)) {
            err = "internal: the sphere is not symmetric under g -> -g";
            return VLOC_E_SPHERE;
        }
        p.mirror[i] = m;
        const bool zero = s.h == 0 && s.k == 0;
        if (zero || s.h > 0 || (s.h == 0 && s.k > 0)) {
            const int32_t l0 = zero ? 0 : s.lmin;
            p.half_off[i] = (int32_t)(p.half_hkl.size() / 3);
            for (int32_t l = l0; l < s.lmin + s.count; ++l) {
                p.half_hkl.push_back(s.h);
                p.half_hkl.push_back(s.k);
                p.half_hkl.push_back(l);
            }
        }
    }
    return VLOC_OK;
}

vloc_status build_host_plan(HostPlan &p, const int32_t grid[3], const double cell[9], double ecut,
                            const double k[3], const vloc_options *opt, std::string &err,
                            const Occupied *cover)
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
    if (p.opt.deal < 0 || p.opt.deal > 3) {
        err = "unknown deal mode";
        return VLOC_E_INVALID;
    }
    if (p.opt.sticks_per_group < 0 || p.opt.sticks_per_group > 64 || p.opt.band_chunk < 0 ||
        p.opt.plane_rows < 0 || p.opt.plane_threads < 0 || p.opt.plane_threads > 1024 ||
        (p.opt.plane_threads % 64) != 0 || p.opt.plane_xwaves < 0 ||
        (p.opt.plane_threads > 512 && p.opt.precision != VLOC_F64) ||
        p.opt.plane_xwaves * 64 > (p.opt.plane_threads ? p.opt.plane_threads : 512) ||
        p.opt.plane_xmode < 0 || p.opt.plane_xmode > 6 || p.opt.gamma < 0 ||
        p.opt.gamma > 1) {
        err = "option out of range (sticks_per_group 0..64, plane_threads 0 or 64..512 step 64 "
              "(FP64: up to 1024), "
              "plane_xwaves <= plane_threads / 64, plane_xmode 0..6, gamma 0..1)";
        return VLOC_E_INVALID;
    }
    p.gamma = p.opt.gamma != 0;
    if (p.gamma && (!k || k[0] != 0.0 || k[1] != 0.0 || k[2] != 0.0)) {
        err = "the real (gamma) mode needs k = 0";
        return VLOC_E_INVALID;
    }
    for (int i = 0; i < 3; ++i) {
        p.grid[i] = grid[i];
        p.kpt[i] = k[i];
        if (grid[i] < 1 || grid[i] > kMaxLine) {
            err = "grid dimension outside [1, " + std::to_string(kMaxLine) + "]";
            return VLOC_E_GRID;
        }
        int r = grid[i];
        for (int f : {2, 3, 5})
            while (r % f == 0) r /= f;
        if (r != 1) {
            err = "grid dimension " + std::to_string(grid[i]) +
                  " has a prime factor other than 2, 3 and 5";
            return VLOC_E_GRID;
        }
    }
    if (!split_length(grid[0], p.sx) || !split_length(grid[1], p.sy) ||
        !split_length(grid[2], p.sz)) {
        err = "internal: no two-codelet split of a 2,3,5-smooth grid dimension";
        return VLOC_E_GRID;
    }
    // Row-block layout of the plane kernel: blocks of L2y = 8 rows and an x
    // split with L2x = 8 (the compiled kernels)
    if (p.opt.plane_xmode == 5) {
        Split *sp[2] = {&p.sx, &p.sy};
        for (int a = 0; a < 2; ++a) {
            if (p.opt.split[a]) continue;
            const int L = grid[a];
            if (L % 8 || !is_codelet(L / 8)) {
                err = "the row-block layout (plane_xmode 5) needs N1 and N2 = 8 L1 with L1 a "
                      "codelet length";
                return VLOC_E_INVALID;
            }
            sp[a]->L1 = L / 8;
            sp[a]->L2 = 8;
        }
    }
    {
        Split *sp[3] = {&p.sx, &p.sy, &p.sz};
        for (int a = 0; a < 3; ++a) {
            const int l1 = p.opt.split[a];
            if (!l1) continue;
            const int L = grid[a];
            if (l1 < 0 || L % l1 || !is_codelet(l1) || !is_codelet(L / l1)) {
                err = "split[" + std::to_string(a) + "] = " + std::to_string(l1) +
                      " does not split " + std::to_string(L) + " into two codelet lengths";
                return VLOC_E_INVALID;
            }
            sp[a]->L1 = l1;
            sp[a]->L2 = L / l1;
        }
    }
    // workgroups of more than 512 threads have registers for codelets of at
    // most 16 points
    const bool big_codelet = std::max(std::max(p.sx.L1, p.sx.L2), std::max(p.sy.L1, p.sy.L2)) > 16;
    if (big_codelet && p.opt.plane_threads > 512) {
        err = "plane_threads > 512 needs x and y codelets of at most 16 points";
        return VLOC_E_INVALID;
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
    if (cover) {
        p.hmin = std::min(p.hmin, cover->hmin);
        p.hmax = std::max(p.hmax, cover->hmax);
        p.kmin = std::min(p.kmin, cover->kmin);
        p.kmax = std::max(p.kmax, cover->kmax);
        lmin = std::min(lmin, cover->lmin);
        lmax = std::max(lmax, cover->lmax);
    }
    p.lmin = lmin;
    p.lmax = lmax;
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
    p.zx = zero_mask(p.sx, p.hmin, p.hmax);
    p.fx = full_mask(p.sx, p.hmin, p.hmax);
    p.zy = zero_mask(p.sy, p.kmin, p.kmax);
    p.zz = zero_mask(p.sz, lmin, lmax);

    // ---- launch geometry
    const int es = p.elem_bytes();
    const int Lz = grid[2];
    // stick kernels: FP64 groups of ~21 sticks on 256 threads, FP32 groups of
    // ~32 sticks on 384 threads (measured best at 96^3)
    int tasks_per_stick = std::max(p.sz.L1, p.sz.L2);
    const int want_threads = es == 16 ? 256 : 384;
    p.group_cap = p.opt.sticks_per_group ? p.opt.sticks_per_group
                                         : std::max(1, want_threads / tasks_per_stick);
    p.group_cap = std::min<int32_t>(p.group_cap, (int32_t)p.sticks.size());
    p.ldz = Lz + 1;
    {
        // the stick kernels keep a group's lines and the z-stage twiddles in LDS
        const int64_t cap = (160 * 1024 / es - Lz) / (Lz + 1);
        if (p.group_cap > cap) {
            if (p.opt.sticks_per_group) {
                char buf[200];
                std::snprintf(buf, sizeof buf,
                         "sticks_per_group %d: the stick kernels' LDS holds at most %lld "
                         "sticks of %d points",
                         p.opt.sticks_per_group, (long long)cap, Lz);
                err = buf;
                return VLOC_E_INVALID;
            }
            p.group_cap = (int32_t)std::max<int64_t>(1, cap);
        }
    }
    const int64_t nst = p.nst();

    // ---- units of the deal: one stick, or in the real (gamma) mode a stick of
    // the half sphere with its mirror (-h, -k), which the stick kernels need in
    // one workgroup; the (0, 0) stick is its own mirror
    std::vector<std::vector<int32_t>> units;
    if (p.gamma) {
        vloc_status s = build_gamma_tables(p, err);
        if (s != VLOC_OK) return s;
        for (int64_t i = 0; i < nst; ++i) {
            const Stick &st = p.sticks[i];
            if (st.h == 0 && st.k == 0)
                units.push_back({(int32_t)i});
            else if (st.h > 0 || (st.h == 0 && st.k > 0))
                units.push_back({(int32_t)i, p.mirror[i]});
        }
        // a group holds whole units: at most group_cap / 2 pairs
        p.group_cap = 2 * std::max<int32_t>(1, p.group_cap / 2);
    } else {
        for (int64_t i = 0; i < nst; ++i) units.push_back({(int32_t)i});
    }
    const int64_t nunits = (int64_t)units.size();
    const int32_t upg = p.gamma ? p.group_cap / 2 : p.group_cap; // units per group
    p.ngroups = (int32_t)((nunits + upg - 1) / upg);
    p.stick_threads = (int)std::min<int64_t>(
        512, std::max<int64_t>(64, ((int64_t)std::min<int64_t>(p.group_cap, nst) *
                                        tasks_per_stick + 63) / 64 * 64));

    // ---- deal (Sec. 3.2): sort by descending count, ties in canonical order
    std::vector<int32_t> order(nunits);
    std::iota(order.begin(), order.end(), 0);
    if (p.opt.deal == VLOC_DEAL_GREEDY || p.opt.deal == VLOC_DEAL_SNAKE)
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return p.sticks[units[a][0]].count > p.sticks[units[b][0]].count;
        });
    p.group_of_stick.assign(nst, 0);
    std::vector<std::vector<int32_t>> members(p.ngroups);
    for (int64_t r = 0; r < nunits; ++r) {
        int32_t g;
        if (p.opt.deal == VLOC_DEAL_CONTIGUOUS) {
            g = (int32_t)(r / upg);
        } else {
            g = (int32_t)(r % p.ngroups);
            if (p.opt.deal == VLOC_DEAL_SNAKE && ((r / p.ngroups) & 1)) g = p.ngroups - 1 - g;
        }
        for (int32_t s : units[order[r]]) {
            p.group_of_stick[s] = g;
            members[g].push_back(s);
        }
    }
    p.stick_of_slot.clear();
    p.group_start.assign(p.ngroups, 0);
    p.group_size.assign(p.ngroups, 0);
    for (int32_t g = 0; g < p.ngroups; ++g) {
        p.group_start[g] = (int32_t)p.stick_of_slot.size();
        p.group_size[g] = (int32_t)members[g].size();
        for (int32_t s : members[g]) p.stick_of_slot.push_back(s);
    }

    // ---- plane kernel sizing: the occupied plane (nxo x N2, column stride
    // ldy) plus, per wavefront, a batch of rb full x rows of padded length rl
    p.ldy = grid[1] + 1;
    p.ldx = grid[0] + 1;
    const int64_t plane_bytes = (int64_t)p.nxo * p.ldy * es;
    const int64_t lds_max = 160 * 1024;
    p.plane_rl = p.sx.L1 * (p.sx.L2 + 1);
    p.plane_rl += ((p.sx.L2 - p.plane_rl) % 16 + 16) % 16; // same rule as the kernel
    const int nwaves = (p.opt.plane_threads ? p.opt.plane_threads : 512) / 64;
    p.plane_threads = nwaves * 64;
    // Choose (x waves, rows per batch) by an estimate of the plane time in
    // wave instructions: a stage with more than 64 tasks costs whole extra
    // rounds.  The y pass runs on all 4 SIMDs; the x pass on min(4, xw) of them
    // and no faster than its slowest wave, with a latency charge of 1/(2 xw);
    // the sum is divided by the workgroups that fit on a CU (LDS-bound, <= 2).
    auto log2i = [](int v) { double l = 0; while (v > 1) { v >>= 1; l += 1; } return l; };
    const double cA = 3.0 * p.sx.L1 * log2i(p.sx.L1) + 4.0 * (p.sx.L1 - 1) + 20.0;
    const double cB = 6.0 * p.sx.L2 * log2i(p.sx.L2) + 2.0 * p.sx.L2 + 30.0;
    const double cAy = 3.0 * p.sy.L1 * log2i(p.sy.L1) + 4.0 * (p.sy.L1 - 1) + 20.0;
    const double cBy = 3.0 * p.sy.L2 * log2i(p.sy.L2) + 30.0;
    const int N2 = grid[1];
    const double ycost = 2.0 * (((int64_t)p.nxo * p.sy.L2 + 63) / 64 * cAy +
                                ((int64_t)p.nxo * p.sy.L1 + 63) / 64 * cBy);
    double best = 1e300;
    int best_xw = 0, best_rb = 0;
    for (int xw = 1; xw <= nwaves; ++xw) {
        if (p.opt.plane_xwaves && xw != p.opt.plane_xwaves) continue;
        const int rpw = (N2 + xw - 1) / xw;
        for (int rb = 1; rb <= rpw; ++rb) {
            // (plane_rows sizes the parts instead when the parted plane is asked for)
            if (p.opt.plane_rows && p.opt.plane_xmode != 6 &&
                rb != std::min<int>(p.opt.plane_rows, rpw))
                continue;
            const int64_t lds = plane_bytes + (int64_t)xw * rb * p.plane_rl * es;
            if (lds > lds_max) break;
            double total = 0, slowest = 0;
            for (int w = 0; w < xw; ++w) {
                int rows = std::min(rpw, std::max(0, N2 - w * rpw));
                double c = 0;
                for (int y = 0; y < rows; y += rb) {
                    int nr = std::min(rb, rows - y);
                    c += 2 * cA * ((nr * p.sx.L2 + 63) / 64) + cB * ((nr * p.sx.L1 + 63) / 64);
                }
                total += c;
                slowest = std::max(slowest, c);
            }
            const int nwg = (int)std::min<int64_t>(2, lds_max / lds);
            double tx = std::max(total / std::min(4, xw), slowest) * (1.0 + 0.5 / xw);
            double t = (ycost / 4.0 + tx) / nwg;
            if (t < best - 1e-9 || (std::abs(t - best) <= 1e-9 && xw > best_xw)) {
                best = t;
                best_xw = xw;
                best_rb = rb;
            }
        }
    }
    if (best_xw == 0) {
        err = "occupied plane does not fit in LDS";
        return VLOC_E_GRID;
    }
    p.plane_xw = best_xw;
    p.plane_rb = best_rb;
    p.plane_rows = best_rb;
    p.plane_lds = (int32_t)(plane_bytes + (int64_t)best_xw * best_rb * p.plane_rl * es);
    // Quad x pass: one lane quad per row holds a whole row in registers, so
    // the occupied plane is the only LDS.  Compiled for N1 = 4 xq with
    // xq in {6, 18, 20, 24} and the y split each goes with.
    {
        int xq = (grid[0] % 4 == 0) ? grid[0] / 4 : 0;
        bool have = (xq == 24 && p.sy.L1 == 8 && p.sy.L2 == 12) ||
                    (xq == 6 && p.sy.L1 == 4 && p.sy.L2 == 6) ||
                    (xq == 18 && p.sy.L1 == 8 && p.sy.L2 == 12) ||
                    (xq == 20 && p.sy.L1 == 8 && p.sy.L2 == 10);
        int qthreads = ((4 * grid[1] + 63) / 64) * 64;
        bool fits = have && qthreads <= 512 && plane_bytes <= lds_max;
        // measured slower than the row buffers in both precisions at 96^3, so
        // only used when asked for
        bool want = p.opt.plane_xmode == 2;
        if (p.opt.plane_xmode == 2 && (!fits || p.opt.plane_threads > 512)) {
            err = "quad x pass not available for this grid";
            return VLOC_E_INVALID;
        }
        if (want && fits) {
            p.plane_xq = xq;
            p.plane_threads = p.opt.plane_threads ? std::max<int>(p.opt.plane_threads, qthreads)
                                                  : qthreads;
            p.plane_xw = 0;
            p.plane_rb = 1;
            p.plane_rows = 0;
            p.plane_lds = (int32_t)plane_bytes;
        }
    }
    // Full plane: the whole plane in LDS and the x pass in place over all
    // threads (no row buffers).  The default wherever it fits; the row-buffer
    // layout otherwise or when asked for.
    {
        // the plane, then the y and x stage twiddles and the column k ranges
        const int64_t full_bytes = (int64_t)grid[0] * p.ldy * es +
                                   (int64_t)(grid[0] + grid[1]) * es + (int64_t)p.nxo * 8;
        const bool fits = full_bytes <= lds_max;
        if ((p.opt.plane_xmode == 3 || p.opt.plane_xmode == 4) && !fits) {
            err = "the full plane does not fit in LDS (plane_xmode 3 or 4)";
            return VLOC_E_INVALID;
        }
        if (p.opt.plane_xmode == 5) {
            // row blocks: column stride N2 + 7, one 768-thread workgroup per CU
            const int64_t rb_bytes = (int64_t)grid[0] * (grid[1] + 7) * es +
                                     (int64_t)(grid[0] + grid[1]) * es;
            if (rb_bytes > lds_max || !fits) {
                err = "the row-block layout (plane_xmode 5) does not fit in LDS";
                return VLOC_E_INVALID;
            }
            if (p.opt.precision != VLOC_F64 || big_codelet ||
                (p.opt.plane_threads && p.opt.plane_threads != 768) ||
                (int64_t)p.nxo * p.sy.L2 > 768) {
                err = "the row-block layout (plane_xmode 5) needs FP64, 768 plane threads, "
                      "codelets of at most 16 points and nxo * 8 <= 768";
                return VLOC_E_INVALID;
            }
            p.plane_full = 3;
            p.plane_xq = 0;
            p.plane_xw = 0;
            p.plane_rb = 0;
            p.plane_rows = 0;
            p.plane_lds = (int32_t)std::max(full_bytes, rb_bytes);
            p.plane_threads = 768;
        } else if (fits && (p.opt.plane_xmode >= 3 || p.opt.plane_xmode == 0)) {
            p.plane_full = p.opt.plane_xmode == 4 ? 2 : 1;
            p.plane_xq = 0;
            p.plane_xw = 0;
            p.plane_rb = 0;
            p.plane_rows = 0;
            p.plane_lds = (int32_t)full_bytes;
            p.plane_threads = p.opt.plane_threads ? p.opt.plane_threads
                                                  : (es == 16 && !big_codelet ? 1024 : 512);
            // The direct y form of the plane kernel holds nxo L2y y stage-A
            // tasks, one per thread in FP64 (more than 512 threads), two in FP32.
            // Unless the y split was asked for, take the swapped split when
            // only it fits (128^3 FP32, |G| <= 32: 65 x 16 tasks do not fit
            // 1024, 65 x 8 do); the form saves the scatter, the gather and
            // three barriers per plane.
            const int64_t dcap = es == 16 ? (p.plane_threads > 512 ? p.plane_threads : 0)
                                          : 2LL * p.plane_threads;
            if (!p.opt.split[1] && dcap > 0 && p.sy.L1 != p.sy.L2 &&
                (int64_t)p.nxo * p.sy.L2 > dcap && (int64_t)p.nxo * p.sy.L1 <= dcap) {
                std::swap(p.sy.L1, p.sy.L2);
                p.zy = zero_mask(p.sy, p.kmin, p.kmax);
            }
        }
    }
    // Parted plane: the occupied columns (nxo x N2) for the y pass and one row
    // buffer of N2 / P rows (N1 x (N2 / P + 1)) for the x pass, sharing the
    // LDS; the x pass runs part by part and the rows of the other parts wait
    // in a per-workgroup device scratch of nxo x N2 values.  P divides L1y, so
    // that the rows of one y stage-B line lie in one part.  The default where
    // the whole plane does not fit (measured faster than the row buffers: FP64
    // at 128^3 on 768 threads, the only FP64 width with registers for its
    // 16-point stages; FP32 at 144^3 and 160^3 on 1024); plane_rows asks for
    // N2 / P rows per part.
    if (p.opt.plane_xmode == 6 || (p.opt.plane_xmode == 0 && !p.plane_full)) {
        const int nthr = p.opt.plane_threads ? p.opt.plane_threads
                                             : (big_codelet ? 512 : (es == 16 ? 768 : 1024));
        // unless asked otherwise, the longer y codelet first: shorter y
        // stage-B lines to hold across the part barrier
        Split sx = p.sx, sy = p.sy;
        if (!p.opt.split[1] && sy.L1 < sy.L2) std::swap(sy.L1, sy.L2);
        const int64_t cbytes = (int64_t)p.nxo * p.ldy * es;
        const int64_t extra = (int64_t)(grid[0] + grid[1]) * es + (int64_t)p.nxo * 8;
        int parts = 0;
        int64_t lds = 0;
        for (int P = 2; P <= sy.L1 && !parts; ++P) {
            if (sy.L1 % P) continue;
            const int rpp = grid[1] / P;
            if (p.opt.plane_rows && p.opt.plane_rows != rpp) continue;
            const int64_t rbytes = (int64_t)grid[0] * (rpp + 1) * es;
            const int64_t tot = std::max(cbytes, rbytes) + extra;
            if (tot <= lds_max) {
                parts = P;
                lds = tot;
            }
        }
        const bool ok = parts > 0 && (int64_t)p.nxo * (sy.L1 / parts) <= nthr &&
                        (!big_codelet || nthr <= 512);
        if (p.opt.plane_xmode == 6 && !ok) {
            err = "the parted plane (plane_xmode 6) needs a part size N2 / P with P dividing "
                  "L1y whose row buffer fits in LDS, and nxo * L1y / P <= plane_threads";
            return VLOC_E_INVALID;
        }
        if (ok) {
            p.sx = sx;
            p.sy = sy;
            p.zx = zero_mask(p.sx, p.hmin, p.hmax);
            p.fx = full_mask(p.sx, p.hmin, p.hmax);
            p.zy = zero_mask(p.sy, p.kmin, p.kmax);
            p.plane_full = 4;
            p.plane_parts = parts;
            p.plane_xq = 0;
            p.plane_xw = 0;
            p.plane_rb = 0;
            p.plane_rows = grid[1] / parts;
            p.plane_lds = (int32_t)lds;
            p.plane_threads = nthr;
        }
    }
    // per occupied x-plane: first k (mod N2) and the span of k from the first
    // to the last stick of the plane.  On a skewed cell with a k-shift the
    // sticks of one x-plane need not be contiguous in k (the sphere's section
    // at fixed h can miss every integer l at some k between two that it
    // meets); those positions are holes, zero in the y pass's input.
    p.col_kmin.assign(p.nxo, 0);
    p.col_kcnt.assign(p.nxo, 0);
    p.holes.clear();
    {
        std::vector<int32_t> kmin(p.nxo, INT32_MAX), kmax(p.nxo, INT32_MIN);
        for (const Stick &s : p.sticks) {
            int hc = s.h - p.hmin;
            kmin[hc] = std::min(kmin[hc], s.k);
            kmax[hc] = std::max(kmax[hc], s.k);
        }
        std::vector<int32_t> seen(p.nxo, 0);
        for (const Stick &s : p.sticks) seen[s.h - p.hmin]++;
        for (int hc = 0; hc < p.nxo; ++hc) {
            if (!seen[hc]) continue;
            p.col_kmin[hc] = ((kmin[hc] % grid[1]) + grid[1]) % grid[1];
            p.col_kcnt[hc] = kmax[hc] - kmin[hc] + 1;
        }
        // sticks are in canonical (h, k) order: walk each plane's k values
        size_t i = 0;
        while (i < p.sticks.size()) {
            const int32_t h = p.sticks[i].h;
            int32_t next_k = p.sticks[i].k;
            for (; i < p.sticks.size() && p.sticks[i].h == h; ++i) {
                for (int32_t kk = next_k; kk < p.sticks[i].k; ++kk) {
                    p.holes.push_back(h);
                    p.holes.push_back(kk);
                }
                next_k = p.sticks[i].k + 1;
            }
        }
    }

    // ---- band chunk: at most as many launch bands as keep the stick buffer
    // within 256 MiB (measured at 96^3: larger chunks amortise the kernel
    // boundaries; beyond this size nothing more is gained); a call's bands are
    // then cut into equal chunks of at most this size
    int64_t per_band = (int64_t)Lz * nst * es;
    int64_t chunk = std::max<int64_t>(1, (256LL << 20) / per_band);
    if (p.opt.band_chunk) chunk = p.opt.band_chunk;
    // stick-kernel blocks of one launch (chunk * ngroups) stay below 2^31
    chunk = std::min<int64_t>(chunk, INT32_MAX / std::max<int32_t>(1, p.ngroups));
    p.band_chunk = (int32_t)std::min<int64_t>(chunk, 1 << 20);
    // the density passes also keep the FP64 partial planes live, which share
    // the device's 256 MB last-level cache with the stick buffer: there the
    // automatic chunk keeps the stick buffer within 176 MiB (measured at 128^3:
    // 54 instead of 81 FP32 bands per launch, 27 instead of 40 FP64)
    int64_t dchunk = std::max<int64_t>(1, (176LL << 20) / per_band);
    p.density_chunk = p.opt.band_chunk ? p.band_chunk
                                       : (int32_t)std::min<int64_t>(dchunk, p.band_chunk);
    return VLOC_OK;
}

} // namespace vloc
