// api.cpp -- the C ABI of libvloc (declared in include/vloc.h).
//
// A plan is built on the host (plan.cpp); its device tables are uploaded on
// first use.  vloc_apply runs, per band chunk, K1 (stick z-transforms), K2
// (plane kernel with the potential) and K3 (stick z-transforms back, 1/N,
// gather) on the plan's stream, with the stick buffer S of one chunk reused
// in place by K2.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"

using namespace vloc;

struct vloc_plan_s {
    HostPlan hp;
    hipStream_t stream = nullptr;
    bool uploaded = false;
    int device = -1;
    int4 *d_slot = nullptr;
    int2 *d_groups = nullptr;
    int2 *d_cols = nullptr;
    void *d_tw[3] = {nullptr, nullptr, nullptr};
    double2 *d_twx64 = nullptr;
    void *d_S = nullptr;
    size_t S_bytes = 0;
    double *d_partial = nullptr; // density partial planes
    size_t partial_bytes = 0;
    Geometry geo{};
    // kernel timing: events[4*i .. 4*i+3] bracket K1, K2, K3 of chunk launch i
    bool timing = false;
    std::vector<hipEvent_t> events;
    size_t events_used = 0;
    std::vector<int> rec_modes;
};

namespace {

thread_local std::string g_err;

vloc_status fail(vloc_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

vloc_status hip_fail(hipError_t e, const char *where)
{
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return VLOC_E_DEVICE;
}

void free_device(vloc_plan p)
{
    if (p->d_slot) (void)hipFree(p->d_slot);
    if (p->d_groups) (void)hipFree(p->d_groups);
    if (p->d_cols) (void)hipFree(p->d_cols);
    if (p->d_twx64) (void)hipFree(p->d_twx64);
    p->d_twx64 = nullptr;
    p->d_cols = nullptr;
    for (void *&t : p->d_tw)
        if (t) (void)hipFree(t), t = nullptr;
    if (p->d_S) (void)hipFree(p->d_S);
    if (p->d_partial) (void)hipFree(p->d_partial);
    p->d_partial = nullptr;
    p->partial_bytes = 0;
    p->d_slot = nullptr;
    p->d_groups = nullptr;
    p->d_S = nullptr;
    p->S_bytes = 0;
    p->uploaded = false;
}

vloc_status upload(vloc_plan p)
{
    if (p->uploaded) return VLOC_OK;
    const HostPlan &h = p->hp;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return fail(VLOC_E_DEVICE, "no HIP device available");
    if ((e = hipGetDevice(&p->device)) != hipSuccess) return hip_fail(e, "hipGetDevice");

    const int64_t nst = h.nst();
    std::vector<int4> slot(nst);
    for (int64_t s = 0; s < nst; ++s) {
        const Stick &st = h.sticks[h.stick_of_slot[s]];
        int lm = st.lmin % h.grid[2];
        if (lm < 0) lm += h.grid[2];
        int kp = st.k % h.grid[1];
        if (kp < 0) kp += h.grid[1];
        slot[s] = make_int4(st.offset, st.count, lm, (st.h - h.hmin) * h.ldy + kp);
    }
    std::vector<int2> groups(h.ngroups);
    for (int g = 0; g < h.ngroups; ++g) groups[g] = make_int2(h.group_start[g], h.group_size[g]);

    std::vector<int2> cols(h.nxo);
    for (int c = 0; c < h.nxo; ++c) cols[c] = make_int2(h.col_kmin[c], h.col_kcnt[c]);
    if ((e = hipMalloc(&p->d_slot, sizeof(int4) * nst)) != hipSuccess) goto nomem;
    if ((e = hipMalloc(&p->d_cols, sizeof(int2) * h.nxo)) != hipSuccess) goto nomem;
    if ((e = hipMemcpy(p->d_cols, cols.data(), sizeof(int2) * h.nxo, hipMemcpyHostToDevice)) !=
        hipSuccess)
        goto devfail;
    if ((e = hipMalloc(&p->d_groups, sizeof(int2) * h.ngroups)) != hipSuccess) goto nomem;
    if ((e = hipMemcpy(p->d_slot, slot.data(), sizeof(int4) * nst, hipMemcpyHostToDevice)) !=
        hipSuccess)
        goto devfail;
    if ((e = hipMemcpy(p->d_groups, groups.data(), sizeof(int2) * h.ngroups,
                       hipMemcpyHostToDevice)) != hipSuccess)
        goto devfail;
    {
        const Split *sp[3] = {&h.sx, &h.sy, &h.sz};
        for (int a = 0; a < 3; ++a) {
            std::vector<double> t64 = twiddle_table(sp[a]->L);
            size_t bytes;
            const void *src;
            std::vector<float> t32;
            if (h.opt.precision == VLOC_F32) {
                t32.assign(t64.begin(), t64.end());
                bytes = t32.size() * sizeof(float);
                src = t32.data();
            } else {
                bytes = t64.size() * sizeof(double);
                src = t64.data();
            }
            if ((e = hipMalloc(&p->d_tw[a], bytes)) != hipSuccess) goto nomem;
            if ((e = hipMemcpy(p->d_tw[a], src, bytes, hipMemcpyHostToDevice)) != hipSuccess)
                goto devfail;
        }
    }
    {
        std::vector<double> t64 = twiddle_table(h.sx.L);
        if ((e = hipMalloc(&p->d_twx64, t64.size() * sizeof(double))) != hipSuccess) goto nomem;
        if ((e = hipMemcpy(p->d_twx64, t64.data(), t64.size() * sizeof(double),
                           hipMemcpyHostToDevice)) != hipSuccess)
            goto devfail;
    }
    {
        Geometry &g = p->geo;
        g.N1 = h.grid[0];
        g.N2 = h.grid[1];
        g.N3 = h.grid[2];
        g.L1x = h.sx.L1;
        g.L2x = h.sx.L2;
        g.L1y = h.sy.L1;
        g.L2y = h.sy.L2;
        g.L1z = h.sz.L1;
        g.L2z = h.sz.L2;
        g.nxo = h.nxo;
        g.hmin_mod = ((h.hmin % g.N1) + g.N1) % g.N1;
        g.ldy = h.ldy;
        g.ldx = h.ldx;
        g.ldz = h.ldz;
        g.rows = h.plane_rows;
        g.rb = h.plane_rb;
        g.rl = h.plane_rl;
        g.xw = h.plane_xw;
        g.xq = h.plane_xq;
        g.zx = h.zx;
        g.zy = h.zy;
        g.zz = h.zz;
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) !=
                hipSuccess ||
            cus < 1)
            cus = 256;
        const int per_cu = std::max(1, std::min(2, (160 * 1024) / std::max(1, h.plane_lds)));
        g.resident_plane_wgs = cus * per_cu;
        g.nsub = 1;
        g.nst = (int)nst;
        g.npw = (int)h.npw();
        g.ngroups = h.ngroups;
        int cap = 0;
        for (int s : h.group_size) cap = s > cap ? s : cap;
        g.group_cap = cap;
        g.inv_n = 1.0 / ((double)g.N1 * g.N2 * g.N3);
    }
    p->uploaded = true;
    return VLOC_OK;
nomem:
    free_device(p);
    (void)hipGetLastError();
    return fail(VLOC_E_NOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
devfail:
    free_device(p);
    return hip_fail(e, "table upload");
}

vloc_status ensure_scratch(vloc_plan p, int64_t chunk)
{
    size_t need = (size_t)chunk * p->hp.grid[2] * (size_t)p->hp.nst() * p->hp.elem_bytes();
    if (need <= p->S_bytes) return VLOC_OK;
    const char *f = std::getenv("VLOC_TEST_FAIL_ALLOC");
    if (f && f[0] == '1') return fail(VLOC_E_NOMEM, "stick buffer allocation refused (test hook)");
    if (p->d_S) {
        hipError_t e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        (void)hipFree(p->d_S);
        p->d_S = nullptr;
        p->S_bytes = 0;
    }
    hipError_t e = hipMalloc(&p->d_S, need);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        p->d_S = nullptr;
        return fail(VLOC_E_NOMEM, "stick buffer allocation failed: " +
                                      std::string(hipGetErrorString(e)));
    }
    p->S_bytes = need;
    return VLOC_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return na && nb && x < y + nb && y < x + na;
}

DevTables tables(vloc_plan p)
{
    DevTables t;
    t.slot_info = p->d_slot;
    t.groups = p->d_groups;
    t.cols = p->d_cols;
    t.twx = p->d_tw[0];
    t.twy = p->d_tw[1];
    t.twz = p->d_tw[2];
    t.twx64 = p->d_twx64;
    t.partial = p->d_partial;
    t.wts = nullptr;
    return t;
}

// Next four events for one chunk (created on demand, reused after a read).
hipError_t next_events(vloc_plan p, hipEvent_t *ev)
{
    while (p->events.size() < p->events_used + 4) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        p->events.push_back(e);
    }
    for (int i = 0; i < 4; ++i) ev[i] = p->events[p->events_used + i];
    p->events_used += 4;
    return hipSuccess;
}

template <typename T>
vloc_status run_chunks(vloc_plan p, int mode, const void *in, int64_t nbands, const void *V,
                       void *out, const double *wts = nullptr)
{
    const HostPlan &h = p->hp;
    const int64_t chunk = nbands < h.band_chunk ? nbands : h.band_chunk;
    vloc_status s = ensure_scratch(p, chunk);
    if (s != VLOC_OK) return s;
    const Geometry &g = p->geo;
    DevTables t = tables(p);
    t.wts = wts;
    hipError_t e;
    for (int64_t b0 = 0; b0 < nbands; b0 += chunk) {
        int nb = (int)((nbands - b0) < chunk ? (nbands - b0) : chunk);
        hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
        if (p->timing) {
            if ((e = next_events(p, ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");
            p->rec_modes.push_back(mode);
            (void)hipEventRecord(ev[0], p->stream);
        }
        if (mode != MODE_R2G) {
            e = launch_stick_fwd<T>(g, t, in, b0, nb, p->d_S, h.stick_threads, p->stream);
            if (e != hipSuccess) return hip_fail(e, "stick forward launch");
        }
        if (p->timing) (void)hipEventRecord(ev[1], p->stream);
        void *psi = mode == MODE_G2R ? out : (mode == MODE_R2G ? const_cast<void *>(in) : nullptr);
        e = launch_plane<T>(g, t, mode, p->d_S, V, psi, b0, nb, h.plane_threads, h.plane_lds,
                            p->stream);
        if (e != hipSuccess) return hip_fail(e, "plane launch");
        if (p->timing) (void)hipEventRecord(ev[2], p->stream);
        if (mode != MODE_G2R && mode != MODE_DENSITY) {
            e = launch_stick_bwd<T>(g, t, p->d_S, out, b0, nb, h.stick_threads, p->stream);
            if (e != hipSuccess) return hip_fail(e, "stick backward launch");
        }
        if (p->timing) (void)hipEventRecord(ev[3], p->stream);
    }
    return VLOC_OK;
}

vloc_status dispatch(vloc_plan p, int mode, const void *in, int64_t nbands, const void *V,
                     void *out)
{
    vloc_status s = upload(p);
    if (s != VLOC_OK) return s;
    if (p->hp.opt.precision == VLOC_F32) return run_chunks<float>(p, mode, in, nbands, V, out);
    return run_chunks<double>(p, mode, in, nbands, V, out);
}

} // namespace

extern "C" {

vloc_status vloc_plan_create_ex(vloc_plan *plan, const int32_t grid[3], const double cell[9],
                                double ecut, const double k[3], const vloc_options *opt)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan pointer is NULL");
    *plan = nullptr;
    vloc_plan p = new (std::nothrow) vloc_plan_s();
    if (!p) return fail(VLOC_E_NOMEM, "host allocation failed");
    std::string err;
    vloc_status s;
    try {
        s = build_host_plan(p->hp, grid, cell, ecut, k, opt, err);
    } catch (const std::bad_alloc &) {
        s = VLOC_E_NOMEM;
        err = "host allocation failed";
    }
    if (s != VLOC_OK) {
        delete p;
        return fail(s, err);
    }
    *plan = p;
    g_err.clear();
    return VLOC_OK;
}

vloc_status vloc_plan_create(vloc_plan *plan, const int32_t grid[3], const double cell[9],
                             double ecut, const double k[3])
{
    return vloc_plan_create_ex(plan, grid, cell, ecut, k, nullptr);
}

vloc_status vloc_plan_destroy(vloc_plan plan)
{
    if (!plan) return VLOC_OK;
    if (plan->uploaded || plan->d_S || !plan->events.empty()) {
        (void)hipStreamSynchronize(plan->stream);
        free_device(plan);
        for (hipEvent_t e : plan->events) (void)hipEventDestroy(e);
    }
    delete plan;
    return VLOC_OK;
}

vloc_status vloc_set_stream(vloc_plan plan, void *hip_stream)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    plan->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return VLOC_OK;
}

vloc_status vloc_apply(vloc_plan plan, const void *c, int64_t nbands, const void *V, void *out)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (nbands == 0) return VLOC_OK;
    if (!c || !V || !out) return fail(VLOC_E_INVALID, "NULL c, V or out");
    const HostPlan &h = plan->hp;
    size_t es = (size_t)h.elem_bytes();
    size_t cbytes = (size_t)nbands * (size_t)h.npw() * es;
    size_t vbytes = (size_t)h.grid[0] * h.grid[1] * h.grid[2] * (es / 2);
    if (overlaps(out, cbytes, c, cbytes) || overlaps(out, cbytes, V, vbytes))
        return fail(VLOC_E_ALIAS, "out overlaps c or V");
    if (((uintptr_t)c | (uintptr_t)out) % es || (uintptr_t)V % (es / 2))
        return fail(VLOC_E_INVALID, "misaligned c, V or out");
    return dispatch(plan, MODE_APPLY, c, nbands, V, out);
}

vloc_status vloc_g2r(vloc_plan plan, const void *c, int64_t nbands, void *psi_r)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (nbands == 0) return VLOC_OK;
    if (!c || !psi_r) return fail(VLOC_E_INVALID, "NULL c or psi_r");
    const HostPlan &h = plan->hp;
    size_t es = (size_t)h.elem_bytes();
    size_t cbytes = (size_t)nbands * (size_t)h.npw() * es;
    size_t pbytes = (size_t)nbands * h.grid[0] * h.grid[1] * h.grid[2] * es;
    if (overlaps(psi_r, pbytes, c, cbytes)) return fail(VLOC_E_ALIAS, "psi_r overlaps c");
    return dispatch(plan, MODE_G2R, c, nbands, nullptr, psi_r);
}

vloc_status vloc_r2g(vloc_plan plan, const void *psi_r, int64_t nbands, void *c_out)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (nbands == 0) return VLOC_OK;
    if (!c_out || !psi_r) return fail(VLOC_E_INVALID, "NULL psi_r or c_out");
    const HostPlan &h = plan->hp;
    size_t es = (size_t)h.elem_bytes();
    size_t cbytes = (size_t)nbands * (size_t)h.npw() * es;
    size_t pbytes = (size_t)nbands * h.grid[0] * h.grid[1] * h.grid[2] * es;
    if (overlaps(psi_r, pbytes, c_out, cbytes)) return fail(VLOC_E_ALIAS, "c_out overlaps psi_r");
    return dispatch(plan, MODE_R2G, psi_r, nbands, nullptr, c_out);
}

vloc_status vloc_plan_enable_timing(vloc_plan plan, int32_t enable)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    plan->timing = enable != 0;
    return VLOC_OK;
}

vloc_status vloc_plan_read_timing(vloc_plan plan, double ms[3], int64_t launches[3])
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    double acc[3] = {0, 0, 0};
    int64_t cnt[3] = {0, 0, 0};
    for (size_t i = 0; 4 * i + 3 < plan->events_used; ++i) {
        hipEvent_t *ev = &plan->events[4 * i];
        hipError_t e = hipEventSynchronize(ev[3]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        int mode = plan->rec_modes[i];
        for (int k = 0; k < 3; ++k) {
            if ((k == 0 && mode == MODE_R2G) || (k == 2 && (mode == MODE_G2R || mode == MODE_DENSITY)))
                continue;
            float t = 0.f;
            e = hipEventElapsedTime(&t, ev[k], ev[k + 1]);
            if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
            acc[k] += t;
            cnt[k] += 1;
        }
    }
    plan->events_used = 0;
    plan->rec_modes.clear();
    if (ms) std::memcpy(ms, acc, sizeof acc);
    if (launches) std::memcpy(launches, cnt, sizeof cnt);
    return VLOC_OK;
}

vloc_status vloc_band_dot(vloc_plan plan, const void *a, const void *b, int64_t nbands, double *e)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (nbands == 0) return VLOC_OK;
    if (!a || !b || !e) return fail(VLOC_E_INVALID, "NULL a, b or e");
    vloc_status s = upload(plan);
    if (s != VLOC_OK) return s;
    hipError_t err = plan->hp.opt.precision == VLOC_F32
                         ? launch_band_dot<float>(a, b, plan->hp.npw(), nbands, e, plan->stream)
                         : launch_band_dot<double>(a, b, plan->hp.npw(), nbands, e, plan->stream);
    return err == hipSuccess ? VLOC_OK : hip_fail(err, "band dot launch");
}

vloc_status vloc_weighted_sum(vloc_plan plan, const double *x, const double *w, int64_t nbands,
                              double *E)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (!x || !w || !E) return fail(VLOC_E_INVALID, "NULL x, w or E");
    vloc_status s = upload(plan);
    if (s != VLOC_OK) return s;
    hipError_t err = launch_weighted_sum(x, w, nbands, E, plan->stream);
    return err == hipSuccess ? VLOC_OK : hip_fail(err, "weighted sum launch");
}

vloc_status vloc_scale_bands(vloc_plan plan, const void *x, int64_t nbands, const double *w,
                             const double *scale, double factor, void *y)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (nbands == 0) return VLOC_OK;
    if (!x || !y) return fail(VLOC_E_INVALID, "NULL x or y");
    vloc_status s = upload(plan);
    if (s != VLOC_OK) return s;
    const int64_t npw = plan->hp.npw();
    hipError_t err =
        plan->hp.opt.precision == VLOC_F32
            ? launch_scale_bands<float>(x, npw, nbands, w, scale, factor, y, plan->stream)
            : launch_scale_bands<double>(x, npw, nbands, w, scale, factor, y, plan->stream);
    return err == hipSuccess ? VLOC_OK : hip_fail(err, "band scaling launch");
}

vloc_status vloc_density(vloc_plan plan, const void *c, int64_t nbands, const double *w,
                         const double *scale, double *rho)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (nbands == 0) return VLOC_OK;
    if (!c || !w || !rho) return fail(VLOC_E_INVALID, "NULL c, w or rho");
    if (plan->hp.plane_xq) return fail(VLOC_E_INVALID, "density needs the row-buffer x pass");
    vloc_status s = upload(plan);
    if (s != VLOC_OK) return s;
    HostPlan &h = plan->hp;
    Geometry &g = plan->geo;
    const int64_t N = (int64_t)h.grid[0] * h.grid[1] * h.grid[2];
    const int64_t chunk = nbands < h.band_chunk ? nbands : h.band_chunk;
    // band subsets per launch: items N3 * nsub fill the resident workgroups in
    // whole rounds where possible (fewest idle slots, then fewest subsets)
    {
        const int R = std::max(1, g.resident_plane_wgs);
        const int lo = std::max(1, (R + h.grid[2] - 1) / h.grid[2]);
        int best = lo;
        double best_w = 2.0;
        for (int ns = lo; ns <= 4 * lo && ns <= chunk; ++ns) {
            const int64_t items = (int64_t)h.grid[2] * ns;
            const double rounds = (double)((items + R - 1) / R);
            const double waste = rounds * R / (double)items;
            if (waste < best_w - 1e-9) {
                best_w = waste;
                best = ns;
            }
        }
        g.nsub = (int)std::min<int64_t>(best, chunk);
    }
    const size_t need = (size_t)g.nsub * (size_t)N * sizeof(double);
    if (need > plan->partial_bytes) {
        if (plan->d_partial) {
            hipError_t e = hipStreamSynchronize(plan->stream);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            (void)hipFree(plan->d_partial);
            plan->d_partial = nullptr;
            plan->partial_bytes = 0;
        }
        hipError_t e = hipMalloc(&plan->d_partial, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            plan->d_partial = nullptr;
            return fail(VLOC_E_NOMEM, "density buffer allocation failed");
        }
        plan->partial_bytes = need;
    }
    hipError_t e = launch_fill_f64(plan->d_partial, (int64_t)g.nsub * N, 0.0, plan->stream);
    if (e != hipSuccess) return hip_fail(e, "fill launch");
    s = h.opt.precision == VLOC_F32 ? run_chunks<float>(plan, MODE_DENSITY, c, nbands, nullptr,
                                                        nullptr, w)
                                    : run_chunks<double>(plan, MODE_DENSITY, c, nbands, nullptr,
                                                         nullptr, w);
    if (s != VLOC_OK) return s;
    e = launch_density_reduce(plan->d_partial, g.nsub, N, g.inv_n, scale, rho, plan->stream);
    return e == hipSuccess ? VLOC_OK : hip_fail(e, "density reduce launch");
}

vloc_status vloc_plan_npw(vloc_plan plan, int64_t *npw)
{
    if (!plan || !npw) return fail(VLOC_E_INVALID, "NULL argument");
    *npw = plan->hp.npw();
    return VLOC_OK;
}

vloc_status vloc_plan_gvectors(vloc_plan plan, int32_t *hkl)
{
    if (!plan || !hkl) return fail(VLOC_E_INVALID, "NULL argument");
    std::memcpy(hkl, plan->hp.hkl.data(), plan->hp.hkl.size() * sizeof(int32_t));
    return VLOC_OK;
}

vloc_status vloc_plan_sticks(vloc_plan plan, int64_t *nsticks, int32_t *table)
{
    if (!plan || !nsticks) return fail(VLOC_E_INVALID, "NULL argument");
    *nsticks = plan->hp.nst();
    if (table) {
        for (size_t i = 0; i < plan->hp.sticks.size(); ++i) {
            const Stick &s = plan->hp.sticks[i];
            table[5 * i] = s.h;
            table[5 * i + 1] = s.k;
            table[5 * i + 2] = s.offset;
            table[5 * i + 3] = s.count;
            table[5 * i + 4] = s.lmin;
        }
    }
    return VLOC_OK;
}

vloc_status vloc_plan_balance(vloc_plan plan, int64_t *ngroups, int64_t *pw_per_group)
{
    if (!plan || !ngroups) return fail(VLOC_E_INVALID, "NULL argument");
    const HostPlan &h = plan->hp;
    *ngroups = h.ngroups;
    if (pw_per_group) {
        for (int g = 0; g < h.ngroups; ++g) pw_per_group[g] = 0;
        for (size_t i = 0; i < h.sticks.size(); ++i)
            pw_per_group[h.group_of_stick[i]] += h.sticks[i].count;
    }
    return VLOC_OK;
}

vloc_status vloc_plan_stick_groups(vloc_plan plan, int32_t *group_of_stick)
{
    if (!plan || !group_of_stick) return fail(VLOC_E_INVALID, "NULL argument");
    std::memcpy(group_of_stick, plan->hp.group_of_stick.data(),
                plan->hp.group_of_stick.size() * sizeof(int32_t));
    return VLOC_OK;
}

vloc_status vloc_plan_layout(vloc_plan plan, int32_t out[14])
{
    if (!plan || !out) return fail(VLOC_E_INVALID, "NULL argument");
    const HostPlan &h = plan->hp;
    int32_t v[14] = {h.sx.L1,      h.sx.L2,         h.sy.L1,      h.sy.L2, h.sz.L1,
                     h.sz.L2,      h.group_cap,     h.band_chunk, h.plane_rows,
                     h.plane_threads, h.plane_lds, h.nxo,        h.plane_xw,
                     h.plane_xq ? 2 : 1};
    std::memcpy(out, v, sizeof v);
    return VLOC_OK;
}

const char *vloc_status_string(vloc_status s)
{
    switch (s) {
    case VLOC_OK: return "ok";
    case VLOC_E_INVALID: return "invalid argument";
    case VLOC_E_GRID: return "unsupported grid";
    case VLOC_E_CELL: return "invalid cell";
    case VLOC_E_SPHERE: return "invalid or aliasing cutoff sphere";
    case VLOC_E_ALIAS: return "output overlaps an input";
    case VLOC_E_NOMEM: return "out of memory";
    case VLOC_E_DEVICE: return "HIP device error";
    }
    return "unknown status";
}

const char *vloc_last_error(void) { return g_err.c_str(); }

} // extern "C"
