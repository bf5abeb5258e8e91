// api.cpp -- the C ABI of libvloc (declared in include/vloc.h).
//
// A plan is built on the host (plan.cpp); its device tables are uploaded on
// first use.  vloc_apply runs, per band chunk, K1 (stick z-transforms), K2
// (plane kernel with the potential) and K3 (stick z-transforms back, 1/N,
// gather) on the plan's stream, with the stick buffer S of one chunk reused
// in place by K2.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"

using namespace vloc;

// Device side shared by a plan and a batch: the tables of one or more member
// plans (concatenated, one segment per member), the stick buffer, the
// density partial planes and the timing events.
struct Engine {
    std::vector<const HostPlan *> members;
    hipStream_t stream = nullptr;
    bool uploaded = false;
    int device = -1;
    int4 *d_slot = nullptr;
    int2 *d_groups = nullptr;
    int2 *d_cols = nullptr;
    int4 *d_gam = nullptr;
    int *d_yslot = nullptr;
    int *d_holes = nullptr;
    void *d_tw[3] = {nullptr, nullptr, nullptr};
    double2 *d_twx64 = nullptr;
    std::vector<int> slot_off, group_off, col_off, hole_off, nholes;
    void *d_S = nullptr;
    size_t S_bytes = 0;
    double *d_partial = nullptr; // density partial planes
    size_t partial_bytes = 0;
    void *d_VT = nullptr;        // potential in the full-plane kernel's order
    void *d_parts = nullptr;     // parted plane: nxo x N2 values per resident workgroup
    Geometry geo{};
    // kernel timing: events[4*i .. 4*i+3] bracket K1, K2, K3 of launch i
    bool timing = false;
    std::vector<hipEvent_t> events;
    size_t events_used = 0;
    std::vector<int> rec_modes;
    // orders work across a change of stream (the stick buffer is reused)
    hipEvent_t order_ev = nullptr;
    // LDS bytes of the plane launches when the members' own sizes differ (a
    // batch on its members' own occupied ranges); 0 = the first member's
    int32_t plane_lds = 0;
};

static int32_t plane_lds(const Engine &E)
{
    return E.plane_lds ? E.plane_lds : E.members[0]->plane_lds;
}

struct vloc_plan_s {
    HostPlan hp;
    Engine eng;
    bool borrowed = false; // member of a batch: freed with the batch
};

struct vloc_batch_s {
    std::vector<vloc_plan_s *> plans; // members, owned
    Engine eng;
    int32_t lds = 0;                  // LDS bytes of the batch's plane launches
    int64_t band_chunk = 0;           // bands per launch over all k-points; 0 = all
    // HIP graph of the last call's launches, replayed while the call's
    // pointers and band counts stay the same
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uintptr_t> graph_key;
    int64_t graphs_captured = 0, graph_launches = 0;
};

// Scratch of vloc_apply_noalloc: the potential in the plane kernel's order,
// then the stick buffer of one band chunk.  Each GPU the library runs on holds
// its own copy until the process ends, and every call on that GPU shares it.
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

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

template <typename P>
void free_ptr(P *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_device(Engine &E)
{
    free_ptr(E.d_slot);
    free_ptr(E.d_groups);
    free_ptr(E.d_cols);
    free_ptr(E.d_gam);
    free_ptr(E.d_yslot);
    free_ptr(E.d_holes);
    free_ptr(E.d_twx64);
    for (void *&t : E.d_tw) free_ptr(t);
    free_ptr(E.d_S);
    free_ptr(E.d_partial);
    free_ptr(E.d_VT);
    free_ptr(E.d_parts);
    E.partial_bytes = 0;
    E.S_bytes = 0;
    E.uploaded = false;
}

// Waits for the engine's stream and frees everything it holds.
void release(Engine &E)
{
    if (E.uploaded || E.d_S || !E.events.empty()) {
        (void)hipStreamSynchronize(E.stream);
        free_device(E);
        for (hipEvent_t e : E.events) (void)hipEventDestroy(e);
        E.events.clear();
    }
    if (E.order_ev) {
        (void)hipEventDestroy(E.order_ev);
        E.order_ev = nullptr;
    }
}

// Makes `s` the engine's stream.  Work already enqueued on the old stream
// uses the engine's stick buffer and arranged potential, which the next call
// reuses: the new stream first waits for everything queued on the old one.
vloc_status switch_stream(Engine &E, hipStream_t s)
{
    if (s == E.stream) return VLOC_OK;
    if (E.uploaded || E.d_S) {
        hipError_t e = hipSuccess;
        if (!E.order_ev) e = hipEventCreateWithFlags(&E.order_ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(E.order_ev, E.stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, E.order_ev, 0);
        if (e != hipSuccess) return hip_fail(e, "ordering the stream change");
    }
    E.stream = s;
    return VLOC_OK;
}

template <typename V>
hipError_t upload_vec(V *&dst, const std::vector<V> &src)
{
    hipError_t e = hipMalloc(&dst, sizeof(V) * std::max<size_t>(1, src.size()));
    if (e != hipSuccess) return e;
    if (src.empty()) return hipSuccess;
    return hipMemcpy(dst, src.data(), sizeof(V) * src.size(), hipMemcpyHostToDevice);
}

vloc_status upload(Engine &E)
{
    if (E.uploaded) return VLOC_OK;
    const HostPlan &h = *E.members[0];
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return fail(VLOC_E_DEVICE, "no HIP device available");
    if ((e = hipGetDevice(&E.device)) != hipSuccess) return hip_fail(e, "hipGetDevice");

    // member tables, concatenated: slots and groups relative to the member
    std::vector<int4> slot, gam;
    std::vector<int2> groups, cols;
    std::vector<int> yslot, holes;
    E.slot_off.clear();
    E.group_off.clear();
    E.col_off.clear();
    E.hole_off.clear();
    E.nholes.clear();
    int cap = 0;
    for (const HostPlan *m : E.members) {
        E.slot_off.push_back((int)slot.size());
        E.group_off.push_back((int)groups.size());
        E.col_off.push_back((int)cols.size());
        E.hole_off.push_back((int)holes.size());
        E.nholes.push_back((int)(m->holes.size() / 2));
        for (size_t i = 0; i + 1 < m->holes.size(); i += 2) {
            const int32_t hh = m->holes[i], kk = m->holes[i + 1];
            int kp = kk % m->grid[1];
            if (kp < 0) kp += m->grid[1];
            int col = hh - m->hmin;
            if (m->plane_full && m->plane_full != 4)
                col = ((hh % m->grid[0]) + m->grid[0]) % m->grid[0];
            holes.push_back(col * m->ldy + kp);
        }
        for (int64_t s = 0; s < m->nst(); ++s) {
            const Stick &st = m->sticks[m->stick_of_slot[s]];
            int lm = st.lmin % m->grid[2];
            if (lm < 0) lm += m->grid[2];
            int kp = st.k % m->grid[1];
            if (kp < 0) kp += m->grid[1];
            // plane position: occupied column h - hmin (row buffers, parted plane), or in
            // the whole plane column h mod N1
            int col = st.h - m->hmin;
            if (m->plane_full && m->plane_full != 4)
                col = ((st.h % m->grid[0]) + m->grid[0]) % m->grid[0];
            slot.push_back(make_int4(st.offset, st.count, lm, col * m->ldy + kp));
        }
        for (int g = 0; g < m->ngroups; ++g) {
            groups.push_back(make_int2(m->group_start[g], m->group_size[g]));
            cap = std::max(cap, m->group_size[g]);
        }
        if (m->gamma) {
            // per slot: source offset, kind, -lmin of (0, 0), mirror's index in the group
            std::vector<int32_t> slot_of(m->nst());
            for (int64_t s = 0; s < m->nst(); ++s) slot_of[m->stick_of_slot[s]] = (int32_t)s;
            for (int64_t s = 0; s < m->nst(); ++s) {
                const int32_t i = m->stick_of_slot[s];
                const Stick &st = m->sticks[i];
                const int32_t mi = m->mirror[i];
                const int32_t rel = slot_of[mi] - m->group_start[m->group_of_stick[i]];
                if (st.h == 0 && st.k == 0)
                    gam.push_back(make_int4(m->half_off[i], 2, -st.lmin, rel));
                else if (m->half_off[i] >= 0)
                    gam.push_back(make_int4(m->half_off[i], 0, 0, rel));
                else
                    gam.push_back(make_int4(m->half_off[mi] + st.count - 1, 1, 0, rel));
            }
        }
        for (int c = 0; c < m->nxo; ++c) cols.push_back(make_int2(m->col_kmin[c], m->col_kcnt[c]));
        if (h.plane_full) {
            // slot of each (occupied x-plane, row) position, -1 where no stick
            const size_t y0 = yslot.size();
            yslot.resize(y0 + (size_t)m->nxo * m->grid[1], -1);
            for (int64_t s = 0; s < m->nst(); ++s) {
                const Stick &st = m->sticks[m->stick_of_slot[s]];
                int kp = st.k % m->grid[1];
                if (kp < 0) kp += m->grid[1];
                yslot[y0 + (size_t)(st.h - m->hmin) * m->grid[1] + kp] = (int)s;
            }
        }
    }
    if ((e = upload_vec(E.d_slot, slot)) != hipSuccess) goto devfail;
    if ((e = upload_vec(E.d_groups, groups)) != hipSuccess) goto devfail;
    if ((e = upload_vec(E.d_cols, cols)) != hipSuccess) goto devfail;
    if (!gam.empty() && (e = upload_vec(E.d_gam, gam)) != hipSuccess) goto devfail;
    if (!yslot.empty() && (e = upload_vec(E.d_yslot, yslot)) != hipSuccess) goto devfail;
    if (!holes.empty() && (e = upload_vec(E.d_holes, holes)) != hipSuccess) goto devfail;
    if (h.plane_full) {
        const size_t vbytes = (size_t)h.grid[0] * h.grid[1] * h.grid[2] * (h.elem_bytes() / 2);
        if ((e = hipMalloc(&E.d_VT, vbytes)) != hipSuccess) goto devfail;
    }
    {
        const Split *sp[3] = {&h.sx, &h.sy, &h.sz};
        for (int a = 0; a < 3; ++a) {
            // stage twiddles W_L^{n2 k1} arranged [n2][k1]
            const std::vector<double> nat = twiddle_table(sp[a]->L);
            std::vector<double> t64(nat.size());
            for (int n2 = 0; n2 < sp[a]->L2; ++n2)
                for (int k1 = 0; k1 < sp[a]->L1; ++k1) {
                    const int j = n2 * k1, d = n2 * sp[a]->L1 + k1;
                    t64[2 * d] = nat[2 * j];
                    t64[2 * d + 1] = nat[2 * j + 1];
                }
            if (h.opt.precision == VLOC_F32) {
                std::vector<float> t32(t64.begin(), t64.end());
                float *d = nullptr;
                e = upload_vec(d, t32);
                E.d_tw[a] = d;
            } else {
                double *d = nullptr;
                e = upload_vec(d, t64);
                E.d_tw[a] = d;
            }
            if (e != hipSuccess) goto devfail;
        }
    }
    {
        std::vector<double> t64 = twiddle_table(h.sx.L);
        double *d = nullptr;
        e = upload_vec(d, t64);
        E.d_twx64 = reinterpret_cast<double2 *>(d);
        if (e != hipSuccess) goto devfail;
    }
    {
        Geometry &g = E.geo;
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
        g.nxo_magic = ((1ull << 40) + (unsigned)h.nxo - 1) / (unsigned)h.nxo;
        g.hmin_mod = ((h.hmin % g.N1) + g.N1) % g.N1;
        g.ldy = h.ldy;
        g.ldx = h.ldx;
        g.ldz = h.ldz;
        g.rb = h.plane_rb;
        g.rl = h.plane_rl;
        g.xw = h.plane_xw;
        g.xq = h.plane_xq;
        // masks that hold for every member (members on their own occupied
        // ranges differ in them)
        g.zx = h.zx;
        g.zy = h.zy;
        g.zz = h.zz;
        g.fx = h.fx;
        for (const HostPlan *m : E.members) {
            g.zx &= m->zx;
            g.zy &= m->zy;
            g.zz &= m->zz;
            g.fx &= m->fx;
        }
        g.full = h.plane_full;
        g.parts = h.plane_parts;
        g.parts_elems = std::max(h.nxo * h.ldy, h.grid[0] * (h.plane_parts
                                                                 ? h.grid[1] / h.plane_parts + 1
                                                                 : 0));
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, E.device) !=
                hipSuccess ||
            cus < 1)
            cus = 256;
        const int per_cu = std::max(1, std::min(2, (160 * 1024) / std::max(1, plane_lds(E))));
        g.resident_plane_wgs = cus * per_cu;
        if (h.plane_full == 4) {
            // one scratch region per workgroup of the persistent plane grid
            const size_t pb = (size_t)g.resident_plane_wgs * h.nxo * h.grid[1] * h.elem_bytes();
            if ((e = hipMalloc(&E.d_parts, pb)) != hipSuccess) goto devfail;
        }
        g.nsub = 1;
        g.group_cap = cap;
        g.gamma = h.gamma ? 1 : 0;
        g.inv_n = 1.0 / ((double)g.N1 * g.N2 * g.N3);
    }
    E.uploaded = true;
    return VLOC_OK;
devfail:
    free_device(E);
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory)
        return fail(VLOC_E_NOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    return hip_fail(e, "table upload");
}

vloc_status ensure_scratch(Engine &E, size_t need)
{
    if (need <= E.S_bytes) return VLOC_OK;
    const char *f = std::getenv("VLOC_TEST_FAIL_ALLOC");
    if (f && f[0] == '1') return fail(VLOC_E_NOMEM, "stick buffer allocation refused (test hook)");
    if (E.d_S) {
        hipError_t e = hipStreamSynchronize(E.stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        free_ptr(E.d_S);
        E.S_bytes = 0;
    }
    hipError_t e = hipMalloc(&E.d_S, need);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        E.d_S = nullptr;
        return fail(VLOC_E_NOMEM, "stick buffer allocation failed: " +
                                      std::string(hipGetErrorString(e)));
    }
    E.S_bytes = need;
    return VLOC_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return na && nb && x < y + nb && y < x + na;
}

DevTables tables(const Engine &E)
{
    DevTables t;
    t.slot_info = E.d_slot;
    t.groups = E.d_groups;
    t.cols = E.d_cols;
    t.twx = E.d_tw[0];
    t.twy = E.d_tw[1];
    t.twz = E.d_tw[2];
    t.twx64 = E.d_twx64;
    t.partial = E.d_partial;
    t.wts = nullptr;
    t.gam = E.d_gam;
    t.yslot = E.d_yslot;
    t.holes = E.d_holes;
    t.parts = E.d_parts;
    return t;
}

// Next four events for one launch (created on demand, reused after a read).
hipError_t next_events(Engine &E, hipEvent_t *ev)
{
    while (E.events.size() < E.events_used + 4) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        E.events.push_back(e);
    }
    for (int i = 0; i < 4; ++i) ev[i] = E.events[E.events_used + i];
    E.events_used += 4;
    return hipSuccess;
}

// Band range [b0, b0 + nb) of one member, as a segment.
struct Part {
    int member;
    int64_t b0;
    int nb;
};

// Segment of member `member` for its launch bands [b0, b0 + nb): caller data
// pointers of its first band, its stick-buffer offset and its table rows.  In
// the real mode a launch band is a pair of the caller's bands.
void fill_seg(const Engine &E, int member, const void *in, void *out, int64_t nbands, int64_t b0,
              int nb, long long s_off, int band_lo, int blk_lo, Seg &s)
{
    const HostPlan &m = *E.members[member];
    const size_t es = (size_t)m.elem_bytes();
    const int64_t per = m.gamma ? 2 : 1; // caller bands per launch band
    const int64_t first = per * b0;      // first caller band of the segment
    s.in = in ? static_cast<const char *>(in) + first * m.npw_io() * es : nullptr;
    s.out = out ? static_cast<char *>(out) + first * m.npw_io() * es : nullptr;
    s.nbr = (int)std::min<int64_t>(per * nb, nbands - first);
    s.s_off = s_off;
    s.nst = (int)m.nst();
    s.npw = (int)m.npw_io();
    s.ngroups = m.ngroups;
    s.slot_off = E.slot_off[member];
    s.group_off = E.group_off[member];
    s.col_off = E.col_off[member];
    s.hole_off = E.hole_off[member];
    s.nholes = E.nholes[member];
    s.nxo = m.nxo;
    s.hmin_mod = ((m.hmin % m.grid[0]) + m.grid[0]) % m.grid[0];
    s.nxo_magic = ((1ull << 40) + (unsigned)m.nxo - 1) / (unsigned)m.nxo;
    s.band_lo = band_lo;
    s.nb = nb;
    s.blk_lo = blk_lo;
}

// The launches of one call: the caller's bands of every member, concatenated
// in member order, cut into chunks of at most `chunk` bands; a chunk holds one
// segment per member it touches.  With own > 0, a member of at least `own`
// launch bands instead gets launches of its own (its bands cut into equal
// chunks of at most `chunk`), and only the smaller members share launches: a
// launch of one segment runs the plane kernel's direct y form, and a member
// that large fills the device by itself.  In the real mode a launch band is a
// pair of the caller's bands.  Returns the stick-buffer bytes of the largest
// chunk.
size_t make_launches(const Engine &E, const void *const *in, void *const *out,
                     const int64_t *nbands, int64_t chunk, std::vector<Launch> &ls,
                     int64_t own = 0, int64_t own_cap = 0)
{
    ls.clear();
    const int nm = (int)E.members.size();
    const int N3 = E.members[0]->grid[2];
    size_t need = 0;
    std::vector<Part> cur;
    int64_t cur_bands = 0;
    std::vector<Part> solo;
    auto emit = [&](std::vector<Part> &cur) {
        if (cur.empty()) return;
        Launch L{};
        L.nseg = (int)cur.size();
        long long s_off = 0;
        int band_lo = 0, blk_lo = 0;
        for (size_t i = 0; i < cur.size(); ++i) {
            const Part &p = cur[i];
            fill_seg(E, p.member, in ? in[p.member] : nullptr, out ? out[p.member] : nullptr,
                     nbands[p.member], p.b0, p.nb, s_off, band_lo, blk_lo, L.seg[i]);
            const HostPlan &m = *E.members[p.member];
            s_off += (long long)p.nb * N3 * m.nst();
            band_lo += p.nb;
            blk_lo += p.nb * m.ngroups;
        }
        L.nbt = band_lo;
        L.nblk = blk_lo;
        need = std::max(need, (size_t)s_off * (size_t)E.members[0]->elem_bytes());
        ls.push_back(L);
        cur.clear();
    };
    auto flush = [&]() {
        emit(cur);
        cur_bands = 0;
    };
    for (int m = 0; m < nm; ++m) {
        const int64_t units = E.members[m]->gamma ? (nbands[m] + 1) / 2 : nbands[m];
        if (own > 0 && units >= own) {
            const int64_t nch = (units + own_cap - 1) / own_cap;
            const int64_t each = (units + nch - 1) / nch;
            for (int64_t b = 0; b < units; b += each) {
                solo.push_back(Part{m, b, (int)std::min(each, units - b)});
                emit(solo);
            }
            continue;
        }
        int64_t b = 0;
        while (b < units) {
            int64_t take = std::min(units - b, chunk - cur_bands);
            cur.push_back(Part{m, b, (int)take});
            cur_bands += take;
            b += take;
            if (cur_bands == chunk) flush();
        }
    }
    flush();
    return need;
}

// Enqueues K1 -> K2 -> K3 of every launch on stream st.  mode APPLY takes
// V; G2R / R2G / DENSITY (one member) take psi / weights indexed from the
// launch's first band.
template <typename T>
vloc_status run_launches(Engine &E, int mode, const Launch *ls, size_t nl, const void *V,
                         void *psi, const double *wts, hipStream_t st, bool timed, void *S,
                         void *VT, bool arrange = true)
{
    const HostPlan &h = *E.members[0];
    const Geometry &g = E.geo;
    DevTables t = tables(E);
    t.wts = wts;
    hipError_t e;
    int64_t band0 = 0;
    if ((mode == MODE_APPLY || mode == MODE_APPLY_DENSITY) && g.full && nl > 0) {
        // the potential in the full-plane kernel's order, once per call (with
        // arrange false, VT already holds it)
        if (arrange && (e = launch_arrange_v<T>(g, V, VT, st)) != hipSuccess)
            return hip_fail(e, "potential arrangement launch");
        V = VT;
    }
    for (size_t li = 0; li < nl; ++li) {
        const Launch &L = ls[li];
        hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
        if (timed) {
            if ((e = next_events(E, ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");
            E.rec_modes.push_back(mode);
            (void)hipEventRecord(ev[0], st);
        }
        if (mode != MODE_R2G) {
            e = launch_stick_fwd<T>(g, t, L, S, h.stick_threads, st);
            if (e != hipSuccess) return hip_fail(e, "stick forward launch");
        }
        if (timed) (void)hipEventRecord(ev[1], st);
        e = launch_plane<T>(g, t, L, mode, S, V, psi, band0, h.plane_threads, plane_lds(E), st);
        if (e != hipSuccess) return hip_fail(e, "plane launch");
        if (timed) (void)hipEventRecord(ev[2], st);
        if (mode != MODE_G2R && mode != MODE_DENSITY) {
            e = launch_stick_bwd<T>(g, t, L, S, h.stick_threads, st);
            if (e != hipSuccess) return hip_fail(e, "stick backward launch");
        }
        if (timed) (void)hipEventRecord(ev[3], st);
        band0 += L.nbt;
    }
    return VLOC_OK;
}

// One plan: its bands in chunks of the plan's band_chunk.
vloc_status dispatch(vloc_plan p, int mode, const void *in, int64_t nbands, const void *V,
                     void *out, const double *wts = nullptr, int64_t max_chunk = 0)
{
    Engine &E = p->eng;
    vloc_status s = upload(E);
    if (s != VLOC_OK) return s;
    std::vector<Launch> ls;
    const void *ins[1] = {mode == MODE_R2G ? nullptr : in};
    void *outs[1] = {(mode == MODE_APPLY || mode == MODE_R2G || mode == MODE_APPLY_DENSITY)
                         ? out
                         : nullptr};
    // equal chunks of at most band_chunk launch bands (no short last chunk)
    const int64_t units = p->hp.gamma ? (nbands + 1) / 2 : nbands;
    const int64_t bc = max_chunk > 0 ? max_chunk : p->hp.band_chunk;
    const int64_t nch = (units + bc - 1) / bc;
    const int64_t chunk = nch > 0 ? (units + nch - 1) / nch : 1;
    size_t need = make_launches(E, ins, outs, &nbands, chunk, ls);
    if ((s = ensure_scratch(E, need)) != VLOC_OK) return s;
    void *psi = mode == MODE_G2R ? out : (mode == MODE_R2G ? const_cast<void *>(in) : nullptr);
    if (p->hp.opt.precision == VLOC_F32)
        return run_launches<float>(E, mode, ls.data(), ls.size(), V, psi, wts, E.stream, E.timing,
                                   E.d_S, E.d_VT);
    return run_launches<double>(E, mode, ls.data(), ls.size(), V, psi, wts, E.stream, E.timing,
                                E.d_S, E.d_VT);
}

vloc_status read_timing(Engine &E, double ms[3], int64_t launches[3])
{
    double acc[3] = {0, 0, 0};
    int64_t cnt[3] = {0, 0, 0};
    for (size_t i = 0; 4 * i + 3 < E.events_used; ++i) {
        hipEvent_t *ev = &E.events[4 * i];
        hipError_t e = hipEventSynchronize(ev[3]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        int mode = E.rec_modes[i];
        for (int k = 0; k < 3; ++k) {
            if ((k == 0 && mode == MODE_R2G) ||
                (k == 2 && (mode == MODE_G2R || mode == MODE_DENSITY)))
                continue;
            float t = 0.f;
            e = hipEventElapsedTime(&t, ev[k], ev[k + 1]);
            if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
            acc[k] += t;
            cnt[k] += 1;
        }
    }
    E.events_used = 0;
    E.rec_modes.clear();
    if (ms) std::memcpy(ms, acc, sizeof acc);
    if (launches) std::memcpy(launches, cnt, sizeof cnt);
    return VLOC_OK;
}

// Device address of `scratch` on each GPU, looked up once per device with that
// device current (in host code the array's name is only a stand-in for it).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

vloc_status scratch_address(int dev, void **ptr)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(VLOC_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return VLOC_OK;
}

void drop_graph(vloc_batch b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_key.clear();
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
    p->eng.members.assign(1, &p->hp);
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
    if (plan->borrowed) return fail(VLOC_E_INVALID, "plan belongs to a batch");
    release(plan->eng);
    delete plan;
    return VLOC_OK;
}

vloc_status vloc_set_stream(vloc_plan plan, void *hip_stream)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    return switch_stream(plan->eng, reinterpret_cast<hipStream_t>(hip_stream));
}

vloc_status vloc_apply(vloc_plan plan, const void *c, int64_t nbands, const void *V, void *out)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (nbands == 0) return VLOC_OK;
    if (!c || !V || !out) return fail(VLOC_E_INVALID, "NULL c, V or out");
    const HostPlan &h = plan->hp;
    size_t es = (size_t)h.elem_bytes();
    size_t cbytes = (size_t)nbands * (size_t)h.npw_io() * es;
    size_t vbytes = (size_t)h.grid[0] * h.grid[1] * h.grid[2] * (es / 2);
    if (overlaps(out, cbytes, c, cbytes) || overlaps(out, cbytes, V, vbytes))
        return fail(VLOC_E_ALIAS, "out overlaps c or V");
    if (((uintptr_t)c | (uintptr_t)out) % es || (uintptr_t)V % (es / 2))
        return fail(VLOC_E_INVALID, "misaligned c, V or out");
    return dispatch(plan, MODE_APPLY, c, nbands, V, out);
}

vloc_status vloc_apply_noalloc(vloc_plan plan, const void *c, int64_t nbands, const void *V,
                               void *out)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (nbands == 0) return VLOC_OK;
    if (!c || !V || !out) return fail(VLOC_E_INVALID, "NULL c, V or out");
    const HostPlan &h = plan->hp;
    Engine &E = plan->eng;
    const size_t es = (size_t)h.elem_bytes();
    const size_t cbytes = (size_t)nbands * (size_t)h.npw_io() * es;
    const size_t nvox = (size_t)h.grid[0] * h.grid[1] * h.grid[2];
    if (overlaps(out, cbytes, c, cbytes) || overlaps(out, cbytes, V, nvox * (es / 2)))
        return fail(VLOC_E_ALIAS, "out overlaps c or V");
    if (((uintptr_t)c | (uintptr_t)out) % es || (uintptr_t)V % (es / 2))
        return fail(VLOC_E_INVALID, "misaligned c, V or out");
    // the arranged potential, then the stick buffer of as many bands as fit
    const size_t vt = h.plane_full ? (nvox * (es / 2) + 255) / 256 * 256 : 0;
    const size_t per_band = (size_t)h.grid[2] * (size_t)h.nst() * es;
    if (vt + per_band > kScratchBytes) {
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "one band needs %zu bytes of scratch (potential %zu + stick buffer %zu); "
                      "the allocation-free path has %zu",
                      vt + per_band, vt, per_band, kScratchBytes);
        return fail(VLOC_E_INVALID, buf);
    }
    if (!E.uploaded)
        return fail(VLOC_E_INVALID, "the plan's tables are not on the device yet (they are "
                                    "uploaded by its first vloc_apply call)");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != E.device) return fail(VLOC_E_INVALID, "the current device is not the plan's");
    void *base = nullptr;
    vloc_status s = scratch_address(dev, &base);
    if (s != VLOC_OK) return s;
    void *VT = base;
    void *S = static_cast<char *>(base) + vt;
    // equal chunks of at most this many launch bands, as vloc_apply cuts them
    const int64_t cap = std::min<int64_t>(h.band_chunk, (int64_t)((kScratchBytes - vt) / per_band));
    const int64_t units = h.gamma ? (nbands + 1) / 2 : nbands;
    const int64_t nch = (units + cap - 1) / cap;
    const int64_t chunk = (units + nch - 1) / nch;
    const bool f32 = h.opt.precision == VLOC_F32;
    for (int64_t b0 = 0, i = 0; b0 < units; b0 += chunk, ++i) {
        Launch L{};
        const int nb = (int)std::min<int64_t>(chunk, units - b0);
        L.nseg = 1;
        fill_seg(E, 0, c, out, nbands, b0, nb, 0, 0, 0, L.seg[0]);
        L.nbt = nb;
        L.nblk = nb * h.ngroups;
        // the first chunk arranges the potential into VT (whole-plane layout);
        // the later ones read it from there
        s = f32 ? run_launches<float>(E, MODE_APPLY, &L, 1, V, nullptr, nullptr, E.stream, false,
                                      S, VT, i == 0)
                : run_launches<double>(E, MODE_APPLY, &L, 1, V, nullptr, nullptr, E.stream, false,
                                       S, VT, i == 0);
        if (s != VLOC_OK) return s;
    }
    return VLOC_OK;
}

vloc_status vloc_g2r(vloc_plan plan, const void *c, int64_t nbands, void *psi_r)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (nbands == 0) return VLOC_OK;
    if (!c || !psi_r) return fail(VLOC_E_INVALID, "NULL c or psi_r");
    if (plan->hp.gamma) return fail(VLOC_E_INVALID, "real-mode plans only apply");
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
    if (plan->hp.gamma) return fail(VLOC_E_INVALID, "real-mode plans only apply");
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
    plan->eng.timing = enable != 0;
    return VLOC_OK;
}

vloc_status vloc_plan_read_timing(vloc_plan plan, double ms[3], int64_t launches[3])
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    return read_timing(plan->eng, ms, launches);
}

vloc_status vloc_band_dot(vloc_plan plan, const void *a, const void *b, int64_t nbands, double *e)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (nbands == 0) return VLOC_OK;
    if (!a || !b || !e) return fail(VLOC_E_INVALID, "NULL a, b or e");
    if (plan->hp.gamma) return fail(VLOC_E_INVALID, "real-mode plans only apply");
    vloc_status s = upload(plan->eng);
    if (s != VLOC_OK) return s;
    hipStream_t st = plan->eng.stream;
    hipError_t err = plan->hp.opt.precision == VLOC_F32
                         ? launch_band_dot<float>(a, b, plan->hp.npw(), nbands, e, st)
                         : launch_band_dot<double>(a, b, plan->hp.npw(), nbands, e, st);
    return err == hipSuccess ? VLOC_OK : hip_fail(err, "band dot launch");
}

vloc_status vloc_weighted_sum(vloc_plan plan, const double *x, const double *w, int64_t nbands,
                              double *E)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (!x || !w || !E) return fail(VLOC_E_INVALID, "NULL x, w or E");
    vloc_status s = upload(plan->eng);
    if (s != VLOC_OK) return s;
    hipError_t err = launch_weighted_sum(x, w, nbands, E, plan->eng.stream);
    return err == hipSuccess ? VLOC_OK : hip_fail(err, "weighted sum launch");
}

vloc_status vloc_scale_bands(vloc_plan plan, const void *x, int64_t nbands, const double *w,
                             const double *scale, double factor, void *y)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (nbands == 0) return VLOC_OK;
    if (!x || !y) return fail(VLOC_E_INVALID, "NULL x or y");
    if (plan->hp.gamma) return fail(VLOC_E_INVALID, "real-mode plans only apply");
    vloc_status s = upload(plan->eng);
    if (s != VLOC_OK) return s;
    const int64_t npw = plan->hp.npw();
    hipStream_t st = plan->eng.stream;
    hipError_t err = plan->hp.opt.precision == VLOC_F32
                         ? launch_scale_bands<float>(x, npw, nbands, w, scale, factor, y, st)
                         : launch_scale_bands<double>(x, npw, nbands, w, scale, factor, y, st);
    return err == hipSuccess ? VLOC_OK : hip_fail(err, "band scaling launch");
}

} // extern "C"

namespace {

// Density passes: checks, band subsets per launch, zeroed FP64 partial planes;
// then the plane kernel in `mode` (DENSITY or APPLY_DENSITY) and the fixed-order
// reduction of the partial planes into rho.
vloc_status density_pass(vloc_plan plan, int mode, const void *c, int64_t nbands, const void *V,
                         void *out, const double *w, const double *scale, double *rho)
{
    if (plan->hp.gamma) return fail(VLOC_E_INVALID, "real-mode plans only apply");
    if (plan->hp.plane_xq) return fail(VLOC_E_INVALID, "density needs the row-buffer x pass");
    Engine &E = plan->eng;
    vloc_status s = upload(E);
    if (s != VLOC_OK) return s;
    HostPlan &h = plan->hp;
    Geometry &g = E.geo;
    const int64_t N = (int64_t)h.grid[0] * h.grid[1] * h.grid[2];
    const int64_t dchunk = h.density_chunk > 0 ? h.density_chunk : h.band_chunk;
    const int64_t chunk = nbands < dchunk ? nbands : dchunk;
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
    if (need > E.partial_bytes) {
        if (E.d_partial) {
            hipError_t e = hipStreamSynchronize(E.stream);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            free_ptr(E.d_partial);
            E.partial_bytes = 0;
        }
        hipError_t e = hipMalloc(&E.d_partial, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            E.d_partial = nullptr;
            return fail(VLOC_E_NOMEM, "density buffer allocation failed");
        }
        E.partial_bytes = need;
    }
    hipError_t e = launch_fill_f64(E.d_partial, (int64_t)g.nsub * N, 0.0, E.stream);
    if (e != hipSuccess) return hip_fail(e, "fill launch");
    s = dispatch(plan, mode, c, nbands, V, out, w, dchunk);
    if (s != VLOC_OK) return s;
    e = launch_density_reduce(g, E.d_partial, g.nsub, scale, rho, E.stream);
    return e == hipSuccess ? VLOC_OK : hip_fail(e, "density reduce launch");
}

} // namespace

extern "C" {

vloc_status vloc_density(vloc_plan plan, const void *c, int64_t nbands, const double *w,
                         const double *scale, double *rho)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (nbands == 0) return VLOC_OK;
    if (!c || !w || !rho) return fail(VLOC_E_INVALID, "NULL c, w or rho");
    return density_pass(plan, MODE_DENSITY, c, nbands, nullptr, nullptr, w, scale, rho);
}

vloc_status vloc_apply_density(vloc_plan plan, const void *c, int64_t nbands, const void *V,
                               void *out, const double *w, double *rho)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (nbands < 0) return fail(VLOC_E_INVALID, "nbands < 0");
    if (nbands == 0) return VLOC_OK;
    if (!c || !V || !out || !w || !rho) return fail(VLOC_E_INVALID, "NULL c, V, out, w or rho");
    const HostPlan &h = plan->hp;
    const size_t es = (size_t)h.elem_bytes();
    const size_t cbytes = (size_t)nbands * (size_t)h.npw_io() * es;
    const size_t nvox = (size_t)h.grid[0] * h.grid[1] * h.grid[2];
    if (overlaps(out, cbytes, c, cbytes) || overlaps(out, cbytes, V, nvox * (es / 2)) ||
        overlaps(rho, nvox * 8, out, cbytes) || overlaps(rho, nvox * 8, c, cbytes) ||
        overlaps(rho, nvox * 8, V, nvox * (es / 2)))
        return fail(VLOC_E_ALIAS, "out or rho overlaps an input, or each other");
    if (((uintptr_t)c | (uintptr_t)out) % es || (uintptr_t)V % (es / 2) || (uintptr_t)rho % 8)
        return fail(VLOC_E_INVALID, "misaligned c, V, out or rho");
    return density_pass(plan, MODE_APPLY_DENSITY, c, nbands, V, out, w, nullptr, rho);
}

vloc_status vloc_scale_real(vloc_plan plan, const double *x, int64_t n, const double *scale,
                            double factor, double *y)
{
    if (!plan) return fail(VLOC_E_INVALID, "plan is NULL");
    if (n < 0) return fail(VLOC_E_INVALID, "n < 0");
    if (n == 0) return VLOC_OK;
    if (!x || !y) return fail(VLOC_E_INVALID, "NULL x or y");
    vloc_status s = upload(plan->eng);
    if (s != VLOC_OK) return s;
    hipError_t e = launch_scale_real(x, n, scale, factor, y, plan->eng.stream);
    return e == hipSuccess ? VLOC_OK : hip_fail(e, "real scaling launch");
}

vloc_status vloc_plan_npw(vloc_plan plan, int64_t *npw)
{
    if (!plan || !npw) return fail(VLOC_E_INVALID, "NULL argument");
    *npw = plan->hp.npw_io();
    return VLOC_OK;
}

vloc_status vloc_plan_gvectors(vloc_plan plan, int32_t *hkl)
{
    if (!plan || !hkl) return fail(VLOC_E_INVALID, "NULL argument");
    const std::vector<int32_t> &v = plan->hp.gamma ? plan->hp.half_hkl : plan->hp.hkl;
    std::memcpy(hkl, v.data(), v.size() * sizeof(int32_t));
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
                     h.plane_full ? 2 + h.plane_full : (h.plane_xq ? 2 : 1)};
    std::memcpy(out, v, sizeof v);
    return VLOC_OK;
}

/* ------------------------------------------------------------- batches */

vloc_status vloc_batch_create(vloc_batch *batch, const int32_t grid[3], const double cell[9],
                              double ecut, int32_t nk, const double *kpts,
                              const vloc_options *opt)
{
    if (!batch) return fail(VLOC_E_INVALID, "batch pointer is NULL");
    *batch = nullptr;
    if (nk < 1 || nk > kMaxSeg) return fail(VLOC_E_INVALID, "nk must be in [1, 8]");
    if (!kpts) return fail(VLOC_E_INVALID, "kpts is NULL");
    if (opt && opt->gamma) return fail(VLOC_E_INVALID, "batches run the complex mode only");
    vloc_batch b = new (std::nothrow) vloc_batch_s();
    if (!b) return fail(VLOC_E_NOMEM, "host allocation failed");
    std::string err;
    vloc_status s = VLOC_OK;
    try {
        // pass 1: each k-point's own sphere and occupied ranges
        Occupied u{};
        for (int i = 0; i < nk && s == VLOC_OK; ++i) {
            vloc_plan p = new vloc_plan_s();
            p->borrowed = true;
            b->plans.push_back(p);
            s = build_host_plan(p->hp, grid, cell, ecut, kpts + 3 * i, opt, err);
            p->eng.members.assign(1, &p->hp);
            if (s != VLOC_OK) break;
            const HostPlan &h = p->hp;
            if (i == 0) u = Occupied{h.hmin, h.hmax, h.kmin, h.kmax, h.lmin, h.lmax};
            u.hmin = std::min(u.hmin, h.hmin);
            u.hmax = std::max(u.hmax, h.hmax);
            u.kmin = std::min(u.kmin, h.kmin);
            u.kmax = std::max(u.kmax, h.kmax);
            u.lmin = std::min(u.lmin, h.lmin);
            u.lmax = std::max(u.lmax, h.lmax);
        }
        // The whole-plane layouts (x pass spread over the workgroup or rows
        // owned by wavefronts) keep each member on its own occupied range:
        // launch segments carry their occupied x-planes, the engine takes the
        // zero and full masks that hold for every member and the largest LDS
        // size.  Every other layout sizes LDS or row buffers by the occupied
        // range, so the members are laid out again on the union of the ranges.
        bool own = s == VLOC_OK;
        for (size_t i = 0; own && i < b->plans.size(); ++i) {
            const HostPlan &h = b->plans[i]->hp, &h0 = b->plans[0]->hp;
            own = (h.plane_full == 1 || h.plane_full == 2) && h.plane_full == h0.plane_full &&
                  h.plane_threads == h0.plane_threads && h.sx.L1 == h0.sx.L1 &&
                  h.sy.L1 == h0.sy.L1 && h.sz.L1 == h0.sz.L1;
        }
        if (s == VLOC_OK && !own) {
            for (int i = 0; i < nk && s == VLOC_OK; ++i) {
                vloc_plan p = b->plans[i];
                p->hp = HostPlan();
                s = build_host_plan(p->hp, grid, cell, ecut, kpts + 3 * i, opt, err, &u);
                p->eng.members.assign(1, &p->hp);
            }
        }
        if (s == VLOC_OK) {
            const HostPlan &h0 = b->plans[0]->hp;
            int32_t lds = 0;
            for (vloc_plan p : b->plans) lds = std::max(lds, p->hp.plane_lds);
            for (vloc_plan p : b->plans) {
                const HostPlan &h = p->hp;
                if ((!own && (h.nxo != h0.nxo || h.hmin != h0.hmin || h.zx != h0.zx ||
                              h.zy != h0.zy || h.zz != h0.zz || h.plane_lds != h0.plane_lds)) ||
                    h.plane_full != h0.plane_full || h.plane_xw != h0.plane_xw ||
                    h.plane_rb != h0.plane_rb || h.plane_xq != h0.plane_xq ||
                    h.plane_threads != h0.plane_threads) {
                    s = VLOC_E_INVALID;
                    err = "internal: batch members disagree on the plane layout";
                }
            }
            // one LDS size for every launch (the member plans' own calls keep theirs)
            b->lds = lds;
            b->eng.plane_lds = lds;
            for (vloc_plan p : b->plans) b->eng.members.push_back(&p->hp);
            b->band_chunk = opt ? opt->band_chunk : 0;
        }
    } catch (const std::bad_alloc &) {
        s = VLOC_E_NOMEM;
        err = "host allocation failed";
    }
    if (s != VLOC_OK) {
        for (vloc_plan p : b->plans) delete p;
        delete b;
        return fail(s, err);
    }
    *batch = b;
    g_err.clear();
    return VLOC_OK;
}

vloc_status vloc_batch_destroy(vloc_batch batch)
{
    if (!batch) return VLOC_OK;
    (void)hipStreamSynchronize(batch->eng.stream);
    drop_graph(batch);
    if (batch->cap_stream) (void)hipStreamDestroy(batch->cap_stream);
    release(batch->eng);
    for (vloc_plan p : batch->plans) {
        release(p->eng);
        delete p;
    }
    delete batch;
    return VLOC_OK;
}

vloc_status vloc_batch_plan(vloc_batch batch, int32_t ik, vloc_plan *plan)
{
    if (!batch || !plan) return fail(VLOC_E_INVALID, "NULL argument");
    if (ik < 0 || ik >= (int32_t)batch->plans.size()) return fail(VLOC_E_INVALID, "ik out of range");
    *plan = batch->plans[ik];
    return VLOC_OK;
}

vloc_status vloc_batch_set_stream(vloc_batch batch, void *hip_stream)
{
    if (!batch) return fail(VLOC_E_INVALID, "batch is NULL");
    return switch_stream(batch->eng, reinterpret_cast<hipStream_t>(hip_stream));
}

vloc_status vloc_batch_use_graph(vloc_batch batch, int32_t enable)
{
    if (!batch) return fail(VLOC_E_INVALID, "batch is NULL");
    batch->use_graph = enable != 0;
    if (!batch->use_graph) {
        (void)hipStreamSynchronize(batch->eng.stream);
        drop_graph(batch);
    }
    return VLOC_OK;
}

vloc_status vloc_batch_apply(vloc_batch batch, const void *const *c, const int64_t *nbands,
                             const void *V, void *const *out)
{
    if (!batch) return fail(VLOC_E_INVALID, "batch is NULL");
    if (!c || !nbands || !out) return fail(VLOC_E_INVALID, "NULL c, nbands or out array");
    const int nk = (int)batch->plans.size();
    const HostPlan &h0 = batch->plans[0]->hp;
    const size_t es = (size_t)h0.elem_bytes();
    const size_t vbytes = (size_t)h0.grid[0] * h0.grid[1] * h0.grid[2] * (es / 2);
    int64_t total = 0;
    for (int i = 0; i < nk; ++i) {
        if (nbands[i] < 0) return fail(VLOC_E_INVALID, "nbands < 0");
        total += nbands[i];
    }
    if (total == 0) return VLOC_OK;
    if (!V) return fail(VLOC_E_INVALID, "V is NULL");
    if ((uintptr_t)V % (es / 2)) return fail(VLOC_E_INVALID, "misaligned V");
    for (int i = 0; i < nk; ++i) {
        if (!nbands[i]) continue;
        if (!c[i] || !out[i]) return fail(VLOC_E_INVALID, "NULL c or out of a k-point with bands");
        if (((uintptr_t)c[i] | (uintptr_t)out[i]) % es)
            return fail(VLOC_E_INVALID, "misaligned c or out");
        const size_t ob = (size_t)nbands[i] * (size_t)batch->plans[i]->hp.npw() * es;
        if (overlaps(out[i], ob, V, vbytes)) return fail(VLOC_E_ALIAS, "out overlaps V");
        for (int j = 0; j < nk; ++j) {
            if (!nbands[j]) continue;
            const size_t cb = (size_t)nbands[j] * (size_t)batch->plans[j]->hp.npw() * es;
            if (overlaps(out[i], ob, c[j], cb)) return fail(VLOC_E_ALIAS, "out overlaps a c");
            if (j != i && overlaps(out[i], ob, out[j], cb))
                return fail(VLOC_E_ALIAS, "two outputs overlap");
        }
    }
    Engine &E = batch->eng;
    vloc_status s = upload(E);
    if (s != VLOC_OK) return s;
    int maxg = 1;
    for (vloc_plan p : batch->plans) maxg = std::max(maxg, p->hp.ngroups);
    // equal chunks of at most band_chunk bands (automatic: the members' stick
    // buffers of one chunk within 256 MiB), each one launch per kernel
    int64_t cmax = batch->band_chunk;
    if (cmax <= 0) {
        int64_t per_band = 0;
        for (vloc_plan p : batch->plans)
            per_band = std::max<int64_t>(per_band, (int64_t)h0.grid[2] * p->hp.nst() * es);
        cmax = std::max<int64_t>(1, (256LL << 20) / per_band);
    }
    cmax = std::min<int64_t>(cmax, INT32_MAX / maxg);
    cmax = std::min<int64_t>(cmax, INT32_MAX / h0.grid[2]);
    // k-points of at least half a chunk, or with planes enough to fill the
    // resident plane workgroups eight times over, get launches of their own
    // (one segment each: the direct y form of the plane kernel); the others
    // share launches, cut into equal chunks
    const int64_t fill = (8LL * std::max(1, E.geo.resident_plane_wgs) + h0.grid[2] - 1) /
                         h0.grid[2];
    const int64_t own = std::max<int64_t>(1, std::min<int64_t>((cmax + 1) / 2, fill));
    int64_t shared = 0;
    for (int i = 0; i < nk; ++i)
        if (nbands[i] < own) shared += nbands[i];
    const int64_t nch = std::max<int64_t>(1, (shared + cmax - 1) / cmax);
    const int64_t chunk = std::max<int64_t>(1, (shared + nch - 1) / nch);
    std::vector<Launch> ls;
    size_t need = make_launches(E, c, out, nbands, chunk, ls, own, cmax);
    if ((s = ensure_scratch(E, need)) != VLOC_OK) return s;
    const bool f32 = h0.opt.precision == VLOC_F32;
    if (!batch->use_graph) {
        return f32 ? run_launches<float>(E, MODE_APPLY, ls.data(), ls.size(), V, nullptr, nullptr,
                                         E.stream, E.timing, E.d_S, E.d_VT)
                   : run_launches<double>(E, MODE_APPLY, ls.data(), ls.size(), V, nullptr,
                                          nullptr, E.stream, E.timing, E.d_S, E.d_VT);
    }
    // graph path: capture the launches once per set of pointers and counts
    std::vector<uintptr_t> key;
    key.push_back((uintptr_t)V);
    key.push_back((uintptr_t)E.d_S);
    for (int i = 0; i < nk; ++i) {
        key.push_back((uintptr_t)c[i]);
        key.push_back((uintptr_t)out[i]);
        key.push_back((uintptr_t)nbands[i]);
    }
    hipError_t e;
    if (!batch->exec || key != batch->graph_key) {
        if (batch->exec) {
            if ((e = hipStreamSynchronize(E.stream)) != hipSuccess)
                return hip_fail(e, "hipStreamSynchronize");
        }
        drop_graph(batch);
        if (!batch->cap_stream &&
            (e = hipStreamCreateWithFlags(&batch->cap_stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "hipStreamCreateWithFlags");
        if ((e = hipStreamBeginCapture(batch->cap_stream, hipStreamCaptureModeRelaxed)) !=
            hipSuccess)
            return hip_fail(e, "hipStreamBeginCapture");
        s = f32 ? run_launches<float>(E, MODE_APPLY, ls.data(), ls.size(), V, nullptr, nullptr,
                                      batch->cap_stream, false, E.d_S, E.d_VT)
                : run_launches<double>(E, MODE_APPLY, ls.data(), ls.size(), V, nullptr, nullptr,
                                       batch->cap_stream, false, E.d_S, E.d_VT);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(batch->cap_stream, &g);
        if (s != VLOC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        batch->graph = g;
        if ((e = hipGraphInstantiateWithFlags(&batch->exec, g, 0)) != hipSuccess) {
            batch->exec = nullptr;
            drop_graph(batch);
            return hip_fail(e, "hipGraphInstantiate");
        }
        batch->graph_key = key;
        batch->graphs_captured++;
    }
    if ((e = hipGraphLaunch(batch->exec, E.stream)) != hipSuccess)
        return hip_fail(e, "hipGraphLaunch");
    batch->graph_launches++;
    return VLOC_OK;
}

vloc_status vloc_batch_enable_timing(vloc_batch batch, int32_t enable)
{
    if (!batch) return fail(VLOC_E_INVALID, "batch is NULL");
    batch->eng.timing = enable != 0;
    return VLOC_OK;
}

vloc_status vloc_batch_read_timing(vloc_batch batch, double ms[3], int64_t launches[3])
{
    if (!batch) return fail(VLOC_E_INVALID, "batch is NULL");
    return read_timing(batch->eng, ms, launches);
}

vloc_status vloc_batch_info(vloc_batch batch, int64_t out[4])
{
    if (!batch || !out) return fail(VLOC_E_INVALID, "NULL argument");
    out[0] = (int64_t)batch->plans.size();
    out[1] = batch->band_chunk;
    out[2] = batch->graphs_captured;
    out[3] = batch->graph_launches;
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
