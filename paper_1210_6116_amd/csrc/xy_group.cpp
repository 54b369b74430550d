// xy_group.cpp -- continuous batching of PCC runs (the xy_group_* calls of
// include/xy.h).  Requests live in one device arena (first-fit sub-allocation,
// so admission never calls the allocator) and every running request is swept in
// the same kernel launches as the others; the per-replica descriptors and the
// tile -> replica table are rebuilt between rounds when the set changes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/xy.h"
#include "xy_device.hpp"
#include "xy_host.hpp"
#include "xy_launch.hpp"

using namespace xyhost;

namespace {

// First-fit allocator over [0, size) with coalescing of free neighbours.
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free;  // offset -> length
    void init(size_t n)
    {
        size = n;
        free.clear();
        free[0] = n;
    }
    bool take(size_t n, size_t *off)
    {
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t at = it->first + n;
                free.erase(it);
                if (rest) free[at] = rest;
                return true;
            }
        }
        return false;
    }
    void give(size_t off, size_t n)
    {
        auto it = free.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free.erase(nx);
        }
        if (it != free.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free.erase(it);
            }
        }
    }
};

struct Slot {
    bool used = false, running = false, needs_init = false, reported = false;
    xy_params p{};
    Plan plan;               // single-replica layout
    size_t off = 0, bytes = 0;
    int64_t target = 0, done = 0;
    xy::RepState *st = nullptr;
};

size_t slot_bytes(const Plan &P) { return align_up(P.lay[0].end) + align_up(sizeof(xy::RepState)); }

}  // namespace

struct xy_group {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *mem = nullptr;
    Arena arena;
    xy_pcc pcc{};
    std::vector<Slot> slots;
    bool dirty = true;
    bool poisoned = false;
    // device tables of the running replicas (rebuilt when the set changes)
    xy::RepDesc *d_reps = nullptr;
    uint32_t *d_tile_rep = nullptr;
    uint32_t *d_fin_rep = nullptr;  // replica of every finalisation chunk (at most one per tile)
    int64_t tile_cap = 0;
    std::vector<int32_t> order;  // running slot ids in descriptor order
    xy::Launch lc{};
    std::vector<int32_t> finished;
};

namespace {

int gfail(xy_group *g, hipError_t e, const char *what)
{
    if (g) g->poisoned = true;
    return fail(XY_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define GCHECK(g, expr)                                    \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return gfail(g, e_, #expr); \
    } while (0)

int check_group(xy_group *g)
{
    if (!g) return fail(XY_EINVAL, "group is NULL");
    if (g->poisoned) return fail(XY_ESTATE, "group was poisoned by an earlier device error");
    return XY_OK;
}

int plan_request(const xy_params *p, Plan &P)
{
    int rc = make_plan(p, 1, P);
    if (rc) return rc;
    if (P.label_bits != 32) return fail(XY_EINVAL, "serving requests need 32-bit labels (L <= 32768)");
    return XY_OK;
}

// Rebuilds the descriptor and tile tables of the running requests and
// initialises the spins of newly admitted ones.
int rebuild(xy_group *g)
{
    g->order.clear();
    std::vector<xy::RepDesc> descs;
    std::vector<uint32_t> tile_rep, fin_rep;
    int64_t base = 0, fbase = 0;
    int32_t max_th = 1, utw = -1, uth = -1;
    for (int32_t s = 0; s < (int32_t)g->slots.size(); ++s) {
        Slot &sl = g->slots[s];
        if (!sl.running) continue;
        const int32_t k = (int32_t)g->order.size();
        g->order.push_back(s);
        xy::RepDesc d;
        fill_desc(sl.plan, 0, sl.p, g->mem + sl.off, sl.st, base, fbase, k, d);
        descs.push_back(d);
        const Resolved &r = sl.plan.res[0];
        for (int64_t t = 0; t < r.ntiles; ++t) tile_rep.push_back((uint32_t)k);
        for (int64_t c = 0; c < r.fin_chunks; ++c) fin_rep.push_back((uint32_t)k);
        base += r.ntiles;
        fbase += r.fin_chunks;
        max_th = std::max(max_th, r.TH);
        utw = (utw < 0 || utw == r.TW) ? r.TW : 0;
        uth = (uth < 0 || uth == r.TH) ? r.TH : 0;
    }
    if (base > g->tile_cap) return fail(XY_EBUDGET, "tile table overflow");
    const int32_t n = (int32_t)descs.size();
    GCHECK(g, hipStreamSynchronize(g->stream));
    if (n) {
        GCHECK(g, hipMemcpy(g->d_reps, descs.data(), n * sizeof(xy::RepDesc), hipMemcpyHostToDevice));
        GCHECK(g, hipMemcpy(g->d_tile_rep, tile_rep.data(), tile_rep.size() * sizeof(uint32_t),
                            hipMemcpyHostToDevice));
        GCHECK(g, hipMemcpy(g->d_fin_rep, fin_rep.data(), fin_rep.size() * sizeof(uint32_t),
                            hipMemcpyHostToDevice));
    }
    xy::Launch &lc = g->lc;
    lc.reps = g->d_reps;
    lc.tile_rep = g->d_tile_rep;
    lc.nrep = n;
    lc.label_bits = 32;
    lc.max_th = max_th;
    lc.big_index = 0;
    lc.uniform_tw = utw;
    lc.uniform_th = uth;
    lc.gtile0 = 0;
    lc.gtile_end = base;
    lc.fin_rep = g->d_fin_rep;
    lc.nfin = fbase;
    for (int32_t k = 0; k < n; ++k) {
        Slot &sl = g->slots[g->order[k]];
        if (!sl.needs_init) continue;
        GCHECK(g, xy::launch_init_spins(g->d_reps, k, sl.plan.res[0].N, sl.p.start, g->stream));
        GCHECK(g, xy::launch_init_fourier(g->d_reps, k, sl.plan.res[0].L, g->stream));
        GCHECK(g, xy::launch_edge_refresh(g->d_reps, k, sl.plan.res[0].ntiles, g->stream));
        sl.needs_init = false;
    }
    if (n) GCHECK(g, xy::launch_init_dir(g->d_reps, n, g->stream));
    GCHECK(g, hipStreamSynchronize(g->stream));
    g->dirty = false;
    return XY_OK;
}

}  // namespace

extern "C" {

int xy_group_bytes(const xy_params *p, size_t *bytes)
{
    if (!bytes) return fail(XY_EINVAL, "bytes pointer is NULL");
    Plan P;
    int rc = plan_request(p, P);
    if (rc) return rc;
    *bytes = slot_bytes(P);
    return XY_OK;
}

int xy_group_create(size_t budget_bytes, int32_t max_slots, const xy_pcc *c, void *hip_stream, xy_group **out)
{
    if (!out || !c) return fail(XY_EINVAL, "NULL argument");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 65536) return fail(XY_EINVAL, "max_slots=%d outside [1, 65536]", max_slots);
    if (budget_bytes < (1u << 20)) return fail(XY_EINVAL, "budget of %zu bytes is too small", budget_bytes);
    if (c->window < 1 || !(c->dbeta0 > 0.0) || !(c->dbeta_min >= 0.0) || c->halve_every < 0)
        return fail(XY_EINVAL, "bad PCC rule");
    if (c->rule != XY_PCC_HELICITY)
        return fail(XY_EINVAL, "serving groups run the helicity-modulus PCC rule only (rule %d)", c->rule);
    xy_group *g = new (std::nothrow) xy_group;
    if (!g) return fail(XY_ENOMEM, "host allocation failed");
    g->pcc = *c;
    g->slots.resize(max_slots);
    // smallest tiles hold 64 x 16 sites and a site needs at least 8 bytes
    g->tile_cap = (int64_t)(budget_bytes / (64 * 16 * 8)) + max_slots;
    const size_t tables = align_up(max_slots * sizeof(xy::RepDesc)) + 2 * align_up(g->tile_cap * sizeof(uint32_t));
    void *mem = nullptr;
    hipError_t e = hipMalloc(&mem, budget_bytes + tables);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete g;
        return fail(XY_ENOMEM, "hipMalloc of %zu bytes failed: %s", budget_bytes + tables, hipGetErrorString(e));
    }
    g->mem = static_cast<char *>(mem);
    g->arena.init(budget_bytes);
    g->d_reps = reinterpret_cast<xy::RepDesc *>(g->mem + budget_bytes);
    g->d_tile_rep = reinterpret_cast<uint32_t *>(g->mem + budget_bytes + align_up(max_slots * sizeof(xy::RepDesc)));
    g->d_fin_rep = g->d_tile_rep + align_up(g->tile_cap * sizeof(uint32_t)) / sizeof(uint32_t);
    if (hip_stream) {
        g->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            xy_group_free(g);
            return fail(XY_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
        }
        g->own_stream = true;
    }
    *out = g;
    return XY_OK;
}

int xy_group_add(xy_group *g, const xy_params *p, int64_t nsweeps, int32_t *slot)
{
    int rc = check_group(g);
    if (rc) return rc;
    if (!slot) return fail(XY_EINVAL, "slot pointer is NULL");
    if (nsweeps < 1) return fail(XY_EINVAL, "nsweeps=%lld < 1", (long long)nsweeps);
    Plan P;
    rc = plan_request(p, P);
    if (rc) return rc;
    const size_t bytes = slot_bytes(P);
    if (bytes > g->arena.size)
        return fail(XY_EINVAL, "a request of %zu bytes can never fit the group's budget of %zu bytes", bytes,
                    g->arena.size);
    int32_t s = -1;
    for (int32_t k = 0; k < (int32_t)g->slots.size(); ++k)
        if (!g->slots[k].used) {
            s = k;
            break;
        }
    if (s < 0) return fail(XY_EBUDGET, "all %zu slots are in use", g->slots.size());
    size_t off = 0;
    if (!g->arena.take(bytes, &off)) return fail(XY_EBUDGET, "no %zu free bytes in the group's arena", bytes);
    Slot &sl = g->slots[s];
    sl = Slot();
    sl.used = sl.running = sl.needs_init = true;
    sl.p = *p;
    sl.plan = P;
    sl.off = off;
    sl.bytes = bytes;
    sl.target = nsweeps;
    sl.st = reinterpret_cast<xy::RepState *>(g->mem + off + align_up(P.lay[0].end));
    xy::RepState st;
    std::memset(&st, 0, sizeof st);
    st.beta = p->beta;
    GCHECK(g, hipMemcpy(sl.st, &st, sizeof st, hipMemcpyHostToDevice));
    g->dirty = true;
    *slot = s;
    return XY_OK;
}

int xy_group_round(xy_group *g, int64_t max_sweeps, int64_t *ran)
{
    int rc = check_group(g);
    if (rc) return rc;
    if (max_sweeps < 1) return fail(XY_EINVAL, "max_sweeps=%lld < 1", (long long)max_sweeps);
    if (g->dirty) {
        rc = rebuild(g);
        if (rc) return rc;
    }
    int64_t k = max_sweeps;
    for (int32_t s : g->order) k = std::min(k, g->slots[s].target - g->slots[s].done);
    if (g->order.empty()) k = 0;
    if (ran) *ran = k;
    if (k == 0) return XY_OK;
    const int32_t n = (int32_t)g->order.size();
    xy::FlipArgs fa;
    std::memset(&fa, 0, sizeof fa);
    fa.nrep = n;
    fa.window = g->pcc.window;
    fa.dbeta0 = g->pcc.dbeta0;
    fa.dbeta_min = g->pcc.dbeta_min;
    fa.halve_every = g->pcc.halve_every;
    fa.target = g->pcc.target;
    Pipe pp;
    auto plain = [](int, auto launch) { return launch(); };
    for (int64_t j = 0; j < k; ++j) {
        // the next sweep's links may be activated in this pass only if no
        // running request ends a PCC window (and so changes beta) here
        bool window_ends = false;
        for (int32_t s : g->order)
            if ((g->slots[s].done + j + 1) % g->pcc.window == 0) window_ends = true;
        const int next = j + 1 < k ? (window_ends ? NEXT_SPEC : NEXT_FUSE) : NEXT_END;
        GCHECK(g, enqueue_sweep_lc(g->lc, g->d_reps, n, fa, next, pp, g->stream, plain));
    }
    GCHECK(g, hipStreamSynchronize(g->stream));
    for (int32_t s : g->order) {
        Slot &sl = g->slots[s];
        sl.done += k;
        if (sl.done >= sl.target) {
            sl.running = false;
            g->finished.push_back(s);
            g->dirty = true;
        }
    }
    return XY_OK;
}

int xy_group_poll(xy_group *g, int32_t *slots, int32_t cap, int32_t *n)
{
    int rc = check_group(g);
    if (rc) return rc;
    if (!n || (cap > 0 && !slots)) return fail(XY_EINVAL, "NULL argument");
    int32_t m = 0;
    while (m < cap && !g->finished.empty()) {
        slots[m++] = g->finished.front();
        g->finished.erase(g->finished.begin());
    }
    *n = m;
    return XY_OK;
}

int xy_group_result(xy_group *g, int32_t slot, xy_obs *last, double *beta, double *beta_mean)
{
    int rc = check_group(g);
    if (rc) return rc;
    if (slot < 0 || slot >= (int32_t)g->slots.size() || !g->slots[slot].used)
        return fail(XY_EINVAL, "slot %d is not in use", slot);
    xy::RepState st;
    GCHECK(g, hipStreamSynchronize(g->stream));
    GCHECK(g, hipMemcpy(&st, g->slots[slot].st, sizeof st, hipMemcpyDeviceToHost));
    if (last) *last = st.last;
    if (beta) *beta = st.beta;
    if (beta_mean) *beta_mean = st.beta_n ? st.beta_sum / (double)st.beta_n : st.beta;
    return XY_OK;
}

int xy_group_get_state(xy_group *g, int32_t slot, float *cos_out, float *sin_out)
{
    int rc = check_group(g);
    if (rc) return rc;
    if (slot < 0 || slot >= (int32_t)g->slots.size() || !g->slots[slot].used)
        return fail(XY_EINVAL, "slot %d is not in use", slot);
    if (!cos_out || !sin_out) return fail(XY_EINVAL, "output pointer is NULL");
    const Slot &sl = g->slots[slot];
    if (sl.needs_init) return fail(XY_ESTATE, "slot %d has not run a round yet", slot);
    const size_t bytes = (size_t)sl.plan.res[0].N * sizeof(float);
    GCHECK(g, hipStreamSynchronize(g->stream));
    GCHECK(g, hipMemcpy(cos_out, g->mem + sl.off + sl.plan.lay[0].c, bytes, hipMemcpyDeviceToHost));
    GCHECK(g, hipMemcpy(sin_out, g->mem + sl.off + sl.plan.lay[0].s, bytes, hipMemcpyDeviceToHost));
    return XY_OK;
}

int xy_group_release(xy_group *g, int32_t slot)
{
    int rc = check_group(g);
    if (rc) return rc;
    if (slot < 0 || slot >= (int32_t)g->slots.size() || !g->slots[slot].used)
        return fail(XY_EINVAL, "slot %d is not in use", slot);
    Slot &sl = g->slots[slot];
    if (sl.running) return fail(XY_ESTATE, "slot %d is still running", slot);
    g->arena.give(sl.off, sl.bytes);
    sl = Slot();
    return XY_OK;
}

int xy_group_info(xy_group *g, size_t *used_bytes, int32_t *running)
{
    int rc = check_group(g);
    if (rc) return rc;
    size_t used = 0;
    int32_t r = 0;
    for (const Slot &sl : g->slots) {
        if (sl.used) used += sl.bytes;
        if (sl.running) ++r;
    }
    if (used_bytes) *used_bytes = used;
    if (running) *running = r;
    return XY_OK;
}

int xy_group_free(xy_group *g)
{
    if (!g) return XY_OK;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    if (g->mem) (void)hipFree(g->mem);
    if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
    return XY_OK;
}

}  // extern "C"
