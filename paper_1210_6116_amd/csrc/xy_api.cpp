// xy_api.cpp -- host side of the C ABI declared in include/xy.h: parameter
// checks, the device memory layout of a handle, and the per-sweep launch
// sequence (bonds + tile labelling, merge across tiles, flip + reductions).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/xy.h"
#include "xy_device.hpp"
#include "xy_launch.hpp"
#include "xy_host.hpp"

namespace xyhost {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}


size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int ilog2(int64_t v)
{
    int k = 0;
    while ((int64_t(1) << k) < v) ++k;
    return k;
}




int check_params(const xy_params *p, int32_t n)
{
    if (!p) return fail(XY_EINVAL, "params pointer is NULL");
    if (n < 1 || n > (1 << 20)) return fail(XY_EINVAL, "n_replicas=%d outside [1, 2^20]", n);
    for (int32_t k = 0; k < n; ++k) {
        const xy_params &q = p[k];
        if (q.L < 2 || q.L > 65536 || (q.L & (q.L - 1)) != 0)
            return fail(XY_EINVAL, "replica %d: L=%lld is not a power of two in [2, 65536]", k, (long long)q.L);
        if (!(q.beta >= 0.0 && q.beta <= 1e4))
            return fail(XY_EINVAL, "replica %d: beta=%g outside [0, 1e4]", k, q.beta);
        if (q.label_bits != 0 && q.label_bits != 32 && q.label_bits != 64)
            return fail(XY_EINVAL, "replica %d: label_bits=%d is not 0, 32 or 64", k, q.label_bits);
        if (q.label_bits == 32 && q.L * q.L >= (int64_t(1) << 32))
            return fail(XY_EINVAL, "replica %d: L=%lld needs 64-bit labels", k, (long long)q.L);
        if (q.start != XY_START_HOT && q.start != XY_START_COLD)
            return fail(XY_EINVAL, "replica %d: start=%d unknown", k, q.start);
        if (q.tile_rows != 0 && q.tile_rows != 16 && q.tile_rows != 32 && q.tile_rows != 64)
            return fail(XY_EINVAL, "replica %d: tile_rows=%d is not 0, 16, 32 or 64", k, q.tile_rows);
    }
    return XY_OK;
}

int make_plan(const xy_params *p, int32_t n, Plan &P)
{
    int rc = check_params(p, n);
    if (rc) return rc;
    P.n = n;
    bool need64 = false, want32 = false, want64 = false;
    int64_t maxN = 0;
    for (int32_t k = 0; k < n; ++k) {
        const int64_t N = p[k].L * p[k].L;
        maxN = std::max(maxN, N);
        if (N >= (int64_t(1) << 32)) need64 = true;
        if (p[k].label_bits == 32) want32 = true;
        if (p[k].label_bits == 64) want64 = true;
    }
    if (want32 && (need64 || want64)) return fail(XY_EINVAL, "replicas disagree on the label width");
    P.label_bits = (need64 || want64) ? 64 : 32;
    // 64-bit site indices are needed above 2^30 sites; XY_WIDE_INDEX=1 selects
    // them for any size (the same kernels with wider index arithmetic; tests)
    const char *wide = std::getenv("XY_WIDE_INDEX");
    P.big_index = maxN > (int64_t(1) << 30) || (wide && wide[0] == '1');
    size_t off = 0;
    P.res.resize(n);
    P.lay.resize(n);
    P.total_tiles = 0;
    for (int32_t k = 0; k < n; ++k) {
        Resolved &r = P.res[k];
        r.L = p[k].L;
        r.N = r.L * r.L;
        const int rows = p[k].tile_rows ? p[k].tile_rows : 32;
        r.TW = (int32_t)std::min<int64_t>(r.L, 64);
        r.TH = (int32_t)std::min<int64_t>(r.L, rows);
        r.ntx = (int32_t)(r.L / r.TW);
        r.nty = (int32_t)(r.L / r.TH);
        r.nb = 2 * (r.TW + r.TH);
        r.ntiles = (int64_t)r.ntx * r.nty;
        r.fin_chunks = (int32_t)((r.ntiles + xy::kFinSpan - 1) / xy::kFinSpan);
        P.total_fin += r.fin_chunks;
        P.max_th = std::max(P.max_th, r.TH);
        P.uniform_tw = (P.uniform_tw < 0 || P.uniform_tw == r.TW) ? r.TW : 0;
        P.uniform_th = (P.uniform_th < 0 || P.uniform_th == r.TH) ? r.TH : 0;
        P.total_tiles += r.ntiles;
        RepLayout &l = P.lay[k];
        const size_t words = (size_t)std::max<int64_t>(1, (r.N + 31) / 32);
        const size_t nodes = (size_t)r.ntiles * r.nb;
        l.c = off;
        off = align_up(off + (size_t)r.N * 4);
        l.s = off;
        off = align_up(off + (size_t)r.N * 4);
        // edge copies and link planes are double-buffered: the fused pass reads
        // the neighbours' edge copies of sweep t (slot t&1) while it writes
        // those of sweep t+1.  Labels and the forest have one buffer: a tile
        // reads its own labels of sweep t before it overwrites them.
        for (int q = 0; q < 2; ++q) {
            l.edge[q] = off;
            off = align_up(off + (size_t)r.ntiles * (r.TH + r.TW) * sizeof(float2));
            l.bx[q] = off;
            off = align_up(off + words * 4);
            l.by[q] = off;
            off = align_up(off + words * 4);
        }
        // the second candidate's link planes (a flip that activates the next
        // sweep's links for both betas its PCC step may choose)
        l.bxs = off;
        off = align_up(off + words * 4);
        l.bys = off;
        off = align_up(off + words * 4);
        l.lab = off;
        off = align_up(off + (size_t)r.N * sizeof(uint16_t));
        l.bslot = off;
        off = align_up(off + nodes);
        l.node = off;
        off = align_up(off + nodes * sizeof(unsigned long long));
        l.cross = off;
        off = align_up(off + (size_t)r.ntiles * 2 * sizeof(unsigned long long));
        l.ecoin = off;
        off = align_up(off + (size_t)r.ntiles * 4 * sizeof(unsigned long long));
        l.ecnt = off;
        off = align_up(off + (size_t)r.ntiles * 2 * sizeof(uint32_t));
        l.partials = off;
        off = align_up(off + (size_t)r.ntiles * xy::kNumSums * sizeof(double));
        l.partials2 = off;
        off = align_up(off + (size_t)r.fin_chunks * xy::kNumSums * sizeof(double));
        l.fourier = off;
        off = align_up(off + (size_t)r.L * 2 * sizeof(double));
        l.end = off;
    }
    P.off_reps = off;
    off = align_up(off + n * sizeof(xy::RepDesc));
    P.off_state = off;
    off = align_up(off + n * sizeof(xy::RepState));
    P.off_tile_rep = off;
    if (n > 1) off = align_up(off + (size_t)P.total_tiles * sizeof(uint32_t));
    P.off_fin_rep = off;
    if (n > 1) off = align_up(off + (size_t)P.total_fin * sizeof(uint32_t));
    P.off_obs = off;
    off = align_up(off + (size_t)(2 * kTraceChunk + 1) * n * sizeof(xy_obs));
    P.total = off;
    return XY_OK;
}

void fill_desc(const Plan &P, int32_t k, const xy_params &p, char *A, xy::RepState *st, int64_t tile_base,
               int64_t fin_base, int32_t idx, xy::RepDesc &d)
{
    const Resolved &r = P.res[k];
    const RepLayout &l = P.lay[k];
    std::memset(&d, 0, sizeof d);
    d.c = reinterpret_cast<float *>(A + l.c);
    d.s = reinterpret_cast<float *>(A + l.s);
    for (int q = 0; q < 2; ++q) {
        d.bx[q] = reinterpret_cast<uint32_t *>(A + l.bx[q]);
        d.by[q] = reinterpret_cast<uint32_t *>(A + l.by[q]);
        d.edge[q] = reinterpret_cast<float2 *>(A + l.edge[q]);
    }
    d.bxs = reinterpret_cast<uint32_t *>(A + l.bxs);
    d.bys = reinterpret_cast<uint32_t *>(A + l.bys);
    d.lab = reinterpret_cast<uint16_t *>(A + l.lab);
    d.bslot = reinterpret_cast<uint8_t *>(A + l.bslot);
    d.node = reinterpret_cast<unsigned long long *>(A + l.node);
    d.cross = reinterpret_cast<unsigned long long *>(A + l.cross);
    d.ecoin = reinterpret_cast<unsigned long long *>(A + l.ecoin);
    d.ecnt = reinterpret_cast<uint32_t *>(A + l.ecnt);
    d.partials = reinterpret_cast<double *>(A + l.partials);
    d.partials2 = reinterpret_cast<double *>(A + l.partials2);
    d.fourier = reinterpret_cast<double *>(A + l.fourier);
    d.st = st;
    d.L = r.L;
    d.N = r.N;
    d.ntiles = r.ntiles;
    d.tile_base = tile_base;
    d.seed = p.seed;
    d.rep = p.replica;
    d.log2L = ilog2(r.L);
    d.TW = r.TW;
    d.TH = r.TH;
    d.log2TW = ilog2(r.TW);
    d.ntx = r.ntx;
    d.nty = r.nty;
    d.nb = r.nb;
    d.fin_chunks = r.fin_chunks;
    d.fin_base = fin_base;
    d.idx = idx;
}


int plan_link_labels(int64_t L, int32_t label_bits, int32_t tile_rows, LinkLabelJob &J)
{
    xy_params p;
    std::memset(&p, 0, sizeof p);
    p.L = L;
    p.label_bits = label_bits;
    p.tile_rows = tile_rows;
    if (label_bits != 32 && label_bits != 64) return fail(XY_EINVAL, "label_bits=%d is not 32 or 64", label_bits);
    int rc = make_plan(&p, 1, J.plan);
    if (rc) return rc;
    const Resolved &r = J.plan.res[0];
    const size_t nodes = (size_t)r.ntiles * r.nb;
    static_assert(sizeof(xy::RepState) <= 512 && sizeof(xy::RepDesc) <= 512, "scratch header too small");
    J.off_state = 0;
    J.off_desc = 512;
    J.off_lab = 1024;
    J.off_bslot = align_up(J.off_lab + (size_t)r.N * sizeof(uint16_t));
    J.off_node = align_up(J.off_bslot + nodes);
    J.off_cross = align_up(J.off_node + nodes * sizeof(unsigned long long));
    J.total = align_up(J.off_cross + (size_t)r.ntiles * 2 * sizeof(unsigned long long));
    return XY_OK;
}

void link_label_desc(const LinkLabelJob &J, char *mem, const uint32_t *d_bx, const uint32_t *d_by, xy::RepDesc &d)
{
    const Resolved &r = J.plan.res[0];
    std::memset(&d, 0, sizeof d);
    d.lab = reinterpret_cast<uint16_t *>(mem + J.off_lab);
    d.bslot = reinterpret_cast<uint8_t *>(mem + J.off_bslot);
    d.node = reinterpret_cast<unsigned long long *>(mem + J.off_node);
    d.cross = reinterpret_cast<unsigned long long *>(mem + J.off_cross);
    for (int q = 0; q < 2; ++q) {
        d.bx[q] = const_cast<uint32_t *>(d_bx);
        d.by[q] = const_cast<uint32_t *>(d_by);
    }
    d.st = reinterpret_cast<xy::RepState *>(mem + J.off_state);
    d.L = r.L;
    d.N = r.N;
    d.ntiles = r.ntiles;
    d.log2L = ilog2(r.L);
    d.TW = r.TW;
    d.TH = r.TH;
    d.log2TW = ilog2(r.TW);
    d.ntx = r.ntx;
    d.nty = r.nty;
    d.nb = r.nb;
}

hipError_t enqueue_link_labels(const LinkLabelJob &J, char *mem, void *d_labels, hipStream_t s)
{
    const Resolved &r = J.plan.res[0];
    const xy::RepDesc *d_rep = reinterpret_cast<const xy::RepDesc *>(mem + J.off_desc);
    xy::Launch lc;
    lc.reps = d_rep;
    lc.tile_rep = nullptr;
    lc.nrep = 1;
    lc.label_bits = J.plan.label_bits;
    lc.max_th = r.TH;
    lc.big_index = J.plan.big_index;
    lc.uniform_tw = J.plan.uniform_tw;
    lc.uniform_th = J.plan.uniform_th;
    lc.gtile0 = 0;
    lc.gtile_end = r.ntiles;
    lc.fin_rep = nullptr;
    lc.nfin = 0;  // no finalisation here
    hipError_t e = xy::launch_tile(lc, xy::TILE_PLANES, s);
    if (e == hipSuccess) e = xy::launch_merge(lc, false, false, s);
    if (e == hipSuccess) e = xy::launch_flatten(d_rep, 0, r.N, J.plan.big_index, d_labels, J.plan.label_bits, s);
    return e;
}

}  // namespace xyhost

using namespace xyhost;

struct xy_handle {
    Plan plan;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *arena = nullptr;
    bool own_arena = false;
    std::vector<xy::RepDesc> reps;
    xy::RepDesc *d_reps = nullptr;
    xy::RepState *d_state = nullptr;
    uint32_t *d_tile_rep = nullptr;
    uint32_t *d_fin_rep = nullptr;
    xy_obs *d_trace = nullptr, *d_wmean = nullptr, *d_meas = nullptr;
    bool poisoned = false;
    // timing
    bool timing = false;
    struct Ev {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Ev> ev_used;
    std::vector<hipEvent_t> ev_pool;
    double ms[XY_K_COUNT] = {};
    int64_t launches[XY_K_COUNT] = {};
    // wrapping-check buffers of the percolation rule (allocated on first use)
    char *perc_mem = nullptr;
    int32_t dedup = XY_DEDUP_WAVE;  // merge's pair deduplication and edges per wave (xy_set_merge)
    int32_t merge_epw = 1;
    int32_t inpass = 0;             // the labelling tile pass unites the tile edges itself (xy_set_merge_in_pass)
    // captured sweep sequence (xy_sweep_graph)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int64_t graph_n = 0;
    int32_t graph_merge = 1;  // the merge choices the graph was captured with
};

namespace {

int hip_fail(xy_handle *h, hipError_t e, const char *what)
{
    if (h) h->poisoned = true;
    return fail(XY_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHECK(h, expr)                                    \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(h, e_, #expr); \
    } while (0)

int check_handle(xy_handle *h)
{
    if (!h) return fail(XY_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(XY_ESTATE, "handle was poisoned by an earlier device error");
    return XY_OK;
}

xy::Launch launch_all(xy_handle *h)
{
    xy::Launch lc;
    lc.reps = h->d_reps;
    lc.tile_rep = h->d_tile_rep;
    lc.nrep = h->plan.n;
    lc.label_bits = h->plan.label_bits;
    lc.max_th = h->plan.max_th;
    lc.big_index = h->plan.big_index;
    lc.uniform_tw = h->plan.uniform_tw;
    lc.uniform_th = h->plan.uniform_th;
    lc.gtile0 = 0;
    lc.gtile_end = h->plan.total_tiles;
    lc.fin_rep = h->d_fin_rep;
    lc.nfin = h->plan.total_fin;
    lc.dedup = h->dedup;
    lc.merge_epw = h->merge_epw;
    lc.inpass = h->inpass;
    return lc;
}

hipError_t take_event(xy_handle *h, hipEvent_t *e)
{
    if (!h->ev_pool.empty()) {
        *e = h->ev_pool.back();
        h->ev_pool.pop_back();
        return hipSuccess;
    }
    // timing events only: no system-scope fence (cache writeback and
    // invalidation) when they are recorded, so that they bracket the kernels
    // alone; they are read after the stream has been synchronised
    return hipEventCreateWithFlags(e, hipEventDisableSystemFence);
}

// Runs `launch` bracketed by timing events when timing is on.
template <typename F>
hipError_t timed(xy_handle *h, int kind, F launch)
{
    if (!h->timing) return launch();
    xy_handle::Ev ev;
    hipError_t e0 = take_event(h, &ev.a);
    if (e0 != hipSuccess) return e0;
    e0 = take_event(h, &ev.b);
    if (e0 != hipSuccess) return e0;
    ev.kind = kind;
    hipError_t e = hipSuccess;
    if (kind == XY_K_WRAP) {
        // several kernels: events around them on the stream
        e = hipEventRecord(ev.a, h->stream);
        if (e != hipSuccess) return e;
        e = launch();
        if (e != hipSuccess) return e;
        e = hipEventRecord(ev.b, h->stream);
    } else {
        // one kernel: the events take its own start and end
        xy::next_launch_events() = xy::KernelEvents{ev.a, ev.b};
        e = launch();
        const bool unused = xy::next_launch_events().start != nullptr;
        xy::next_launch_events() = xy::KernelEvents{};
        if (e != hipSuccess) return e;
        if (unused) {  // nothing was launched: an empty interval
            e = hipEventRecord(ev.a, h->stream);
            if (e == hipSuccess) e = hipEventRecord(ev.b, h->stream);
        }
    }
    if (e != hipSuccess) return e;
    h->ev_used.push_back(ev);
    return e;
}

// Enqueues one sweep of every replica (pp carries the launch state between the
// sweeps of one call).  fuse_next: the flip of this sweep also activates and
// labels the links of the next one, and its finalisation runs with the next
// sweep's edge coins (allowed only when beta cannot change in between, i.e.
// not at the end of a PCC window, and only if another sweep follows).
int enqueue_sweep(xy_handle *h, const xy::FlipArgs &fa, int next, Pipe &pp)
{
    const xy::Launch lc = launch_all(h);
    hipEvent_t sweep_begin = nullptr;
    if (h->timing) {
        HIPCHECK(h, take_event(h, &sweep_begin));
        HIPCHECK(h, hipEventRecord(sweep_begin, h->stream));
    }
    auto timer = [&](int kind, auto launch) { return timed(h, kind, launch); };
    HIPCHECK(h, enqueue_sweep_lc(lc, h->d_reps, h->plan.n, fa, next, pp, h->stream, timer));
    if (h->timing) {
        xy_handle::Ev ev;
        ev.kind = XY_K_SWEEP;
        ev.a = sweep_begin;
        HIPCHECK(h, take_event(h, &ev.b));
        HIPCHECK(h, hipEventRecord(ev.b, h->stream));
        h->ev_used.push_back(ev);
    }
    return XY_OK;
}

xy::FlipArgs no_pcc(const xy_handle *h)
{
    xy::FlipArgs fa;
    std::memset(&fa, 0, sizeof fa);
    fa.nrep = h->plan.n;
    return fa;
}

int read_state(xy_handle *h, int32_t rep, xy::RepState *out)
{
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipMemcpy(out, h->d_state + rep, sizeof *out, hipMemcpyDeviceToHost));
    return XY_OK;
}

// Buffers of the wrapping check for every replica (two forest copies and two
// arrays of per-node potentials), allocated on the first percolation-rule call
// and named in the replicas' descriptors from then on.
int ensure_wrap_buffers(xy_handle *h)
{
    if (h->perc_mem) return XY_OK;
    const Plan &P = h->plan;
    size_t total = 0;
    std::vector<size_t> off(P.n);
    for (int32_t k = 0; k < P.n; ++k) {
        const Resolved &r = P.res[k];
        if (r.L > xy::kWrapMaxL)
            return fail(XY_EINVAL, "replica %d: the percolation rule needs L <= %lld (L=%lld)", k,
                        (long long)xy::kWrapMaxL, (long long)r.L);
        off[k] = total;
        total += align_up(4 * (size_t)r.ntiles * r.nb * sizeof(unsigned long long));
    }
    char *mem = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&mem), total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(XY_ENOMEM, "hipMalloc of %zu bytes for the wrapping check failed: %s", total,
                    hipGetErrorString(e));
    }
    for (int32_t k = 0; k < P.n; ++k) {
        const size_t words = (size_t)P.res[k].ntiles * P.res[k].nb;
        unsigned long long *w = reinterpret_cast<unsigned long long *>(mem + off[k]);
        h->reps[k].node_cut[0] = w;
        h->reps[k].node_cut[1] = w + words;
        h->reps[k].pstate[0] = w + 2 * words;
        h->reps[k].pstate[1] = w + 3 * words;
    }
    h->perc_mem = mem;
    // the stream may still run sweeps that read the descriptors: copy in order
    HIPCHECK(h, hipMemcpyAsync(h->d_reps, h->reps.data(), P.n * sizeof(xy::RepDesc), hipMemcpyHostToDevice,
                               h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return XY_OK;
}

int check_rep(xy_handle *h, int32_t rep)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (rep < 0 || rep >= h->plan.n) return fail(XY_EINVAL, "replica %d outside [0, %d)", rep, h->plan.n);
    return XY_OK;
}

}  // namespace

extern "C" {

const char *xy_last_error(void) { return g_err.c_str(); }

int xy_bytes_required(const xy_params *p, int32_t n, size_t *bytes)
{
    if (!bytes) return fail(XY_EINVAL, "bytes pointer is NULL");
    Plan P;
    int rc = make_plan(p, n, P);
    if (rc) return rc;
    *bytes = P.total;
    return XY_OK;
}

int xy_alloc(const xy_params *p, int32_t n, void *hip_stream, void *arena, size_t arena_bytes,
             xy_handle **out)
{
    if (!out) return fail(XY_EINVAL, "out pointer is NULL");
    *out = nullptr;
    xy_handle *h = new (std::nothrow) xy_handle;
    if (!h) return fail(XY_ENOMEM, "host allocation failed");
    int rc = make_plan(p, n, h->plan);
    if (rc) {
        delete h;
        return rc;
    }
    const Plan &P = h->plan;
    if (arena) {
        if (arena_bytes < P.total) {
            delete h;
            return fail(XY_ENOMEM, "arena of %zu bytes is smaller than the %zu required", arena_bytes, P.total);
        }
        if (reinterpret_cast<uintptr_t>(arena) % kAlign) {
            delete h;
            return fail(XY_EINVAL, "arena is not %zu-byte aligned", kAlign);
        }
        h->arena = static_cast<char *>(arena);
    } else {
        void *mem = nullptr;
        hipError_t e = hipMalloc(&mem, P.total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete h;
            return fail(XY_ENOMEM, "hipMalloc of %zu bytes failed: %s", P.total, hipGetErrorString(e));
        }
        h->arena = static_cast<char *>(mem);
        h->own_arena = true;
    }
    if (hip_stream) {
        h->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            xy_free(h);
            return fail(XY_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
        }
        h->own_stream = true;
    }
    char *A = h->arena;
    h->d_reps = reinterpret_cast<xy::RepDesc *>(A + P.off_reps);
    h->d_state = reinterpret_cast<xy::RepState *>(A + P.off_state);
    h->d_tile_rep = n > 1 ? reinterpret_cast<uint32_t *>(A + P.off_tile_rep) : nullptr;
    h->d_fin_rep = n > 1 ? reinterpret_cast<uint32_t *>(A + P.off_fin_rep) : nullptr;
    h->d_trace = reinterpret_cast<xy_obs *>(A + P.off_obs);
    h->d_wmean = h->d_trace + kTraceChunk * n;
    h->d_meas = h->d_wmean + kTraceChunk * n;
    h->reps.resize(n);
    std::vector<xy::RepState> states(n);
    std::vector<uint32_t> tile_rep, fin_rep;
    if (n > 1) tile_rep.resize(P.total_tiles);
    if (n > 1) fin_rep.resize(P.total_fin);
    int64_t base = 0, fbase = 0;
    for (int32_t k = 0; k < n; ++k) {
        const Resolved &r = P.res[k];
        fill_desc(P, k, p[k], A, h->d_state + k, base, fbase, k, h->reps[k]);
        for (int64_t tt = 0; tt < r.ntiles && n > 1; ++tt) tile_rep[base + tt] = (uint32_t)k;
        for (int64_t c = 0; c < r.fin_chunks && n > 1; ++c) fin_rep[fbase + c] = (uint32_t)k;
        base += r.ntiles;
        fbase += r.fin_chunks;
        xy::RepState &s = states[k];
        std::memset(&s, 0, sizeof s);
        s.beta = p[k].beta;
    }
    // a HIP failure from here on releases the handle (its arena and stream)
    // before returning: the caller receives no handle to free
    auto init = [&]() -> int {
        HIPCHECK(h, hipMemcpy(h->d_reps, h->reps.data(), n * sizeof(xy::RepDesc), hipMemcpyHostToDevice));
        HIPCHECK(h, hipMemcpy(h->d_state, states.data(), n * sizeof(xy::RepState), hipMemcpyHostToDevice));
        if (n > 1) {
            HIPCHECK(h, hipMemcpy(h->d_tile_rep, tile_rep.data(), tile_rep.size() * sizeof(uint32_t),
                                  hipMemcpyHostToDevice));
            HIPCHECK(h, hipMemcpy(h->d_fin_rep, fin_rep.data(), fin_rep.size() * sizeof(uint32_t),
                                  hipMemcpyHostToDevice));
        }
        for (int32_t k = 0; k < n; ++k) {
            HIPCHECK(h, xy::launch_init_spins(h->d_reps, k, P.res[k].N, p[k].start, h->stream));
            HIPCHECK(h, xy::launch_init_fourier(h->d_reps, k, P.res[k].L, h->stream));
            HIPCHECK(h, xy::launch_edge_refresh(h->d_reps, k, P.res[k].ntiles, h->stream));
        }
        HIPCHECK(h, xy::launch_init_dir(h->d_reps, n, h->stream));
        HIPCHECK(h, hipStreamSynchronize(h->stream));
        return XY_OK;
    };
    rc = init();
    if (rc) {
        const std::string msg = g_err;
        xy_free(h);
        g_err = msg;
        return rc;
    }
    *out = h;
    return XY_OK;
}

int xy_free(xy_handle *h)
{
    if (!h) return XY_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (auto &e : h->ev_used) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (auto &e : h->ev_pool) (void)hipEventDestroy(e);
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->perc_mem) (void)hipFree(h->perc_mem);
    if (h->own_arena && h->arena) (void)hipFree(h->arena);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return XY_OK;
}

int xy_sweep(xy_handle *h, int64_t nsweeps, xy_obs *trace)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (nsweeps < 0) return fail(XY_EINVAL, "nsweeps=%lld is negative", (long long)nsweeps);
    const int32_t n = h->plan.n;
    Pipe pp;
    for (int64_t k = 0; k < nsweeps; ++k) {
        xy::FlipArgs fa = no_pcc(h);
        if (trace) {
            fa.trace = h->d_trace;
            fa.trace_row = k % kTraceChunk;
        }
        // a sweep whose trace row is copied back right after it is not fused
        // (its finalisation must not be deferred past the copy)
        const bool fuse = k + 1 < nsweeps && !(trace && fa.trace_row == kTraceChunk - 1);
        rc = enqueue_sweep(h, fa, fuse ? NEXT_FUSE : NEXT_END, pp);
        if (rc) return rc;
        if (trace && (fa.trace_row == kTraceChunk - 1 || k == nsweeps - 1)) {
            const int64_t first = k - fa.trace_row;
            HIPCHECK(h, hipMemcpyAsync(trace + first * n, h->d_trace, (fa.trace_row + 1) * n * sizeof(xy_obs),
                                       hipMemcpyDeviceToHost, h->stream));
            HIPCHECK(h, hipStreamSynchronize(h->stream));
        }
    }
    return XY_OK;
}

int xy_sweep_graph(xy_handle *h, int64_t nsweeps, int64_t replays)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (nsweeps < 1 || replays < 0)
        return fail(XY_EINVAL, "nsweeps=%lld replays=%lld", (long long)nsweeps, (long long)replays);
    if (h->timing) return fail(XY_ESTATE, "per-kernel timing is on; graphs capture no events");
    if (!h->graph_exec || h->graph_n != nsweeps || h->graph_merge != h->dedup * 4 + h->merge_epw) {
        if (h->graph_exec) HIPCHECK(h, hipGraphExecDestroy(h->graph_exec));
        if (h->graph) HIPCHECK(h, hipGraphDestroy(h->graph));
        h->graph_exec = nullptr;
        h->graph = nullptr;
        HIPCHECK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed));
        Pipe pp;
        for (int64_t k = 0; k < nsweeps && rc == XY_OK; ++k)
            rc = enqueue_sweep(h, no_pcc(h), k + 1 < nsweeps ? NEXT_FUSE : NEXT_END, pp);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(h->stream, &graph);
        if (rc) return rc;
        if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
        h->graph = graph;
        HIPCHECK(h, hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
        h->graph_n = nsweeps;
        h->graph_merge = h->dedup * 4 + h->merge_epw;
    }
    for (int64_t r = 0; r < replays; ++r) HIPCHECK(h, hipGraphLaunch(h->graph_exec, h->stream));
    return XY_OK;
}

int xy_measure(xy_handle *h, xy_obs *out)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!out) return fail(XY_EINVAL, "out pointer is NULL");
    const xy::Launch lc = launch_all(h);
    HIPCHECK(h, xy::launch_measure(lc, h->stream));
    HIPCHECK(h, xy::launch_finalize(lc, no_pcc(h), h->d_meas, h->stream));
    HIPCHECK(h, hipMemcpyAsync(out, h->d_meas, h->plan.n * sizeof(xy_obs), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return XY_OK;
}

int xy_pcc_step(xy_handle *h, const xy_pcc *c, int64_t nsteps, xy_obs *window_mean)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!c) return fail(XY_EINVAL, "pcc pointer is NULL");
    if (nsteps < 1) return fail(XY_EINVAL, "nsteps=%lld < 1", (long long)nsteps);
    if (c->window < 1) return fail(XY_EINVAL, "window=%lld < 1", (long long)c->window);
    if (!(c->dbeta0 > 0.0) || !(c->dbeta_min >= 0.0) || c->halve_every < 0 || !std::isfinite(c->target))
        return fail(XY_EINVAL, "bad PCC schedule (dbeta0=%g dbeta_min=%g halve_every=%lld target=%g)",
                    c->dbeta0, c->dbeta_min, (long long)c->halve_every, c->target);
    if (c->rule != XY_PCC_HELICITY && c->rule != XY_PCC_PERCOLATION)
        return fail(XY_EINVAL, "PCC rule %d unknown", c->rule);
    if (c->rule == XY_PCC_PERCOLATION) {
        rc = ensure_wrap_buffers(h);
        if (rc) return rc;
    }
    const int32_t n = h->plan.n;
    Pipe pp;
    for (int64_t k = 0; k < nsteps; ++k) {
        for (int64_t w = 0; w < c->window; ++w) {
            xy::FlipArgs fa = no_pcc(h);
            fa.window = c->window;
            fa.dbeta0 = c->dbeta0;
            fa.dbeta_min = c->dbeta_min;
            fa.halve_every = c->halve_every;
            fa.target = c->target;
            fa.rule = c->rule;
            if (window_mean) {
                fa.wmean = h->d_wmean;
                fa.wrow = k % kTraceChunk;
            }
            // inside a window beta cannot change: fuse; at its end the step
            // moves beta by +-dbeta: activate the next sweep's links for both
            rc = enqueue_sweep(h, fa, w + 1 < c->window ? NEXT_FUSE : (k + 1 < nsteps ? NEXT_SPEC : NEXT_END), pp);
            if (rc) return rc;
        }
        const int64_t row = k % kTraceChunk;
        if (window_mean && (row == kTraceChunk - 1 || k == nsteps - 1)) {
            const int64_t first = k - row;
            HIPCHECK(h, hipMemcpyAsync(window_mean + first * n, h->d_wmean, (row + 1) * n * sizeof(xy_obs),
                                       hipMemcpyDeviceToHost, h->stream));
            HIPCHECK(h, hipStreamSynchronize(h->stream));
        }
    }
    return XY_OK;
}

int xy_get_state(xy_handle *h, int32_t rep, float *cos_out, float *sin_out)
{
    int rc = check_rep(h, rep);
    if (rc) return rc;
    if (!cos_out || !sin_out) return fail(XY_EINVAL, "output pointer is NULL");
    const xy::RepDesc &d = h->reps[rep];
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipMemcpy(cos_out, d.c, d.N * sizeof(float), hipMemcpyDeviceToHost));
    HIPCHECK(h, hipMemcpy(sin_out, d.s, d.N * sizeof(float), hipMemcpyDeviceToHost));
    return XY_OK;
}

int xy_set_state(xy_handle *h, int32_t rep, const float *cos_in, const float *sin_in)
{
    int rc = check_rep(h, rep);
    if (rc) return rc;
    if (!cos_in || !sin_in) return fail(XY_EINVAL, "input pointer is NULL");
    const xy::RepDesc &d = h->reps[rep];
    for (int64_t i = 0; i < d.N; ++i) {
        const double n2 = (double)cos_in[i] * cos_in[i] + (double)sin_in[i] * sin_in[i];
        if (!(std::fabs(n2 - 1.0) <= 1e-3))
            return fail(XY_EINVAL, "spin %lld has squared length %g, not 1", (long long)i, n2);
    }
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipMemcpy(d.c, cos_in, d.N * sizeof(float), hipMemcpyHostToDevice));
    HIPCHECK(h, hipMemcpy(d.s, sin_in, d.N * sizeof(float), hipMemcpyHostToDevice));
    HIPCHECK(h, xy::launch_edge_refresh(h->d_reps, rep, d.ntiles, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return XY_OK;
}

int xy_flatten_labels(xy_handle *h, int32_t rep, void *d_out, int32_t out_bits)
{
    int rc = check_rep(h, rep);
    if (rc) return rc;
    if (!d_out) return fail(XY_EINVAL, "output pointer is NULL");
    if (out_bits != 32 && out_bits != 64) return fail(XY_EINVAL, "out_bits=%d is not 32 or 64", out_bits);
    const xy::RepDesc &d = h->reps[rep];
    if (out_bits == 32 && d.N > (int64_t(1) << 32))
        return fail(XY_EINVAL, "labels of %lld sites need 64 bits", (long long)d.N);
    xy::RepState s;
    rc = read_state(h, rep, &s);
    if (rc) return rc;
    if (s.t == 0) return fail(XY_ESTATE, "replica %d has not swept yet", rep);
    HIPCHECK(h, xy::launch_flatten(h->d_reps, rep, d.N, h->plan.big_index, d_out, out_bits, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return XY_OK;
}

int xy_get_labels(xy_handle *h, int32_t rep, int64_t *out)
{
    int rc = check_rep(h, rep);
    if (rc) return rc;
    if (!out) return fail(XY_EINVAL, "output pointer is NULL");
    const xy::RepDesc &d = h->reps[rep];
    void *tmp = nullptr;
    const hipError_t ea = hipMalloc(&tmp, d.N * sizeof(int64_t));
    if (ea != hipSuccess) {
        // only the temporary buffer is missing: the handle stays usable, and
        // the allocation error must not be reported by the next launch
        (void)hipGetLastError();
        return fail(XY_ENOMEM, "hipMalloc of %lld label bytes failed: %s", (long long)(d.N * sizeof(int64_t)),
                    hipGetErrorString(ea));
    }
    rc = xy_flatten_labels(h, rep, tmp, 64);
    if (rc == XY_OK) {
        const hipError_t e = hipMemcpy(out, tmp, d.N * sizeof(int64_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = hip_fail(h, e, "label copy");
    }
    (void)hipFree(tmp);
    return rc;
}

int xy_get_bonds(xy_handle *h, int32_t rep, uint32_t *bx, uint32_t *by)
{
    int rc = check_rep(h, rep);
    if (rc) return rc;
    if (!bx || !by) return fail(XY_EINVAL, "output pointer is NULL");
    xy::RepState s;
    rc = read_state(h, rep, &s);
    if (rc) return rc;
    if (s.t == 0) return fail(XY_ESTATE, "replica %d has not swept yet", rep);
    const xy::RepDesc &d = h->reps[rep];
    const size_t words = (size_t)std::max<int64_t>(1, (d.N + 31) / 32);
    HIPCHECK(h, hipMemcpy(bx, d.bx[(s.t - 1) & 1], words * 4, hipMemcpyDeviceToHost));
    HIPCHECK(h, hipMemcpy(by, d.by[(s.t - 1) & 1], words * 4, hipMemcpyDeviceToHost));
    return XY_OK;
}

int xy_get_views(xy_handle *h, int32_t rep, xy_views *out)
{
    int rc = check_rep(h, rep);
    if (rc) return rc;
    if (!out) return fail(XY_EINVAL, "output pointer is NULL");
    xy::RepState s;
    rc = read_state(h, rep, &s);
    if (rc) return rc;
    if (s.t == 0) return fail(XY_ESTATE, "replica %d has not swept yet", rep);
    const xy::RepDesc &d = h->reps[rep];
    const int par = (int)((s.t - 1) & 1);
    *out = xy_views{};
    out->cos_plane = d.c;
    out->sin_plane = d.s;
    out->bond_x = d.bx[par];
    out->bond_y = d.by[par];
    out->L = d.L;
    out->label_bits = h->plan.label_bits;
    out->sweep = s.t;
    return XY_OK;
}

int xy_set_beta(xy_handle *h, int32_t rep, double beta)
{
    int rc = check_rep(h, rep);
    if (rc) return rc;
    if (!(beta >= 0.0 && beta <= 1e4)) return fail(XY_EINVAL, "beta=%g outside [0, 1e4]", beta);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    HIPCHECK(h, hipMemcpy(&h->d_state[rep].beta, &beta, sizeof beta, hipMemcpyHostToDevice));
    return XY_OK;
}

int xy_get_beta(xy_handle *h, int32_t rep, double *beta)
{
    int rc = check_rep(h, rep);
    if (rc) return rc;
    if (!beta) return fail(XY_EINVAL, "output pointer is NULL");
    xy::RepState s;
    rc = read_state(h, rep, &s);
    if (rc) return rc;
    *beta = s.beta;
    return XY_OK;
}

int xy_get_sweep(xy_handle *h, int32_t rep, uint64_t *sweep, double r[2])
{
    int rc = check_rep(h, rep);
    if (rc) return rc;
    xy::RepState s;
    rc = read_state(h, rep, &s);
    if (rc) return rc;
    if (sweep) *sweep = s.t;
    if (r) {
        r[0] = s.dir[s.t & 1][0];
        r[1] = s.dir[s.t & 1][1];
    }
    return XY_OK;
}

int xy_label_links(int64_t L, int32_t label_bits, int32_t tile_rows, const uint32_t *d_bx, const uint32_t *d_by,
                   void *d_labels, void *hip_stream)
{
    if (!d_bx || !d_by || !d_labels) return fail(XY_EINVAL, "device pointer is NULL");
    LinkLabelJob J;
    int rc = plan_link_labels(L, label_bits, tile_rows, J);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    char *mem = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&mem), J.total);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // not left for the next launch to report
        return fail(XY_ENOMEM, "hipMalloc failed: %s", hipGetErrorString(e));
    }
    xy::RepDesc d;
    link_label_desc(J, mem, d_bx, d_by, d);
    xy::RepState st;
    std::memset(&st, 0, sizeof st);
    e = hipMemcpy(mem + J.off_state, &st, sizeof st, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(mem + J.off_desc, &d, sizeof d, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = enqueue_link_labels(J, mem, d_labels, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(mem);
    if (e != hipSuccess) return fail(XY_EDEVICE, "labelling failed: %s", hipGetErrorString(e));
    return XY_OK;
}

int xy_set_merge(xy_handle *h, int32_t dedup, int32_t edges_per_wave)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (dedup != XY_DEDUP_WAVE && dedup != XY_DEDUP_NEIGHBOUR && dedup != XY_DEDUP_HASH)
        return fail(XY_EINVAL, "merge deduplication policy %d unknown", dedup);
    if (edges_per_wave != 1 && edges_per_wave != 2 && edges_per_wave != 4)
        return fail(XY_EINVAL, "edges_per_wave=%d is not 1, 2 or 4", edges_per_wave);
    h->dedup = dedup;
    h->merge_epw = edges_per_wave;
    return XY_OK;
}

int xy_set_merge_in_pass(xy_handle *h, int32_t on)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (on != 0 && on != 1) return fail(XY_EINVAL, "xy_set_merge_in_pass: on=%d is not 0 or 1", on);
    h->inpass = on;
    return XY_OK;
}

int xy_timing(xy_handle *h, int32_t enable)
{
    int rc = check_handle(h);
    if (rc) return rc;
    h->timing = enable != 0;
    return XY_OK;
}

int xy_timing_read(xy_handle *h, double *ms, int64_t *launches, double *samples, int64_t cap,
                   int64_t *nsamples)
{
    int rc = check_handle(h);
    if (rc) return rc;
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    int64_t ns = 0;
    for (auto &e : h->ev_used) {
        float t = 0.f;
        HIPCHECK(h, hipEventElapsedTime(&t, e.a, e.b));
        h->ms[e.kind] += t;
        h->launches[e.kind] += 1;
        if (e.kind == XY_K_SWEEP && samples && ns < cap) samples[ns++] = t;
        h->ev_pool.push_back(e.a);
        h->ev_pool.push_back(e.b);
    }
    h->ev_used.clear();
    if (nsamples) *nsamples = ns;
    for (int k = 0; k < XY_K_COUNT; ++k) {
        if (ms) ms[k] = h->ms[k];
        if (launches) launches[k] = h->launches[k];
        h->ms[k] = 0.0;
        h->launches[k] = 0;
    }
    return XY_OK;
}

}  // extern "C"
