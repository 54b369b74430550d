// xy_kernels.hip -- gfx950 kernels of one Swendsen-Wang sweep of the 2D
// classical XY model with Wolff's embedded-cluster formalism, the fused
// observable reductions, and the generalized PCC beta step (Komura & Okabe,
// arXiv:1210.6116: Eq. (Hc); the SW / PCC paragraphs; the helicity-modulus
// definitions of e and s; the simulation paragraph for the PCC parameters).
//
// The lattice is cut into tiles of 64 columns (one wave64 lane per column) by
// TH rows; one workgroup owns a tile and each of its waves a band of rows.  A
// sweep t is:
//   k_tile<BONDS>  mirror-direction projections, link activation (bit planes),
//                  in-tile union-find in LDS (row runs from wave ballots, a
//                  scan-line pass, unions where a run meets two labels, band
//                  seams), 16-bit tile-local labels, the tile's edge slots and
//                  boundary nodes, the links over its right and bottom edges
//   k_merge        union of the boundary nodes joined by every active link that
//                  leaves a tile (lock-free 64-bit atomicMin on (key, node): the
//                  root of a cluster carries its smallest site)
//   k_resolve      coin of the cluster at every edge position of every tile
//   k_tile<FLIP>   coins (a tile's own roots from its rows' Philox blocks, the
//                  others from the edge coins), reflection of flipped clusters
//                  in FP64 with one rounding to the FP32 state, the ten sums of
//                  the flipped state
//   k_finalize     sums of the tiles' partials in chunks; the last chunk of a
//                  replica finishes it: observables, PCC window and beta step,
//                  sweep counter
// k_tile<FUSED> does FLIP for sweep t and BONDS for sweep t+1 in one pass over
// the spins (whenever beta cannot change in between); the finalisation of such
// a flip then runs in two stages beside the next merge and edge coins.
// Built with -ffp-contract=off: the FP64 expressions below are evaluated
// operation by operation, exactly as written.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>

#include "xy_device.hpp"
#include "xy_launch.hpp"

namespace xy {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

enum : int { M_BONDS = 0, M_FLIP = 1, M_FUSED = 2, M_PLANES = 3, M_SPEC = 4, M_PLSEL = 5 };

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ const RepDesc &rep_of(const RepDesc *__restrict__ reps,
                                                 const uint32_t *__restrict__ tile_rep,
                                                 int32_t nrep, int64_t gtile, int64_t &lt)
{
    const RepDesc &R = reps[nrep == 1 ? 0 : tile_rep[gtile]];
    lt = gtile - R.tile_base;
    return R;
}

__device__ __forceinline__ int band_rows(int TH) { return TH >= kWaves ? TH / kWaves : 1; }

// XCD-aware order.  Blocks are dispatched to the 8 XCDs in turn, so the blocks
// an XCD receives (block j with j = x mod kXcds, counted from a block whose
// index is a multiple of kXcds) take one contiguous band of the n work items
// (tiles, or tile edges), W per block: neighbouring tiles, and the forest
// entries they write and read, share that XCD's L2 in every kernel.  Returns
// n for a slot past the end of its band.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_item(int64_t j, int W, int q, int64_t n)
{
    const int64_t per = (n + kXcds - 1) / kXcds;
    const int64_t k = (j / kXcds) * W + q;
    return k < per ? (j % kXcds) * per + k : n;
}
static int64_t xcd_blocks(int64_t n, int W)
{
    const int64_t per = (n + kXcds - 1) / kXcds;
    return kXcds * ((per + W - 1) / W);
}
__host__ __device__ __forceinline__ int64_t xcd_pad(int64_t b) { return (b + kXcds - 1) / kXcds * kXcds; }

// Point on the unit circle: a uniform point of the unit disk by rejection from
// [-1,1]^2, scaled to unit length (only correctly rounded FP64 operations).
__device__ void disk_point(uint64_t seed, uint32_t rep, uint32_t tag, uint32_t idx, uint32_t tword,
                           bool attempts_in_word0, double *ox, double *oy)
{
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (uint32_t k = 0; k < (uint32_t)kMaxAttempts; ++k) {
        const U4 w = attempts_in_word0 ? philox4x32_10(k, rep, tword, tag, k0, k1)
                                       : philox4x32_10(idx, rep, k, tag, k0, k1);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
        for (int pair = 0; pair < 2; ++pair) {
            const double vx = 2.0 * unif64(ws[2 * pair]) - 1.0;
            const double vy = 2.0 * unif64(ws[2 * pair + 1]) - 1.0;
            const double q = vx * vx + vy * vy;
            if (q > 0.0 && q < 1.0) {
                const double n = sqrt(q);
                *ox = vx / n;
                *oy = vy / n;
                return;
            }
        }
    }
    *ox = 1.0;
    *oy = 0.0;
}

__device__ __forceinline__ void compute_direction(const RepDesc &R, uint64_t t)
{
    double rx, ry;
    disk_point(R.seed, R.rep, TAG_DIR, 0u, (uint32_t)t, true, &rx, &ry);
    R.st->dir[t & 1][0] = rx;
    R.st->dir[t & 1][1] = ry;
}

// Exact (FP64) link decision, in the operation order of the definition:
// a = c rx + s ry; x = ((2 beta) a_i) a_j; active iff x > 0 and exp(-x) < 1 - u.
__device__ __noinline__ bool bond_exact(float fci, float fsi, float fcj, float fsj, double rx, double ry,
                                        double beta, uint32_t w, unsigned long long *ties)
{
    const double ci = fci, si = fsi, cj = fcj, sj = fsj;
    const double ai = ci * rx + si * ry;
    const double aj = cj * rx + sj * ry;
    const double xb = ((2.0 * beta) * ai) * aj;
    const double e = (xb > 0.0) ? exp(-xb) : 1.0;
    const double omu = 1.0 - unif64(w);
    if (fabs(e - omu) < kTieEps) atomicAdd(ties, 1ull);
    return e < omu;
}

// FP32 decision with a guard band.  With y = -(2 beta log2 e) a_i a_j,
// exp(-x) = 2^y, and the link is active iff u < 1 - exp(-x), i.e. iff
// d = w - (1 - 2^min(y, 0)) 2^32 < 0 for the Philox word w = u 2^32.  For
// unit spins the FP32 value of d is within ~2e-6 (1 + beta) 2^32 of the exact
// one, so outside |d| <= G 2^32 both precisions agree; inside it the FP64
// decision is taken.
struct BondCtx {
    double rx, ry, beta;
    float rxf, ryf, bl, gw;  // bl = -2 beta log2 e; gw = G 2^32
    unsigned long long *ties;
};

__device__ __forceinline__ float bond_proj(const BondCtx &B, float2 v)
{
    return __builtin_fmaf(v.x, B.rxf, v.y * B.ryf);
}

// d for the link (i, j), given bai = bl a_i
__device__ __forceinline__ float bond_margin(float bai, float aj, uint32_t w)
{
    const float e = __builtin_amdgcn_exp2f(fminf(bai * aj, 0.0f));
    return __builtin_fmaf(e, 4294967296.0f, (float)w - 4294967296.0f);
}

// Inclusive prefix maximum over the 64 lanes of a wave with DPP moves:
// shifts by 1, 2, 4, 8 inside each row of 16 lanes, then the last lane of
// row 0 (2) into row 1 (3), then the last lane of row 1 into rows 2 and 3.
// Lanes without a source keep 0, the identity of the maximum of unsigned keys.
__device__ __forceinline__ uint32_t wave_prefix_max(uint32_t v)
{
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return v;
}

// The v of lane ^ OFF: by ds_swizzle inside each half of the wave (bit-mask
// mode: xor OFF) or by ds_bpermute across the halves, so no exchange spends
// vector instructions on lane indices.
template <int OFF>
__device__ __forceinline__ double lane_xor(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    int lo2, hi2;
    if constexpr (OFF == 32) {
        const int addr = (int)((threadIdx.x & 63) ^ 32) << 2;
        lo2 = __builtin_amdgcn_ds_bpermute(addr, lo);
        hi2 = __builtin_amdgcn_ds_bpermute(addr, hi);
    } else {
        constexpr int pat = (OFF << 10) | 0x1F;  // and 0x1F, or 0, xor OFF
        lo2 = __builtin_amdgcn_ds_swizzle(lo, pat);
        hi2 = __builtin_amdgcn_ds_swizzle(hi, pat);
    }
    return __hiloint2double(hi2, lo2);
}

// v plus the v of lane ^ OFF: a butterfly step (the same pairs as
// __shfl_xor, so the same sums bit for bit).
template <int OFF>
__device__ __forceinline__ double xor_add(double v)
{
    return v + lane_xor<OFF>(v);
}

// One recursive-halving step over K values at lane distance D: the lane whose
// bit D is clear keeps the first half (adding its partner's first half), the
// other keeps the second half (stored first), so half as many values go
// through the exchange as in a butterfly over all of them.
template <int K, int D>
__device__ __forceinline__ void halve(double (&w)[K])
{
    const bool upper = (threadIdx.x & D) != 0;
#pragma unroll
    for (int i = 0; i < K / 2; ++i) {
        const double keep = upper ? w[i + K / 2] : w[i];
        const double send = upper ? w[i] : w[i + K / 2];
        w[i] = keep + lane_xor<D>(send);
    }
}

// Sums over the 64 lanes of the wave of K values per lane (K = 4 or 8):
// recursive halving over the top log2 K lane bits, then butterfly steps over
// the rest.  On return lane l holds the sum of value l >> (6 - log2 K), so the
// lanes l with l % (64 / K) == 0 hold one sum each.  A fixed order of
// additions: the same sums in every run.
template <int K>
__device__ __forceinline__ double wave_sums_split(double (&w)[K])
{
    static_assert(K == 4 || K == 8, "K = 4 or 8");
    double r;
    if constexpr (K == 8) {
        halve<8, 32>(w);
        double u[4] = {w[0], w[1], w[2], w[3]};
        halve<4, 16>(u);
        double z[2] = {u[0], u[1]};
        halve<2, 8>(z);
        r = xor_add<4>(z[0]);
    } else {
        halve<4, 32>(w);
        double z[2] = {w[0], w[1]};
        halve<2, 16>(z);
        r = xor_add<8>(z[0]);
        r = xor_add<4>(r);
    }
    r = xor_add<2>(r);
    return xor_add<1>(r);
}

// Sum of v over the 64 lanes of the wave, in every lane.
__device__ __forceinline__ double wave_total(double v)
{
    v = xor_add<32>(v);
    v = xor_add<16>(v);
    v = xor_add<8>(v);
    v = xor_add<4>(v);
    v = xor_add<2>(v);
    return xor_add<1>(v);
}

// Bit `lane` of the wave-uniform mask m selects a (set) or b, as one
// v_cndmask with m as its lane mask.
__device__ __forceinline__ uint32_t lane_select(uint64_t m, uint32_t a, uint32_t b)
{
    return __builtin_amdgcn_inverse_ballot_w64(m) ? a : b;
}
// Bit `lane` of the wave-uniform mask m, as a lane predicate (m itself serves
// as the mask of a branch or a select: no vector instruction)
__device__ __forceinline__ bool lane_bit(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// ------------------------------------------------------- union-find in LDS
__device__ __forceinline__ uint32_t lds_load(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x with path halving (x skips to its grandparent at every step);
// the stores are benign for the same reason as in global memory below.
__device__ __forceinline__ uint32_t find_lds(uint32_t *lab, uint32_t x)
{
    while (true) {
        const uint32_t p = lds_load(&lab[x]);
        if (p == x) return x;
        const uint32_t g = lds_load(&lab[p]);
        if (g == p) return p;
        __hip_atomic_store(&lab[x], g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = g;
    }
}

__device__ void union_lds(uint32_t *lab, uint32_t a, uint32_t b)
{
    while (true) {
        a = find_lds(lab, a);
        b = find_lds(lab, b);
        if (a == b) return;
        if (a > b) {
            const uint32_t tmp = a;
            a = b;
            b = tmp;
        }
        const uint32_t old = atomicMin(&lab[b], a);
        if (old == b) return;
        b = old;  // b was hooked meanwhile: merge a with its new parent
    }
}

// --------------------------------------- hand-off between blocks of a launch
// Data one block of a launch hands to another: stored with agent-scope
// (relaxed atomic) accesses, which are coherent across the chip's L2 caches,
// completed (stores_done) before the block signals with an atomic, and read
// with agent-scope loads by a block that has seen the signal.  No L2
// write-back or invalidation is needed: the plain stores and loads of a
// launch stay in the L2 of their own XCD.
template <typename T>
__device__ __forceinline__ void st_agent(XY_G T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_agent(const XY_G T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Waits until every store of the thread is complete (the agent-scope ones are
// then visible to every block); the compiler moves no access across it.
__device__ __forceinline__ void stores_done()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// ------------------------------------------- forest of boundary components
// Entry of node n: (key << 32) | parent.  A root is its own parent; a parent's
// key is never larger than its child's, so a root carries the smallest key,
// i.e. the smallest site, of everything united under it.

// Root entries of nodes a and b, the two paths walked in step (their loads
// overlap), with intermediate pointer jumping: every node on a path is
// re-pointed at its grandparent.  An entry only ever moves to an ancestor in
// the same set and roots are never overwritten, so these plain stores are
// benign while other threads hook roots; a hook such a store may undo is
// always followed by the union of the hooked root's former parent.
__device__ void find_pair(XY_G unsigned long long *P, uint32_t a, uint32_t b, unsigned long long &ra,
                          unsigned long long &rb)
{
    unsigned long long ea = P[a], eb = P[b];
    uint32_t pa = a, pb = b;  // the nodes whose entries ea, eb are
    bool da = (uint32_t)ea == a, db = (uint32_t)eb == b;
    while (!(da && db)) {
        unsigned long long ga = 0, gb = 0;
        if (!da) ga = P[(uint32_t)ea];
        if (!db) gb = P[(uint32_t)eb];
        if (!da) {
            const uint32_t par = (uint32_t)ea;
            if ((uint32_t)ga == par) {
                da = true;
            } else {
                P[pa] = ga;
                pa = par;
            }
            ea = ga;
        }
        if (!db) {
            const uint32_t par = (uint32_t)eb;
            if ((uint32_t)gb == par) {
                db = true;
            } else {
                P[pb] = gb;
                pb = par;
            }
            eb = gb;
        }
    }
    ra = ea;
    rb = eb;
}

// Lock-free union: the root with the larger key is hooked under the other
// with a 64-bit atomic minimum.  If the hooked node stopped being a root
// meanwhile, the union continues with the parent it had got.
__device__ void union_nodes(XY_G unsigned long long *P, uint32_t a, uint32_t b)
{
    while (true) {
        unsigned long long ra, rb;
        find_pair(P, a, b, ra, rb);
        if (ra == rb) return;
        if (ra > rb) {
            const unsigned long long tmp = ra;
            ra = rb;
            rb = tmp;
        }
        const unsigned long long old =
            __hip_atomic_fetch_min(&P[(uint32_t)rb], ra, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == rb) return;
        a = (uint32_t)ra;
        b = (uint32_t)old;
    }
}

// Key (smallest site) of the cluster of node n; read only.
__device__ __forceinline__ uint32_t root_key(const XY_G unsigned long long *P, uint32_t n)
{
    unsigned long long e = P[n];
    while ((uint32_t)e != n) {
        n = (uint32_t)e;
        e = P[n];
    }
    return (uint32_t)(e >> 32);
}

// Flip coin of the cluster whose smallest site is key, in sweep t.
__device__ __forceinline__ bool coin_of(const RepDesc &R, uint32_t t, uint32_t key)
{
    const U4 o = philox4x32_10(key >> 7, R.rep, t, TAG_FLIP, (uint32_t)R.seed, (uint32_t)(R.seed >> 32));
    const uint32_t wi = (key >> 5) & 3u;
    const uint32_t w = wi == 0 ? o.x : wi == 1 ? o.y : wi == 2 ? o.z : o.w;
    return (w >> (key & 31u)) & 1u;
}

// --------------------------------------------- reductions (fixed order)
template <int K, int NW>
__device__ __forceinline__ void block_sum(double (&v)[K], double *red /* NW*K */)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_total(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[wave * K + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = red[k];
            for (int w2 = 1; w2 < NW; ++w2) s += red[w2 * K + k];
            v[k] = s;
        }
    }
}

// First half of block_sum: each wave's sums into red[wave * K + k]; after a
// later barrier the sums over the waves finish it (the tile kernel reuses a
// barrier it needs anyway).
template <int K>
__device__ __forceinline__ void wave_sums(double (&v)[K], double *red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if constexpr (K == 4 || K == 8) {
        // (v is consumed)
        const double r = wave_sums_split<K>(v);
        constexpr int S = 64 / K;
        if (lane % S == 0) red[wave * K + lane / S] = r;
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = wave_total(v[k]);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) red[wave * K + k] = v[k];
        }
    }
}

// The Fourier sums from a lane's column sums (v[4], v[5] over the rows it
// holds): every site of column x carries the same factor e^{i 2 pi x / L}.
template <typename IT>
__device__ __forceinline__ void fourier_terms(const RepDesc &R, IT x0, bool col, double (&v)[kNumSums])
{
    if (!col) return;
    const XY_G double *f = gmem(R.fourier) + 2 * (x0 + (IT)(threadIdx.x & 63));
    const double cs = f[0], sn = f[1];
    v[6] = v[4] * cs;
    v[7] = v[4] * sn;
    v[8] = v[5] * cs;
    v[9] = v[5] * sn;
}

__device__ __forceinline__ void store_partials(const RepDesc &R, int64_t lt, const double (&v)[kNumSums])
{
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kNumSums; ++k) gmem(R.partials)[k * R.ntiles + lt] = v[k];
    }
}

// Observables from the six sums (the definitions' formulas); one thread.
__device__ __forceinline__ void obs_from_sums(const double *S, double N, double beta, xy_obs *o)
{
    o->E = -(S[0] + S[2]) / N;
    o->m2 = (S[4] * S[4] + S[5] * S[5]) / (N * N);
    o->ex = S[0] / N;
    o->sx = S[1] / N;
    o->ey = S[2] / N;
    o->sy = S[3] / N;
    o->ups_x = o->ex - beta * N * o->sx * o->sx;
    o->mk2 = (S[6] * S[6] + S[7] * S[7] + S[8] * S[8] + S[9] * S[9]) / (N * N);
}

// --------------------------------------------------------------- init
__global__ __launch_bounds__(kThreads) void k_init_spins(const RepDesc *__restrict__ reps, int32_t r,
                                                          int32_t start)
{
    const RepDesc &R = reps[r];
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < R.N; i += stride) {
        double x = 1.0, y = 0.0;
        if (start == XY_START_HOT) disk_point(R.seed, R.rep, TAG_INIT, (uint32_t)i, 0u, false, &x, &y);
        R.c[i] = (float)x;
        R.s[i] = (float)y;
    }
}

// Edge copies (first column, then first row of every tile) of the current
// spins, for the sweep that comes next; needed whenever the host sets spins.
__global__ __launch_bounds__(128) void k_edge_refresh(const RepDesc *__restrict__ reps, int32_t r)
{
    const RepDesc &R = reps[r];
    const int64_t lt = blockIdx.x;
    const Tile<uint64_t> T = make_tile<uint64_t>(R, lt);
    float2 *e = R.edge[R.st->t & 1] + lt * (T.TH + T.TW);
    for (int k = threadIdx.x; k < T.TH + T.TW; k += blockDim.x) {
        const uint64_t i = k < T.TH ? T.site(k, 0) : T.site(0, k - T.TH);
        e[k] = make_float2(R.c[i], R.s[i]);
    }
    // the tile's edge arrival counts start at zero
    if (threadIdx.x < 2) R.ecnt[2 * lt + threadIdx.x] = 0u;
}

// (cos, sin)(2 pi x / L) of every column x, for the Fourier sums.
__global__ __launch_bounds__(kThreads) void k_init_fourier(const RepDesc *__restrict__ reps, int32_t r)
{
    const RepDesc &R = reps[r];
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < R.L; x += (int64_t)gridDim.x * kThreads) {
        double sn, cs;
        sincospi(2.0 * (double)x / (double)R.L, &sn, &cs);
        gmem(R.fourier)[2 * x] = cs;
        gmem(R.fourier)[2 * x + 1] = sn;
    }
}

__global__ void k_init_dir(const RepDesc *__restrict__ reps, int32_t nrep)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep) return;
    compute_direction(reps[r], reps[r].st->t);
}

// ----------------------------------------------------------- the tile kernel
// LDS: spin[(TH+1)*(TW+1)] float2 (tile + right halo column + bottom halo row;
//        after the link pass reused for lab[TW*TH] u32, the tile-local
//        union-find of the labelling, and the waves' column sums)
//      | bxm[TH], bym[TH] u64 row masks of active links
//      | rcoin[TH], scoin[4] u64 flip coins of rows and of edge positions
// BT = rows per wave known at compile time (tiles of 64 x NW*BT for NW waves;
// every loop over a wave's rows is unrolled and its independent loads are
// issued together); BT = 0 is the general path (4 waves) for lattices
// narrower than 64 and for batches of mixed tile shapes.
// The unions of the links over tile edge (tile lt, edge 0 right / 1 bottom)
// inside a labelling tile pass, by one wave, once both of its tiles have
// handed over their slots, nodes and link masks; tab: the wave's 64 words of
// LDS.
__device__ void edge_unions_in_pass(const RepDesc &R, int64_t lt, int edge, uint32_t *tab);

template <typename IT, int MODE, int BT, int NW>
// Occupancy target: 7 waves per SIMD with 32-bit site indices (at most 72
// VGPRs; 64 x 32 tiles take 18 KB of LDS per block), 6 with 64-bit indices,
// except for M_SPEC (7: its few spills cost less than the wave gained).
__global__ __launch_bounds__(NW * 64)
__attribute__((amdgpu_waves_per_eu(sizeof(IT) == 4 ? 7 : (MODE == M_SPEC ? 7 : 6)))) void k_tile(
    const RepDesc *__restrict__ reps, const uint32_t *__restrict__ tile_rep, int32_t nrep, int64_t gtile0,
    int64_t gtile_end, FlipArgs fa)
{
    // M_SPEC: flip of sweep t and the links of sweep t+1 for both betas the
    // PCC step after sweep t may choose, no labelling; M_PLSEL: labels of a
    // sweep from the link planes of the beta that was chosen
    constexpr bool FLIP = MODE == M_FLIP || MODE == M_FUSED || MODE == M_SPEC;
    constexpr bool BONDS = MODE == M_BONDS || MODE == M_FUSED || MODE == M_SPEC;
    constexpr bool CCL = MODE != M_FLIP && MODE != M_SPEC;
    constexpr bool NEXT = MODE == M_FUSED || MODE == M_SPEC;    // activates the links of sweep t+1
    constexpr bool FROM_PLANES = MODE == M_PLANES || MODE == M_PLSEL;
    constexpr bool FIXED = BT > 0;
    constexpr int BMAX = FIXED ? BT : 16;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NT = NW * 64;  // threads of the block: NW waves of BT rows (fixed tiles)
    constexpr int kPairSums = 4;  // link sums: cos and sin of the x links, of the y links
    __shared__ double red[NW * kPairSums];

    const int64_t gtile = gtile0 + xcd_item(blockIdx.x, 1, 0, gtile_end - gtile0);
    if (gtile >= gtile_end) return;
    int64_t lt;
    const RepDesc &R = rep_of(reps, tile_rep, nrep, gtile, lt);
    const Tile<IT> T = make_tile<IT>(R, lt);
    const int TW = FIXED ? 64 : T.TW, TH = FIXED ? NW * BT : T.TH, SS = TW + 1;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int B = FIXED ? BT : band_rows(TH), yb = wave * B;
    XY_G RepState *st = gmem(R.st);
    // site (yb + k, lane) belongs to this tile (always, for fixed tiles)
    auto own = [&](int k) -> bool { return FIXED || (yb + k < TH && lane < TW); };
    XY_G float *__restrict__ cp = gmem(R.c);
    XY_G float *__restrict__ sp = gmem(R.s);
    // with 64-bit site indices, per-site accesses add the tile's first site to
    // the (scalar) base and keep the offset inside the tile (below 2^21) 32-bit
    constexpr bool WIDE = sizeof(IT) == 8;
    XY_G float *__restrict__ cpw = cp + (WIDE ? T.base : (IT)0);
    XY_G float *__restrict__ spw = sp + (WIDE ? T.base : (IT)0);
    auto woff = [&](int k, int x) -> uint32_t { return (uint32_t)((yb + k) << T.log2L) + (uint32_t)x; };
    // the wave's own spins and labels first: their addresses do not depend on
    // the sweep counter, so these loads overlap its read
    float c0[BMAX], s0[BMAX];
    uint32_t lv[BMAX];  // labels of the flipped sweep (flip modes)

    if constexpr (!FROM_PLANES) {
#pragma unroll
        for (int k = 0; k < B; ++k) {
            if (own(k)) {
                if constexpr (WIDE) {
                    // (2^32-site lattices: each pass streams the arrays once,
                    // past caches far smaller than them)
                    const uint32_t i = woff(k, lane);
                    c0[k] = __builtin_nontemporal_load(&gel(cpw, i));
                    s0[k] = __builtin_nontemporal_load(&gel(spw, i));
                    if constexpr (FLIP)
                        lv[k] = __builtin_nontemporal_load(&gel(gmem((const uint16_t *)R.lab) + T.base, i));
                } else {
                    const IT i = T.site(yb + k, lane);
                    c0[k] = gel(cp, i);
                    s0[k] = gel(sp, i);
                    if constexpr (FLIP) lv[k] = gel(gmem((const uint16_t *)R.lab), i);
                }
            }
        }
    }
    const uint64_t t = cload(&R.st->t);
    const int par = (int)(t & 1);
    const uint64_t tb = NEXT ? t + 1 : t;  // sweep whose links this launch activates
    const int pb = (int)(tb & 1);

    // spin area: the spins with their halo; after the link pass the labelling's
    // union-find and the waves' column sums
    float2 *spin = (float2 *)smem;
    const int sarea = max((TH + 1) * SS * (int)sizeof(float2), TW * TH * (int)sizeof(uint32_t) + NT * 16);
    uint64_t *bxm = (uint64_t *)(smem + sarea);
    uint64_t *bym = bxm + TH;
    uint64_t *rcoin = bym + TH;   // TH words: coins of the tile's rows
    uint64_t *scoin = rcoin + TH; // 4 words: coins of the edge positions
    uint64_t *bxm2 = scoin + 4;   // M_SPEC: the row masks of the second beta
    uint64_t *bym2 = bxm2 + TH;
    uint32_t *lab_s = (uint32_t *)smem;  // after the link pass
    const int64_t ecount = TH + TW;

    if constexpr (FLIP) {
        const XY_G float2 *__restrict__ eg = gmem(R.edge[par]);
        const double rx = cload(&R.st->dir[par][0]), ry = cload(&R.st->dir[par][1]);
        // (2 a) r = a (2 r) exactly: doubling is exact in binary floating point
        const double rx2 = 2.0 * rx, ry2 = 2.0 * ry;
        const bool renorm = ((t + 1) % kRenormEvery) == 0;
        const uint32_t tf = (uint32_t)t;
        auto reflect = [&](bool f, float &c1, float &s1) {
            if (f) {
                const double c = c1, s = s1;
                const double a = c * rx + s * ry;
                c1 = (float)(c - a * rx2);
                s1 = (float)(s - a * ry2);
            }
        };
        auto renormalise = [&](float &c1, float &s1) {
            const double c = c1, s = s1;
            const double n = sqrt(c * c + s * s);
            c1 = (float)(c / n);
            s1 = (float)(s / n);
        };
        // halo: right column and bottom row of the neighbouring tiles (spins
        // before the sweep from their edge copies, coins from their edge-position
        // coins), flipped here exactly as their owners flip them
        const XY_G unsigned long long *__restrict__ ec = gmem(R.ecoin);
        float2 he = make_float2(0.f, 0.f);
        int hslot = -1;
        bool hcoin = false;
        if (wave == 0 && lane < TH) {
            const int64_t nt = T.right_tile();
            const int q = 2 * TW + lane;  // the neighbour's left column
            hcoin = (ec[nt * 4 + (q >> 6)] >> (q & 63)) & 1ull;
            he = ldf2(eg + nt * ecount + lane);
            hslot = lane * SS + TW;
        } else if (wave == 1 && lane < TW) {
            const int64_t nt = T.down_tile();
            hcoin = (ec[nt * 4] >> lane) & 1ull;  // the neighbour's top row
            he = ldf2(eg + nt * ecount + TH + lane);
            hslot = TH * SS + lane;
        }
        // coins of the clusters that reach the tile's edge (bit p of scoin: the
        // coin of edge position p, drawn after the merge; a boundary label
        // names its slot, itself an edge position), and of clusters inside the
        // tile (rooted at one of its sites): the Philox block holding a row's
        // sites, bit x of rcoin[y] for site (y, x).  For 64-column tiles the two
        // arrays are one bit string indexed by the label.
        if (threadIdx.x < 4) scoin[threadIdx.x] = ec[lt * 4 + threadIdx.x];
        if (threadIdx.x >= 64 && threadIdx.x < 64 + TH) {
            const int y = threadIdx.x - 64;
            const IT site0 = T.site(y, 0);
            const U4 o = philox4x32_10((uint32_t)(site0 >> 7), R.rep, tf, TAG_FLIP, (uint32_t)R.seed,
                                       (uint32_t)(R.seed >> 32));
            const uint32_t wi = (uint32_t)(site0 >> 5) & 3u;
            const uint32_t ws[4] = {o.x, o.y, o.z, o.w};
            const uint64_t two = ((uint64_t)(wi < 3 ? ws[wi + 1] : 0u) << 32) | ws[wi];
            rcoin[y] = two >> ((uint32_t)site0 & 31u);
        }
        if (hslot >= 0) {
            float c1 = he.x, s1 = he.y;
            reflect(hcoin, c1, s1);
            if (renorm) renormalise(c1, s1);
            spin[hslot] = make_float2(c1, s1);
        }
        __syncthreads();
        // the wave's sites: reflections, then (every kRenormEvery sweeps, the
        // same in every lane) the renormalisation, then the stores; the
        // spins of the sweep are updated in place
#pragma unroll
        for (int k = 0; k < B; ++k) {
            if (own(k)) {
                const uint32_t l = lv[k];
                bool f;
                if constexpr (FIXED) {
                    // (the bit field extract takes its offset modulo 32)
                    f = __builtin_amdgcn_ubfe(((const uint32_t *)rcoin)[l >> 5], l, 1u) != 0u;
                } else {
                    const uint32_t nsite = (uint32_t)(TW * TH), q = l - nsite;
                    f = l >= nsite ? ((scoin[q >> 6] >> (q & 63u)) & 1ull)
                                   : ((rcoin[l >> T.log2TW] >> (l & (uint32_t)(TW - 1))) & 1ull);
                }
                reflect(f, c0[k], s0[k]);
            }
        }
        if (renorm) {
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (own(k)) renormalise(c0[k], s0[k]);
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            if (own(k)) {
                const float c1 = c0[k], s1 = s0[k];
                // every site is stored, flipped or not: lines written in
                // part (cluster edges) cost the memory more than whole lines
                if constexpr (WIDE) {
                    // streaming stores (2^32-site lattices)
                    __builtin_nontemporal_store(c1, &gel(cpw, woff(k, lane)));
                    __builtin_nontemporal_store(s1, &gel(spw, woff(k, lane)));
                } else {
                    gel(cp, T.site(yb + k, lane)) = c1;
                    gel(sp, T.site(yb + k, lane)) = s1;
                }
                spin[(yb + k) * SS + lane] = make_float2(c1, s1);
            }
        }
        __syncthreads();
        // edge copies (first column, first row) of the flipped tile for sweep t+1
        XY_G float2 *en = gmem(R.edge[par ^ 1]) + lt * ecount;
        if (wave == 2 && lane < TH)
            stf2(en + lane, spin[lane * SS]);
        else if (wave == 3 && lane < TW)
            stf2(en + TH + lane, spin[lane]);
    } else if constexpr (MODE == M_BONDS) {
        // spins before the sweep: own sites from the planes, halo from edge copies
        const XY_G float2 *__restrict__ eg = gmem(R.edge[par]);
        if (wave == 0 && lane < TW)
            spin[TH * SS + lane] = ldf2(eg + T.down_tile() * ecount + TH + lane);
        else if (wave == 1 && lane < TH)
            spin[lane * SS + TW] = ldf2(eg + T.right_tile() * ecount + lane);
#pragma unroll
        for (int k = 0; k < B; ++k)
            if (own(k)) spin[(yb + k) * SS + lane] = make_float2(c0[k], s0[k]);
        __syncthreads();
    }

    // ---- link sums of the flipped tile and / or link activation of sweep tb
    double v[kPairSums] = {};
    double cs = 0.0, ss = 0.0;  // the lane's column sums of cos and sin
    // link masks of the wave's own rows, kept in scalar registers (fixed tiles)
    constexpr bool RMASK = FIXED && BONDS && CCL;
    bool two = false;  // M_SPEC: the PCC step after this sweep moves beta (two candidates)
    uint64_t xrow[RMASK ? BMAX : 1], yrow[RMASK ? BMAX : 1];
    if constexpr (FLIP || BONDS) {
        BondCtx ctx, ctx2;
        uint32_t key0 = 0, key1 = 0;
        if constexpr (BONDS) {
            ctx.rx = cload(&R.st->dir[pb][0]);
            ctx.ry = cload(&R.st->dir[pb][1]);
            ctx.beta = cload(&R.st->beta);
            ctx.rxf = (float)ctx.rx;
            ctx.ryf = (float)ctx.ry;
            ctx.ties = (unsigned long long *)&st->ties[pb];
            if constexpr (MODE == M_SPEC) {
                // the PCC step at the end of this sweep's window moves beta by
                // +-db (the finalisation's own expressions): links for both
                // candidates, the first as beta + db (or beta if no step ends)
                const double beta = ctx.beta;
                if (fa.window > 0 && cload(&R.st->acc_n) + 1 >= fa.window) {
                    double db = fa.dbeta0;
                    if (fa.halve_every > 0) {
                        const int64_t halvings = cload(&R.st->pcc_k) / fa.halve_every;
                        db = ldexp(fa.dbeta0, -(int)(halvings < 200 ? halvings : 200));
                    }
                    if (db < fa.dbeta_min) db = fa.dbeta_min;
                    two = true;
                    ctx.beta = beta + db;
                    ctx2 = ctx;
                    ctx2.beta = beta + (-db);
                    ctx2.bl = (float)(-2.0 * ctx2.beta * 1.4426950408889634);
                    ctx2.gw = (float)(1e-5 * (1.0 + ctx2.beta) * 4294967296.0);
                    ctx2.ties = (unsigned long long *)&st->ties_spec[1];
                }
                ctx.ties = (unsigned long long *)&st->ties_spec[0];
                if (lt == 0 && threadIdx.x == 0) st->beta_cand = ctx.beta;
            }
            ctx.bl = (float)(-2.0 * ctx.beta * 1.4426950408889634);
            ctx.gw = (float)(1e-5 * (1.0 + ctx.beta) * 4294967296.0);
            key0 = (uint32_t)R.seed;
            key1 = (uint32_t)(R.seed >> 32);
        }
        // the decisions of one row of links for the betas of c: margins
        // against the Philox words, the FP64 definition inside the guard band
        auto decide = [&](const BondCtx &c, float bai, float pr, float pd, uint32_t wx, uint32_t wy, float2 a,
                          float2 r, float2 d, uint64_t &mx, uint64_t &my) {
            const float dx = bond_margin(bai, pr, wx);
            const float dy = bond_margin(bai, pd, wy);
            mx = __ballot(dx < 0.0f);
            my = __ballot(dy < 0.0f);
            if (__ballot(fabsf(dx) <= c.gw) | __ballot(fabsf(dy) <= c.gw)) {
                // some lane inside the guard band (rare)
                bool xa = dx < 0.0f, ya = dy < 0.0f;
                if (fabsf(dx) <= c.gw) xa = bond_exact(a.x, a.y, r.x, r.y, c.rx, c.ry, c.beta, wx, c.ties);
                if (fabsf(dy) <= c.gw) ya = bond_exact(a.x, a.y, d.x, d.y, c.rx, c.ry, c.beta, wy, c.ties);
                mx = __ballot(xa);
                my = __ballot(ya);
            }
        };
        float padn = 0.0f;  // M_SPEC: projection of the row below
        U4 w = {0u, 0u, 0u, 0u};
        // a row's values below are the next row's own: carried, not recomputed
        double cdn = 0.0, sdn = 0.0;
        float badn = 0.0f;  // bl a of the row below
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int y = yb + k;
            if (!FIXED && y >= TH) break;
            uint64_t mx = 0, my = 0;  // active links of the row (BONDS)
            uint64_t mx2 = 0, my2 = 0;  // M_SPEC: for the second beta
            if (FIXED || lane < TW) {
                const float2 a = spin[y * SS + lane];
                const float2 r = spin[y * SS + lane + 1];
                const float2 d = spin[(y + 1) * SS + lane];
                if constexpr (FLIP) {
                    // FP64 link sums; fused multiply-adds (the sums are compared
                    // with a tolerance, not bit for bit)
                    const double ci = k == 0 ? (double)a.x : cdn, si = k == 0 ? (double)a.y : sdn;
                    const double cr = r.x, sr = r.y, cd = d.x, sd = d.y;
                    v[0] = fma(ci, cr, fma(si, sr, v[0]));
                    v[1] = fma(si, cr, fma(-ci, sr, v[1]));
                    v[2] = fma(ci, cd, fma(si, sd, v[2]));
                    v[3] = fma(si, cd, fma(-ci, sd, v[3]));
                    cs += ci;
                    ss += si;
                    cdn = cd;
                    sdn = sd;
                }
                if constexpr (BONDS) {
                    const IT gy = T.y0 + (IT)y;
                    // one Philox block serves the vertical site pair (2m, 2m+1)
                    if (FIXED ? (k % 2 == 0) : (k == 0 || (gy & 1) == 0))
                        w = philox4x32_10((uint32_t)(((gy >> 1) << T.log2L) + T.x0 + (IT)lane), R.rep,
                                          (uint32_t)tb, TAG_BOND, key0, key1);
                    // fixed tiles start on even rows and bands have an even
                    // number of rows, so the pair half is the row's parity in the band
                    const bool odd = FIXED && BT % 2 == 0 ? (k & 1) : (gy & 1);
                    const uint32_t wx = odd ? w.z : w.x;
                    const uint32_t wy = odd ? w.w : w.y;
                    if constexpr (MODE == M_SPEC) {
                        // projections shared by both betas
                        const float pa = k == 0 ? bond_proj(ctx, a) : padn;
                        const float pd = bond_proj(ctx, d), pr = bond_proj(ctx, r);
                        padn = pd;
                        decide(ctx, ctx.bl * pa, pr, pd, wx, wy, a, r, d, mx, my);
                        if (two) decide(ctx2, ctx2.bl * pa, pr, pd, wx, wy, a, r, d, mx2, my2);
                    } else {
                        const float bai = k == 0 ? ctx.bl * bond_proj(ctx, a) : badn;
                        const float ad = bond_proj(ctx, d);
                        badn = ctx.bl * ad;
                        decide(ctx, bai, bond_proj(ctx, r), ad, wx, wy, a, r, d, mx, my);
                    }
                }
            }
            if constexpr (BONDS) {
                if (lane == 0) {
                    bxm[y] = mx;
                    bym[y] = my;
                    if constexpr (MODE == M_SPEC) {
                        bxm2[y] = mx2;
                        bym2[y] = my2;
                    }
                }
                if constexpr (RMASK) {
                    xrow[k] = mx;
                    yrow[k] = my;
                }
            }
        }
    }
    // sums of the flipped tile.  The four link sums are reduced per wave now
    // and folded by thread 0 after the next barrier.  The column sums of cos
    // and sin go to the spin area after that barrier (the spins are read by
    // then), behind the edge-slot table; after the following barrier the last
    // wave adds them up per column, forms the four Fourier sums (every site of
    // column x carries e^{i 2 pi x / L}) and reduces those and the two site sums.
    double *colsum = (double *)(smem + (size_t)TW * TH * sizeof(uint32_t));
    auto fold_link_sums = [&]() {
        if (threadIdx.x < kPairSums) {
            const int k = threadIdx.x;
            double a = red[k];
#pragma unroll
            for (int w2 = 1; w2 < NW; ++w2) a += red[w2 * kPairSums + k];
            gmem(R.partials)[k * R.ntiles + lt] = a;
        }
        colsum[(wave * 64 + lane) * 2] = lane < TW ? cs : 0.0;
        colsum[(wave * 64 + lane) * 2 + 1] = lane < TW ? ss : 0.0;
    };
    auto fold_site_sums = [&]() {
        if (wave == NW - 1) {
            double f[6] = {colsum[lane * 2], colsum[lane * 2 + 1], 0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int w2 = 1; w2 < NW; ++w2) {
                f[0] += colsum[(w2 * 64 + lane) * 2];
                f[1] += colsum[(w2 * 64 + lane) * 2 + 1];
            }
            if (lane < TW) {
                const XY_G double *fo = gmem(R.fourier) + 2 * (T.x0 + (IT)lane);
                const double ck = fo[0], sk = fo[1];
                f[2] = f[0] * ck;
                f[3] = f[0] * sk;
                f[4] = f[1] * ck;
                f[5] = f[1] * sk;
            }
            double f8[8] = {f[0], f[1], f[2], f[3], f[4], f[5], 0.0, 0.0};
            const double r = wave_sums_split<8>(f8);
            if ((lane & 7) == 0 && lane < 48) gmem(R.partials)[(kPairSums + (lane >> 3)) * R.ntiles + lt] = r;
        }
    };
    // active-link bit planes of sweep tb from the row masks in LDS
    auto write_planes = [&](const uint64_t *xm, const uint64_t *ym, XY_G uint32_t *gbx, XY_G uint32_t *gby) {
        if (TW == 64) {
            for (int j = threadIdx.x; j < 2 * TH; j += NT) {
                const int y = j >> 1, half = j & 1;
                const IT word = (T.site(y, 0) >> 5) + (IT)half;
                gbx[word] = (uint32_t)(xm[y] >> (32 * half));
                gby[word] = (uint32_t)(ym[y] >> (32 * half));
            }
        } else {
            // narrow lattice (L < 64): the tile spans whole rows, so whole words
            const int nbits = TW * TH;
            const int nwords = nbits >= 32 ? nbits >> 5 : 1;
            for (int j = threadIdx.x; j < nwords; j += NT) {
                uint32_t vx = 0u, vy = 0u;
                for (int b = 0; b < 32; ++b) {
                    const int p = j * 32 + b;
                    if (p >= nbits) break;
                    const int y = p >> T.log2TW, x = p & (TW - 1);
                    vx |= (uint32_t)((xm[y] >> x) & 1ull) << b;
                    vy |= (uint32_t)((ym[y] >> x) & 1ull) << b;
                }
                const IT word = (T.base >> 5) + (IT)j;
                gbx[word] = vx;
                gby[word] = vy;
            }
        }
    };
    if constexpr (FLIP) {
        wave_sums<kPairSums>(v, red);
        if constexpr (!CCL) {
            __syncthreads();
            fold_link_sums();
            if constexpr (MODE == M_SPEC) {
                // the candidates' planes: the first in the slot of sweep t+1,
                // the second (if the step can move beta) in the spare planes
                write_planes(bxm, bym, gmem(R.bx[pb]), gmem(R.by[pb]));
                if (two) write_planes(bxm2, bym2, gmem(R.bxs), gmem(R.bys));
            }
            __syncthreads();
            fold_site_sums();
            return;
        }
    }
    if constexpr (MODE == M_PLSEL) {
        // the finalisation chose beta: the links of this sweep are the
        // planes of the candidate it matches; the second candidate's planes
        // are copied into the sweep's slot, and its near ties counted
        const bool second = cload(&R.st->beta) != cload(&R.st->beta_cand);
        XY_G uint32_t *gbx = gmem(R.bx[pb]), *gby = gmem(R.by[pb]);
        const XY_G uint32_t *sbx = second ? gmem((const uint32_t *)R.bxs) : gbx;
        const XY_G uint32_t *sby = second ? gmem((const uint32_t *)R.bys) : gby;
        if (TW == 64) {
            for (int y = threadIdx.x; y < TH; y += NT) {
                const IT word = T.site(y, 0) >> 5;
                const uint32_t x0 = sbx[word], x1 = sbx[word + 1], y0 = sby[word], y1 = sby[word + 1];
                bxm[y] = ((uint64_t)x1 << 32) | x0;
                bym[y] = ((uint64_t)y1 << 32) | y0;
                if (second) {
                    gbx[word] = x0;
                    gbx[word + 1] = x1;
                    gby[word] = y0;
                    gby[word + 1] = y1;
                }
            }
        } else {
            for (int y = threadIdx.x; y < TH; y += NT) {
                uint64_t mx = 0, my = 0;
                for (int x = 0; x < TW; ++x) {
                    const IT i = T.site(y, x);
                    mx |= (uint64_t)((sbx[i >> 5] >> (i & 31)) & 1u) << x;
                    my |= (uint64_t)((sby[i >> 5] >> (i & 31)) & 1u) << x;
                }
                bxm[y] = mx;
                bym[y] = my;
            }
            if (second) {
                __syncthreads();  // (uniform: second is the same in every thread)
                write_planes(bxm, bym, gbx, gby);
            }
        }
        if (lt == 0 && threadIdx.x == 0) {
            st->ties[pb] += st->ties_spec[second ? 1 : 0];
            st->ties_spec[0] = 0ull;
            st->ties_spec[1] = 0ull;
        }
    }
    if constexpr (MODE == M_PLANES) {
        const XY_G uint32_t *gbx = gmem(R.bx[pb]), *gby = gmem(R.by[pb]);
        for (int y = threadIdx.x; y < TH; y += NT) {
            uint64_t mx = 0, my = 0;
            for (int x = 0; x < TW; ++x) {
                const IT i = T.site(y, x);
                mx |= (uint64_t)((gbx[i >> 5] >> (i & 31)) & 1u) << x;
                my |= (uint64_t)((gby[i >> 5] >> (i & 31)) & 1u) << x;
            }
            bxm[y] = mx;
            bym[y] = my;
        }
    }
    if constexpr (!CCL) return;

    __syncthreads();
    if constexpr (FLIP) fold_link_sums();
    const uint32_t NONE = 0xFFFFFFFFu;
    if constexpr (BONDS) write_planes(bxm, bym, gmem(R.bx[pb]), gmem(R.by[pb]));

    // ---- in-tile labelling of sweep tb
    if (lt == 0 && threadIdx.x == 0) st->tl = tb;
    const uint64_t twmask = TW == 64 ? ~0ull : ((1ull << (TW & 63)) - 1ull);
    const uint64_t inner = twmask >> 1;  // link x -> x+1 stays inside the tile
    const uint64_t below = (1ull << lane) - 1ull;
    auto xrow_mask = [&](int k) -> uint64_t {
        if constexpr (RMASK) return xrow[k];
        else return uniform_u64(bxm[yb + k]);
    };
    auto yrow_mask = [&](int k) -> uint64_t {
        if constexpr (RMASK) return yrow[k];
        else return uniform_u64(bym[yb + k]);
    };
    // 1) each wave scans its band of rows top-down.  A run of x-links takes
    //    the smallest label among the runs above that it touches through a
    //    y-link (segmented prefix minimum over the run's lanes, then read at
    //    the run's last lane); a run touching two different labels records
    //    their union; a run touching none is labelled by its first site.
    //    Labels are sites of this band only, so the waves do not interact.
    uint32_t lprev = NONE;
    uint32_t pend = 0u;  // bit k: a union of row k is left to the loop after the scan
#pragma unroll
    for (int k = 0; k < B; ++k) {
        const int y = yb + k;
        if (!FIXED && y >= TH) break;
        const bool act = FIXED || lane < TW;
        const uint64_t xm = xrow_mask(k) & inner;
        const uint64_t ends = ~xm;  // bit x: the run through x ends at x
        const uint32_t end = (uint32_t)__builtin_ctzll(ends & ~below);
        // segmented minimum as an unsegmented maximum of (run index, 0xFFFF - label):
        // run indices grow with the lane, so a lane's prefix maximum comes from
        // its own run.  A lane offers the label above it (through a y-link) or
        // else its own site; labels above are smaller than the row's sites, so
        // the run's minimum is the smallest label above, or else its first site.
        // Labels of a tile are below 2^12.
        const uint64_t up = k > 0 ? yrow_mask(k - 1) : 0ull;  // lanes with a y-link from above
        const uint32_t c2 = lane_select(up, lprev, (uint32_t)(y * TW) + (uint32_t)lane);
        const uint32_t run_id = __builtin_amdgcn_mbcnt_hi((uint32_t)(ends >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)ends, 0u));
        const uint32_t key = (run_id << 16) | (0xFFFFu - c2);
        const uint32_t pm = (uint32_t)__builtin_amdgcn_ds_bpermute((int)end << 2, (int)wave_prefix_max(key));
        const uint32_t lab = 0xFFFFu - (pm & 0xFFFFu);
        if (act) lab_s[y * TW + lane] = lab;
        if (k > 0) {
            // a lane whose label above differs from its run's records their
            // union, unless its left neighbour in the run offers the same label
            // (lane 0 has no left neighbour: bit 0 of xm << 1 is clear, so its
            // cleft, zero, is never looked at)
            const uint32_t cleft =
                (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c2, 0x138, 0xf, 0xf, true);  // wave_shr:1
            const uint64_t need = up & __ballot(c2 != lab) & ~((xm << 1) & __ballot(cleft == c2));
            pend = lane_bit(need) ? pend | (1u << k) : pend;
        }
        lprev = lab;
    }
    // the unions the scan recorded, all rows in one loop: the site above and
    // the site itself stand for the two labels (every site's entry holds its
    // label, and the unions only ever point an entry at another member of
    // its set)
    while (pend) {
        const int k = __builtin_ctz(pend);
        pend &= pend - 1u;
        const uint32_t q = (uint32_t)((yb + k) * TW + lane);
        union_lds(lab_s, q - (uint32_t)TW, q);
    }
    __syncthreads();
    if constexpr (FLIP) fold_site_sums();
    // 2) the seams between bands: y-links from a wave's last row; a link
    //    whose left neighbour joins the same two runs is skipped
    {
        const int y = yb + B - 1;
        if (y < TH - 1 && (FIXED || lane < TW)) {
            const uint64_t vv = bym[y] & twmask;
            const uint64_t h0 = bxm[y] & inner, h1 = bxm[y + 1] & inner;
            const uint64_t need = vv & ~(vv & (vv << 1) & (h0 << 1) & (h1 << 1));
            if (lane_bit(need))
                union_lds(lab_s, (uint32_t)(y * TW + lane), (uint32_t)((y + 1) * TW + lane));
        }
    }
    __syncthreads();
    // 3) tile-local roots of the wave's sites, and of every edge position
    //    (one thread each) with the smallest edge position per root: the
    //    slot of a component that reaches the tile's edge
    //    Nothing is united any more, so the walks only read, and the rows'
    //    walks advance together (their loads of one step are issued at once).
    const int NB = R.nb;
    const int p = threadIdx.x;  // NB <= 256 edge positions
    uint32_t lr[BMAX], nx[BMAX];
    uint32_t proot = p < NB ? lds_load(&lab_s[T.edge_local(p)]) : 0u;
#pragma unroll
    for (int k = 0; k < B; ++k) lr[k] = own(k) ? lds_load(&lab_s[(yb + k) * TW + lane]) : 0u;
    uint32_t pnx = lds_load(&lab_s[proot]);
#pragma unroll
    for (int k = 0; k < B; ++k) nx[k] = lds_load(&lab_s[lr[k]]);
    while (true) {
        bool more = pnx != proot;
#pragma unroll
        for (int k = 0; k < B; ++k) more = more || nx[k] != lr[k];
        if (!more) break;
        if (pnx != proot) {
            proot = pnx;
            pnx = lds_load(&lab_s[proot]);
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            if (nx[k] != lr[k]) {
                lr[k] = nx[k];
                nx[k] = lds_load(&lab_s[lr[k]]);
            }
        }
    }
    // the smallest edge position of a root is marked in the root's own entry
    // (kMark | 255 - p, so the largest mark wins), once every walk is done
    constexpr uint32_t kMark = 0x80000000u;
    auto slot_of = [&](uint32_t root) -> uint32_t {
        const uint32_t m = lab_s[root];
        return m >= kMark ? 255u - (m & 0xFFu) : NONE;
    };
    __syncthreads();
    if (p < NB) atomicMax(&lab_s[proot], kMark | (255u - (uint32_t)p));
    __syncthreads();
    // 4) edge slots and boundary nodes of the tile
    //    (with fa.inpass other blocks of this launch read them: agent-scope
    //    stores; plain ones otherwise, which the L2 combines)
    auto put = [&](auto *p, auto v) {
        if (fa.inpass) st_agent(p, v);
        else *p = v;
    };
    if (p < NB) {
        const uint32_t sl = slot_of(proot);
        const int64_t nbase = lt * NB;
        put(gmem(R.bslot) + nbase + p, (uint8_t)sl);
        if (sl == (uint32_t)p)
            put(gmem(R.node) + nbase + p,
                ((unsigned long long)(uint32_t)T.site_of_local((int)proot) << 32) | (uint32_t)(nbase + p));
    }
    //    and the links over the right and bottom edges
    if (wave == 0) {
        const bool xr = lane < TH && ((bxm[lane] >> (TW - 1)) & 1ull);
        const uint64_t xm = __ballot(xr);
        if (lane == 0) {
            XY_G unsigned long long *cr = gmem(R.cross);
            put(cr + 2 * lt, (unsigned long long)xm);
            put(cr + 2 * lt + 1, (unsigned long long)(bym[TH - 1] & twmask));
        }
    }
    // 5) tile-local labels.  The lane index is taken afresh (mbcnt) so that
    //    the site offsets of the first loads need not stay live through the
    //    kernel.
    XY_G uint16_t *labn = gmem(R.lab);
    const int lane2 = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
#pragma unroll
    for (int k = 0; k < B; ++k) {
        if (own(k)) {
            const uint32_t sl = slot_of(lr[k]);
            const uint16_t v = (uint16_t)(sl != NONE ? (uint32_t)(TW * TH) + sl : lr[k]);
            if constexpr (WIDE) __builtin_nontemporal_store(v, &gel(labn + T.base, woff(k, lane2)));
            else gel(labn, T.site(yb + k, lane2)) = v;
        }
    }
    if (!fa.inpass) return;
    // 6) with fa.inpass the tile edges are united in this pass instead of by
    //    a merge kernel.  Once the tile's slots, nodes and masks above are
    //    complete (waited for after the labels, so that the stores of both
    //    overlap), the tile counts itself at the four edges it touches (its
    //    right and bottom edges, the left tile's right edge, the upper tile's
    //    bottom edge); the second of an edge's two tiles to arrive unites that
    //    edge (one wave per edge) and clears its count for the next sweep.
    //    No block waits for another.
    __shared__ int64_t edge_owner[4];
    __shared__ int edge_go[4];
    stores_done();
    __syncthreads();
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;
        const int64_t owner = q < 2 ? lt : q == 2 ? T.left_tile() : T.up_tile();
        XY_G uint32_t *cnt = gmem(R.ecnt) + 2 * owner + (q & 1);
        const uint32_t before = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (before == 1u) st_agent(cnt, 0u);
        edge_owner[q] = owner;
        edge_go[q] = before == 1u;
    }
    __syncthreads();
    if (wave < 4 && edge_go[wave]) edge_unions_in_pass(R, edge_owner[wave], wave & 1, (uint32_t *)smem + wave * 64);
}

// ------------------------------------------------- merge across tiles
// One wave per tile edge (0: right, TH links; 1: bottom, TW links).  Every
// active link over the edge unites the boundary nodes of its two end
// components, once per distinct pair of nodes in the wave.  Reads
// are contiguous (the edge's link mask and the two rows of edge slots); the
// unions touch only the forest of boundary nodes.
__device__ void finish_sweep(const RepDesc &R, const FlipArgs &fa, xy_obs *measure_out, const double (&tot)[kNumSums]);

// Finalisation of a sweep in two stages, the same arithmetic on every path:
// (1) one block per chunk of kFinSpan tiles sums the tiles' partials;
// (2) one block per replica sums the chunks and finishes the sweep.  After a
// fused flip both run beside work that runs anyway (stage 1 in the first
// blocks of the merge, stage 2 in the first blocks of the edge coins); on its
// own, k_finalize runs stage 1 and the last block of each replica stage 2.
template <int U = 4, int KG = kNumSums>
__device__ __forceinline__ void fin_chunk(const RepDesc *__restrict__ reps, const uint32_t *__restrict__ fin_rep,
                                          int32_t nrep, int64_t b, double *red, bool agent = false);
__device__ __forceinline__ void fin_replica(const RepDesc &R, const FlipArgs &fa, xy_obs *measure_out, double *red,
                                            bool agent = false);

// cut 0: the sweep's forest.  cut 1 / 2 (wrapping check): the copy node_cut[0]
// / node_cut[1] of the forest, merged without the links that cross the
// lattice's seam along x (right edges of the last tile column) / along y
// (bottom edges of the last tile row).
// The unions of tile edge gw (2 x tile + 0: right edge, + 1: bottom edge).
// One tile edge of the merge: the lane's link over it (the node pair its two
// end components are slots of) and the node array the unions go to.
struct EdgeLinks {
    uint32_t a, b;                  // boundary nodes of the link's two ends
    uint64_t m;                     // the edge's active links (bit = lane)
    bool on;                        // the lane's link is active and not cut
    int nlinks;                     // links over the edge
    XY_G unsigned long long *P;     // forest the unions go to
};

template <bool CUT>
__device__ __forceinline__ EdgeLinks edge_links(const RepDesc *__restrict__ reps,
                                                const uint32_t *__restrict__ tile_rep, int32_t nrep, int64_t gtile0,
                                                int64_t gw, int32_t next_dir, int32_t cut)
{
    const int lane = threadIdx.x & 63;
    const int64_t gtile = gtile0 + (gw >> 1);
    const int edge = (int)(gw & 1);
    int64_t lt;
    const RepDesc &R = rep_of(reps, tile_rep, nrep, gtile, lt);
    const Tile<uint64_t> T = make_tile<uint64_t>(R, lt);
    const int NB = R.nb;
    EdgeLinks e;
    e.nlinks = edge ? T.TW : T.TH;
    e.a = 0;
    e.b = 0;
    if (lane < e.nlinks) {  // read with the link mask, not after it
        const XY_G uint8_t *bsl = gmem(R.bslot);
        const int64_t nt = edge ? T.down_tile() : T.right_tile();
        const int pa = edge ? T.TW + lane : 2 * T.TW + T.TH + lane;  // own bottom row / right column
        const int pn = edge ? lane : 2 * T.TW + lane;                 // neighbour's top row / left column
        e.a = (uint32_t)(lt * NB) + bsl[lt * NB + pa];
        e.b = (uint32_t)(nt * NB) + bsl[nt * NB + pn];
    }
    e.m = gmem(R.cross)[2 * lt + edge];
    const bool seam =
        CUT && ((cut == 1 && edge == 0 && T.tx == T.ntx - 1) || (cut == 2 && edge == 1 && T.ty == T.nty - 1));
    e.on = !seam && lane < e.nlinks && ((e.m >> lane) & 1ull);
    e.P = gmem(CUT ? R.node_cut[cut - 1] : R.node);
    // mirror direction of the sweep after the one labelled last
    if (next_dir && lt == 0 && edge == 0 && lane == 0) compute_direction(R, R.st->tl + 1);
    return e;
}

// Does the lane lead the union of its pair?  dedup 0: one union per distinct
// pair of the edge (the lowest lane holding a pair not seen yet leads it, and
// every lane with the same pair drops out); dedup 1: a lane drops out only
// when the lane before it holds the same pair (a tuning choice: the
// partition, and so every root and coin, is the same either way).
// dedup 2: one lane per pair found through a 64-entry table in the wave's
// LDS (tab): every lane whose link asks for a union writes its index to the
// entry its pair hashes to (the lowest lane wins) and leads if it won or if
// the winner holds another pair (a collision: then copies of that pair may
// all lead, and a union repeated changes nothing).
template <int DEDUP>
__device__ __forceinline__ bool leads(const EdgeLinks &e, uint32_t *tab)
{
    const int lane = threadIdx.x & 63;
    bool lead = false;
    if constexpr (DEDUP == 2) {
        const bool want = e.on && e.a != e.b;
        tab[lane] = 64u;
        const uint32_t h = ((e.a ^ (e.b << 7)) * 0x9E3779B1u) >> 26;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (want) __hip_atomic_fetch_min(&tab[h], (uint32_t)lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t w = want ? tab[h] & 63u : (uint32_t)lane;
        const uint32_t wa = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(w << 2), (int)e.a);
        const uint32_t wb = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(w << 2), (int)e.b);
        lead = want && (w == (uint32_t)lane || wa != e.a || wb != e.b);
    } else if constexpr (DEDUP == 0) {
        uint64_t todo = __ballot(e.on && e.a != e.b);
        while (todo) {
            const int l = __ffsll((long long)todo) - 1;
            const uint32_t la = __shfl(e.a, l), lb = __shfl(e.b, l);
            lead = lead || lane == l;
            todo &= ~__ballot(e.on && e.a == la && e.b == lb);
        }
    } else {
        const uint32_t pa = __shfl_up(e.a, 1), pb = __shfl_up(e.b, 1);
        const bool prev_on = lane > 0 && ((e.m >> (lane - 1)) & 1ull) && lane - 1 < e.nlinks;
        lead = e.on && e.a != e.b && !(prev_on && pa == e.a && pb == e.b);
    }
    return lead;
}

__device__ void edge_unions_in_pass(const RepDesc &R, int64_t lt, int edge, uint32_t *tab)
{
    const int lane = threadIdx.x & 63;
    const Tile<uint64_t> T = make_tile<uint64_t>(R, lt);
    const int NB = R.nb;
    EdgeLinks e;
    e.nlinks = edge ? T.TW : T.TH;
    e.a = 0;
    e.b = 0;
    // the two tiles' slots and the owner's mask, stored by blocks of this
    // launch: agent-scope loads
    const XY_G uint8_t *bsl = gmem(R.bslot);
    const int64_t nt = edge ? T.down_tile() : T.right_tile();
    if (lane < e.nlinks) {
        const int pa = edge ? T.TW + lane : 2 * T.TW + T.TH + lane;  // own bottom row / right column
        const int pn = edge ? lane : 2 * T.TW + lane;                 // neighbour's top row / left column
        e.a = (uint32_t)(lt * NB) + ld_agent(bsl + lt * NB + pa);
        e.b = (uint32_t)(nt * NB) + ld_agent(bsl + nt * NB + pn);
    }
    e.m = ld_agent(gmem(R.cross) + 2 * lt + edge);
    e.on = lane < e.nlinks && ((e.m >> lane) & 1ull);
    e.P = gmem(R.node);
    if (leads<2>(e, tab)) union_nodes(e.P, e.a, e.b);
}

// DEDUP and EPW: the merge schedule (pair deduplication, tile edges per
// wave); CUT: a forest copy of the wrapping check (cut 1 or 2)
template <int DEDUP, int EPW, bool CUT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_merge(
    const RepDesc *__restrict__ reps, const uint32_t *__restrict__ tile_rep, const uint32_t *__restrict__ fin_rep,
    int32_t nrep, int64_t gtile0, int64_t gtile_end, int32_t next_dir, int64_t nfin, int32_t cut)
{
    // the first nfin blocks: deferred finalisation, stage 1 (chunk c of
    // replica r; first in the grid, so that they overlap the unions)
    if (blockIdx.x < nfin) {
        __shared__ double red[kWaves * kNumSums];
        fin_chunk(reps, fin_rep, nrep, blockIdx.x, red);
        return;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (blockIdx.x < xcd_pad(nfin)) return;
    const int64_t nw = 2 * (gtile_end - gtile0);  // tile edges
    if constexpr (EPW == 1) {
        const int64_t gw = xcd_item(blockIdx.x - xcd_pad(nfin), kWaves, wave, nw);
        if (gw >= nw) return;
        const EdgeLinks e = edge_links<CUT>(reps, tile_rep, nrep, gtile0, gw, next_dir, cut);
        __shared__ uint32_t tab_s[DEDUP == 2 ? kWaves * 64 : 1];
        if (leads<DEDUP>(e, tab_s + (DEDUP == 2 ? wave * 64 : 0))) union_nodes(e.P, e.a, e.b);
    } else {
        // EPW tile edges per wave: their links read together, then the
        // leading pairs of all of them packed into the wave's lanes (through
        // its part of LDS), so that their unions run side by side rather
        // than one edge after the other
        __shared__ uint2 pair_s[kWaves][EPW * 64];
        __shared__ uint8_t edge_s[kWaves][EPW * 64];
        __shared__ uint32_t tab_s[DEDUP == 2 ? kWaves * 64 : 1];
        EdgeLinks e[EPW];
        int ne = 0;  // edges of this wave (the same in every lane)
#pragma unroll
        for (int q = 0; q < EPW; ++q) {
            const int64_t gw = xcd_item(blockIdx.x - xcd_pad(nfin), kWaves * EPW, wave * EPW + q, nw);
            if (gw >= nw) break;
            e[q] = edge_links<CUT>(reps, tile_rep, nrep, gtile0, gw, next_dir, cut);
            ne = q + 1;
        }
        uint32_t n = 0;  // pairs packed (the same in every lane)
#pragma unroll
        for (int q = 0; q < EPW; ++q) {
            if (q >= ne) break;
            const bool lead = leads<DEDUP>(e[q], tab_s + (DEDUP == 2 ? wave * 64 : 0));
            const uint64_t bm = __ballot(lead);
            if (lead) {
                const uint32_t r =
                    n + __builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
                pair_s[wave][r] = make_uint2(e[q].a, e[q].b);
                edge_s[wave][r] = (uint8_t)q;
            }
            n += (uint32_t)__popcll(bm);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (uint32_t j = (uint32_t)lane; j < n; j += 64) {
            const uint2 pr = pair_s[wave][j];
            const int q = edge_s[wave][j];
            XY_G unsigned long long *P = e[0].P;
#pragma unroll
            for (int q2 = 1; q2 < EPW; ++q2)
                if (q == q2) P = e[q2].P;
            union_nodes(P, pr.x, pr.y);
        }
    }
}

// ------------------------------------------------- coins of edge positions
// After the merge: every used slot (the smallest edge position of its tile
// component) finds the smallest site of its cluster and draws that cluster's
// flip coin; then every edge position takes the coin of its slot.  Bit p of
// ecoin[4 * tile + p / 64] is the coin of the cluster at edge position p (a
// boundary label's slot is itself an edge position).  One wave per tile: lane
// l holds positions l, l + 64, l + 128, l + 192 (NB <= 256), walks their
// paths to the roots together, and the coins are exchanged by ballots.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_resolve(const RepDesc *__restrict__ reps,
                                                       const uint32_t *__restrict__ tile_rep, int32_t nrep,
                                                       int64_t gtile0, int64_t gtile_end, int64_t nfin, FlipArgs fa,
                                                       const uint32_t *__restrict__ fin_rep, int32_t inpass)
{
    // the first nfin blocks: deferred finalisation (first in the grid, to
    // overlap the coins).  inpass == 0: stage 2 (the chunks of replica r,
    // then the sweep); the merge kernel ran stage 1.  inpass != 0: no merge
    // kernel ran: block b sums chunk b (stage 1), hands it over with an
    // agent-scope store and counts itself in its replica's fin_done; the
    // block that completes the count runs stage 2 and clears it.
    if (blockIdx.x < nfin) {
        __shared__ double red[kWaves * kNumSums];
        if (!inpass) {
            fin_replica(reps[blockIdx.x], fa, nullptr, red);
            return;
        }
        __shared__ int last;
        // (four tiles per thread for four sums at a time: the kernel is held
        // to 64 VGPRs)
        fin_chunk<4, 4>(reps, fin_rep, nrep, blockIdx.x, red, true);
        const RepDesc &R = reps[nrep == 1 ? 0 : fin_rep[blockIdx.x]];
        if (threadIdx.x == 0) {
            stores_done();
            const uint32_t done = __hip_atomic_fetch_add(&R.st->fin_done, 1u, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
            last = done + 1 == (uint32_t)R.fin_chunks;
            if (last) __hip_atomic_store(&R.st->fin_done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (last) fin_replica(R, fa, nullptr, red, true);
        return;
    }
    constexpr int G = 4;  // groups of 64 edge positions
    const int lane = threadIdx.x & 63;
    if (blockIdx.x < xcd_pad(nfin)) return;
    const int64_t gtile =
        gtile0 + xcd_item(blockIdx.x - xcd_pad(nfin), kWaves, threadIdx.x >> 6, gtile_end - gtile0);
    if (gtile >= gtile_end) return;
    int64_t lt;
    const RepDesc &R = rep_of(reps, tile_rep, nrep, gtile, lt);
    // mirror direction of the sweep after the one labelled last (drawn by
    // the merge kernel when there is one)
    if (inpass && lt == 0 && lane == 0) compute_direction(R, R.st->tl + 1);
    const int NB = R.nb;
    const XY_G uint8_t *bs = gmem(R.bslot) + lt * NB;
    const XY_G unsigned long long *P = gmem(R.node);
    uint32_t sl[G], n[G];
    unsigned long long e[G];
    bool used[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int p = g * 64 + lane;
        sl[g] = p < NB ? bs[p] : 0u;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int p = g * 64 + lane;
        used[g] = p < NB && sl[g] == (uint32_t)p;
        n[g] = (uint32_t)(lt * NB + p);
        e[g] = used[g] ? P[n[g]] : 0ull;
    }
    // roots: a root's entry names itself and holds the cluster's smallest site
    while (true) {
        bool more = false;
#pragma unroll
        for (int g = 0; g < G; ++g) more = more || (used[g] && (uint32_t)e[g] != n[g]);
        if (!__ballot(more)) break;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (used[g] && (uint32_t)e[g] != n[g]) {
                n[g] = (uint32_t)e[g];
                e[g] = P[n[g]];
            }
        }
    }
    const uint64_t t = cload(&R.st->tl);  // the sweep labelled last
    // the used slots' keys packed in rank order into the wave's part of LDS,
    // so that the Philox blocks of the coins run once per 64 used slots
    // rather than once per group of 64 positions
    __shared__ uint32_t keys_s[kWaves * G * 64];
    uint32_t *ks = keys_s + (threadIdx.x >> 6) * (G * 64);
    uint32_t rank[G];
    uint32_t nused = 0;  // the same in every lane
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint64_t bm = __ballot(used[g]);
        rank[g] = nused + __builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
        if (used[g]) ks[rank[g]] = (uint32_t)(e[g] >> 32);
        nused += (uint32_t)__popcll(bm);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint64_t cb[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        const uint32_t r = (uint32_t)(q * 64 + lane);
        cb[q] = (uint32_t)(q * 64) < nused ? __ballot(r < nused && coin_of(R, (uint32_t)t, ks[r])) : 0ull;
    }
    uint64_t cm[G];  // bit l of cm[g]: the coin of used position g * 64 + l
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t q = rank[g] >> 6;
        const uint64_t w = q == 0 ? cb[0] : q == 1 ? cb[1] : q == 2 ? cb[2] : cb[3];
        cm[g] = __ballot(used[g] && ((w >> (rank[g] & 63u)) & 1ull));
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t q = sl[g] >> 6;
        const uint64_t w = q == 0 ? cm[0] : q == 1 ? cm[1] : q == 2 ? cm[2] : cm[3];
        const uint64_t m2 = __ballot(g * 64 + lane < NB && ((w >> (sl[g] & 63u)) & 1ull));
        if (lane == 0) gmem(R.ecoin)[lt * 4 + g] = m2;
    }
}

// ------------------------------------------------- wrapping check
// Does some cluster of the sweep labelled last wind around the periodic
// lattice?  Along x: cut the torus open along its x seam (the links from
// column L-1 to column 0 removed: the forest copy merged with cut 1).  Every
// cluster of the torus falls into clusters of the cut lattice ("sheets"), and
// the seam links join sheets: link (L-1, y) -> (0, y) steps from the sheet of
// its left end to the sheet of its right end, one column further along x.
// Give every sheet a potential phi (unwrapped x offset in units of L) with
// phi(right end's sheet) = phi(left end's sheet) + 1 along every active seam
// link: a cluster winds along x exactly when some closed walk over sheets and
// seam links crosses the seam a nonzero net number of times, i.e. when no
// potentials satisfy every seam link of it.  The block propagates the
// smallest sheet id of each cluster over the seam links together with the
// potential it implies (a sheet takes both from a neighbour only when the id
// is smaller than its own, so ids and potentials settle), then checks every
// seam link.  Along y the same with cut 2 and the links (x, L-1) -> (x, 0).
// First the forest copies, taken before the sweep's forest is merged; the
// replica's wrap bits of the sweep start as 4 (checked).
__global__ __launch_bounds__(kThreads) void k_copy_nodes(const RepDesc *__restrict__ reps,
                                                          const uint32_t *__restrict__ tile_rep, int32_t nrep,
                                                          int64_t gtile0)
{
    int64_t lt;
    const RepDesc &R = rep_of(reps, tile_rep, nrep, gtile0 + blockIdx.x, lt);
    const int NB = R.nb;
    const XY_G unsigned long long *src = gmem(R.node) + lt * NB;
    XY_G unsigned long long *d0 = gmem(R.node_cut[0]) + lt * NB;
    XY_G unsigned long long *d1 = gmem(R.node_cut[1]) + lt * NB;
    for (int p = threadIdx.x; p < NB; p += kThreads) {
        const unsigned long long v = src[p];
        d0[p] = v;
        d1[p] = v;
    }
    if (lt == 0 && threadIdx.x == 0) {
        XY_G RepState *st = gmem(R.st);
        st->wrap[st->tl & 1] = 4u;
    }
}

// A check whose propagation found no settled state within its round limit
// (cannot happen: every round with a change lowers some sheet's id) is
// reported with bit 8 instead of looping on.
constexpr uint32_t kWrapUnsettled = 8u;

__global__ __launch_bounds__(kThreads) void k_wrap(const RepDesc *__restrict__ reps)
{
    const int d = blockIdx.x & 1;  // 0: along x, 1: along y
    const RepDesc &R = reps[blockIdx.x >> 1];
    __shared__ uint32_t ra[kWrapMaxL], rb[kWrapMaxL];  // sheets of the seam links' ends
    __shared__ int changed, wound;
    const int64_t L = R.L;
    const int TW = R.TW, TH = R.TH, NB = R.nb, log2TW = R.log2TW, log2TH = __ffs(TH) - 1;
    XY_G RepState *st = gmem(R.st);
    const uint64_t tl = st->tl;
    const XY_G uint8_t *bsl = gmem(R.bslot);
    const XY_G unsigned long long *P = gmem(R.node_cut[d]);
    XY_G unsigned long long *S = gmem(R.pstate[d]);
    const XY_G uint32_t *plane = gmem(d == 0 ? R.bx[tl & 1] : R.by[tl & 1]);
    constexpr uint32_t NONE = 0xFFFFFFFFu;
    constexpr uint32_t kBias = 0x80000000u;
    // forest node of the edge position p of tile lt, followed to its root
    auto sheet = [&](int64_t lt, int p) -> uint32_t {
        uint32_t n = (uint32_t)(lt * NB) + bsl[lt * NB + p];
        unsigned long long e = P[n];
        while ((uint32_t)e != n) {
            n = (uint32_t)e;
            e = P[n];
        }
        return n;
    };
    for (int64_t j = threadIdx.x; j < L; j += kThreads) {
        // the seam link from a = (xa, ya) to b = (xb, yb)
        const int64_t xa = d == 0 ? L - 1 : j, ya = d == 0 ? j : L - 1;
        const int64_t xb = d == 0 ? 0 : j, yb = d == 0 ? j : 0;
        const int64_t ia = ya * L + xa;
        uint32_t u = NONE, v = NONE;
        if ((plane[ia >> 5] >> (ia & 31)) & 1u) {
            const int64_t lta = (ya >> log2TH) * R.ntx + (xa >> log2TW);
            const int64_t ltb = (yb >> log2TH) * R.ntx + (xb >> log2TW);
            // a: right column / bottom row of its tile; b: left column / top row
            const int pa = d == 0 ? 2 * TW + TH + (int)(ya & (TH - 1)) : TW + (int)(xa & (TW - 1));
            const int pb = d == 0 ? 2 * TW + (int)(yb & (TH - 1)) : (int)(xb & (TW - 1));
            u = sheet(lta, pa);
            v = sheet(ltb, pb);
        }
        ra[j] = u;
        rb[j] = v;
    }
    __syncthreads();
    for (int64_t j = threadIdx.x; j < L; j += kThreads) {
        if (ra[j] != NONE) {
            S[ra[j]] = ((unsigned long long)ra[j] << 32) | kBias;
            S[rb[j]] = ((unsigned long long)rb[j] << 32) | kBias;
        }
    }
    auto sload = [&](uint32_t n) {
        return __hip_atomic_load(&S[n], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    bool settled = false;
    for (int64_t round = 0; round < 4 * L + 64; ++round) {
        __syncthreads();
        if (threadIdx.x == 0) changed = 0;
        __syncthreads();
        int mine = 0;
        for (int64_t j = threadIdx.x; j < L; j += kThreads) {
            const uint32_t u = ra[j], v = rb[j];
            if (u == NONE) continue;
            const unsigned long long su = sload(u), sv = sload(v);
            const uint32_t lu = (uint32_t)(su >> 32), lv = (uint32_t)(sv >> 32);
            // phi(v) = phi(u) + 1
            if (lu < lv) {
                const unsigned long long want = ((unsigned long long)lu << 32) | (uint32_t)((uint32_t)su + 1u);
                unsigned long long expect = sv;
                __hip_atomic_compare_exchange_strong(&S[v], &expect, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP);
                mine = 1;
            } else if (lv < lu) {
                const unsigned long long want = ((unsigned long long)lv << 32) | (uint32_t)((uint32_t)sv - 1u);
                unsigned long long expect = su;
                __hip_atomic_compare_exchange_strong(&S[u], &expect, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP);
                mine = 1;
            }
        }
        if (mine) changed = 1;
        __syncthreads();
        if (!changed) {
            settled = true;
            break;
        }
    }
    if (threadIdx.x == 0) wound = 0;
    __syncthreads();
    for (int64_t j = threadIdx.x; j < L; j += kThreads) {
        const uint32_t u = ra[j], v = rb[j];
        if (u == NONE) continue;
        const unsigned long long su = sload(u), sv = sload(v);
        if ((su >> 32) == (sv >> 32) && (uint32_t)sv != (uint32_t)su + 1u) wound = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        atomicOr((uint32_t *)&st->wrap[tl & 1], (wound ? 1u << d : 0u) | (settled ? 0u : kWrapUnsettled));
}

// ------------------------------------------------- finalise a sweep
// A replica's per-tile partials are summed in a fixed order (chunks of
// kFinSpan tiles, then the chunks), and finish_sweep forms the observables,
// runs the PCC window / beta step and advances the sweep counter.
// measure_out != null: observables of the current configuration only (no
// counters touched).
//
// Sums of the per-tile partials of replica R over the tiles [j0, j1), in a
// fixed order (thread j takes tiles j0 + j, j0 + j + NT, ...); thread 0 gets
// the totals.
template <int NT, int U = 4, int KG = kNumSums>
__device__ void sum_partials(const RepDesc &R, int64_t j0, int64_t j1, double (&tot)[kNumSums], double *red)
{
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) tot[k] = 0.0;
    const int64_t nt = R.ntiles;
    const XY_G double *pt = gmem(R.partials);
    // the sums in groups of KG; per group U tiles per thread per round, their
    // loads issued together (every sum still adds its tiles in the same order)
#pragma unroll
    for (int g = 0; g < kNumSums; g += KG) {
        int64_t j = j0 + threadIdx.x;
        for (; j + (U - 1) * NT < j1; j += U * NT) {
            double x[U][KG];
#pragma unroll
            for (int q = 0; q < U; ++q)
#pragma unroll
                for (int k = 0; k < KG; ++k)
                    if (g + k < kNumSums) x[q][k] = pt[(g + k) * nt + j + q * NT];
#pragma unroll
            for (int q = 0; q < U; ++q)
#pragma unroll
                for (int k = 0; k < KG; ++k)
                    if (g + k < kNumSums) tot[g + k] += x[q][k];
        }
        for (; j < j1; j += NT) {
#pragma unroll
            for (int k = 0; k < KG; ++k)
                if (g + k < kNumSums) tot[g + k] += pt[(g + k) * nt + j];
        }
    }
    block_sum<kNumSums, NT / 64>(tot, red);
}

// Observables from the totals, the PCC window / beta step and the sweep
// counter (one thread).  measure_out != null: observables only.
__device__ void finish_sweep(const RepDesc &R, const FlipArgs &fa, xy_obs *measure_out, const double (&tot)[kNumSums])
{
    RepState *st = R.st;
    const uint64_t t = st->t;
    const double beta = st->beta;
    const double N = (double)R.N;
    xy_obs o;
    obs_from_sums(tot, N, beta, &o);
    o.beta = beta;
    if (measure_out) {
        o.sweep = t;
        o.near_ties = 0;
        o.wrap = 0;
        o.perc = -1.0;
        measure_out[R.idx] = o;
        return;
    }
    const int par = (int)(t & 1);
    o.sweep = t + 1;
    o.near_ties = st->ties[par];
    o.wrap = fa.rule == XY_PCC_PERCOLATION ? st->wrap[par] : 0u;
    o.perc = fa.rule == XY_PCC_PERCOLATION ? ((o.wrap & 3u) ? 1.0 : 0.0) : -1.0;
    st->ties_total += o.near_ties;
    st->ties[par] = 0ull;
    st->last = o;
    if (fa.trace) fa.trace[fa.trace_row * fa.nrep + R.idx] = o;
    if (fa.window > 0) {
        double *acc = st->acc;
        acc[0] += o.E;
        acc[1] += o.m2;
        acc[2] += o.ex;
        acc[3] += o.sx;
        acc[4] += o.ey;
        acc[5] += o.sy;
        acc[6] += o.ups_x;
        acc[7] += N * o.sx * o.sx;
        acc[8] += o.mk2;
        acc[9] += o.perc;
        st->wrap_acc |= (uint32_t)o.wrap;
        st->acc_n += 1;
        if (st->acc_n >= fa.window) {
            const double W = (double)fa.window;
            const double mean_ex = acc[2] / W, mean_ns2 = acc[7] / W;
            // helicity rule: beta*Upsilon of the window; percolation rule: the
            // fraction of its sweeps in which some cluster wound around the lattice
            const double bu = fa.rule == XY_PCC_PERCOLATION ? acc[9] / W : beta * (mean_ex - beta * mean_ns2);
            double db = fa.dbeta0;
            if (fa.halve_every > 0) {
                const int64_t halvings = st->pcc_k / fa.halve_every;
                db = ldexp(fa.dbeta0, -(int)(halvings < 200 ? halvings : 200));
            }
            if (db < fa.dbeta_min) db = fa.dbeta_min;
            const double nb = beta + ((bu < fa.target) ? db : -db);
            if (fa.wmean) {
                xy_obs m;
                m.sweep = t + 1;
                m.beta = nb;
                m.E = acc[0] / W;
                m.m2 = acc[1] / W;
                m.ex = acc[2] / W;
                m.sx = acc[3] / W;
                m.ey = acc[4] / W;
                m.sy = acc[5] / W;
                m.ups_x = acc[6] / W;
                m.mk2 = acc[8] / W;
                m.near_ties = 0;
                m.wrap = st->wrap_acc;
                m.perc = acc[9] / W;
                fa.wmean[fa.wrow * fa.nrep + R.idx] = m;
            }
            st->beta = nb;
            st->beta_sum += nb;
            st->beta_n += 1;
            st->pcc_k += 1;
            for (int k = 0; k < 10; ++k) acc[k] = 0.0;
            st->wrap_acc = 0u;
            st->acc_n = 0;
        }
    }
    st->t = t + 1;
}

// Stage 1: chunk b of the launch (replica fin_rep[b]) into its partials2 row.
template <int U, int KG>
__device__ __forceinline__ void fin_chunk(const RepDesc *__restrict__ reps, const uint32_t *__restrict__ fin_rep,
                                          int32_t nrep, int64_t b, double *red, bool agent)
{
    const RepDesc &R = reps[nrep == 1 ? 0 : fin_rep[b]];
    const int64_t c = b - R.fin_base;
    double tot[kNumSums];
    sum_partials<kThreads, U, KG>(R, c * kFinSpan, std::min<int64_t>((c + 1) * kFinSpan, R.ntiles), tot, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kNumSums; ++k) {
            if (agent) st_agent(gmem(R.partials2) + c * kNumSums + k, tot[k]);
            else gmem(R.partials2)[c * kNumSums + k] = tot[k];
        }
    }
}

// Stage 2: the chunk sums of replica R in a fixed order, then the sweep.
__device__ __forceinline__ void fin_replica(const RepDesc &R, const FlipArgs &fa, xy_obs *measure_out, double *red,
                                            bool agent)
{
    double tot[kNumSums];
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) tot[k] = 0.0;
    const XY_G double *p2 = gmem(R.partials2);
    for (int64_t c = threadIdx.x; c < R.fin_chunks; c += kThreads) {
#pragma unroll
        for (int k = 0; k < kNumSums; ++k) tot[k] += agent ? ld_agent(p2 + c * kNumSums + k) : p2[c * kNumSums + k];
    }
    block_sum<kNumSums, kWaves>(tot, red);
    if (threadIdx.x == 0) finish_sweep(R, fa, measure_out, tot);
}

// Both stages in one launch: every chunk block adds itself to its replica's
// count after its stores (release); the block that completes the count
// (acquire) finishes the replica and resets the count for the next launch.
__global__ __launch_bounds__(kThreads) void k_finalize(const RepDesc *__restrict__ reps,
                                                        const uint32_t *__restrict__ fin_rep, int32_t nrep,
                                                        FlipArgs fa, xy_obs *measure_out)
{
    __shared__ double red[kWaves * kNumSums];
    __shared__ int last;
    fin_chunk(reps, fin_rep, nrep, blockIdx.x, red);
    const RepDesc &R = reps[nrep == 1 ? 0 : fin_rep[blockIdx.x]];
    if (threadIdx.x == 0) {
        const uint32_t done = __hip_atomic_fetch_add(&R.st->fin_done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = done + 1 == (uint32_t)R.fin_chunks;
        if (last) R.st->fin_done = 0u;
    }
    __syncthreads();
    if (!last) return;
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
    fin_replica(R, fa, measure_out, red);
}

// ------------------------------------------------- measure (no update)
template <typename IT>
__global__ __launch_bounds__(kThreads) void k_measure(const RepDesc *__restrict__ reps,
                                                       const uint32_t *__restrict__ tile_rep,
                                                       int32_t nrep, int64_t gtile0)
{
    __shared__ double red[kWaves * kNumSums];
    int64_t lt;
    const RepDesc &R = rep_of(reps, tile_rep, nrep, gtile0 + blockIdx.x, lt);
    const Tile<IT> T = make_tile<IT>(R, lt);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int B = band_rows(T.TH), yb = wave * B;
    const IT Lm = T.L - 1;
    double v[kNumSums] = {};
    for (int k = 0; k < B; ++k) {
        const int y = yb + k;
        if (y < T.TH && lane < T.TW) {
            const IT gy = T.y0 + (IT)y, gx = T.x0 + (IT)lane;
            const IT i = (gy << T.log2L) + gx;
            const IT jr = (gy << T.log2L) + ((gx + 1) & Lm);
            const IT jd = (((gy + 1) & Lm) << T.log2L) + gx;
            const double ci = R.c[i], si = R.s[i], cr = R.c[jr], sr = R.s[jr], cd = R.c[jd], sd = R.s[jd];
            v[0] += ci * cr + si * sr;
            v[1] += si * cr - ci * sr;
            v[2] += ci * cd + si * sd;
            v[3] += si * cd - ci * sd;
            v[4] += ci;
            v[5] += si;
        }
    }
    fourier_terms(R, T.x0, lane < T.TW, v);
    block_sum<kNumSums, kWaves>(v, red);
    store_partials(R, lt, v);
}

// ------------------------------------------------- canonical labels
// Label of every site of replica r (sweep labelled last): the smallest site of its
// cluster (tile-local root, or the key of its boundary node's root).
template <typename IT>
__global__ __launch_bounds__(kThreads) void k_flatten(const RepDesc *__restrict__ reps, int32_t r, void *out,
                                                       int32_t out_bits)
{
    const RepDesc &R = reps[r];
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const int log2TH = __ffs(R.TH) - 1;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < R.N; i += stride) {
        const IT y = (IT)i >> R.log2L, x = (IT)i & (IT)(R.L - 1);
        const int64_t lt = (int64_t)(y >> log2TH) * R.ntx + (int64_t)(x >> R.log2TW);
        const uint32_t l = gmem(R.lab)[i];
        const uint32_t nsite = (uint32_t)R.TH << R.log2TW;
        uint64_t key;
        if (l >= nsite) {
            key = root_key(gmem(R.node), (uint32_t)(lt * R.nb) + (l - nsite));
        } else {
            const Tile<IT> T = make_tile<IT>(R, lt);
            key = (uint64_t)T.site_of_local((int)l);
        }
        if (out_bits == 64)
            gmem((uint64_t *)out)[i] = key;
        else
            gmem((uint32_t *)out)[i] = (uint32_t)key;
    }
}

// ====================================================== host-side launchers
size_t lds_bytes_tile(int TH)
{
    // spin area: the spins with their halo, later the labelling's union-find
    // and the column sums of the waves (8 waves for 64-row tiles, else 4)
    const size_t spins = (size_t)(TH + 1) * 65 * sizeof(float2);
    const size_t later = (size_t)64 * TH * sizeof(uint32_t) + (size_t)(TH >= 64 ? 8 : 4) * 64 * 2 * sizeof(double);
    return std::max(spins, later) + (size_t)(5 * TH + 4) * sizeof(uint64_t);
}

// Element-wise kernels over N sites loop with a grid stride: a dispatch holds
// fewer than 2^32 work-items, and N reaches 2^32.
constexpr int64_t kMaxStrideBlocks = 1 << 20;


KernelEvents &next_launch_events()
{
    static thread_local KernelEvents ev;
    return ev;
}

// Launch of a kernel; with events set by next_launch_events() (a timed
// launch), the kernel's own start and end are recorded into them (the
// dispatch's timestamps, not the stream's progress around it) and the events
// are used up.
template <typename K, typename... A>
static void launch_k(K kern, dim3 grid, dim3 block, uint32_t lds, hipStream_t s, A... args)
{
    KernelEvents &ev = next_launch_events();
    if (ev.start) {
        const KernelEvents e = ev;
        ev = KernelEvents{};
        hipExtLaunchKernelGGL(kern, grid, block, lds, s, e.start, e.stop, 0u, args...);
    } else {
        hipLaunchKernelGGL(kern, grid, block, lds, s, args...);
    }
}

hipError_t launch_init_spins(const RepDesc *d_reps, int32_t r, int64_t N, int32_t start, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((N + kThreads - 1) / kThreads, kMaxStrideBlocks);
    launch_k(k_init_spins, dim3((unsigned)blocks), dim3(kThreads), 0, s, d_reps, r, start);
    return hipGetLastError();
}

hipError_t launch_init_fourier(const RepDesc *d_reps, int32_t r, int64_t L, hipStream_t s)
{
    launch_k(k_init_fourier, dim3((unsigned)((L + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, d_reps,
                       r);
    return hipGetLastError();
}

hipError_t launch_edge_refresh(const RepDesc *d_reps, int32_t r, int64_t ntiles, hipStream_t s)
{
    launch_k(k_edge_refresh, dim3((unsigned)ntiles), dim3(128), 0, s, d_reps, r);
    return hipGetLastError();
}

hipError_t launch_init_dir(const RepDesc *d_reps, int32_t nrep, hipStream_t s)
{
    launch_k(k_init_dir, dim3((nrep + 63) / 64), dim3(64), 0, s, d_reps, nrep);
    return hipGetLastError();
}

template <int MODE, int BT, int NW>
static void tile_dispatch_bt(const Launch &lc, const FlipArgs &fa, hipStream_t s)
{
    const size_t lds = lds_bytes_tile(lc.max_th);
    const dim3 grid((unsigned)xcd_blocks(lc.gtile_end - lc.gtile0, 1)), block(NW * 64);
    if (lc.big_index)
        launch_k((k_tile<uint64_t, MODE, BT, NW>), grid, block, lds, s, lc.reps, lc.tile_rep, lc.nrep,
                           lc.gtile0, lc.gtile_end, fa);
    else
        launch_k((k_tile<uint32_t, MODE, BT, NW>), grid, block, lds, s, lc.reps, lc.tile_rep, lc.nrep,
                           lc.gtile0, lc.gtile_end, fa);
}

// Fixed-size tiles of 64 columns when every replica of the launch has that
// shape: 8 rows per wave, 4 waves (32 rows) or 8 waves (64 rows), or 4 rows per
// wave for 16-row tiles; the general path (4 waves) otherwise.
template <int MODE>
static void tile_dispatch(const Launch &lc, const FlipArgs &fa, hipStream_t s)
{
    if (MODE != M_PLANES && lc.uniform_th == 64 && lc.uniform_tw == 64)
        tile_dispatch_bt<MODE, 8, 8>(lc, fa, s);
    else if (MODE != M_PLANES && lc.uniform_th == 32 && lc.uniform_tw == 64)
        tile_dispatch_bt<MODE, 8, 4>(lc, fa, s);
    else if (MODE != M_PLANES && lc.uniform_th == 16 && lc.uniform_tw == 64)
        tile_dispatch_bt<MODE, 4, 4>(lc, fa, s);
    else
        tile_dispatch_bt<MODE, 0, 4>(lc, fa, s);
}

hipError_t launch_tile(const Launch &lc, int mode, hipStream_t s, const FlipArgs *fa)
{
    FlipArgs f;
    if (fa) f = *fa;
    else std::memset(&f, 0, sizeof f);
    f.inpass = lc.inpass;
    switch (mode) {
    case TILE_BONDS: tile_dispatch<M_BONDS>(lc, f, s); break;
    case TILE_FLIP: tile_dispatch<M_FLIP>(lc, f, s); break;
    case TILE_FUSED: tile_dispatch<M_FUSED>(lc, f, s); break;
    case TILE_PLANES: tile_dispatch<M_PLANES>(lc, f, s); break;
    case TILE_SPEC: tile_dispatch<M_SPEC>(lc, f, s); break;
    case TILE_PLSEL: tile_dispatch<M_PLSEL>(lc, f, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_merge(const Launch &lc, bool next_dir, bool fin, hipStream_t s)
{
    const int epw = lc.merge_epw == 4 ? 4 : lc.merge_epw == 2 ? 2 : 1;
    const int64_t nblk = xcd_blocks(2 * (lc.gtile_end - lc.gtile0), kWaves * epw);  // epw tile edges per wave
    const int64_t nfin = fin ? lc.nfin : 0;
    const dim3 grid((unsigned)(xcd_pad(nfin) + nblk)), block(kThreads);
    auto go = [&](auto kern) {
        launch_k(kern, grid, block, 0, s, lc.reps, lc.tile_rep, lc.fin_rep, lc.nrep, lc.gtile0,
                           lc.gtile_end, (int32_t)next_dir, nfin, (int32_t)0);
    };
    switch (lc.dedup * 4 + epw) {
    case 1: go(k_merge<0, 1, false>); break;
    case 2: go(k_merge<0, 2, false>); break;
    case 4: go(k_merge<0, 4, false>); break;
    case 5: go(k_merge<1, 1, false>); break;
    case 6: go(k_merge<1, 2, false>); break;
    case 8: go(k_merge<1, 4, false>); break;
    case 9: go(k_merge<2, 1, false>); break;
    case 10: go(k_merge<2, 2, false>); break;
    default: go(k_merge<2, 4, false>); break;
    }
    return hipGetLastError();
}

hipError_t launch_merge_cut(const Launch &lc, int cut, hipStream_t s)
{
    if (cut != 1 && cut != 2) return hipErrorInvalidValue;
    const int64_t nblk = xcd_blocks(2 * (lc.gtile_end - lc.gtile0), kWaves);
    auto go = [&](auto kern) {
        launch_k(kern, dim3((unsigned)nblk), dim3(kThreads), 0, s, lc.reps, lc.tile_rep, lc.fin_rep,
                           lc.nrep, lc.gtile0, lc.gtile_end, (int32_t)0, (int64_t)0, (int32_t)cut);
    };
    if (lc.dedup == 0) go(k_merge<0, 1, true>);
    else if (lc.dedup == 1) go(k_merge<1, 1, true>);
    else go(k_merge<2, 1, true>);
    return hipGetLastError();
}

hipError_t launch_copy_nodes(const Launch &lc, hipStream_t s)
{
    launch_k(k_copy_nodes, dim3((unsigned)(lc.gtile_end - lc.gtile0)), dim3(kThreads), 0, s, lc.reps,
                       lc.tile_rep, lc.nrep, lc.gtile0);
    return hipGetLastError();
}

hipError_t launch_wrap(const Launch &lc, hipStream_t s)
{
    launch_k(k_wrap, dim3((unsigned)(2 * lc.nrep)), dim3(kThreads), 0, s, lc.reps);
    return hipGetLastError();
}

hipError_t launch_resolve(const Launch &lc, const FlipArgs *fin, hipStream_t s)
{
    const int64_t ntile = lc.gtile_end - lc.gtile0;
    FlipArgs fa;
    if (fin) fa = *fin;
    else std::memset(&fa, 0, sizeof fa);
    // the finalisation's blocks: one per replica (stage 2), or one per chunk
    // (both stages) when the tile pass united the edges
    const int64_t nfin = fin ? (lc.inpass ? lc.nfin : lc.nrep) : 0;
    launch_k(k_resolve, dim3((unsigned)(xcd_pad(nfin) + xcd_blocks(ntile, kWaves))), dim3(kThreads), 0, s,
             lc.reps, lc.tile_rep, lc.nrep, lc.gtile0, lc.gtile_end, nfin, fa, lc.fin_rep, (int32_t)lc.inpass);
    return hipGetLastError();
}

hipError_t launch_measure(const Launch &lc, hipStream_t s)
{
    const dim3 grid((unsigned)(lc.gtile_end - lc.gtile0)), block(kThreads);
    if (lc.big_index)
        launch_k((k_measure<uint64_t>), grid, block, 0, s, lc.reps, lc.tile_rep, lc.nrep, lc.gtile0);
    else
        launch_k((k_measure<uint32_t>), grid, block, 0, s, lc.reps, lc.tile_rep, lc.nrep, lc.gtile0);
    return hipGetLastError();
}

hipError_t launch_finalize(const Launch &lc, const FlipArgs &fa, xy_obs *measure_out, hipStream_t s)
{
    launch_k(k_finalize, dim3((unsigned)lc.nfin), dim3(kThreads), 0, s, lc.reps, lc.fin_rep, lc.nrep, fa,
                       measure_out);
    return hipGetLastError();
}

hipError_t launch_flatten(const RepDesc *d_reps, int32_t r, int64_t N, bool big_index, void *d_out,
                          int32_t out_bits, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((N + kThreads - 1) / kThreads, kMaxStrideBlocks);
    if (big_index)
        launch_k((k_flatten<uint64_t>), dim3((unsigned)blocks), dim3(kThreads), 0, s, d_reps, r, d_out,
                           out_bits);
    else
        launch_k((k_flatten<uint32_t>), dim3((unsigned)blocks), dim3(kThreads), 0, s, d_reps, r, d_out,
                           out_bits);
    return hipGetLastError();
}

}  // namespace xy
