// xy_device.hpp -- device-side building blocks of the MI355X Swendsen-Wang /
// PCC engine for the 2D classical XY model (Komura & Okabe, arXiv:1210.6116):
// the counter-based random stream, the per-replica descriptors shared by every
// kernel, and the lattice geometry of a labelling tile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/xy.h"

namespace xy {

// ---------------------------------------------------------------------------
// Random stream: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Every
// number the sweep draws is a pure function of (seed, counter), so a replica's
// trajectory does not depend on launch shape, batching or tile size.
// Counter layout (word0, word1 = replica, word2, word3 = tag):
//   BOND (pair = (y>>1)*L + x, rep, t, 1): words 0,1 = x-link, y-link of site
//        (x, 2*(y>>1)); words 2,3 the same for site (x, 2*(y>>1)+1)
//   FLIP (root>>7, rep, t, 2): coin of cluster root r = bit (r&31) of word (r>>5)&3
//        (drawn where needed: per tile row for the tile's own roots, per slot
//        for roots found through the boundary forest)
//   DIR  (k, rep, t, 3), INIT (site, rep, k, 4): k-th attempt of a rejection
//        draw of a point in the unit disk
// ---------------------------------------------------------------------------
enum : uint32_t { TAG_BOND = 1u, TAG_FLIP = 2u, TAG_DIR = 3u, TAG_INIT = 4u };
constexpr int kMaxAttempts = 16;      // rejection draws (two candidates each)
constexpr uint64_t kRenormEvery = 1024;  // spins rescaled to unit length after sweeps t with (t+1) % this == 0
constexpr double kTieEps = 1e-9;         // |u - p| below this counts as a near tie

// Global-memory view of a pointer.  Data reached through a descriptor would
// otherwise be accessed with flat instructions, whose completion is counted
// together with LDS traffic (every LDS wait would also wait for them).
#define XY_G __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ XY_G T *gmem(T *p)
{
    return (XY_G T *)p;
}

__device__ __forceinline__ float2 ldf2(const XY_G float2 *p)
{
    const unsigned long long u = *(const XY_G unsigned long long *)p;
    return make_float2(__uint_as_float((uint32_t)u), __uint_as_float((uint32_t)(u >> 32)));
}

__device__ __forceinline__ void stf2(XY_G float2 *p, float2 v)
{
    *(XY_G unsigned long long *)p =
        ((unsigned long long)__float_as_uint(v.y) << 32) | (unsigned long long)__float_as_uint(v.x);
}

// Read through the constant address space: for a uniform address this is a
// scalar load, allowed only for data no kernel running it writes (the sweep
// counter, direction and beta in the kernels that only read them).
#define XY_C __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ T cload(const T *p)
{
    return *(const XY_C T *)p;
}

// Values that are the same in every lane (read from memory the kernel also
// writes, so the compiler keeps them in vector registers) moved to scalar
// registers, with everything derived from them.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Element i of a global array.  With 32-bit site indices (N <= 2^30) the byte
// offset fits 32 bits, so the access can take a scalar base and one 32-bit
// vector offset (shared by arrays of the same element size) instead of a
// 64-bit vector address per access.
template <typename T>
__device__ __forceinline__ XY_G T &gel(XY_G T *base, uint32_t i)
{
    return *(XY_G T *)((XY_G char *)base + (uint32_t)(i * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ XY_G T &gel(XY_G T *base, uint64_t i)
{
    return base[i];
}
template <typename T>
__device__ __forceinline__ const XY_G T &gel(const XY_G T *base, uint32_t i)
{
    return *(const XY_G T *)((const XY_G char *)base + (uint32_t)(i * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ const XY_G T &gel(const XY_G T *base, uint64_t i)
{
    return base[i];
}

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0, n2;
        if (round < 2) {
            // the first two rounds: where the counter's upper words are the
            // same in every lane (as in the sweep's draws) half of these
            // products and exclusive ors are scalar; grouping the key with
            // them keeps them so
            n0 = (uint32_t)(p1 >> 32) ^ (c1 ^ k0);
            n2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);
        } else {
            // three-input exclusive or in one instruction (truth table 0x96)
            n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
            n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        }
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ double unif64(uint32_t w) { return (double)w * (1.0 / 4294967296.0); }

// ---------------------------------------------------------------------------
// Replica descriptors.  A handle owns an array of RepDesc (read-only during a
// sweep) and RepState (mutated on the device: beta, sweep counter, direction,
// PCC window, reduction counters).
// ---------------------------------------------------------------------------
// Scx, Ssx, Scy, Ssy, sum cos, sum sin, then the Fourier sums at k = 2 pi / L
// along x: sum cos e^{ikx} (real, imaginary), sum sin e^{ikx} (real, imaginary)
constexpr int kNumSums = 10;
constexpr int64_t kFinSpan = 1024;  // tiles per chunk of the two-stage finalisation

struct RepState {
    double beta;
    uint64_t t;              // sweeps completed (flips finalised)
    uint64_t tl;             // the sweep whose links were activated and labelled last
    double dir[2][2];        // mirror direction of sweep t in slot t&1
    unsigned long long ties[2];  // near ties of sweep t in slot t&1
    uint32_t fin_done;       // chunks finalised in the running finalisation launch
    uint32_t wrap_acc;       // union of the wrap bits of the running PCC window
    uint32_t wrap[2];        // wrap bits of sweep tl in slot tl&1 (4 | x | 2y; percolation rule only)
    double acc[10];          // PCC window sums: E, m2, ex, sx, ey, sy, ups_x, N sx^2, mk2, wrapping indicator
    double beta_cand;        // the first of the two betas a flip with both candidates' links activated
    unsigned long long ties_spec[2];  // near ties of those links, per candidate
    int64_t acc_n;           // sweeps in the running window
    int64_t pcc_k;           // PCC steps taken (halving schedule)
    uint64_t ties_total;
    double beta_sum;         // sum of beta after each PCC step
    int64_t beta_n;          // PCC steps summed
    xy_obs last;             // observables after the latest sweep
};

// Labels of the sweep labelled last (one buffer each: a tile reads its own
// labels of sweep t before it writes those of sweep t + 1, and nothing reads
// the forest of sweep t once its edge coins are drawn):
//   lab[i]   16 bits per site, tile-local: the tile-local index y*TW + x of the
//            smallest site of i's component inside its tile, or TW*TH + s
//            when that component touches the tile's edge, s being its slot
//   bslot    per tile NB = 2*(TW+TH) bytes: for every edge position p (top row,
//            bottom row, left column, right column) the slot of its component,
//            which is the smallest edge position of that component
//   node     per tile NB packed words, one per used slot: (key << 32) | parent,
//            key = global index of the smallest site of the parent's component;
//            a root's parent is itself.  Node id = tile * NB + slot.
//   cross    per tile two words: active links over the right edge (bit y) and
//            over the bottom edge (bit x)
//   ecoin    per tile four words (one buffer): bit p = flip coin of the cluster
//            at edge position p, drawn between the merge and the flip

struct RepDesc {
    float *c, *s;            // spin planes, N floats each
    uint16_t *lab;           // tile-local labels
    uint32_t *bx[2], *by[2]; // active-link bit planes of sweep t in slot t&1
    uint32_t *bxs, *bys;     // the second beta's candidate planes (flip with both candidates' links)
    uint8_t *bslot;          // edge positions -> slot
    unsigned long long *node;     // boundary-component forest
    unsigned long long *cross;    // links over the right / bottom tile edges
    unsigned long long *ecoin;    // per tile 4 words: flip coin of the cluster at every edge position
    uint32_t *ecnt;          // per tile 2 counters (right, bottom edge): its tiles' arrivals in a tile pass
                             // that unites the edges itself (zero between launches)
    float2 *edge[2];         // spins before sweep t in slot t&1: per tile, its first column (TH) then first row (TW)
    double *partials;        // kNumSums planes of per-tile sums: partials[k * ntiles + tile]
    double *partials2;       // chunk sums of the partials, fin_chunks x kNumSums
    double *fourier;         // cos(2 pi x / L), sin(2 pi x / L) at [2x], [2x+1], x = 0 .. L-1
    // wrapping check (percolation rule; null unless the handle allocated it):
    // node_cut[d] a copy of the forest merged without the links that cross the
    // lattice's seam along x (d = 0) or y (d = 1); pstate[d] per forest node
    // (component label << 32) | (potential + 2^31) of the check
    unsigned long long *node_cut[2];
    unsigned long long *pstate[2];
    RepState *st;
    int64_t L, N;
    int64_t ntiles, tile_base;  // tiles of this replica, first global tile id
    uint64_t seed;
    uint32_t rep;
    int32_t log2L, TW, TH, log2TW, ntx, nty;
    int32_t nb;              // edge positions (and slots) per tile, 2 * (TW + TH)
    int32_t fin_chunks;      // chunks of kFinSpan tiles (finalisation)
    int64_t fin_base;        // global index of the replica's first chunk in its launch
    int32_t idx;             // position of the replica in its handle
};

// Tile geometry in the site-index type IT (uint32_t when N <= 2^30, so that
// byte offsets of 4-byte arrays fit 32 bits; uint64_t otherwise).  TW =
// min(L, 64) columns (one wave64 lane per column) by TH rows; tile (tx, ty)
// covers columns tx*TW.. and rows ty*TH..
template <typename IT>
struct Tile {
    IT L, x0, y0, base;
    int32_t log2L, TW, TH, log2TW, tx, ty, ntx, nty;
    __device__ __forceinline__ IT site(int ly, int lx) const { return base + ((IT)ly << log2L) + (IT)lx; }
    __device__ __forceinline__ bool contains(IT i) const
    {
        const IT y = i >> log2L, x = i & (L - 1);
        return y >= y0 && y < y0 + (IT)TH && x >= x0 && x < x0 + (IT)TW;
    }
    __device__ __forceinline__ int local(IT i) const
    {
        const IT y = i >> log2L, x = i & (L - 1);
        return (int)(((y - y0) << log2TW) + (x - x0));
    }
    // tile-local index of edge position p (top row, bottom row, left column,
    // right column; corners appear twice)
    __device__ __forceinline__ int edge_local(int p) const
    {
        if (p < TW) return p;
        if (p < 2 * TW) return ((TH - 1) << log2TW) + (p - TW);
        if (p < 2 * TW + TH) return (p - 2 * TW) << log2TW;
        return ((p - 2 * TW - TH) << log2TW) + TW - 1;
    }
    __device__ __forceinline__ IT site_of_local(int q) const { return site(q >> log2TW, q & (TW - 1)); }
    // tiles to the right and below (periodic; ntx and nty are powers of two)
    __device__ __forceinline__ int64_t right_tile() const { return (int64_t)ty * ntx + ((tx + 1) & (ntx - 1)); }
    __device__ __forceinline__ int64_t down_tile() const { return (int64_t)((ty + 1) & (nty - 1)) * ntx + tx; }
    __device__ __forceinline__ int64_t left_tile() const { return (int64_t)ty * ntx + ((tx - 1) & (ntx - 1)); }
    __device__ __forceinline__ int64_t up_tile() const { return (int64_t)((ty - 1) & (nty - 1)) * ntx + tx; }
};

template <typename IT>
__device__ __forceinline__ Tile<IT> make_tile(const RepDesc &R, int64_t lt)
{
    Tile<IT> T;
    T.L = (IT)R.L;
    T.log2L = R.log2L;
    T.TW = R.TW;
    T.TH = R.TH;
    T.log2TW = R.log2TW;
    T.ntx = R.ntx;
    T.nty = R.nty;
    T.tx = (int32_t)(lt & (R.ntx - 1));
    T.ty = (int32_t)(lt >> (R.log2L - R.log2TW));
    T.x0 = (IT)T.tx * (IT)R.TW;
    T.y0 = (IT)T.ty * (IT)R.TH;
    T.base = (T.y0 << T.log2L) + T.x0;
    return T;
}

}  // namespace xy
