// xy_host.hpp -- host-side internals shared by the handle API (xy_api.cpp)
// and the serving group API (xy_group.cpp): parameter checks and the device
// memory layout of a set of replicas.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/xy.h"
#include "xy_device.hpp"
#include "xy_launch.hpp"

namespace xyhost {

constexpr size_t kAlign = 256;
constexpr int64_t kTraceChunk = 256;  // sweeps (or PCC steps) per trace copy-back

int fail(int code, const char *fmt, ...);
size_t align_up(size_t x);
int ilog2(int64_t v);

struct Resolved {
    int64_t L, N;
    int32_t TW, TH, ntx, nty, nb;
    int64_t ntiles;
    int32_t fin_chunks;  // finalisation chunks, ceil(ntiles / kFinSpan)
};

// Per-replica byte layout inside an arena.
struct RepLayout {
    size_t c, s, lab, bx[2], by[2], bxs, bys, bslot, node, cross, edge[2], ecoin, ecnt, partials, partials2, fourier,
        end;
};

struct Plan {
    int32_t n = 0, label_bits = 32, max_th = 1, uniform_tw = -1, uniform_th = -1;
    bool big_index = false;
    std::vector<Resolved> res;
    std::vector<RepLayout> lay;
    size_t off_reps = 0, off_state = 0, off_tile_rep = 0, off_fin_rep = 0, off_obs = 0, total = 0;
    int64_t total_tiles = 0, total_fin = 0;
};

int check_params(const xy_params *p, int32_t n);
int make_plan(const xy_params *p, int32_t n, Plan &P);
// Descriptor of replica k of plan P whose buffers start at base (layout P.lay[k]).
void fill_desc(const Plan &P, int32_t k, const xy_params &p, char *base, xy::RepState *st, int64_t tile_base,
               int64_t fin_base, int32_t idx, xy::RepDesc &d);
// Standalone labelling of a given link set (xy_label_links and its variant
// without allocation): the plan of one replica and the byte layout of its
// scratch (state and descriptor, tile-local labels, edge slots, forest,
// edge-link masks).
struct LinkLabelJob {
    Plan plan;
    size_t off_state = 0, off_desc = 0, off_lab = 0, off_bslot = 0, off_node = 0, off_cross = 0, total = 0;
};
int plan_link_labels(int64_t L, int32_t label_bits, int32_t tile_rows, LinkLabelJob &J);
// Descriptor of the labelling whose scratch starts at the device address mem.
void link_label_desc(const LinkLabelJob &J, char *mem, const uint32_t *d_bx, const uint32_t *d_by, xy::RepDesc &d);
// Tile labelling from the bit planes, merge across tiles and canonical labels
// into d_labels; the scratch must already hold the state and the descriptor.
hipError_t enqueue_link_labels(const LinkLabelJob &J, char *mem, void *d_labels, hipStream_t s);
// Launch state carried from one sweep to the next inside a sequence.
struct Pipe {
    bool ready = false;        // the links of the next sweep are activated and labelled
    bool fin_pending = false;  // the last flip's finalisation is still to run
    xy::FlipArgs fa_pending;   // its arguments
    bool spec = false;         // the last flip activated the next sweep's links for both candidate betas
};

// What the flip of a sweep does besides flipping: END the sequence (flip,
// finalisation); FUSE the links and labels of the next sweep into it (beta
// cannot change in between); SPEC activate the next sweep's links for both
// betas the PCC step after this sweep may choose (the next sweep labels the
// links of the chosen one instead of activating them from the spins again).
enum { NEXT_END = 0, NEXT_FUSE = 1, NEXT_SPEC = 2 };

// One sweep of every replica in lc: links + tile labels (unless pp.ready; from
// the chosen candidate's planes if pp.spec), merge of the boundary components
// (with the deferred finalisation of the previous sweep), edge coins, then the
// flip as `next` says: with its finalisation (END, SPEC), or fused with the
// next sweep's links, whose finalisation runs with the next sweep's merge and
// edge coins (FUSE).  A sequence must end with NEXT_END.  timer(kind, launch)
// runs each launch (and may bracket it with events).
template <typename Timer>
hipError_t enqueue_sweep_lc(const xy::Launch &lc_in, const xy::RepDesc *d_reps, int32_t nrep, const xy::FlipArgs &fa,
                            int next, Pipe &pp, hipStream_t s, Timer &&timer)
{
    hipError_t e = hipSuccess;
    // percolation rule: the wrapping check copies the forest before the
    // merge, so the edges are united by the merge kernel, not in the tile pass
    const bool perc = fa.rule == XY_PCC_PERCOLATION;
    xy::Launch lc = lc_in;
    if (perc) lc.inpass = 0;
    if (!pp.ready) {
        if (pp.spec)
            e = timer(XY_K_PLSEL, [&] { return xy::launch_tile(lc, xy::TILE_PLSEL, s); });
        else
            e = timer(XY_K_BONDS, [&] { return xy::launch_tile(lc, xy::TILE_BONDS, s); });
        if (e != hipSuccess) return e;
    }
    pp.spec = false;
    // percolation rule: the wrapping check of the sweep just labelled (forest
    // copies before the merge, their merges without the seam links after it)
    if (perc) {
        e = timer(XY_K_WRAP, [&] { return xy::launch_copy_nodes(lc, s); });
        if (e != hipSuccess) return e;
    }
    // the merge kernel, unless the labelling tile pass united the edges
    // (then the coins also draw the next direction and run both stages of a
    // deferred finalisation)
    if (!lc.inpass) {
        e = timer(XY_K_MERGE, [&] { return xy::launch_merge(lc, true, pp.fin_pending, s); });
        if (e != hipSuccess) return e;
    }
    if (perc) {
        e = timer(XY_K_WRAP, [&] {
            hipError_t e2 = xy::launch_merge_cut(lc, 1, s);
            if (e2 == hipSuccess) e2 = xy::launch_merge_cut(lc, 2, s);
            if (e2 == hipSuccess) e2 = xy::launch_wrap(lc, s);
            return e2;
        });
        if (e != hipSuccess) return e;
    }
    e = timer(XY_K_COINS, [&] { return xy::launch_resolve(lc, pp.fin_pending ? &pp.fa_pending : nullptr, s); });
    if (e != hipSuccess) return e;
    pp.fin_pending = false;
    if (next == NEXT_FUSE) {
        e = timer(XY_K_FUSED, [&] { return xy::launch_tile(lc, xy::TILE_FUSED, s); });
        pp.ready = true;
        pp.fin_pending = true;
        pp.fa_pending = fa;
        return e;
    }
    if (next == NEXT_SPEC)
        e = timer(XY_K_SPEC, [&] { return xy::launch_tile(lc, xy::TILE_SPEC, s, &fa); });
    else
        e = timer(XY_K_FLIP, [&] { return xy::launch_tile(lc, xy::TILE_FLIP, s); });
    if (e != hipSuccess) return e;
    e = timer(XY_K_FINALIZE, [&] { return xy::launch_finalize(lc, fa, nullptr, s); });
    pp.ready = false;
    pp.spec = next == NEXT_SPEC;
    return e;
}

}  // namespace xyhost
