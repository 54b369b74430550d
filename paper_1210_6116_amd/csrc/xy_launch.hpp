// xy_launch.hpp -- host-side launchers of the sweep kernels (internal to libxy).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/xy.h"

namespace xy {

struct RepDesc;

// One launch covers the global tiles [gtile0, gtile_end) of a handle.
struct Launch {
    const RepDesc *reps;      // device array of replica descriptors
    const uint32_t *tile_rep; // device: replica of every global tile (unused if nrep == 1)
    int32_t nrep;
    int32_t label_bits;       // width of canonical labels handed out: 32 or 64
    int32_t max_th;           // largest tile height among the replicas (LDS sizing)
    int32_t big_index;        // 1: 64-bit site indices (some replica has N > 2^30)
    int32_t uniform_tw, uniform_th;  // tile shape shared by every replica, or 0
    int64_t gtile0, gtile_end;
    const uint32_t *fin_rep;  // device: replica of every finalisation chunk (unused if nrep == 1)
    int64_t nfin;             // finalisation chunks of all replicas
    int32_t dedup = 0;        // merge: 0 one union per distinct node pair of a wave, 1 per run of equal neighbours
    int32_t merge_epw = 1;    // merge: tile edges per wave (1, 2 or 4)
    int32_t inpass = 0;       // the labelling tile pass unites the tile edges (no merge kernel)
};

// Modes of the tile kernel.  TILE_SPEC: flip of sweep t and the links of
// sweep t+1 for both betas a PCC step after sweep t may choose (no labels);
// TILE_PLSEL: labels of a sweep from the links of the beta that was chosen.
enum { TILE_BONDS = 0, TILE_FLIP = 1, TILE_FUSED = 2, TILE_PLANES = 3, TILE_SPEC = 4, TILE_PLSEL = 5 };

// Per-launch arguments of the flip kernel's finalisation (observables, PCC).
struct FlipArgs {
    xy_obs *trace;        // device: trace[trace_row * nrep + replica], or null
    int64_t trace_row;
    int32_t nrep;
    int32_t rule;         // XY_PCC_HELICITY, or XY_PCC_PERCOLATION (the sweep's wrapping check ran)
    int64_t window;       // PCC window (0: no PCC accumulation)
    double dbeta0, dbeta_min;
    int64_t halve_every;
    double target;
    xy_obs *wmean;        // device: window means wmean[wrow * nrep + replica], or null
    int64_t wrow;
    int32_t inpass;       // tile passes that label: unite the tile edges themselves (no merge kernel)
    int32_t pad;
};

hipError_t launch_init_spins(const RepDesc *d_reps, int32_t r, int64_t N, int32_t start, hipStream_t s);
hipError_t launch_edge_refresh(const RepDesc *d_reps, int32_t r, int64_t ntiles, hipStream_t s);
hipError_t launch_init_fourier(const RepDesc *d_reps, int32_t r, int64_t L, hipStream_t s);
hipError_t launch_init_dir(const RepDesc *d_reps, int32_t nrep, hipStream_t s);
// fa: the sweep's finalisation arguments (TILE_SPEC reads its PCC rule), or null.
hipError_t launch_tile(const Launch &lc, int mode, hipStream_t s, const FlipArgs *fa = nullptr);
// Union across tile edges; next_dir: also draw the next sweep's direction.
// fin: also the first stage of the deferred finalisation of the previous,
// fused sweep (the second runs with the edge coins, given its arguments).
hipError_t launch_merge(const Launch &lc, bool next_dir, bool fin, hipStream_t s);

// Events the next kernel launch on this thread records its own start and end
// into (set by a caller that times one launch; used up by that launch).
struct KernelEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
KernelEvents &next_launch_events();
// Wrapping check of the sweep labelled last (percolation rule): copies of the
// boundary forest before the merge (copy_nodes), merges of the copies without
// the links across the x seam (cut 1) / the y seam (cut 2), then the check
// itself (wrap) into every replica's state.
hipError_t launch_copy_nodes(const Launch &lc, hipStream_t s);
hipError_t launch_merge_cut(const Launch &lc, int cut, hipStream_t s);
hipError_t launch_wrap(const Launch &lc, hipStream_t s);
constexpr int64_t kWrapMaxL = 4096;  // largest side the wrapping check handles
// Coins of the clusters at tile edges, after the merge; fin != null: the
// second stage of a deferred finalisation.  With lc.inpass (the tile pass
// united the edges, no merge kernel ran) it also runs the first stage and
// draws the next sweep's direction.
hipError_t launch_resolve(const Launch &lc, const FlipArgs *fin, hipStream_t s);
hipError_t launch_measure(const Launch &lc, hipStream_t s);
hipError_t launch_finalize(const Launch &lc, const FlipArgs &fa, xy_obs *measure_out, hipStream_t s);
// Canonical labels (smallest site of each cluster) of replica r, of the sweep
// labelled last, as N values of out_bits (32 or 64) into d_out.
hipError_t launch_flatten(const RepDesc *d_reps, int32_t r, int64_t N, bool big_index, void *d_out,
                          int32_t out_bits, hipStream_t s);
size_t lds_bytes_tile(int TH);

}  // namespace xy
