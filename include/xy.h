/*
 * xy.h -- C ABI of the MI355X Swendsen-Wang / PCC engine for the 2D classical
 * XY model (Komura & Okabe, "Large-scale Monte Carlo simulation of
 * two-dimensional classical XY model using multiple GPUs", arXiv:1210.6116).
 *
 * The model is Eq. (Hc): H = -J sum_<ij> cos(theta_i - theta_j) on an L x L
 * square lattice with periodic boundary conditions, J = 1.  One sweep is the
 * Swendsen-Wang multi-cluster update with Wolff's embedded-cluster formalism
 * (introduction: the SW and PCC paragraphs): draw a mirror direction r, activate
 * every link (i, j) with probability p = 1 - exp(min(0, -2 beta (s_i.r)(s_j.r))),
 * label the connected components of the active links, and reflect every spin of
 * each component, s -> s - 2 (s.r) r, with probability 1/2.  After every sweep
 * the energy, the magnetisation and the helicity-modulus sums are reduced
 * (the e / s definitions of the helicity-modulus paragraph); the generalized
 * probability-changing-cluster controller (the PCC paragraph) moves beta by
 * +-dbeta after each window according to whether beta*Upsilon is below or
 * above 0.636508.
 *
 * Conventions for every call:
 *   - The return value is XY_OK (0) or a negative XY_E* code; nothing throws
 *     or aborts across the ABI.  xy_last_error() gives a message for the last
 *     failing call on the calling thread.
 *   - Invalid arguments return XY_EINVAL and change nothing.  A HIP error
 *     returns XY_EDEVICE and poisons the handle: every later call on it except
 *     xy_free returns XY_ESTATE.
 *   - Work is enqueued on the handle's HIP stream.  Calls that return data to
 *     host memory synchronize that stream before returning; the others are
 *     asynchronous.
 *   - A handle must not be driven from two threads at once.
 *   - Site index i = y*L + x (x fastest).  Host arrays are plain C arrays of
 *     the stated length, owned by the caller.
 */
#ifndef XY_H
#define XY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    XY_OK = 0,
    XY_EINVAL = -1,  /* bad argument */
    XY_ENOMEM = -2,  /* device or host allocation failed, or the arena is too small */
    XY_EDEVICE = -3, /* a HIP call failed; the handle is poisoned */
    XY_ESTATE = -4,  /* the handle is poisoned or in the wrong state for the call */
    XY_EBUDGET = -5  /* serving: no free slot or not enough free budget right now (xy_group_add) */
};

enum { XY_START_HOT = 0 /* independent uniform angles */, XY_START_COLD = 1 /* theta = 0 */ };

typedef struct xy_handle xy_handle;

/* One lattice (replica).  A handle holds n of them, each with its own size,
 * temperature and random stream; they are updated together. */
typedef struct {
    int64_t L;          /* side; a power of two, 2 <= L <= 65536 */
    double beta;        /* inverse temperature (J = 1), 0 <= beta <= 1e4 */
    uint64_t seed;      /* 64-bit Philox4x32-10 key */
    uint32_t replica;   /* stream id (Philox counter word 1) */
    int32_t label_bits; /* width of the canonical labels handed out (xy_flatten_labels):
                           32, 64, or 0 = automatic (64 iff L*L >= 2^32).  Labels are
                           kept per tile in 16 bits, with a 64-bit forest of the
                           components that cross tile edges, whatever this is. */
    int32_t start;      /* XY_START_HOT or XY_START_COLD */
    int32_t tile_rows;  /* rows of a labelling tile: 16, 32, 64, or 0 = automatic */
} xy_params;

/* Observables of one configuration, or means over a PCC window (all per site;
 * paper: Eq. (Hc), the helicity-modulus e and s over x-links, <m^2> = chi/L^2). */
typedef struct {
    uint64_t sweep;     /* sweeps completed by the replica when the sample was taken */
    double beta;        /* beta the sweep ran at (window means: beta after the step) */
    double E;           /* H / N, both link directions */
    double m2;          /* |sum_i s_i / N|^2 */
    double ex, sx;      /* sum over x-links of cos / sin(theta_i - theta_j), over N */
    double ey, sy;      /* the same over y-links */
    double ups_x;       /* ex - beta N sx^2 (sample of the helicity modulus) */
    double mk2;         /* |sum_r s(r) exp(i k x)|^2 / N^2 at k = 2 pi / L: chi(k) / N of the
                           second-moment correlation length (m2 is chi(0) / N) */
    uint64_t near_ties; /* bond decisions of the sweep with |u - p| < 1e-9 */
    uint64_t wrap;      /* percolation-rule runs (XY_PCC_PERCOLATION): 4 | bit 0 if some cluster of the
                           sweep winds around the periodic lattice along x (holds a closed path of active
                           links with nonzero x winding number) | bit 1 the same along y; window means:
                           4 | the union of the window's bits.  0 when the check did not run. */
    double perc;        /* percolation-rule runs: 1 if some cluster winds (along x or y), else 0; window
                           means: the fraction of the window's sweeps in which one did.  -1 when the
                           check did not run. */
} xy_obs;

/* PCC controller (paper: the PCC paragraph and the simulation paragraph:
 * windows of 1000 MCS, dbeta = 0.0005, target 0.636508).  Two rules:
 *   XY_PCC_HELICITY   the generalized rule the paper uses: beta*Upsilon of the
 *                     window (from the means of e_x and N s_x^2) below target
 *                     -> beta += dbeta, otherwise beta -= dbeta;
 *   XY_PCC_PERCOLATION  the original rule of the PCC paragraph (raise or lower
 *                     the temperature according to whether the clusters
 *                     percolate): after every sweep the library checks whether
 *                     some cluster winds around the periodic lattice (along x
 *                     or y; xy_obs.wrap); the fraction P of the window's sweeps
 *                     in which one did below target (e.g. 0.5) -> beta +=
 *                     dbeta, otherwise beta -= dbeta.  Needs L <= 4096. */
enum { XY_PCC_HELICITY = 0, XY_PCC_PERCOLATION = 1 };
typedef struct {
    int64_t window;      /* sweeps per PCC step, >= 1 */
    double dbeta0;       /* step of the first PCC step, > 0 */
    double dbeta_min;    /* floor of the halving schedule, >= 0 */
    int64_t halve_every; /* PCC steps between halvings of dbeta; 0 = never */
    double target;       /* critical beta*Upsilon, e.g. 0.636508; percolation rule: critical P, e.g. 0.5 */
    int32_t rule;        /* XY_PCC_HELICITY or XY_PCC_PERCOLATION */
    int32_t reserved;    /* 0 */
} xy_pcc;

/* Device bytes that xy_alloc needs for these n replicas (arena size). */
int xy_bytes_required(const xy_params *p, int32_t n, size_t *bytes);

/* Creates a handle for n >= 1 replicas p[0..n-1] and initialises their spins
 * (hot or cold start) at sweep 0.  hip_stream: the hipStream_t to enqueue on,
 * or NULL for a stream the library creates.  arena: device memory of at least
 * xy_bytes_required() bytes that the caller owns and keeps alive until
 * xy_free (e.g. a torch tensor), or NULL to let the library allocate.
 * On success *out receives the handle. */
int xy_alloc(const xy_params *p, int32_t n, void *hip_stream, void *arena, size_t arena_bytes,
             xy_handle **out);

/* Runs nsweeps >= 0 sweeps of every replica at its current beta.
 * trace: NULL, or host memory for nsweeps * n xy_obs, filled as
 * trace[k * n + rep] with the observables after sweep k (synchronizes). */
int xy_sweep(xy_handle *h, int64_t nsweeps, xy_obs *trace);

/* Runs replays x nsweeps sweeps: the launch sequence of nsweeps sweeps is
 * captured once into a HIP graph on the handle's stream (kept in the handle and
 * reused while nsweeps stays the same) and the graph is launched replays times.
 * Same results as xy_sweep(h, replays * nsweeps, NULL); asynchronous.  Not
 * allowed while per-kernel timing is on (XY_ESTATE). */
int xy_sweep_graph(xy_handle *h, int64_t nsweeps, int64_t replays);

/* Observables of every replica's current configuration (n xy_obs, host;
 * synchronizes).  near_ties is 0; sweep is the replica's sweep count. */
int xy_measure(xy_handle *h, xy_obs *out);

/* Runs nsteps >= 1 PCC steps of c->window sweeps each, updating every
 * replica's beta on the device after each window.  window_mean: NULL, or host
 * memory for nsteps * n xy_obs receiving the window means (beta = the new
 * beta) as window_mean[k * n + rep] (synchronizes).  The first call with the
 * percolation rule allocates the handle's wrapping-check buffers (four 64-bit
 * words per tile-edge position, kept until xy_free); XY_EINVAL if a replica
 * has L > 4096 for that rule. */
int xy_pcc_step(xy_handle *h, const xy_pcc *c, int64_t nsteps, xy_obs *window_mean);

/* Releases the handle and whatever the library allocated.  xy_free(NULL) is OK. */
int xy_free(xy_handle *h);

/* ---- inspection and control (tests, tooling) ---------------------------- */

/* Copies replica rep's spins to / from host arrays of N = L*L floats.  Spins
 * set must be unit vectors within 1e-3 (the bond test's error bound assumes
 * it); XY_EINVAL otherwise. */
int xy_get_state(xy_handle *h, int32_t rep, float *cos_out, float *sin_out);
int xy_set_state(xy_handle *h, int32_t rep, const float *cos_in, const float *sin_in);

/* Canonical cluster labels (minimum site index of each cluster) of the most
 * recent sweep of replica rep, as N int64 values (host; synchronizes). */
int xy_get_labels(xy_handle *h, int32_t rep, int64_t *out);

/* Active-link bit planes of the most recent sweep of replica rep: bit i of
 * word i/32 of bx (by) is the link (i, right(i)) ((i, down(i))).  Host arrays
 * of ceil(N/32) uint32 each (synchronizes). */
int xy_get_bonds(xy_handle *h, int32_t rep, uint32_t *bx, uint32_t *by);

/* Device views of replica rep after its most recent sweep, for checks that
 * must run where the data is (a lattice of 2^32 sites does not fit a host
 * copy in FP64).  All pointers are device addresses inside the handle's
 * memory, owned by the handle and valid until the next call that sweeps,
 * sets state or frees it; callers only read through them.
 *   cos_plane, sin_plane  N FP32 each, row-major (x fastest): the state
 *   bond_x, bond_y        link bit planes of the sweep, as in xy_get_bonds
 *   label_bits            width of the canonical labels (32 or 64) that
 *                         xy_flatten_labels writes by default
 * XY_ESTATE if the replica has not swept yet. */
typedef struct {
    const float *cos_plane;
    const float *sin_plane;
    const uint32_t *bond_x;
    const uint32_t *bond_y;
    int64_t L;
    int32_t label_bits;
    int32_t reserved;
    uint64_t sweep; /* sweeps completed */
} xy_views;
int xy_get_views(xy_handle *h, int32_t rep, xy_views *out);

/* Canonical cluster labels of the most recent sweep of replica rep (the
 * flatten of the two-level labelling: every site gets the smallest site index
 * of its cluster), written to d_out, caller-owned device memory of N entries
 * of out_bits/8 bytes (out_bits 32 or 64; 32 only if N <= 2^32).  Runs on the
 * handle's stream and synchronizes it. */
int xy_flatten_labels(xy_handle *h, int32_t rep, void *d_out, int32_t out_bits);

/* beta of replica rep: set (takes effect from the next sweep) / read. */
int xy_set_beta(xy_handle *h, int32_t rep, double beta);
int xy_get_beta(xy_handle *h, int32_t rep, double *beta);

/* Sweep counter of replica rep and its mirror direction r for the next sweep. */
int xy_get_sweep(xy_handle *h, int32_t rep, uint64_t *sweep, double r[2]);

/* Standalone labelling of a given link set (the same kernels as the sweep):
 * d_bx, d_by are device bit planes as in xy_get_bonds; d_labels receives N
 * canonical labels (uint32 if label_bits == 32, uint64 if 64) in device memory.
 * Runs on hip_stream (NULL = the default stream) and synchronizes it. */
int xy_label_links(int64_t L, int32_t label_bits, int32_t tile_rows, const uint32_t *d_bx,
                   const uint32_t *d_by, void *d_labels, void *hip_stream);

/* xy_label_links for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same labelling, with its scratch (state and descriptor, tile-local
 * labels, edge slots, boundary forest, edge-link masks) in a fixed 16 MiB
 * device array of the library instead of a per-call allocation.  Each GPU the
 * library runs on holds its own copy of that array until the process ends.
 * Arguments as in xy_label_links; L*L plus the forest must fit the array
 * (L <= 2048 for every tile height; larger lattices: XY_EINVAL, nothing
 * enqueued).  Allocates nothing and does not synchronize: the work is only
 * enqueued on hip_stream (NULL = the default stream), and d_labels is ready
 * once that stream has reached it.  Every call on a GPU uses that GPU's one
 * array, so calls that overlap on one GPU (different streams, or threads)
 * race; calls on one stream are ordered.  The first call on each device takes
 * the array's device address (hipGetSymbolAddress) with that device current. */
int xy_label_links_noalloc(int64_t L, int32_t label_bits, int32_t tile_rows, const uint32_t *d_bx,
                           const uint32_t *d_by, void *d_labels, void *hip_stream);

/* Schedule of the merge across tile edges (tuning choices; results are
 * identical bit for bit whatever they are).  dedup: every active link over a
 * tile edge asks for the union of the boundary components at its two ends, and
 * a wave of 64 such links often repeats a pair:
 *   XY_DEDUP_WAVE       (default) one union per distinct pair of the wave;
 *   XY_DEDUP_NEIGHBOUR  a link is skipped only when the link before it joins
 *                       the same pair (fewer ballots when pairs rarely repeat);
 *   XY_DEDUP_HASH       one union per pair through a 64-entry table in LDS that
 *                       the pairs hash to (a fixed cost per edge; a collision
 *                       only repeats a union).
 * edges_per_wave: 1 (default), 2 or 4 tile edges per wave: their links are
 * read together and the pairs that lead a union packed into the wave's lanes,
 * so that the unions of all of them run side by side (half or a quarter as
 * many waves, each with more unions in flight).  XY_EINVAL for other values. */
enum { XY_DEDUP_WAVE = 0, XY_DEDUP_NEIGHBOUR = 1, XY_DEDUP_HASH = 2 };
int xy_set_merge(xy_handle *h, int32_t dedup, int32_t edges_per_wave);

/* The merge across tile edges inside the labelling tile pass (on = 1) instead
 * of a merge kernel of its own (on = 0, the default): a tile that has stored
 * its edge slots, boundary nodes and edge link masks (agent-scope stores,
 * completed) counts itself at the four tile edges it touches, and the second
 * of an edge's two tiles to arrive unites that edge's links (hash
 * deduplication) before its block ends; no block waits for another.  The edge
 * coins then also run both stages of a deferred finalisation and draw the next
 * sweep's direction.  One kernel fewer per sweep, against unions in the tile
 * pass's tail (a tuning choice, as xy_set_merge: the partition, and every
 * label and coin, is the same either way).  Calls with the percolation rule
 * keep the merge kernel (the wrapping check copies the forest before it).
 * XY_EINVAL for on not 0 or 1. */
int xy_set_merge_in_pass(xy_handle *h, int32_t on);

/* Per-kernel timing with HIP events on the handle's stream: enable (1) or
 * disable (0) recording; read the accumulated milliseconds and launch counts
 * of each kernel class (XY_K_*) and reset them (synchronizes).  XY_K_SWEEP
 * brackets whole sweeps (first kernel of the sweep to its finalize).  With
 * samples non-NULL, up to cap individual sweep durations (ms, in order) are
 * also copied out and *nsamples receives how many. */
enum {
    XY_K_BONDS = 0,    /* link activation + in-tile labelling */
    XY_K_MERGE = 1,    /* union of boundary components across tile edges (+ a deferred finalisation) */
    XY_K_FLIP = 2,     /* cluster coins, reflection, sums */
    XY_K_FUSED = 3,    /* flip of sweep t + links and tile labels of sweep t+1 */
    XY_K_FINALIZE = 4, /* observables, PCC step, counters */
    XY_K_COINS = 5,    /* coins of the clusters at tile edges */
    XY_K_SWEEP = 6,
    XY_K_WRAP = 7,     /* wrapping check of the percolation rule (forest copies, cut merges, check) */
    XY_K_SPEC = 8,     /* flip of sweep t + links of sweep t+1 for both betas its PCC step may choose */
    XY_K_PLSEL = 9,    /* labels of a sweep from the links of the chosen beta */
    XY_K_COUNT = 10
};
int xy_timing(xy_handle *h, int32_t enable);
int xy_timing_read(xy_handle *h, double *ms, int64_t *launches, double *samples, int64_t cap,
                   int64_t *nsamples);

/* ---- serving: continuous batching of PCC runs ------------------------------
 * A group keeps up to max_slots requests (each one lattice with its own L,
 * seed and initial beta, and a number of sweeps to run) resident in one device
 * arena of budget_bytes, and advances all resident requests together: every
 * round runs the same number of sweeps of each of them in the same kernel
 * launches, each sweep followed by its own PCC update with the group's rule c.
 * A request's result does not depend on the other requests in the group.
 * Requests are admitted between rounds as slots and memory free up. */
typedef struct xy_group xy_group;

/* budget_bytes: device memory the group may use (one arena, allocated here);
 * max_slots >= 1; c: PCC rule of every request (XY_PCC_HELICITY only);
 * hip_stream as in xy_alloc. */
int xy_group_create(size_t budget_bytes, int32_t max_slots, const xy_pcc *c, void *hip_stream,
                    xy_group **out);
/* Admits a request of nsweeps >= 1 sweeps (label_bits must resolve to 32).
 * *slot receives its slot id.  XY_EBUDGET if no slot or not enough free
 * memory right now (nothing changes; the request may fit later); XY_EINVAL
 * for bad parameters, and for a request larger than the whole budget (it can
 * never be admitted). */
int xy_group_add(xy_group *g, const xy_params *p, int64_t nsweeps, int32_t *slot);
/* Bytes a request of these parameters occupies in the group's arena. */
int xy_group_bytes(const xy_params *p, size_t *bytes);
/* Runs one round of min(max_sweeps, fewest remaining sweeps) sweeps of every
 * running request (0 if none is running); *ran receives that number.
 * Synchronizes. */
int xy_group_round(xy_group *g, int64_t max_sweeps, int64_t *ran);
/* Slot ids of requests that finished since the previous call (up to cap). */
int xy_group_poll(xy_group *g, int32_t *slots, int32_t cap, int32_t *n);
/* Result of a finished (or running) request: observables after its latest
 * sweep, its current beta, and the mean of beta over its PCC steps. */
int xy_group_result(xy_group *g, int32_t slot, xy_obs *last, double *beta, double *beta_mean);
/* Spins of a request (finished, or running after at least one round) as
 * host arrays of N = L*L floats each (synchronizes).  XY_ESTATE before the
 * request's first round. */
int xy_group_get_state(xy_group *g, int32_t slot, float *cos_out, float *sin_out);
/* Frees a finished request's slot and memory. */
int xy_group_release(xy_group *g, int32_t slot);
/* Bytes in use and running requests. */
int xy_group_info(xy_group *g, size_t *used_bytes, int32_t *running);
int xy_group_free(xy_group *g);

/* Message of the last failing call on this thread ("" if none). */
const char *xy_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* XY_H */
