/*
 * tril.h -- C ABI of libtril: bounding-volume-hierarchy collision detection
 * between two photon beams (Breit-Wheeler pair creation), hand-written HIP
 * kernels for AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Sec. 1 and Sec. 2 of Jansen et al., "Tree Code for
 * Collision Detection of Large Numbers of Particles -- Application for the
 * Breit-Wheeler Process"): photons with position, momentum, energy and
 * macro-particle weight go in; colliding photon pairs, pair counts, the pair
 * yield and the pair-energy spectrum come out.
 *
 * Per time step k (step length dt, window [k dt, (k+1) dt]):
 *   tril_build   -- one bounding-volume hierarchy (a linear BVH over Morton
 *                   codes) over the target beam's photon segments swept over
 *                   the step (boxes enlarged by one step's travel, Sec. 2.1);
 *   tril_collide -- every query photon's swept box, enlarged by an upper
 *                   bound of its collision radius, descends that hierarchy
 *                   (depth-first, a failed box test skips the subtree,
 *                   Sec. 2.2, box test Eq. 5); surviving leaf pairs get the
 *                   exact narrow-phase test:
 *                     s_ij = E_i E_j (1 - u_i.u_j) / (2 m_e^2) > 1   (Eq. 1, 2)
 *                     min over the window of |X_i(t) - X_j(t)|^2 <= r_ij^2,
 *                     r_ij^2 = sqrt(w_i w_j) sigma_BW(s_ij) / pi     (Eq. 1)
 *                   with X(t) = x0 + t p/E (straight lines at c) and hits
 *                   (i, j, k) appended to the caller's pair buffer. The decision
 *                   is that of FP64 arithmetic: a single-precision stage with a
 *                   running bound on its rounding error decides the candidates
 *                   that clear the criterion by more than that bound (plus
 *                   1e-5 r^2), FP64 the rest (precision contract of the paper's
 *                   exact test, Eq. 1 and 2);
 *   tril_stats   -- after the last step: union of the hits over steps (each
 *                   pair kept once, with its first step), sorted ascending by
 *                   (i, j); pair count, yield sum sqrt(w_i w_j), pair-energy
 *                   spectrum and per-step hit counts.
 *
 * Units: um for lengths, um/c for times (c = 1), MeV for energies, MeV/c for
 * momenta. Constants: m_e c^2 = 0.51099895 MeV, r_e = 2.8179403262e-9 um.
 *
 * Memory: every pointer is a DEVICE pointer unless marked "host". The caller
 * owns every input and output buffer and keeps it alive until the stream has
 * passed the call; the context owns the hierarchy and all scratch memory.
 * Every call is asynchronous on the context's HIP stream except tril_stats,
 * which synchronises that stream. One context must not be used from two host
 * threads at once; distinct contexts are independent.
 *
 * Errors: every int-returning call returns TRIL_OK (0) or a negative code;
 * tril_strerror gives its text. On an error no output buffer is written past
 * its capacity.
 */
#ifndef TRIL_H
#define TRIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRIL_OK           0
#define TRIL_E_INVAL     -1  /* bad argument: NULL pointer, dt <= 0, n < 0, bad edges, bad offsets */
#define TRIL_E_NOMEM     -2  /* device allocation failed */
#define TRIL_E_OVERFLOW  -3  /* pair or candidate buffer too small; see tril_stats */
#define TRIL_E_HIP       -4  /* HIP runtime error; tril_last_hip_error gives its text */
#define TRIL_E_NOTIMPL   -5  /* flag or mode not implemented */
#define TRIL_E_STATE     -6  /* call order: collide before any build, or beams of different instance counts */
#define TRIL_E_DATA      -7  /* photon data rejected on the device: non-finite value, E <= 0,
                                  w < 0, or a momentum whose magnitude |p| c differs from E
                                  by more than 1e-12 relative (photons are massless) */
#define TRIL_E_INTERNAL  -8  /* a device-side wait exceeded its bound (should not happen) */

/* tril_params.flags */
#define TRIL_TIMING        0x1u  /* record HIP events around each phase (ms_* in tril_stats_t) */
#define TRIL_SORT_QUERIES_ONCE 0x2u /* Morton-order the query beam at its first step only */
#define TRIL_FP64_NARROW   0x4u  /* decide every candidate in FP64 (no FP32 stage) */
#define TRIL_ANNIHILATE    0x8u  /* photons that collide are consumed: tril_stats keeps a
                                    raw hit only if neither photon was consumed by a hit
                                    before it in the order (step, time of closest approach
                                    inside the step, i, j); Sec. 2.1 (annihilating photons)
                                    and Sec. 2.2 (collisions sorted in time). tril_run
                                    resolves each batch of steps as it finishes and leaves
                                    the photons consumed so far out of the later batches'
                                    hierarchies and queries (same kept hits; the run then
                                    synchronises once per batch) */
#define TRIL_GRID          0x10u /* broad phase on a uniform grid instead of the hierarchy (the
                                    mesh the paper compares its tree against, Sec. 3): per
                                    step, target boxes sorted by the cell of their centre
                                    (about one cell per photon over the step's bounds), each
                                    query scanning the cells its box meets; same candidates'
                                    superset, same narrow phase and results. One instance only
                                    (else TRIL_E_NOTIMPL); tril_run then goes step by step */

typedef struct tril_ctx tril_ctx;
typedef struct tril_mlp tril_mlp;

/* One beam as structure-of-arrays, FP64, length n (all instances together).
 * Positions are at t = 0; photon i is at x_i + t * p_i / E_i at time t.
 * Independent collision instances are contiguous slices given by the host CSR
 * array inst_off[0..n_inst] (inst_off[0] = 0, non-decreasing, inst_off[n_inst] = n);
 * inst_off may be NULL when n_inst == 1. Photons only collide with photons of
 * the same instance of the other beam. Row indices in outputs are global rows. */
typedef struct {
    int64_t n;
    const double *x, *y, *z;      /* device, n each: position at t = 0 [um] */
    const double *px, *py, *pz;   /* device, n each: momentum [MeV/c], |p| c = E to 1e-12
                                     relative (checked on the device, TRIL_E_DATA) */
    const double *E;              /* device, n: energy [MeV], finite and > 0 */
    const double *w;              /* device, n: macro-particle weight, finite and >= 0 */
    int32_t n_inst;               /* >= 1 */
    const int64_t *inst_off;      /* host, n_inst + 1 entries, or NULL if n_inst == 1 */
} tril_beam;

/* Context parameters (copied at tril_create; the host arrays may be freed afterwards). */
typedef struct {
    double dt;                    /* step length [um/c], finite and > 0 */
    uint32_t flags;               /* TRIL_* flags above */
    int32_t n_bins;               /* pair-energy spectrum bins, >= 0 */
    const double *bin_edges;      /* host, n_bins + 1 strictly increasing edges [MeV]; bin b
                                     holds edges[b] <= E_i + E_j < edges[b+1] */
    int64_t cand_cap;             /* broad-phase candidates one step may hold (0 = default) */
    int32_t block_traverse;       /* traversal workgroup size: 64, 128, 256, 512 or 0 = default (64) */
    int32_t step_batch;           /* tril_run: steps per launch, >= 0 (0 = as many as keep one
                                     launch within 2^29 photon-steps with window copies
                                     (kinetic_window != 1, plain regime); otherwise within
                                     2^27, or, for beams of more than 2^22 photons, 32
                                     steps within 2^29) */
    int32_t morton_bits;          /* Morton bits of the sort keys, 3..30, or 0 = automatic:
                                     30 (10 per axis) for tril_build/tril_collide; for tril_run,
                                     which first puts both beams in the order of their full
                                     30-bit codes, as many as fit three 8-bit radix passes
                                     beside the step/instance prefix (18..30). Photons with
                                     equal codes keep their order (stable sort). The pair set
                                     does not depend on it. */
    int32_t kinetic_window;       /* tril_run batches: steps served by one copy of the target
                                     hierarchy, >= 0 (0 = automatic: 32, or 16 while the
                                     descents are of 4 steps or fewer; 1 = a copy per step).
                                     A copy holds the boxes of its window's middle step; a
                                     query tests its internal nodes with its own box widened
                                     by the target instance's motion (the bounds of u dt)
                                     over the steps in between, and every leaf that passes
                                     at the leaf's own box of the query's step. Plain regime
                                     only; the candidates, and so the results, do not depend
                                     on it. */
    int32_t descent_window;       /* tril_run batches with window copies: steps served by one
                                     descent of a copy, 0..32, at most the copy's steps. The
                                     descent tests internal nodes with the hull of the widened
                                     boxes of its first and last steps, and every leaf that
                                     passes at the leaf's own boxes of each of its steps.
                                     0 = automatic: 8 steps at first; every tril_stats call
                                     then halves the length when the runs since the previous
                                     call tested more than 0.45 leaves per descent (and does
                                     not take that length again), or doubles it below 0.13.
                                     The results do not depend on it. */
} tril_params;

/* Caller-owned pair buffer. tril_collide appends raw hits (i, j, step) at
 * positions *count, *count + 1, ... (order unspecified) and adds to *count;
 * entries at positions >= cap are counted but not written. The caller sets
 * *count = 0 before the first step of a run (e.g. with hipMemsetAsync). */
typedef struct {
    int64_t cap;
    int32_t *i;                   /* device, cap: query row (beam passed to tril_collide) */
    int32_t *j;                   /* device, cap: target row (beam passed to tril_build) */
    int32_t *step;                /* device, cap: step index k */
    int64_t *count;               /* device, 1 */
} tril_pairs;

typedef struct {
    int64_t n_pairs;          /* unique colliding pairs (after the union over steps) */
    int64_t n_hits;           /* raw (pair, step) hits */
    int64_t n_candidates;     /* broad-phase candidate pairs, summed over steps */
    int64_t n_node_visits;    /* hierarchy nodes whose box was tested, summed over steps */
    int64_t n_queries;        /* query photons sent into the hierarchy, summed over steps */
    int64_t n_sigma_evals;    /* candidates that needed the cross-section evaluation */
    int64_t n_builds;         /* tril_build calls since the last reset */
    int64_t n_collides;       /* tril_collide calls since the last reset */
    double yield;             /* sum over unique pairs of sqrt(w_i w_j) */
    double *spectrum;         /* host, n_bins, caller-owned, or NULL */
    int64_t *step_counts;     /* host, n_step_counts, caller-owned, or NULL: raw hits per step */
    int32_t n_step_counts;    /* steps 0 .. n_step_counts-1 are counted */
    int32_t descent_window;   /* output: steps per descent of the four-child hierarchy copies
                                 in the tril_run calls these counters cover (0: none) */
    double ms_build;          /* with TRIL_TIMING: summed event time of tril_build */
    double ms_query_prep;     /* with TRIL_TIMING: query boxes + Morton order */
    double ms_traverse;       /* with TRIL_TIMING: traversal kernel */
    double ms_narrow;         /* with TRIL_TIMING: narrow-phase kernel */
    int64_t n_timed_launches; /* traversal launches the ms_* sums cover (one per collide call,
                                 one per step batch of tril_run) */
    int64_t n_fp64_rechecks;  /* candidates the FP32 stage of the narrow phase could not decide
                                 and passed to FP64 (0 with TRIL_FP64_NARROW) */
    int64_t n_leaf_checks;    /* hierarchy copies shared by several steps: leaves whose own box
                                 at the query's step was formed and tested, summed over steps */
} tril_stats_t;

/* Create a context on the caller's HIP stream (hipStream_t, NULL = default stream).
 * Validates p on the host before any device call: TRIL_E_INVAL for NULL ctx/p,
 * non-finite or non-positive dt, n_bins < 0, edges NULL or not strictly increasing,
 * negative cand_cap or an unsupported block size. */
int tril_create(tril_ctx **ctx, const tril_params *p, void *hip_stream);

/* Build the hierarchy over `target` for step `step` (>= 0): swept boxes over
 * [step dt, (step+1) dt], Morton keys, radix sort, hierarchy emission, bottom-up
 * box refit. The target arrays must stay unchanged until the step's tril_collide
 * has passed on the stream. TRIL_E_INVAL on bad sizes/offsets; device-side data
 * errors are reported by tril_stats as TRIL_E_DATA. */
int tril_build(tril_ctx *ctx, const tril_beam *target, int32_t step);

/* Query the last built hierarchy with every photon of `query` at the same step
 * and append the hits to `out`. `query` must have the same n_inst as the target
 * (instance m of the query meets instance m of the target). TRIL_E_STATE if no
 * hierarchy was built or the step differs from the build's step. */
int tril_collide(tril_ctx *ctx, const tril_beam *query, int32_t step, tril_pairs *out);

/* Build + collide for steps k0 .. k0+n_steps-1 in one call; the result is the same
 * as calling tril_build/tril_collide for each step. Steps are processed in batches of
 * m consecutive steps (tril_params.step_batch): one set of launches builds the m
 * per-step hierarchies (separate subtrees keyed by step and instance) and one
 * traversal launch answers the queries of all m steps. Full batches are captured once
 * in a HIP graph and replayed, the step index living in device memory; with
 * TRIL_TIMING every batch runs eagerly with HIP events around each phase. Scratch
 * grows with m x (photons per beam): about 150 bytes per photon-step with a copy per
 * step; with window copies about 170 bytes per photon and copy (boxes, flags, binary and
 * four-child nodes) plus 16 bytes of candidate room per photon-step. */
int tril_run(tril_ctx *ctx, const tril_beam *target, const tril_beam *query,
             int32_t k0, int32_t n_steps, tril_pairs *out);

/* Synchronise the stream, then finish the run held in `pairs`:
 *   * if *count > cap: return TRIL_E_OVERFLOW, leave the buffers untouched and
 *     report the required capacity in out->n_hits;
 *   * with TRIL_ANNIHILATE, first reduce the raw hits to the kept ones (see the flag;
 *     the query and target beams of the last tril_run / tril_collide must still hold
 *     their data): each photon then appears in at most one kept hit, out->n_hits
 *     counts kept hits and the step counts count kept hits per step;
 *   * otherwise rewrite pairs->i/j/step in place as the unique pairs in ascending
 *     (i, j) order with their first step, set *count to the number of unique
 *     pairs, and fill `out` (yield, spectrum, step counts, counters).
 * Counters accumulate over builds/collides since create or tril_reset_counters.
 * Also returns TRIL_E_DATA / TRIL_E_OVERFLOW (candidates) / TRIL_E_INTERNAL for
 * errors flagged on the device during the run. `pairs` may be NULL to read the
 * counters only. */
int tril_stats(tril_ctx *ctx, tril_pairs *pairs, tril_stats_t *out);

/* ---------------------------------------------------------------------------------
 * Pair kinematics (Sec. 1, Eq. pTotal and Eq. Lorentz): the electron and positron each
 * colliding photon pair creates, in the lab frame. Per pair (i a query row, j a target
 * row, k its step), FP64:
 *   E_tot = E_i + E_j, p_tot = p_i + p_j;
 *   CoM lepton momentum p' = sqrt((E_tot^2 - p_tot^2) / 4 - m_e^2) (c = 1; the mass term
 *   of Eq. pTotal squared, as its dimensions require), CoM energy E' = sqrt(p'^2 + m_e^2);
 *   isotropic CoM direction n of the positron (the electron takes -n): cos(theta) =
 *   2 u0 - 1, phi = 2 pi u1, u0, u1 = (word >> 11) 2^-53 of the first two 64-bit words of
 *   Philox4x64-10 (Salmon et al., SC'11) at counter (k, i, j, 0), key (seed, 0);
 *   lab velocity by velocity addition (Eq. Lorentz) of b_CoM = p_tot / E_tot and
 *   b' = +-(p'/E') n: (b_CoM + b'_par + b'_perp sqrt(1 - b_CoM^2)) / (1 + b'.b_CoM), with
 *   b'_par the component of b' along b_CoM and b'_perp = b' - b'_par;
 *   gamma = 1 / sqrt(1 - b^2), E = gamma m_e, p = gamma m_e b.
 * A pair below threshold (s_ij <= 1, never a hit) gets p' = 0: both leptons move with the
 * CoM. Histograms of the positron, each pair weighted by sqrt(w_i w_j): Lorentz factor
 * gamma = E / m_e on caller edges (bin b holds edges[b] <= gamma < edges[b+1]; values
 * outside are dropped) and polar angle of its momentum to +z, n_theta equal bins over
 * [0, pi] (angle pi falls in the last bin).
 * ------------------------------------------------------------------------------- */
#define TRIL_KIN_MAX_BINS 2048

typedef struct {
    uint64_t seed;                /* key word 0 of the direction generator */
    int32_t n_gamma;              /* Lorentz-factor bins, 0 .. TRIL_KIN_MAX_BINS */
    int32_t n_theta;              /* polar-angle bins, 0 .. TRIL_KIN_MAX_BINS */
    const double *gamma_edges;    /* host, n_gamma + 1 finite, strictly increasing; may be
                                     NULL if n_gamma == 0 */
} tril_kin_params;

typedef struct {
    double *gamma_hist;           /* host, n_gamma, caller-owned (NULL if n_gamma == 0) */
    double *theta_hist;           /* host, n_theta, caller-owned (NULL if n_theta == 0) */
    double ms_kernel;             /* output: kernel time from HIP events on the stream */
} tril_kin_out;

/* Leptons and positron histograms of the first n entries of `pairs` (pairs->count is not
 * read; n <= pairs->cap), typically the unique pairs tril_stats leaves in the buffer or the
 * kept hits of TRIL_ANNIHILATE. query and target are the beams the rows index (instance
 * offsets are not used). leptons: device, 8 n doubles (positron E px py pz, then electron E
 * px py pz, per pair), or NULL. Synchronises the context's stream. TRIL_E_INVAL for bad
 * arguments or when a pair names a row outside its beam or a negative step (such pairs are
 * skipped; the others are written). */
int tril_pair_kinematics(tril_ctx *ctx, const tril_beam *query, const tril_beam *target,
                         const tril_pairs *pairs, int64_t n, const tril_kin_params *params,
                         double *leptons, tril_kin_out *out);

/* tril_pair_kinematics for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): no context, no
 * allocation, no synchronisation; everything is enqueued on `stream`. Its scratch (the
 * histogram accumulators, an error flag and up to 2^18 packed photon records, 16 MiB in
 * all) is a device array inside the library that every device holds from the first call
 * on it until the process ends; calls that overlap on one device share it and race.
 * Same leptons and histograms as tril_pair_kinematics for the same arguments (histogram
 * sums up to their order); when the two beams together hold more than 2^18 photons the
 * kernel reads them unpacked. gamma_edges: device, n_gamma + 1 finite, strictly
 * increasing; gamma_hist (n_gamma) and theta_hist (n_theta): device, caller-owned,
 * overwritten; status: device int32, receives TRIL_OK, or TRIL_E_INVAL when the edges are
 * not increasing or a pair names a row outside its beam or a negative step (such pairs are
 * skipped). Returns TRIL_E_INVAL for bad arguments (including n_gamma or n_theta above
 * TRIL_KIN_MAX_BINS, the bins its accumulators hold), TRIL_E_HIP for a launch failure. */
int tril_pair_kinematics_noalloc(const tril_beam *query, const tril_beam *target,
                                 const tril_pairs *pairs, int64_t n, uint64_t seed,
                                 int32_t n_gamma, const double *gamma_edges, int32_t n_theta,
                                 double *leptons, double *gamma_hist, double *theta_hist,
                                 int32_t *status, void *hip_stream);

/* Launch configuration of tril_run (performance only: the results do not depend on it). */
typedef struct {
    int32_t block_traverse;       /* traversal workgroup size: 64, 128, 256 or 512 */
    int32_t step_batch;           /* steps per launch, >= 1 (0 = automatic) */
    int32_t morton_bits;          /* 0 (automatic) or 3..30, as in tril_params */
    int32_t traverse_queue;       /* 0: one traversal workgroup per block of queries (a flat
                                     grid); 1: a persistent grid whose waves take chunks of
                                     1024 queries from device-wide work queues */
    int32_t kinetic_window;       /* steps per copy of the target hierarchy, as in
                                     tril_params (0 = automatic, 1 = per step) */
    int32_t descent_window;       /* steps per descent of a copy, 0..32, as in tril_params
                                     (0 = automatic) */
    double ms_per_step;           /* tril_autotune: measured time per step of the best
                                     configuration (output; ignored by tril_set_tune) */
} tril_tune;

/* Autotuner: time tril_run over steps k0 .. k0+n_probe-1 of the given beams for a set of
 * launch configurations and keep the fastest in the context (and in *best). Coordinate
 * descent: steps per launch (the automatic choice, then 1 .. 128 within 2^27 photon-steps
 * per launch, or within 32 steps' worth for larger beams), then the
 * steps per hierarchy copy (1, 4, 8, 16, 32), then the steps per descent (4, 8, 16, 32,
 * with copies of several steps), then the
 * traversal workgroup size (64 .. 512), then the Morton bits (automatic or 30), then the
 * persistent work-queue traversal against the flat grid. Every
 * configuration runs twice (the first run captures its graphs and sizes the scratch);
 * the second is timed with HIP events on the context stream. Hits go to a scratch buffer
 * owned by the call; the counters are reset at the end (as tril_reset_counters).
 * Synchronises the stream. TRIL_E_INVAL for bad arguments or n_probe < 1. */
int tril_autotune(tril_ctx *ctx, const tril_beam *target, const tril_beam *query, int32_t k0,
                  int32_t n_probe, tril_tune *best);

/* Apply a launch configuration (e.g. one stored from an earlier tril_autotune).
 * TRIL_E_INVAL for values outside the ranges above. */
int tril_set_tune(tril_ctx *ctx, const tril_tune *tune);

/* ---------------------------------------------------------------------------------
 * Statistical (ST) regime (Sec. 2.2, rate between two clouds of particles). Every
 * photon macro-particle is a uniform cloud filling a box of the binning grid's cell
 * size c = (c_x, c_y, c_z) about its position, density n = w / V with V = c_x c_y c_z.
 * Over step k, with mid-step time t_m = k dt + dt/2, the pair (i, j) yields
 *   Y_ij,k = n_i n_j sigma_BW(s_ij) (1 - u_i.u_j) dt V_ov(t_m)
 * (V_ov: intersection volume of the two clouds at t_m; (1 - u_i.u_j) c the two-photon
 * rate factor of the paper's reactivity; sigma = 0 at and below threshold). Yields are
 * summed over steps and over the macro-particle pairs of each bin pair.
 * ------------------------------------------------------------------------------- */

/* Binning grid of one beam: position cell of X(t_bin) in the lab box [lo, hi]
 * (n_pos cells per axis), energy bin log-spaced on [e_lo, e_hi] (n_e bins), polar-angle
 * bin of the direction about `axis` on [0, th_max] (n_th bins); values outside a range
 * fall in its edge bin. bin = (((ix ny + iy) nz + iz) n_e + ie) n_th + ith. */
typedef struct {
    double lo[3], hi[3];          /* [um], hi > lo */
    int32_t n_pos[3];             /* >= 1 each */
    int32_t n_e;                  /* >= 1 */
    double e_lo, e_hi;            /* [MeV], 0 < e_lo < e_hi */
    int32_t n_th;                 /* >= 1 */
    int32_t pad0;
    double th_max;                /* [rad], > 0 */
    double axis[3];               /* unit vector */
    double t_bin;                 /* [um/c] */
} tril_st_grid;

/* Bin index of every photon (device bins[n], -1 for invalid photon data) and, if sums is
 * not NULL, per-bin sums (device sums[8 x number of bins], caller-zeroed, accumulated):
 * w, w E, w ux, w uy, w uz, w X, w Y, w Z (X the position at t_bin). Asynchronous on
 * the HIP stream (NULL = default).
 * TRIL_E_INVAL for bad arguments or more than 2^31 - 1 bins. */
int tril_st_bin(const tril_beam *beam, const tril_st_grid *grid, int32_t *bins, double *sums,
                void *hip_stream);

/* Caller-owned bin-pair table (open addressing): cap slots, a power of two;
 * key[slot] = query bin x n_target_bins + target bin, or -1 for an empty slot;
 * yield[slot] = summed yield. tril_st_exact clears it first. */
typedef struct {
    int64_t cap;
    int64_t *key;                 /* device, cap */
    double *yield;                /* device, cap */
} tril_st_table;

/* Exact ST yields for steps k0 .. k0+n_steps-1: clouds of the target beam in a
 * hierarchy per step (boxes of edges `cell` about the mid-step positions), clouds of the
 * query beam descending it, Y evaluated in FP64 for every overlapping pair and added to
 * the table under (q_bins[i], t_bins[j]). Bins are per caller row (from tril_st_bin);
 * pairs with a negative bin are skipped. *total (host) receives the sum of all yields.
 * Synchronous. TRIL_E_OVERFLOW if the table filled up; TRIL_E_DATA for invalid photon
 * data; TRIL_E_INVAL for bad arguments (cell not finite and > 0, cap not a power of two,
 * n_target_bins < 1 or >= 2^31). Counters accumulate as for tril_run (node visits; cloud
 * pair-steps with a yield in n_candidates). */
int tril_st_exact(tril_ctx *ctx, const tril_beam *target, const int32_t *t_bins,
                  int64_t n_target_bins, const tril_beam *query, const int32_t *q_bins,
                  const double cell[3], int32_t k0, int32_t n_steps, tril_st_table *table,
                  double *total);

/* Exact ST yields with depletion (Sec. 2.2: the rate equation with the loss of collision
 * partners, integrated in closed form). The printed reactivity is read as
 * k = sigma c (1 - cos phi). Per cloud pair (i, j) the exposure over steps k0 ..
 * k0+n_steps-1,
 *   S_ij = sum_k sigma(s_ij) (1 - u_i.u_j) dt V_ov(t_m) / V        (k tau of the closed forms),
 * takes the place of k tau; with a = w_i / V, b = w_j / V, n0 = a + b:
 *   a == b:  n = (n0/2)^2 S / (1 + (n0/2) S)                                      (n_1/2)
 *   a != b:  n = (alpha - 1) alpha n0 (1 - e^X) / (alpha e^X + alpha - 1),         (n_alpha)
 *            alpha = min(a, b) / n0, X = n0 (2 alpha - 1) S,
 * and the pair yields V n (never more than min(w_i, w_j); V n -> the linear yield of
 * tril_st_exact as a S, b S -> 0). Each pair is depleted by its own creations only.
 * pair_table (cleared first, cap a power of two) receives one slot per cloud pair with a
 * positive exposure: key i * target->n + j (caller rows), yield = the pair's depleted yield;
 * table and *total as for tril_st_exact, with depleted yields. Synchronous; errors as for
 * tril_st_exact (TRIL_E_OVERFLOW when either table filled up). */
int tril_st_exact_depleted(tril_ctx *ctx, const tril_beam *target, const int32_t *t_bins,
                           int64_t n_target_bins, const tril_beam *query, const int32_t *q_bins,
                           const double cell[3], int32_t k0, int32_t n_steps,
                           tril_st_table *pair_table, tril_st_table *table, double *total);

/* Individual-particle (IP) regime with swarms (Sec. 2.2): when two macro-particles meet,
 * each is split into real photons with its momentum, spread over its volume and held in an
 * octree, and the real photons are tested one by one. Here macro-particle i is
 * floor(w_i + 1/2) real photons (at most 2^30; more is TRIL_E_DATA) at the centres of the
 * cells of a level-L octree over its cloud box (edges `cell` about its position; 8^L >= n,
 * L smallest); real photon k takes, at level l, the octant given by base-8 digit l of k
 * (lowest digit = top level; digit bits 2, 1, 0 = upper half along x, y, z), so any count
 * spreads evenly. Two real photons collide when their time-synchronous distance over the
 * run window [k0 dt, (k0 + n_steps) dt] comes within r, r^2 = sigma(s) / pi (weight 1 each;
 * s of their macro-particles, s > 1). Macro-particle pairs are found through the hierarchy
 * of the clouds swept over each step. pair_table (cleared first) receives one slot per
 * macro-particle pair whose swept clouds meet above threshold: key i * target->n + j,
 * yield = its number of colliding real pairs (an integer, as a double); table (cleared
 * first) the counts per (q_bins[i], t_bins[j]); *total (host) their sum. No consumption:
 * a real photon may collide with several. Synchronous; errors as for tril_st_exact. */
int tril_ip_swarm(tril_ctx *ctx, const tril_beam *target, const int32_t *t_bins,
                  int64_t n_target_bins, const tril_beam *query, const int32_t *q_bins,
                  const double cell[3], int32_t k0, int32_t n_steps, tril_st_table *pair_table,
                  tril_st_table *table, int64_t *total);

/* ---------------------------------------------------------------------------------
 * Surrogate path of the statistical regime (uses the network declared below).
 *
 * Every occupied bin becomes one cloud: the bin's total weight at its weighted-mean
 * position (at t_bin), mean direction and mean energy. Bin clouds of edge
 * cloud_factor x cell go through the same hierarchy. A bin's mean position lies in its
 * cell at t_bin, so when two macro-particle clouds overlap at time t their bins' mean
 * positions differ by less than 3 cells plus 2 theta |t - t_bin| per axis (theta the
 * largest angle between a photon's direction and its bin's mean direction): with
 * cloud_factor above that bound every overlapping pair of an interior cell is a candidate
 * (3.5 for 10 mrad beams over +-20 um/c of 0.5 um cells; edge cells, which also hold the
 * photons outside the grid, have no such bound). Each candidate bin pair gets
 * Omega_ab = sum over steps of dt V_ov. Features of a bin pair: log E_a, log E_b,
 * log(1 - cos theta_ab), log rho_a, log rho_b, log Omega_ab (rho = total weight / cell
 * volume, theta between the mean directions). The bin-level yield
 * Y0 = rho_a rho_b sigma(s_ab) (1 - cos theta_ab) Omega_ab is the estimate without
 * the network; the network predicts log((Y + eps Y0) / Y0) of the exact bin-pair yield Y,
 * so Y = Y0 (exp(prediction) - eps). Bin pairs the ensemble is unsure of (see gate_mode)
 * are computed exactly.
 * ------------------------------------------------------------------------------- */
typedef struct {
    double cloud_factor;          /* bin cloud edge / cell edge, >= 1 (0 = 3.5) */
    double eps;                   /* floor of the predicted yield ratio (0 = 1e-3) */
    double gate;                  /* ensemble standard deviation above which a bin pair
                                     takes the exact path (0 = 0.01) */
    double scale;                 /* factor on the predicted yields (0 = 1): the ratio of
                                     exact to predicted total on the training rows, which
                                     removes the bias of predicting a mean logarithm */
    int32_t gate_mode;            /* 0 (budget): the bin pairs with the largest uncertainty
                                     contributions u = Yhat x ensemble spread go to the exact
                                     path until the spread of the remaining predicted total,
                                     sqrt(sum u^2), is at most gate x the predicted total;
                                     1 (per pair): every bin pair whose spread exceeds gate;
                                     2 (audit): no bin pair is gated; the total is the sampled
                                     estimate of the exact total (tril_st_audit) with the
                                     network's predictions as its control, which measures and
                                     removes the bias the ensemble members share; its 95%
                                     confidence half-width goes to predicted_spread (relative)
                                     and audit_half_width */
    int32_t pad0;
    int64_t audit_sample;         /* gate_mode 2: expected macro-particles drawn per beam and
                                     replicate (0 = 32768) */
    int32_t audit_reps;           /* gate_mode 2: replicates, 2..64 (0 = 8) */
    int32_t pad1;
    uint64_t audit_seed;          /* gate_mode 2: key of the draws */
} tril_st_sur_params;

typedef struct {
    double total;                 /* surrogate part + exact part */
    double surrogate_part;        /* sum over confident bin pairs of the predicted yield */
    double exact_part;            /* exact yield of the gated bin pairs (audit mode: the
                                     audit's correction, total - surrogate_part) */
    int64_t n_bin_pairs;          /* candidate bin pairs (feature rows) */
    int64_t n_gated;              /* bin pairs sent to the exact path */
    double ms;                    /* event time of the whole call on the context stream */
    double predicted_spread;      /* budget mode: ensemble spread of the surrogate part
                                     relative to the predicted total; audit mode: the 95%
                                     confidence half-width relative to the total */
    double audit_half_width;      /* audit mode: 95% confidence half-width of the total */
    int64_t audit_sampled;        /* audit mode: macro-particles drawn (both beams, all
                                     replicates) */
} tril_st_sur_result;

/* Feature rows of all candidate bin pairs of the two beams' per-bin sums (as written by
 * tril_st_bin) over steps k0 .. k0+n_steps-1: x [n][6] FP32, y0 [n] FP64, key [n]
 * (query bin x n_target_bins + target bin), all device, rows in ascending key order (the
 * same rows in the same order on every call). *n receives the number of rows;
 * TRIL_E_OVERFLOW when it exceeds cap; TRIL_E_NOMEM when the context's bin-pair table
 * could not hold the candidate pairs after growing 64-fold. The two grids must have the
 * same cell. Uses the context's stream and scratch and clears its device error flags.
 * Synchronous. */
int tril_st_features(tril_ctx *ctx, const double *q_sums, const tril_st_grid *q_grid,
                     const double *t_sums, const tril_st_grid *t_grid, int32_t k0, int32_t n_steps,
                     const tril_st_sur_params *params, float *x, double *y0, int64_t *key,
                     int64_t cap, int64_t *n);

/* Training targets of feature rows: target[i] = log((Y + eps y0[i]) / y0[i]) with Y the
 * yield of key[i] in an exact table (0 if absent); y_exact (device, or NULL) receives Y.
 * Asynchronous on the HIP stream. */
int tril_st_targets(const int64_t *key, const double *y0, int64_t n, const tril_st_table *exact,
                    double eps, float *target, double *y_exact, void *hip_stream);

/* Surrogate path for one instance: features, ensemble prediction, gate, and an exact
 * pass (tril_st_exact restricted to the photons of gated bins and to the gated bin
 * pairs) for the gated bin pairs. Synchronous. */
int tril_st_surrogate(tril_ctx *ctx, struct tril_mlp *mlp, const tril_beam *target,
                      const int32_t *t_bins, const double *t_sums, const tril_st_grid *t_grid,
                      const tril_beam *query, const int32_t *q_bins, const double *q_sums,
                      const tril_st_grid *q_grid, int32_t k0, int32_t n_steps,
                      const tril_st_sur_params *params, tril_st_sur_result *out);

/* Sampled estimate of the exact statistical-regime total over steps k0 .. k0+n_steps-1
 * (the sum of tril_st_exact's yields), for instances whose exact pass over all
 * macro-particle pairs is out of reach. Each replicate thins both beams independently
 * (macro-particle i kept with probability pi_i, weight w_i / pi_i, Philox4x64-10 draws
 * keyed by (seed, replicate)), runs the exact pass over the two thinned beams, and adds
 * the known total of a control minus the thinned beams' estimate of it:
 *   T_hat = C + sum_{kept i, j} Y_ij / (pi_i pi_j) - sum_ab c_ab (R_a / W_a) (R_b / W_b),
 * c_ab the control of candidate bin pair (a, b) (the rows of tril_st_features), C their
 * sum, W_a the weight in bin a and R_a the kept weight w_i / pi_i in it. T_hat is unbiased
 * for the exact total (the yield of a cloud pair is linear in each weight, Sec. 2.2, and
 * the two beams are thinned independently) whatever the control; a control close to the
 * yields makes it precise. pi_i = min(1, n_sample (mix c_a w_i / (W_a C) + (1 - mix)
 * w_i / W)), c_a the control summed over bin a's pairs, W the beam's total weight. With a
 * control, a pilot replicate with draws of its own first fits its scale,
 * kappa = (exact pass over the pilot's thinned beams) / (their estimate of C), and every
 * replicate uses kappa c_ab (the pilot is independent of the replicates, which therefore
 * stay unbiased); this removes the arbitrary scale of Y0 and the bias a network's members
 * share. */
typedef struct {
    int64_t n_sample;             /* expected macro-particles drawn per beam and replicate
                                     (0 = 32768) */
    int32_t n_rep;                /* replicates, 2..64 (0 = 8) */
    int32_t control;              /* 0: the network's predicted yields (mlp required, eps and
                                     scale from the surrogate parameters); 1: the bin-level
                                     yield Y0 of the feature rows (no network); 2: none */
    uint64_t seed;                /* key of the draws */
    double mix;                   /* share of pi proportional to the control, [0, 1)
                                     (0 = 0.9) */
} tril_st_audit_params;

typedef struct {
    double estimate;              /* mean of the replicate estimates */
    double half_width;            /* 95% confidence half-width: Student t quantile (n_rep - 1
                                     degrees of freedom) x standard error of the mean */
    double control_total;         /* kappa C */
    double control_scale;         /* kappa (1 without a control) */
    double rep[64];               /* replicate estimates (n_rep of them) */
    int32_t n_rep;
    int32_t pad0;
    int64_t n_sampled[2];         /* query, target macro-particles drawn over all replicates */
    int64_t n_bin_pairs;          /* candidate bin pairs (control rows) */
    double ms;                    /* event time of the whole call on the context stream */
} tril_st_audit_result;

/* Same beams, bins, per-bin sums and grids as tril_st_surrogate; mlp may be NULL unless
 * control is 0; sur_params (or NULL for defaults) gives cloud_factor, eps and scale.
 * Synchronous. TRIL_E_INVAL for bad arguments, TRIL_E_NOTIMPL for more than one
 * instance. */
int tril_st_audit(tril_ctx *ctx, struct tril_mlp *mlp, const tril_beam *target,
                  const int32_t *t_bins, const double *t_sums, const tril_st_grid *t_grid,
                  const tril_beam *query, const int32_t *q_bins, const double *q_sums,
                  const tril_st_grid *q_grid, int32_t k0, int32_t n_steps,
                  const tril_st_sur_params *sur_params, const tril_st_audit_params *params,
                  tril_st_audit_result *out);

/* Calibration factor of the surrogate (the `scale` of tril_st_sur_params): the exact over
 * the predicted total on n feature rows, sum(y_exact) / sum(max(0, y0 (exp(mean) - eps)))
 * with the ensemble mean of the network; x [n][6] FP32, y0 and y_exact [n] FP64, device.
 * The sums are reduced in a fixed order (the same result on every call). Synchronous. */
int tril_st_calibrate(struct tril_mlp *mlp, const float *x, const double *y0,
                      const double *y_exact, int64_t n, double eps, double *scale);

/* ---------------------------------------------------------------------------------
 * Surrogate of the statistical regime: an ensemble of K multilayer perceptrons
 * 6 -> 256 -> 256 -> 256 -> 1 (SiLU) mapping the six features of a bin pair to its log
 * yield; BF16 weights and activations on the matrix cores with FP32 accumulation, FP32
 * master weights trained with Adam on the mean squared error. Parameters of one member,
 * flattened FP32 (133,633): W1 [256][6], b1 [256], W2 [256][256], b2, W3 [256][256], b3,
 * W4 [256], b4 [1]. Inputs and targets are standardised with the model's normalisation
 * (tril_mlp_set_norm or tril_mlp_fit_norm) before the first layer; outputs are returned
 * de-standardised. Device buffers are row-major FP32: x [n][6], y [n].
 * ------------------------------------------------------------------------------- */
/* K members (1..64) initialised from `seed` (He-uniform, member k from its own stream),
 * working on the given HIP stream. */
int tril_mlp_create(tril_mlp **out, int32_t n_members, uint64_t seed, void *hip_stream);
void tril_mlp_destroy(tril_mlp *m);
/* Member's FP32 parameters to or from host memory (n must be 133,633). */
int tril_mlp_set_params(tril_mlp *m, int32_t member, const float *host, int64_t n);
int tril_mlp_get_params(tril_mlp *m, int32_t member, float *host, int64_t n);
/* Normalisation: given (host, 6 means and 6 sd > 0; target mean and sd > 0), or fitted
 * as the column means and standard deviations of the device data x [n][6], y [n]. */
int tril_mlp_set_norm(tril_mlp *m, const float *mu_x, const float *sd_x, float mu_y, float sd_y);
int tril_mlp_fit_norm(tril_mlp *m, const float *x, const float *y, int64_t n);
/* Loss (mean squared error of the standardised output over the n rows, host) and its
 * gradient with respect to every parameter of `member` (host, 133,633), no update. */
int tril_mlp_grad(tril_mlp *m, int32_t member, const float *x, const float *y, int64_t n,
                  float *host_grad, double *host_loss);
/* Train every member for n_steps Adam steps (beta 0.9, 0.999, eps 1e-8, learning rate
 * lr) on minibatches of `batch` rows drawn with replacement by a counter-based hash of
 * (seed, member, step, row). host_loss: NULL or K values, the mean loss of the last tenth
 * of the steps. Synchronous. */
int tril_mlp_train(tril_mlp *m, const float *x, const float *y, int64_t n, int32_t n_steps,
                   int32_t batch, float lr, uint64_t seed, double *host_loss);
/* Ensemble mean and sample standard deviation over the members of the de-standardised
 * output, per row (device, n each). Synchronous. */
int tril_mlp_predict(tril_mlp *m, const float *x, int64_t n, float *mean, float *sdev);

/* Zero the accumulated counters and device error flags (synchronises the context
 * stream). After a call that left a device error flag set, later builds are valid only
 * once this has run: it also clears the hierarchy's scratch that such an interrupted
 * build may have left behind. */
int tril_reset_counters(tril_ctx *ctx);

void tril_destroy(tril_ctx *ctx);
const char *tril_strerror(int code);
/* Text of the last HIP error this thread saw inside the library ("" if none). */
const char *tril_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TRIL_H */
