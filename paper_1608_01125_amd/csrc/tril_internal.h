// Internal declarations of libtril (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "tril.h"

namespace tril {

constexpr double kMe = 0.51099895000;      // electron rest energy [MeV]
constexpr double kRe = 2.8179403262e-9;    // classical electron radius [um]

// Device-side error bits (DevCounters::err).
constexpr uint32_t kErrData = 1u;          // non-finite input, E <= 0, w < 0 or |p| != E
constexpr uint32_t kErrCandOverflow = 2u;  // broad-phase candidate buffer full
constexpr uint32_t kErrSpin = 4u;          // a bounded device loop or stack ran out
constexpr uint32_t kErrPairOverflow = 8u;  // caller pair buffer full
constexpr uint32_t kErrTableFull = 16u;    // statistical-regime bin-pair table full
constexpr uint32_t kErrInternal = 32u;     // an internal invariant failed (four-child forms)

// Breit-Wheeler total cross-section (Eq. 1) [um^2], 0 at and below threshold, written
// as (pi r_e^2 / 2) / s [ (3 - b^4) L - 2 b (2 - b^2) ] with b^2 = (s-1)/s and
// L = 2 log1p(b) + ln s (Eq. 1 with 1 - beta^2 = 1/s, free of its cancellations).
__device__ __forceinline__ double bw_sigma(double s) {
    if (!(s > 1.0)) return 0.0;
    const double k_sig = (0.5 * M_PI) * (kRe * kRe);
    const double b2 = (s - 1.0) / s;
    const double b = sqrt(b2);
    const double L = 2.0 * log1p(b) + log(s);
    const double br = (3.0 - b2 * b2) * L - (2.0 * b) * (2.0 - b2);
    return (k_sig / s) * br;
}

// One internal hierarchy node, 64 bytes: the boxes of its two children and their
// links (c[0] left, c[1] right), so that one load tests both children and a child
// whose box fails is never loaded. A link >= 0 is the id of an internal node; a link
// <= -2 is a leaf holding target element -2 - link (leaf_link / link_elem). The root's
// own box is stored nowhere: a descent starts by testing the root's children. Step s
// of a batch of m steps over n rows owns internal nodes s (n-1) + x, x in [0, n-1).
struct alignas(16) Half {
    float lox, loy, loz;
    int32_t link;
    float hix, hiy, hiz;
    int32_t pad;
};
struct alignas(16) Node {
    Half c[2];
};
static_assert(sizeof(Half) == 32 && sizeof(Node) == 64, "node layout");

// Quantisation frame of one window copy: every leaf box of the copy's step (all
// instances) lies in the box [base, base + 65535 / inv] per axis, so a box of the copy is
// kept as 16-bit cell indices: floor((lo - base) inv) - 1 and ceil((hi - base) inv) + 1
// clamped to [0, 65535] (the one-cell margins cover the FP32 rounding of the products,
// below 0.02 cells).
struct WinFrame {
    float4 base;  // xyz
    float4 inv;   // xyz: cells per unit length
};

// Four-child form of internal node x of a window copy (64 bytes): the node's grandchildren
// (or, where x's child on a side is a leaf, that leaf and an empty slot), so that a descent
// visiting only these forms from the root tests two levels of the binary hierarchy per load
// and halves its chain of dependent loads. Slot k's box, in the copy's frame cells, is
// words 3k..3k+2 (lo x | lo y << 16, lo z | hi x << 16, hi y | hi z << 16; an empty slot
// has lo > hi and meets nothing). Slots 0 and 1 are the children g0 and g0 + 1 of x's left
// child (word 12; internal node ids of the copy or sorted leaf positions), slots 2 and 3
// those of its right child (g2 in word 13); a leaf child of x takes slot 0 or 2 itself. Words
// 14 and 15 hold slots 0, 1 and 2, 3: each slot's subtree energy bound as the top 15 bits of
// its FP32 value rounded up (bits 0-14, 16-30) and its leaf flag (bit 15, 31).
struct alignas(16) CNode4 {
    uint32_t w[16];
};
static_assert(sizeof(CNode4) == 64, "four-child node layout");
// Most steps of one descent over four-child forms: a descent serves consecutive steps of
// one window copy and keeps a leaf's hits as one bit per step of a 32-bit mask.
constexpr int32_t kMaxDescent = 32;
__host__ __device__ inline int32_t leaf_link(int64_t e) { return (int32_t)(-2 - e); }
__host__ __device__ inline int64_t link_elem(int32_t l) { return -2 - (int64_t)l; }

// Parent record of a hierarchy node (internal or leaf), 16 bytes, written by the
// emission kernel for both children of every internal node:
//   parent: id of the parent (-1 for the root, node 0);
//   sib:    id of the sibling, bit 31 set when this node is the right child;
//   lo, hi: the parent's range of sorted leaf positions.
struct alignas(16) PRec {
    int32_t parent;
    int32_t sib;
    int32_t lo;
    int32_t hi;
};
static_assert(sizeof(PRec) == 16, "record layout");

// Swept, padded box of one photon (FP32, rounded outward), 32 bytes.
//   tag: instance index of the photon, or -1 when the photon can collide with
//        nothing (query photons whose best case is below threshold).
struct alignas(16) PBox {
    float lox, loy, loz;
    int32_t tag;
    float hix, hiy, hiz;
    int32_t pad;
};
static_assert(sizeof(PBox) == 32, "box layout");

// Query record of one photon for a batch of steps (48 bytes): a photon moves on a
// straight line, so its swept box at step offset s is the box at offset 0 moved by
// s u dt. lo: the offset-0 box's low corner (FP32, rounded outward, radius pad
// included); inst: its instance, or -1 when it can collide with nothing; d: u dt
// (FP32, nearest); e: its energy rounded up (the threshold prune); w: the box widths
// (FP32, rounded up). The traversal forms lo + s d and lo + s d + w and widens both by a
// bound on that FP32 arithmetic, so the box contains the one the step's own FP64
// computation rounds outward.
struct alignas(16) QRec {
    float lox, loy, loz;
    int32_t inst;
    float dx, dy, dz;
    float e;
    float wx, wy, wz;
    float unused;
};
static_assert(sizeof(QRec) == 48, "query record layout");

// Box at step offset s of a batch from the box at offset 0 (low corner lo0, widths w
// rounded up) and its motion per step d = u dt (FP32, nearest). Each of the rounded
// quantities carries at most 2^-24 relative error: d (as rounded from u dt, scaled by s),
// the fma lo0 + s d, the sum hi = lo + w, and the final widening itself; together less
// than 2^-23 (|lo| + |hi| + s |d|), and the widening is four times that. The result
// contains the box that the step's own FP64 computation rounds outward (whose 1e-12
// relative slack grows by less than 1e-12 s |d| over the batch).
// One axis of it (every axis is formed on its own).
__device__ __forceinline__ void moved_axis(float lo0, float d, float w, float s, float &lo,
                                           float &hi) {
    const float l = fmaf(s, d, lo0);
    const float h = l + w;
    const float e = ((fabsf(l) + fabsf(h)) + s * fabsf(d)) * 0x1p-21f;
    lo = l - e;
    hi = h + e;
}
__device__ __forceinline__ void moved_box(float lox, float loy, float loz, float dx, float dy,
                                          float dz, float wx, float wy, float wz, float s,
                                          float lo[3], float hi[3]) {
    moved_axis(lox, dx, wx, s, lo[0], hi[0]);
    moved_axis(loy, dy, wy, s, lo[1], hi[1]);
    moved_axis(loz, dz, wz, s, lo[2], hi[2]);
}

// Window copies of a batch's hierarchy. Photons move on straight lines, so the box of a
// target leaf at step offset s lies in its box at another offset r moved by (s - r) u dt,
// and u dt of every photon of an instance lies in that instance's per-axis bounds. A
// batch of m steps may therefore keep one copy of the shape per window of W consecutive
// steps, filled with the boxes of the window's middle step r, instead of one per step:
// a query of step s tests internal nodes with its box widened by the instance's motion
// over s - r (plus a rounding slack), which holds every box the subtree's leaves have at
// step s, and tests a leaf that passes against the leaf's own box at step s, formed from
// the leaf's record exactly as the per-step refit forms it. The candidates are those of
// per-step copies; only the internal nodes a query visits change.
__host__ __device__ inline int32_t window_copies(int32_t m, int32_t win) {
    return win > 1 ? (m + win - 1) / win : m;
}
__host__ __device__ inline int32_t window_ref_step(int32_t cp, int32_t win, int32_t m) {
    if (win <= 1) return cp;
    const int32_t a = cp * win;
    const int32_t len = a + win <= m ? win : m - a;
    return a + (len - 1) / 2;
}

// Target record of one sorted leaf position for a batch (48 bytes): the leaf's box at
// step offset 0 (low corner lo, widths w rounded up) and its motion per step d = u dt,
// as the refit forms every step's leaf box from them (moved_box); row: the target row;
// e: the photon's energy rounded up, 0 for a photon that can collide with nothing.
struct alignas(16) TRec {
    float lox, loy, loz;
    int32_t row;
    float dx, dy, dz;
    float e;
    float wx, wy, wz;
    int32_t pad;
};
static_assert(sizeof(TRec) == 48, "target record layout");

// Bounds of u dt over the photons of one target instance, per axis, as FP32 values the
// refit's rounding of u dt cannot leave (lo: lowest, hi: highest; .w unused).
struct WinBound {
    float4 lo, hi;
};

// What a traversal over window copies needs besides the nodes.
struct WinArgs {
    const TRec *trec;      // per sorted target position
    const WinBound *vb;    // per target instance
    const CNode4 *nodes4;  // four-child forms of the copies' nodes (nullptr: binary descent)
    const WinFrame *frames;  // per copy: the quantisation frame of nodes4
    int32_t win;           // steps per copy (>= 2)
    int32_t m;             // steps of the launch
    int64_t n;             // target rows (element of row j at step s: s n + j)
    float reach;           // (m + win + 8) dt + 1e-6: the slack's length term (wslack)
    int32_t dwin;          // four-child forms: steps per descent, 1 .. min(win, kMaxDescent)
};
// Four-child forms: descents of a batch of m steps in copies of win steps, each copy's
// steps split into descents of dwin steps (the last one of a copy shorter).
__host__ __device__ inline int64_t descent_count(int32_t m, int32_t win, int32_t dwin) {
    const int32_t copies = window_copies(m, win);
    const int32_t last = m - (copies - 1) * win;
    return (int64_t)(copies - 1) * ((win + dwin - 1) / dwin) + (last + dwin - 1) / dwin;
}

// Slack of the widened query box on one axis (ql, qh: the query's box at step s). If a
// leaf's box at step s (moved_box, every FP32 operation within 2^-24 relative) meets
// [ql, qh], its coordinates are at most M = max(|ql|, |qh|) plus its width (at most
// 1.01 dt + 1e-11 (1 + M): target boxes carry no radius pad), so the rounding of its
// boxes at s and at the copy's step r, and of the widened box itself, stays below
// (M + (m + 2) dt) 2^-19: the slack below is at least twice that.
__device__ __forceinline__ float wslack(float ql, float qh, float reach) {
    return (fmaxf(fabsf(ql), fabsf(qh)) + reach) * 0x1p-18f;
}

// Philox4x64-10 (Salmon et al., SC'11), the counter-based generator of the pair kinematics
// and of the statistical regime's audit samples.
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

// Philox4x64-10: ten rounds; each round multiplies words 0 and 2 by the two round
// constants into 128-bit products, the high halves crossed with words 1 and 3 and the
// round key, the low halves moved to the odd words; the key advances by the Weyl
// constants between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t x[4], uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t lo0 = kPhiloxM0 * x[0], hi0 = __umul64hi(kPhiloxM0, x[0]);
        const uint64_t lo1 = kPhiloxM1 * x[2], hi1 = __umul64hi(kPhiloxM1, x[2]);
        const uint64_t y0 = hi1 ^ x[1] ^ k0;
        const uint64_t y2 = hi0 ^ x[3] ^ k1;
        x[0] = y0;
        x[1] = lo1;
        x[2] = y2;
        x[3] = lo0;
    }
}

// Counters accumulated on the device across steps. Counters that every wave of a
// large launch updates are spread over kCounterSlots addresses (slot = block index
// modulo kCounterSlots): device-scope atomics to one address serialise at roughly
// 10 ns each, so one address per counter would cost ~0.3 ms per million queries.
constexpr int kCounterSlots = 256;
constexpr int kTravCursors = 8;
struct DevCounters {
    unsigned long long cand_step;      // candidates of the current step (reset per step)
    unsigned long long cand_total;
    unsigned long long sigma_evals;
    unsigned long long fp64_rechecks;  // candidates the FP32 stage left to FP64
    unsigned long long st_pairs;       // statistical regime: cloud pair-steps with a yield
    unsigned long long builds;
    unsigned long long collides;
    unsigned long long trav_next[8];   // work-queue cursors of the persistent traversal
    unsigned int err;
    unsigned int step;                 // current step index (device-resident for graphs)
    unsigned long long visits[kCounterSlots];
    unsigned long long queries[kCounterSlots];
    unsigned long long leaf_checks[kCounterSlots];  // window copies: leaf records read
};

// ---------------------------------------------------------------- radix sort
struct SortScratch {
    uint32_t *hist = nullptr;       // passes x 256
    uint32_t *tile_ctr = nullptr;   // passes
    uint32_t *status = nullptr;     // passes x tiles x 256
    int64_t cap_n = 0;
    int cap_passes = 0;
};
int sort_tile_size();
size_t sort_status_words(int64_t n, int passes);
// Stable LSD sort of (key, value) on the low key_bits bits. keys/vals hold the input;
// the result ends in keys/vals or keys_alt/vals_alt; returns true if in *_alt.
bool radix_sort_u32(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                    int64_t n, int key_bits, const SortScratch &s, unsigned int *err,
                    hipStream_t st);
bool radix_sort_u64(unsigned long long *keys, uint32_t *vals, unsigned long long *keys_alt,
                    uint32_t *vals_alt, int64_t n, int key_bits, const SortScratch &s,
                    unsigned int *err, hipStream_t st);

// ------------------------------------------------------------ hierarchy parts
// Device view of a caller beam plus instance data. A launch covers m consecutive
// steps: virtual element e = s n + i is row i at step offset s, combined instance
// c = s n_inst + (instance of row i).
struct BeamDev {
    int64_t n;                 // rows of the beam (all instances)
    const double *x, *y, *z, *px, *py, *pz, *E, *w;
    int32_t n_inst;
    const int64_t *inst_off;   // device copy, n_inst + 1
    int32_t m;                 // steps covered by the launch (>= 1)
    const int32_t *perm;       // row of this view -> caller's row (nullptr: identity)
    const uint8_t *dead = nullptr;  // per caller row: consumed (annihilation), drops out
};

// Per-instance statistics of a beam over its rows (the same for every step):
// bounds of the positions at t = 0 and of the directions u = p/E (ordered 64-bit
// encodings of doubles), and the largest energy and weight (FP64 bits, both >= 0).
struct InstStats {
    unsigned long long mn[6], mx[6];   // x0 y0 z0 ux uy uz
    unsigned long long emax, wmax;
};
struct StatsPartial {
    InstStats s;
    int32_t inst;   // instance the partial belongs to, -1 = unused slot
    int32_t pad;
};
int64_t stats_partials_needed(int64_t n);

// Sort-key layout for n_comb combined instances and at most max_morton Morton bits:
// 32-bit keys (prefix above the top morton_bits of the 30-bit Morton code) while the
// prefix leaves room for min(max_morton, 27) of them, else 64-bit keys (prefix above
// min(max_morton, 30) Morton bits).
struct KeyLayout {
    bool wide;
    int morton_bits;    // Morton bits kept (top bits of the 30-bit code)
    int prefix_shift;   // key >> prefix_shift = combined instance
    int key_bits;       // bits the sort must order
};
KeyLayout key_layout(int64_t n_comb, int max_morton);

void launch_prologue(DevCounters *c, int kind, int32_t m, hipStream_t st);
void launch_set_step(DevCounters *c, int32_t step, hipStream_t st);
void launch_advance_step(DevCounters *c, int32_t m, hipStream_t st);
void launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t st);

// Per-instance statistics of beam b (rows only; b.m is ignored); flags invalid data
// (light_like: also a momentum whose magnitude differs from E by more than 1e-12
// relative; off for the bin clouds of the statistical regime, whose mean directions are
// shorter than one). rows: NULL, or 8 b.n doubles that receive every row as a 64-B record
// (x y z, px py pz, E w) for launch_gather_rows.
void launch_beam_stats(const BeamDev &b, StatsPartial *partials, InstStats *stats, DevCounters *c,
                       hipStream_t st, bool light_like, double *rows = nullptr);
// Swept boxes of all virtual elements of b plus their sort keys and values (the
// virtual element index). Morton quantisation bounds come from self_stats; query
// padding and the threshold prune from t_stats (target instance statistics).
// Box kind for launch_boxes_keys: the swept segment of a step (on = 0), or the cloud of
// the statistical regime (on = 1): a box of half-widths h about the position at mid-step.
struct CloudBox {
    int on;
    double h[3];
};

// Boxes of all b.m steps at s b.n + i; sort keys (key layout kl, base-instance prefix)
// and row values of step offset key_step only, at i.
// Target leaf boxes of all b.m steps at s b.n + i, formed exactly as the refit forms them.
void launch_leaf_boxes(const BeamDev &b, const CloudBox &cloud, double dt, const DevCounters *c,
                       PBox *out, hipStream_t st);
// rec (queries of the plain regime only, else nullptr): one QRec per row for the batch
void launch_boxes_keys(const BeamDev &b, bool query, const CloudBox &cloud, double dt, double sigma_up,
                       const InstStats *t_stats, const InstStats *self_stats, KeyLayout kl,
                       int32_t key_step, PBox *out, uint32_t *keys32, unsigned long long *keys64,
                       uint32_t *vals, DevCounters *c, hipStream_t st, QRec *rec = nullptr);
// Morton keys of given boxes over given bounds (6 ordered floats), 30 bits.
// dst_soa holds x, y, z, px, py, pz, E, w of src.n rows, array a at offset a * src.n.
// Row k of dst is row order[k] of src (order nullptr: row k); dst_perm[k] is the caller's
// row of it (through src.perm).
void launch_gather_beam(const BeamDev &src, const uint32_t *order, double *dst_soa,
                        int32_t *dst_perm, hipStream_t st);
// The same gather for an order with no locality (a caller's rows into Morton order) from the
// rows' 64-B records (8 src.n doubles written by launch_beam_stats; not overlapping dst_soa):
// each output row reads one record instead of eight scattered words.
void launch_gather_rows(const BeamDev &src, const double *rows, const uint32_t *order,
                        double *dst_soa, int32_t *dst_perm, hipStream_t st);
void launch_morton_u32(const PBox *box, int64_t n, const uint32_t *bounds, uint32_t *keys,
                       uint32_t *vals, hipStream_t st);
// Tree shape over n sorted keys (local ids: internal [0, n-1), leaves n-1 + position).
// inst_root may be NULL (one instance); otherwise the node whose range is exactly one
// instance's run of keys (key >> prefix_shift equal) is recorded there.
void launch_karras_u32(const uint32_t *keys, int64_t n, int prefix_shift, PRec *prec,
                       int32_t *inst_root, hipStream_t st);
void launch_karras_u64(const unsigned long long *keys, int64_t n, int prefix_shift, PRec *prec,
                       int32_t *inst_root, hipStream_t st);
// Root link of each of the b.m x b.n_inst combined instances in the b.m per-step copies
// of the shape: an internal node id, leaf_link(element) for an instance of one row
// (whose box, kept in no node, goes to root_box[combined instance]), -1 for an empty
// one (base_root: the emission's instance roots; sorted_rows: row of each sorted
// position).
// With window copies (win > 1: window_copies(b.m, win) copies), an instance of one row has
// its sorted position as root link and its record written to trec.
void launch_inst_roots(const BeamDev &b, const CloudBox &cloud, double dt, const int32_t *base_root,
                       const uint32_t *sorted_rows, int32_t *inst_root, PBox *root_box,
                       const DevCounters *c, hipStream_t st, int32_t win = 1,
                       TRec *trec = nullptr);
// Quantisation frame of each of the window_copies(m, win) copies of a batch of m steps
// from the first step (device counter) and the per-instance statistics.
void launch_win_frames(const InstStats *stats, int32_t n_inst, double dt, int32_t win, int32_t m,
                       const DevCounters *c, WinFrame *frames, hipStream_t st);
// Four-child forms of the copies x (n - 1) internal nodes (n rows) of window copies, in their
// copies' frames; a child box outside its frame, or children that are not a split and its
// successor, set kErrInternal. inside: NULL, or one byte per internal node of the shape,
// nonzero where the refit has written the node's forms already (the node and its
// descendants lie in one of its chunks); only the other nodes are formed here, in every copy.
void launch_collapse4(const Node *nodes, int64_t n, int32_t copies, const WinFrame *frames,
                      CNode4 *out, unsigned int *err, hipStream_t st,
                      const uint8_t *inside = nullptr);
// Per-instance bounds of u dt of a target beam from its statistics (window copies).
void launch_win_bounds(const InstStats *stats, int32_t n_inst, double dt, WinBound *vb,
                       hipStream_t st);
// Nodes of the b.m steps of view b sharing the shape over its b.n rows, each step's
// leaf boxes computed from the photons (sorted_rows: row of each sorted position;
// flags: b.m (b.n - 1) arrival flags, zero on entry and left zero (the second arrival at
// a node clears its flag; a launch that stops on a device error may leave some set);
// slots: hand-off slots for the
// levels above the chunks, refit_slots_needed(b.n, b.m) of them, or NULL / too few:
// the chunk kernel climbs those levels itself).
int64_t refit_slots_needed(int64_t n, int32_t m);
// Crossing levels of the refit merged level by level (batches of many steps): whether a
// batch of m steps over n rows takes that path, the int32 words of its per-shape
// buffer, and its once-per-batch setup (returns where the sort left the order).
bool refit_by_levels(int64_t n, int32_t m);
int64_t xlevel_ints(int64_t n);
bool enqueue_xlevels(const PRec *prec, int64_t n, int32_t *base, const SortScratch &ss,
                     unsigned int *err, hipStream_t st);
// xbase: the level buffer set up by enqueue_xlevels for this shape (xalt: its result), or
// nullptr for the crossing-level climb through the hand-off slots. win > 1 (plain regime
// only): window copies, window_copies(b.m, win) of them, and every leaf's record in trec
// (b.n entries, by sorted position). nodes4 (window copies only, with frames formed
// beforehand): the four-child forms of every internal node whose descendants all lie in
// one 512-leaf chunk are written from the chunk's merged boxes, and inside (b.n - 1 bytes)
// marks those nodes for launch_collapse4, which forms the others. With nodes4 and
// store_inner false, the binary nodes of the nodes whose parent lies in their chunk too are
// not stored (nothing reads them once their forms exist).
void launch_refit(const BeamDev &b, const CloudBox &cloud, double dt, const uint32_t *sorted_rows,
                  const PRec *prec, int32_t *flags, Node *nodes, int32_t *slots, int64_t slot_cap,
                  int32_t *xbase, bool xalt, const DevCounters *c, unsigned int *err,
                  hipStream_t st, int32_t win = 1, TRec *trec = nullptr,
                  const WinFrame *frames = nullptr, CNode4 *nodes4 = nullptr,
                  uint8_t *inside = nullptr, bool store_inner = true);

// n_int: internal nodes of all steps' trees; root_box: box of each combined instance
// whose root is a leaf; nq: virtual query count (steps x rows).
// qorder: NULL (identity), nq entries (order of all virtual queries) or nq_base entries
// (order of one step, repeated per step).
// ---------------------------------------------------------- uniform-grid broad phase
struct GridDev {
    double lo[3];       // grid origin (step's target box centres, lower bound)
    double inv_cs[3];   // cells per unit length
    int32_t dim[3];
    int32_t n_cells;
    float hmax[3];      // largest half extent of a target box plus rounding slack
};
// Grid of the current step from the target's bounds (g, device), then the cell key of every
// target box centre (keys/vals for the radix sort) and cleared cell ranges (max_cells).
void launch_grid_build(const PBox *tbox, int64_t n, const InstStats *t_stats,
                       const DevCounters *c, double dt, int64_t max_cells, GridDev *g,
                       uint32_t *keys, uint32_t *vals, int32_t *cstart, int32_t *cend,
                       hipStream_t st);
// Cell ranges [cstart, cend) of the sorted target keys.
void launch_grid_ranges(const uint32_t *sorted_keys, int64_t n, int32_t *cstart, int32_t *cend,
                        hipStream_t st);
// Candidates of every query box (in qorder) against the target boxes of the cells its box,
// widened by the largest target half extent, meets.
void launch_grid_query(const GridDev *g, const PBox *tbox, const uint32_t *trows,
                       const int32_t *cstart, const int32_t *cend, const PBox *qbox,
                       const uint32_t *qorder, int64_t nq, int32_t *cand_i, int32_t *cand_j,
                       int64_t cand_cap, DevCounters *c, hipStream_t st);

// Boxes of n query rows at step offset s of a batch, formed from their records exactly as
// the traversal forms them, written at out[perm[row]] (perm nullptr: at out[row]); tag:
// the record's instance (-1: the row can collide with nothing); pad: the row.
void launch_record_boxes(const QRec *qrec, int64_t n, const int32_t *perm, int32_t s, PBox *out,
                         hipStream_t st);
// The narrow phase's device arithmetic on n arguments (which: 0 FP64 a / b, 1 FP64 sqrt,
// 2 FP32 a / b, 3 sqrtf, 4 logf, 5 log1pf, FP32 results widened to FP64).
void launch_math_sweep(int which, int64_t n, const double *a, const double *b, double *out,
                       hipStream_t st);
// Queries from per-step boxes (qbox) or, when qrec is given, from per-row records of the
// batch (element s nq_base + row; n_inst: instances of the query view); win (with qrec
// only): the target hierarchy holds window copies.
void launch_traverse(const Node *nodes, int64_t n_int, const PBox *root_box, const PBox *qbox,
                     const uint32_t *qorder, int64_t order_len, int64_t nq, int64_t nq_base,
                     const int32_t *inst_root, int32_t *cand_i, int32_t *cand_j,
                     int64_t cand_cap, DevCounters *c, int block, hipStream_t st,
                     const QRec *qrec = nullptr, int32_t n_inst = 1, bool queue = false,
                     const WinArgs *win = nullptr);
void launch_narrow(const BeamDev &q, const BeamDev &t, double dt, double sigma_up,
                   const int32_t *cand_i, const int32_t *cand_j, int64_t cand_cap,
                   const tril_pairs &out, DevCounters *c, bool fp32_stage, hipStream_t st);
void launch_pair_eval32(int64_t n, const double *in, double sigma_up, double *out, hipStream_t st);
void launch_pair_eval(int64_t n, const double *in, double *out, hipStream_t st);

// Surrogate network (mlp.hip): 6 -> 256 -> 256 -> 256 -> 1, K members.
constexpr int kMlpIn = 6;
constexpr int kMlpHidden = 256;
constexpr int kMlpSlices = 16;  // K slices of the weight-gradient products (batch rows)
constexpr int64_t kMlpParams = (int64_t)kMlpHidden * kMlpIn + kMlpHidden +
                               2 * ((int64_t)kMlpHidden * kMlpHidden + kMlpHidden) + kMlpHidden + 1;

struct MlpModel {
    int K = 0;
    hipStream_t st = nullptr;
    float *w = nullptr;         // FP32 master parameters, K x kMlpParams
    uint16_t *wb = nullptr;     // BF16 copy
    uint16_t *wbi = nullptr;    // BF16 copy at an aligned member stride (inference)
    float *g = nullptr;         // gradient of one member
    float *am = nullptr, *av = nullptr;  // Adam moments
    float *norm = nullptr;      // input mean [6], sd [6]
    float mu_y = 0.f, sd_y = 1.f;
    int64_t rows = 0;           // scratch capacity (rows of a batch)
    uint16_t *xb = nullptr;
    float *z1 = nullptr, *z2 = nullptr, *z3 = nullptr;
    uint16_t *h1 = nullptr, *h2 = nullptr, *h3 = nullptr;
    float *dz = nullptr, *dz2 = nullptr;
    uint16_t *dzb = nullptr, *dz2b = nullptr;
    float *yhat = nullptr, *dy = nullptr;
    uint16_t *dyb = nullptr;
    float *loss = nullptr;
    int32_t *idx = nullptr;
    float *gpart = nullptr;     // slice partials of the weight gradients (kMlpSlices x H x H)
    int64_t adam_t = 0;
    std::vector<void *> allocs;
    ~MlpModel();
};
int mlp_init(MlpModel *m, int K, uint64_t seed, hipStream_t st);
int mlp_scratch(MlpModel *m, int64_t rows);
void mlp_input(MlpModel *m, const float *x, const int32_t *idx, int64_t n);
void mlp_forward(MlpModel *m, int k, int64_t n, float *yhat_out);
// Inference: refresh the aligned BF16 copy (before the members' forward passes), then one
// fused forward pass of member k.
void mlp_pack_inference(MlpModel *m);
void mlp_fused_forward(MlpModel *m, int k, const float *x, int64_t n, float *out);
void mlp_loss(MlpModel *m, const float *y, const int32_t *idx, int64_t n);
void mlp_backward(MlpModel *m, int k, int64_t n);
void mlp_adam(MlpModel *m, int k, float lr, int64_t t);
void mlp_reduce(MlpModel *m, const float *out, int64_t n, float *mean, float *sdev);
void mlp_cast(MlpModel *m);
void mlp_batch_idx(MlpModel *m, uint64_t seed, int k, int64_t step, int64_t n, int64_t batch);
// Column sums and sums of squares into out[2 c] (written, fixed-order reduction); part:
// scratch of 2 c kMomentSlices doubles; c <= 64.
constexpr int kMomentSlices = 256;
void mlp_moments(const float *a, int64_t n, int c, double *out, double *part, hipStream_t st);
void mlp_gemm(const uint16_t *A, int64_t sam, int64_t sak, const uint16_t *B, int64_t sbk,
              int64_t sbn, int M, int N, int K, int epi, const float *bias, const float *aux,
              float *out, uint16_t *out_bf, float *out_pre, hipStream_t st);

// Statistical regime (st.hip).
struct StGridDev {
    double lo[3], hi[3];
    int32_t n_pos[3];
    int32_t n_e;
    double e_lo, e_hi;
    int32_t n_th;
    double th_max;
    double axis[3];
    double t_bin;
};
struct StCell {
    double c[3];  // cloud box edge lengths (the grid's cell size) [um]
};
constexpr int kStSums = 8;  // per-bin sums: w, w E, w u (3), w X(t_bin) (3)
void launch_st_bin(const BeamDev &b, const StGridDev &g, int32_t *bins, double *sums,
                   hipStream_t st);
void launch_st_records(const double *sums, int64_t n_bins, double t_bin, double *soa, int64_t cap,
                       int32_t *rec_bin, unsigned long long *count, hipStream_t st);
void launch_st_features(const long long *keys, const double *vals, int64_t cap, int64_t n_t_bins,
                        const double *q_sums, const double *t_sums, double vol, float *x,
                        double *y0, long long *key_out, int64_t out_cap, unsigned long long *count,
                        hipStream_t st);
// Feature rows in ascending key order (a deterministic order: the rows are appended in
// the order threads claim slots): sort input, then the permutation of the rows.
void launch_st_keys_iota(const long long *key, int64_t n, unsigned long long *k, uint32_t *v,
                         hipStream_t st);
void launch_st_permute_rows(const float *x, const double *y0, const long long *key,
                            const uint32_t *perm, int64_t n, float *xo, double *y0o,
                            long long *keyo, hipStream_t st);
void launch_st_targets(const long long *key, const double *y0, int64_t n, const long long *tkeys,
                       const double *tvals, int64_t tcap, double eps, float *target, double *y_exact,
                       hipStream_t st);
void launch_st_gate(const long long *key, const double *y0, const float *mean, const float *sdev,
                    int64_t n, double eps, double gate, double scale, int cut, int64_t n_t_bins,
                    long long *filter, int64_t fcap, uint8_t *qmark, uint8_t *tmark, double *slots,
                    unsigned long long *n_flag, unsigned int *err, hipStream_t st);
constexpr int kUncBuckets = 4096;  // uncertainty histogram of the budget gate
void launch_st_unc(const double *y0, const float *mean, const float *sdev, int64_t n, double eps,
                   double scale, double *var_hist, double *slots, hipStream_t st);
// Sampled estimate of the exact statistical-regime total (audit.hip).
void launch_au_control(const long long *key, const double *y0, const float *mean, int64_t n,
                       int mode, double eps, double scale, int64_t n_t_bins, double *ctl, double *pa,
                       double *qb, double *slots, hipStream_t st);
void launch_au_weight(const double *sums, int64_t n_bins, double *slots, hipStream_t st);
void launch_au_sample(const BeamDev &b, const int32_t *bins, const double *sums, const double *pc,
                      double c_tot, double w_tot, double lambda, double mix, uint64_t seed,
                      uint32_t rep, uint32_t side, double *soa, int64_t cap, int32_t *s_bin,
                      int32_t *s_row, double *s_pi, unsigned long long *count, double *R,
                      hipStream_t st);
void launch_au_ctl_sample(const long long *key, const double *ctl, int64_t n, int64_t n_t_bins,
                          const double *Rq, const double *Rt, const double *q_sums,
                          const double *t_sums, double *slots, hipStream_t st);
void launch_au_zero(double *p, int64_t n, hipStream_t st);
// part: 2 x blocks doubles (exact, predicted per block), each a fixed-order sum.
void launch_au_calib(const double *y0, const float *mean, const double *y_exact, int64_t n,
                     double eps, double *part, int blocks, hipStream_t st);
void launch_st_mask_bins(const int32_t *bins, int64_t n, const uint8_t *mark, int32_t *out,
                         hipStream_t st);
void launch_fill_keys(long long *p, int64_t n, hipStream_t st);
void launch_st_clear(long long *keys, double *vals, int64_t cap, double *slots, hipStream_t st);
// Arguments as for launch_traverse.
// Depletion pass over the cloud-pair table (pkeys = i * t.n + j, pvals = exposure): every
// pair's exposure becomes its depleted yield, which is added to the bin-pair table
// (keys/vals, cap a power of two) under (q_bins[i], t_bins[j]); totals into slots.
void launch_st_deplete(long long *pkeys, double *pvals, int64_t pcap, const BeamDev &q,
                       const BeamDev &t, const int32_t *q_bins, const int32_t *t_bins,
                       int64_t n_t_bins, const StCell &cell, long long *keys, double *vals,
                       int64_t cap, double *slots, DevCounters *c, hipStream_t st);
// IP-regime swarms over the macro-particle pairs of the pair table (pkeys = i * t.n + j):
// colliding real-photon pairs of each pair over the window [T0, T0 + Tw] into pvals (as
// doubles), into the bin-pair table under (q_bins[i], t_bins[j]) and into *total.
void launch_swarm(const long long *pkeys, double *pvals, int64_t pcap, const BeamDev &q,
                  const BeamDev &t, const int32_t *q_bins, const int32_t *t_bins,
                  int64_t n_t_bins, const StCell &cell, double T0, double Tw, long long *keys,
                  double *vals, int64_t cap, unsigned long long *total, DevCounters *c,
                  hipStream_t st);
void launch_st_traverse(const Node *nodes, int64_t n_int, const PBox *root_box, const PBox *qbox,
                        const uint32_t *qorder, int64_t order_len, int64_t nq, int64_t nq_base,
                        const int32_t *inst_root,
                        const BeamDev &q, const BeamDev &t, const int32_t *q_bins,
                        const int32_t *t_bins, int64_t n_t_bins, double dt, const StCell &cell,
                        int geometric, const long long *filter, int64_t filter_cap,
                        long long *keys, double *vals, int64_t cap, double *slots, DevCounters *c,
                        hipStream_t st);

// ------------------------------------------------------------ annihilation mode
// Scratch of annihilate_hits: per raw hit (cap) two sort key/value buffer pairs, rank,
// live and kept flags and a copy of (i, j, step); per query photon (cap_q) and target
// photon (cap_t) the lowest live rank and a consumed flag; two counters.
struct AnnScratch {
    unsigned long long *ka = nullptr, *kb = nullptr;
    uint32_t *va = nullptr, *vb = nullptr;
    int32_t *rank = nullptr;
    uint8_t *alive = nullptr, *kept = nullptr;
    int32_t *ti = nullptr, *tj = nullptr, *tk = nullptr;
    int64_t cap = 0;
    int32_t *mq = nullptr, *mt = nullptr;
    uint8_t *cq = nullptr, *ct = nullptr;
    int64_t cap_q = 0, cap_t = 0;
    unsigned long long *counter = nullptr;
};
// Resolve the n raw hits (i, j, step) in p in annihilation mode (rows of the query view
// q and target view t, the callers' beams; steps up to max_step): the kept hits are
// written back to p's first *n_kept entries (order unspecified) and *p.count is set to
// their number. Synchronises the stream (one round trip per resolution round).
// Marks both photons of the first n hits of p consumed (dead_q[i] = dead_t[j] = 1).
void launch_ann_mark(const tril_pairs &p, int64_t n, uint8_t *dead_q, uint8_t *dead_t,
                     hipStream_t st);
hipError_t annihilate_hits(const tril_pairs &p, int64_t n, const BeamDev &q, const BeamDev &t,
                           double dt, int32_t max_step, AnnScratch &a, SortScratch &ss,
                           unsigned int *err, hipStream_t st, int64_t *n_kept);

// ------------------------------------------------------------ pair kinematics
// Leptons of the n pairs (pi[h] a row of q, pj[h] a row of t, pk[h] its step): 8 doubles
// per pair (positron E px py pz, electron E px py pz) to leptons when not null, and the
// positron histograms added to hist (n_gamma Lorentz-factor bins on edges[0..n_gamma], then
// n_theta polar-angle bins; hist zeroed by the caller). A pair naming a row outside its beam
// or a negative step sets bit 1 of *err and is skipped. LDS: (2 n_gamma + 1 + n_theta)
// doubles per workgroup.
// Photon records (64 bytes each) the call will use for n pairs over beams of nq and nt
// photons: nq + nt when the pair list is long enough to pay for packing, else 0.
int64_t pair_kinematics_records(int64_t n, int64_t nq, int64_t nt);
// records: device scratch of pair_kinematics_records(n, q.n, t.n) * 64 bytes, or NULL.
void launch_pair_kinematics(const BeamDev &q, const BeamDev &t, const int32_t *pi,
                            const int32_t *pj, const int32_t *pk, int64_t n, uint64_t seed,
                            double *leptons, const double *edges, int32_t n_gamma,
                            int32_t n_theta, double *hist, unsigned int *err, void *records,
                            hipStream_t st);

// ------------------------------------------------------------------ run stats
struct StatsScratch {
    unsigned long long *keys = nullptr, *keys_alt = nullptr;
    uint32_t *vals = nullptr, *vals_alt = nullptr;
    uint32_t *flags = nullptr, *pos = nullptr, *block_sums = nullptr;
    int32_t *ti = nullptr, *tj = nullptr, *tk = nullptr;
    double *acc = nullptr;                 // [0] yield, [1..n_bins] spectrum
    unsigned long long *ucount = nullptr;  // unique pair count
    unsigned long long *step_counts = nullptr;
    int64_t cap = 0;
    int32_t cap_steps = 0;
};
int stats_block_sums_needed(int64_t n);
// Union over steps, sorted ascending (i, j), first step kept; yield, spectrum,
// per-step counts. Writes the unique pairs back into p.i/j/step. key_bits: bits of the
// largest pair key i * n_target + j.
void run_union_stats(const tril_pairs &p, int64_t n_hits, int64_t n_target, int key_bits, const double *w_q, const double *w_t, const double *E_q, const double *E_t,
                     const double *d_edges, int32_t n_bins, int32_t n_steps_count,
                     StatsScratch &s, SortScratch &ss, unsigned int *err, hipStream_t st);

// Host-side maximum of the cross-section (same formula as the device).
double host_sigma(double s);
double host_sigma_max();

}  // namespace tril
