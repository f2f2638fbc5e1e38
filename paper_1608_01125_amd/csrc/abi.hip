// C ABI of libtril: argument checks, context and scratch ownership, and the
// per-step order of the kernels (build: boxes -> Morton -> sort -> hierarchy
// -> refit; collide: query boxes -> query order -> traversal -> narrow phase).
//
// tril_run processes its steps in batches of m consecutive steps: one set of
// launches builds the m per-step hierarchies (as subtrees with their own roots,
// keyed by step and instance) and one traversal launch answers the queries of all
// m steps. Every decision is the same as for one step at a time; batching only
// fills the GPU with more independent work per launch.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "tril_debug.h"
#include "tril_internal.h"

using namespace tril;

namespace {

thread_local std::string g_last_hip;

int hip_fail(hipError_t e) {
    g_last_hip = hipGetErrorString(e);
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? TRIL_E_NOMEM : TRIL_E_HIP;
}

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return hip_fail(e_);  \
    } while (0)

#define CHK(x)                        \
    do {                              \
        int r_ = (x);                 \
        if (r_ != TRIL_OK) return r_; \
    } while (0)

template <typename T>
int dev_alloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(e);
    }
    return TRIL_OK;
}

template <typename T>
void dev_free(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

int bits_for(uint64_t v) {  // smallest b with v < 2^b
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

// Key width for n_comb combined instances: (instance << 30) | 30-bit Morton code.
int comb_key_bits(int64_t n_comb) { return 30 + bits_for((uint64_t)(n_comb > 1 ? n_comb - 1 : 0)); }

constexpr int64_t kMaxN = (int64_t)1 << 30;       // node ids 2n-1 fit int32, sort counts fit 30 bits
constexpr int64_t kMaxComb = (int64_t)1 << 24;    // combined instances (steps x instances) per launch
constexpr int64_t kBatchBudget = (int64_t)1 << 27;  // default virtual elements per launch
// large beams may take up to kBatchBudgetMax virtual elements per launch (about 140 bytes of
// scratch each) so that a launch still covers kBatchStepsMin steps
constexpr int64_t kBatchBudgetMax = (int64_t)1 << 29;
constexpr int64_t kBatchStepsMin = 32;
// with window copies (the plain regime) a launch's tree buffers hold a copy per window, not
// per step, and its query buffers one record per row: every beam takes up to kBatchBudgetMax
// virtual elements per launch (the whole 400-step run of two 1e6-photon beams in one launch,
// so one order, one emission and one set of launch tails serve all its steps)

}  // namespace

struct WorkBeam {
    double *soa = nullptr;          // x, y, z, px, py, pz, E, w: 8 arrays of n
    int32_t *perm = nullptr;        // working row -> caller row
    int64_t cap = 0;
};

struct tril_mlp {
    MlpModel m;
};

struct tril_ctx {
    hipStream_t st = nullptr;       // caller stream
    hipStream_t gst = nullptr;      // internal stream for graph replay (non-blocking)
    hipEvent_t ev_join_a = nullptr, ev_join_b = nullptr;
    // tril_run batches: the query preparation runs on qst beside the build (fork before the
    // build, join before the traversal), with its own sort scratch
    hipStream_t qst = nullptr;
    hipEvent_t ev_qfork = nullptr, ev_qjoin = nullptr;
    hipEvent_t ev_tfork = nullptr, ev_tjoin = nullptr;  // target re-gather beside the traversal
    double dt = 0.0;
    uint32_t flags = 0;
    int32_t n_bins = 0;
    double *d_edges = nullptr;
    int64_t cand_cap_param = 0;
    int block = 64;
    int trav_queue = 0;             // traversal as a persistent work queue (tril_tune)
    int32_t step_batch = 0;         // steps per launch in tril_run (0 = automatic)
    int32_t kwin = 0;               // steps per tree copy in batches (0 = automatic, 1 = per step)
    int32_t kdesc = 0;              // steps per four-child descent (0 = automatic)
    // automatic descent length: the current one, the lengths given up for reaching too many
    // leaves (bit log2 D), and what the counters held at the last adaptation
    int32_t kdesc_auto = 8;
    uint32_t kdesc_rejected = 0u;
    int64_t ad_checks0 = 0, ad_queries0 = 0;
    bool ad_quad = false;           // a tril_run since then descended four-child forms
    int morton_param = 0;           // Morton bits requested (0 = automatic)
    CloudBox cloud{0, {0.0, 0.0, 0.0}};  // box kind of the builds (statistical regime: clouds)
    double *st_slots = nullptr;     // statistical regime: per-wave yield sums (kCounterSlots)
    // surrogate path scratch: bin clouds, bin-pair overlap table, features, exact fallback
    WorkBeam sr_q, sr_t;
    int32_t *sr_q_bin = nullptr, *sr_t_bin = nullptr;
    int64_t sr_q_cap = 0, sr_t_cap = 0, sr_nq = 0, sr_nt = 0;
    long long *sg_key = nullptr;
    double *sg_val = nullptr;
    int64_t sg_cap = 0;
    float *sf_x = nullptr, *sf_mean = nullptr, *sf_sd = nullptr;
    double *sf_y0 = nullptr;
    int64_t *sf_key = nullptr;
    int64_t sf_cap = 0;
    long long *se_key = nullptr;
    double *se_val = nullptr;
    int64_t se_cap = 0;
    // sampled exact estimate (tril_st_audit): per beam the thinned rows of the last
    // replicate (SoA 8 x au_cap, cell bin, source row, inclusion probability), the per-cell
    // arrays (control sums and kept weights of both beams), the row controls
    double *au_soa[2] = {nullptr, nullptr};
    int32_t *au_bin[2] = {nullptr, nullptr}, *au_row[2] = {nullptr, nullptr};
    double *au_pi[2] = {nullptr, nullptr};
    int64_t au_cap = 0, au_n[2] = {0, 0};
    double *au_cell = nullptr;
    int64_t au_cell_cap = 0;
    double *au_ctl = nullptr;
    int64_t au_ctl_cap = 0;
    unsigned long long *au_count = nullptr;
    int morton_bits = 30;           // Morton bits of the sort keys of the current build/collide
    double sigma_up = 0.0;
    DevCounters *d_cnt = nullptr;
    DevCounters *h_cnt = nullptr;   // pinned host mirror
    // pinned words tril_stats reads back in one round trip: hit count, unique pairs, error
    // flags, yield and spectrum, per-step counts
    unsigned long long *h_pin = nullptr;
    int64_t h_pin_cap = 0;

    // target (hierarchy) state; capacities count virtual elements (steps x rows)
    int64_t t_cap = 0, t_row_cap = 0;  // virtual elements (steps x rows), rows
    int64_t t_comb_cap = 0;
    int32_t t_off_cap = 0;
    int64_t nt = 0;                 // rows of the last target beam
    bool built = false;
    int32_t built_step = -1;
    BeamDev tgt{};
    int64_t *d_t_off = nullptr;
    std::vector<int64_t> h_t_off;
    PBox *t_box = nullptr;
    StatsPartial *t_spart = nullptr;
    InstStats *t_stats = nullptr;
    uint32_t *t_k32a = nullptr, *t_k32b = nullptr;
    unsigned long long *t_k64a = nullptr, *t_k64b = nullptr;
    uint32_t *t_va = nullptr, *t_vb = nullptr;
    PRec *prec = nullptr;
    int32_t *nflags = nullptr;
    Node *nodes = nullptr;
    int32_t *inst_root = nullptr;
    int32_t *inst_base = nullptr;          // instance roots of the shared tree shape
    PBox *root_box = nullptr;              // boxes of combined instances of one row
    TRec *t_rec = nullptr;                 // window copies: per sorted target position
    CNode4 *nodes4 = nullptr;              // window copies: four-child forms of the nodes
    int64_t nodes4_cap = 0;
    uint8_t *t_inside = nullptr;           // window copies: per internal node, formed by the refit
    int64_t inside_cap = 0;
    WinFrame *t_frames = nullptr;          // window copies: quantisation frame per copy
    int32_t frames_cap = 0;
    WinBound *t_wb = nullptr;              // window copies: per target instance, bounds of u dt
    int32_t win_eff = 1;                   // steps per tree copy of the last build
    bool quad = false;                     // the last build has four-child forms
    bool keep_nodes = false;  // store every binary node of window copies (tril_dbg_keep_nodes)
    bool nodes_partial = false;  // the last build stored the binary nodes of chunk tops only
    int32_t *refit_slots = nullptr;        // refit hand-offs to the crossing-level kernel
    int32_t *xlev = nullptr;               // crossing levels of the shape (batches of many steps)
    int64_t refit_slot_cap = 0;
    int64_t n_int = -1;                    // internal nodes of the last build (all steps)
    int32_t tgt_k0 = 0;                    // first step of the last build
    CloudBox tgt_cloud{0, {0.0, 0.0, 0.0}};  // box kind of the last build

    // query state
    int64_t q_cap = 0, q_row_cap = 0;
    int64_t q_comb_cap = 0;
    int32_t q_off_cap = 0;
    int64_t *d_q_off = nullptr;
    std::vector<int64_t> h_q_off;
    PBox *q_box = nullptr;
    QRec *q_rec = nullptr;                 // per-row query records of a batch (plain regime)
    StatsPartial *q_spart = nullptr;
    InstStats *q_stats = nullptr;
    uint32_t *q_keep = nullptr;            // query order kept from a first step (n entries)
    uint32_t *q_k32a = nullptr, *q_k32b = nullptr;
    unsigned long long *q_k64a = nullptr, *q_k64b = nullptr;
    uint32_t *q_va = nullptr, *q_vb = nullptr;
    const uint32_t *q_order = nullptr;     // sorted query rows (points into q_va or q_vb)
    int64_t q_order_len = 0;
    const void *q_order_key = nullptr;     // beam the stored order belongs to
    int64_t q_order_n = -1;

    // candidates of one launch
    int64_t cand_cap = 0;
    int32_t *cand_i = nullptr, *cand_j = nullptr;

    SortScratch ss;
    SortScratch ssq;                       // the query sort of tril_run batches (beside the build)
    StatsScratch sst;
    AnnScratch ann;                        // annihilation-mode resolution
    uint8_t *dead_q = nullptr, *dead_t = nullptr;  // photons consumed in this run (per row)
    int64_t dead_cap_q = 0, dead_cap_t = 0;
    int64_t *ann_count = nullptr;                  // kept hits of one batch (device)
    unsigned long long *swarm_total = nullptr;  // IP regime: colliding real pairs
    GridDev *grid_dev = nullptr;    // uniform-grid broad phase (TRIL_GRID)
    int32_t *grid_start = nullptr, *grid_end = nullptr;
    int64_t grid_cap = 0;
    double *kin_buf = nullptr;             // pair kinematics: edges, histogram bins
    unsigned int *kin_err = nullptr;
    hipEvent_t ev_kin[2] = {nullptr, nullptr};
    double *kin_rec = nullptr;            // packed photon records (8 doubles each)
    int64_t kin_rec_cap = 0;
    int32_t max_step = -1;

    // timing (TRIL_TIMING)
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::array<int, 2>> ev_build, ev_prep, ev_trav, ev_narrow;
    size_t ev_next = 0;
    double ms_acc[4] = {0, 0, 0, 0};   // summed event times of pairs already read and recycled
    int64_t timed_launches = 0;

    // working copies of the two beams for tril_run (two buffers each): rows in the Morton
    // order of the first step of the previous batch, so that the gathers of the build and
    // of the traversal touch nearby memory
    WorkBeam wt[2], wq[2];
    const uint32_t *t_rows = nullptr;      // sorted rows of the last build

    // captured step-batch graphs (one per working-buffer parity)
    // captured batches: a run's first batch (no sorts), the two buffer parities with the
    // re-gather for a following batch, and a last batch without it
    static constexpr int kGraphs = 4;
    hipGraphExec_t gexec[kGraphs] = {};
    std::vector<const void *> gkey[kGraphs];
    int g_next = 0;
    uint64_t alloc_gen = 0;         // bumped on every (re)allocation of scratch

    BeamDev res_t{};                // caller's target beam of the last build or run (statistics)
    BeamDev last_q{};               // caller's query beam of the last collide (statistics)
    BeamDev last_qrec{};            // working view whose rows the query records of the last
                                    // step batch of tril_run describe (m = 0: none)
    int64_t max_nq = 0;
};

namespace {

int ensure_one_sort_scratch(tril_ctx *c, SortScratch &ss, int64_t n) {
    if (n <= ss.cap_n) return TRIL_OK;
    ++c->alloc_gen;
    dev_free(ss.hist);
    dev_free(ss.tile_ctr);
    dev_free(ss.status);
    ss.cap_n = 0;
    CHK(dev_alloc(&ss.hist, 8 * 256));
    CHK(dev_alloc(&ss.tile_ctr, 8));
    CHK(dev_alloc(&ss.status, sort_status_words(n, 8)));
    ss.cap_n = n;
    ss.cap_passes = 8;
    return TRIL_OK;
}

int ensure_sort_scratch(tril_ctx *c, int64_t n) {
    CHK(ensure_one_sort_scratch(c, c->ss, n));
    return ensure_one_sort_scratch(c, c->ssq, n);
}

void free_target(tril_ctx *c) {
    dev_free(c->t_box); dev_free(c->nflags); dev_free(c->nodes); dev_free(c->refit_slots);
    c->t_cap = 0;
    c->refit_slot_cap = 0;
}

void free_target_rows(tril_ctx *c) {
    dev_free(c->t_spart); dev_free(c->t_k32a); dev_free(c->t_k32b);
    dev_free(c->t_k64a); dev_free(c->t_k64b); dev_free(c->t_va); dev_free(c->t_vb);
    dev_free(c->prec); dev_free(c->xlev); dev_free(c->t_rec);
    c->t_row_cap = 0;
}

// Target buffers for launches of up to nv virtual elements over n rows: boxes, nodes
// and arrival flags per element; keys, sort values and the tree shape per row.
int ensure_target(tril_ctx *c, int64_t nv, int64_t n, int64_t n_comb, int32_t n_inst) {
    if (nv > c->t_cap) {
        ++c->alloc_gen;
        free_target(c);
        c->built = false;
        const int64_t m = std::max<int64_t>(nv, 1);
        CHK(dev_alloc(&c->t_box, m));
        CHK(dev_alloc(&c->nflags, m));
        // the refit expects cleared arrival flags and leaves them cleared
        HIPCHK(hipMemset(c->nflags, 0, (size_t)m * sizeof(int32_t)));
        CHK(dev_alloc(&c->nodes, m));  // m' (n' - 1) internal nodes of m' steps over n' rows
        // a launch of m' steps over n' > 512 rows has m' ceil(n' / 512) <= nv / 256 chunks
        // (fewer rows need no hand-offs), 64 slots each
        c->refit_slot_cap = m / 4 + 64;
        CHK(dev_alloc(&c->refit_slots, (size_t)c->refit_slot_cap));
        c->t_cap = m;
    }
    if (n > c->t_row_cap) {
        ++c->alloc_gen;
        free_target_rows(c);
        c->built = false;
        const int64_t m = std::max<int64_t>(n, 1);
        CHK(dev_alloc(&c->t_spart, (size_t)stats_partials_needed(m)));
        CHK(dev_alloc(&c->t_k32a, m)); CHK(dev_alloc(&c->t_k32b, m));
        CHK(dev_alloc(&c->t_k64a, m)); CHK(dev_alloc(&c->t_k64b, m));
        CHK(dev_alloc(&c->t_va, m)); CHK(dev_alloc(&c->t_vb, m));
        CHK(dev_alloc(&c->prec, 2 * m));
        CHK(dev_alloc(&c->xlev, (size_t)xlevel_ints(m)));
        CHK(dev_alloc(&c->t_rec, m));
        c->t_row_cap = m;
    }
    if (n_comb > c->t_comb_cap) {
        ++c->alloc_gen;
        dev_free(c->inst_root); dev_free(c->inst_base); dev_free(c->root_box);
        c->t_comb_cap = 0;
        c->built = false;
        CHK(dev_alloc(&c->inst_root, (size_t)n_comb));
        CHK(dev_alloc(&c->root_box, (size_t)n_comb));
        CHK(dev_alloc(&c->inst_base, (size_t)n_comb));
        c->t_comb_cap = n_comb;
    }
    if (n_inst > c->t_off_cap) {
        ++c->alloc_gen;
        dev_free(c->d_t_off); dev_free(c->t_stats); dev_free(c->t_wb);
        c->t_off_cap = 0;
        CHK(dev_alloc(&c->d_t_off, (size_t)n_inst + 1));
        CHK(dev_alloc(&c->t_stats, (size_t)n_inst));
        CHK(dev_alloc(&c->t_wb, (size_t)n_inst));
        c->t_off_cap = n_inst;
        c->h_t_off.clear();
    }
    return ensure_sort_scratch(c, n);
}

// Query buffers: boxes for nv_box virtual elements (nv when negative), candidates for nv,
// keys and orders per row (n).
int ensure_query(tril_ctx *c, int64_t nv, int64_t n, int64_t n_comb, int32_t n_inst,
                 int64_t nv_box = -1) {
    if (nv_box < 0) nv_box = nv;
    if (nv_box > c->q_cap) {
        ++c->alloc_gen;
        dev_free(c->q_box);
        c->q_cap = 0;
        const int64_t m = std::max<int64_t>(nv_box, 1);
        CHK(dev_alloc(&c->q_box, m));
        c->q_cap = m;
    }
    if (n > c->q_row_cap) {
        ++c->alloc_gen;
        dev_free(c->q_spart); dev_free(c->q_k32a); dev_free(c->q_k32b);
        dev_free(c->q_k64a); dev_free(c->q_k64b); dev_free(c->q_va); dev_free(c->q_vb);
        dev_free(c->q_keep); dev_free(c->q_rec);
        c->q_row_cap = 0;
        c->q_order = nullptr;
        c->q_order_key = nullptr;
        const int64_t m = std::max<int64_t>(n, 1);
        CHK(dev_alloc(&c->q_spart, (size_t)stats_partials_needed(m)));
        CHK(dev_alloc(&c->q_keep, m));
        CHK(dev_alloc(&c->q_rec, m));
        CHK(dev_alloc(&c->q_k32a, m)); CHK(dev_alloc(&c->q_k32b, m));
        CHK(dev_alloc(&c->q_k64a, m)); CHK(dev_alloc(&c->q_k64b, m));
        CHK(dev_alloc(&c->q_va, m)); CHK(dev_alloc(&c->q_vb, m));
        c->q_row_cap = m;
    }
    if (n_comb > c->q_comb_cap) c->q_comb_cap = n_comb;
    if (n_inst > c->q_off_cap) {
        ++c->alloc_gen;
        dev_free(c->d_q_off); dev_free(c->q_stats);
        c->q_off_cap = 0;
        CHK(dev_alloc(&c->d_q_off, (size_t)n_inst + 1));
        CHK(dev_alloc(&c->q_stats, (size_t)n_inst));
        c->q_off_cap = n_inst;
        c->h_q_off.clear();
    }
    const int64_t cap = c->cand_cap_param > 0 ? c->cand_cap_param
                                              : std::max<int64_t>((int64_t)1 << 22, 2 * nv);
    if (cap > c->cand_cap) {
        ++c->alloc_gen;
        dev_free(c->cand_i); dev_free(c->cand_j);
        c->cand_cap = 0;
        CHK(dev_alloc(&c->cand_i, cap));
        CHK(dev_alloc(&c->cand_j, cap));
        c->cand_cap = cap;
    }
    return ensure_sort_scratch(c, n);
}

int check_beam(const tril_beam *b) {
    if (!b) return TRIL_E_INVAL;
    if (b->n < 0 || b->n >= kMaxN) return TRIL_E_INVAL;
    if (b->n_inst < 1 || b->n_inst > kMaxComb) return TRIL_E_INVAL;
    if (b->n > 0 && (!b->x || !b->y || !b->z || !b->px || !b->py || !b->pz || !b->E || !b->w))
        return TRIL_E_INVAL;
    if (b->n_inst > 1) {
        if (!b->inst_off) return TRIL_E_INVAL;
        if (b->inst_off[0] != 0 || b->inst_off[b->n_inst] != b->n) return TRIL_E_INVAL;
        for (int32_t m = 0; m < b->n_inst; ++m)
            if (b->inst_off[m + 1] < b->inst_off[m]) return TRIL_E_INVAL;
    } else if (b->inst_off && (b->inst_off[0] != 0 || b->inst_off[1] != b->n)) {
        return TRIL_E_INVAL;
    }
    return TRIL_OK;
}

int check_pairs(const tril_pairs *p) {
    if (!p || p->cap < 0 || !p->count) return TRIL_E_INVAL;
    if (p->cap > 0 && (!p->i || !p->j || !p->step)) return TRIL_E_INVAL;
    return TRIL_OK;
}

// Copy instance offsets to the device when they changed (synchronous copy from host memory).
int upload_offsets(tril_ctx *c, const tril_beam *b, int64_t *d_off, std::vector<int64_t> &cache) {
    if (b->n_inst <= 1) return TRIL_OK;
    std::vector<int64_t> h(b->inst_off, b->inst_off + b->n_inst + 1);
    if (h == cache) return TRIL_OK;
    HIPCHK(hipStreamSynchronize(c->st));
    HIPCHK(hipMemcpy(d_off, h.data(), h.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    cache = std::move(h);
    return TRIL_OK;
}

BeamDev view(const tril_beam *b, const int64_t *d_off, int32_t m) {
    BeamDev v;
    v.n = b->n;
    v.x = b->x; v.y = b->y; v.z = b->z;
    v.px = b->px; v.py = b->py; v.pz = b->pz;
    v.E = b->E; v.w = b->w;
    v.n_inst = b->n_inst;
    v.inst_off = b->n_inst > 1 ? d_off : nullptr;
    v.m = m;
    v.perm = nullptr;
    return v;
}

void free_work(WorkBeam &w) {
    dev_free(w.soa);
    dev_free(w.perm);
    w.cap = 0;
}

int ensure_work(tril_ctx *c, WorkBeam *w, int64_t n) {
    if (n <= w[0].cap) return TRIL_OK;
    ++c->alloc_gen;
    for (int p = 0; p < 2; ++p) {
        free_work(w[p]);
        const int64_t m = std::max<int64_t>(n, 1);
        CHK(dev_alloc(&w[p].soa, (size_t)(8 * m)));
        CHK(dev_alloc(&w[p].perm, (size_t)m));
        w[p].cap = m;
    }
    return TRIL_OK;
}

// View of a working copy (same rows and instances as the caller's beam b).
BeamDev wview(const tril_beam *b, const int64_t *d_off, int32_t m, const WorkBeam &w) {
    BeamDev v = view(b, d_off, m);
    const int64_t n = b->n;
    v.x = w.soa; v.y = w.soa + n; v.z = w.soa + 2 * n;
    v.px = w.soa + 3 * n; v.py = w.soa + 4 * n; v.pz = w.soa + 5 * n;
    v.E = w.soa + 6 * n; v.w = w.soa + 7 * n;
    v.perm = w.perm;
    return v;
}

// Step offset within a batch of m steps whose Morton order shapes the batch's trees
// (the middle one: no step of the batch is more than m/2 steps from it).
inline int32_t key_step(int32_t m) { return m > 0 ? (m - 1) / 2 : 0; }

// Working copy w of beam b in the order of the Morton codes a batch of b.m steps from the
// device step index sorts it by (its key step, the run's Morton bits, each beam in its own
// frame; the query padding moves no box centre), using the key scratch of its side (sized
// for at least b.n elements). A stable sort of the working copy by the same keys is then
// the identity, so that batch skips its sorts (enqueue_build's presorted, a query
// preparation without sort).
int enqueue_order(tril_ctx *c, const BeamDev &b, bool query_side, WorkBeam &w, hipStream_t st,
                  SortScratch &ss, const double *rows_rec) {
    if (b.n <= 0) return TRIL_OK;
    const KeyLayout kl = key_layout(b.n_inst, c->morton_bits);
    const InstStats *stats = query_side ? c->q_stats : c->t_stats;
    uint32_t *k32a = query_side ? c->q_k32a : c->t_k32a, *k32b = query_side ? c->q_k32b : c->t_k32b;
    unsigned long long *k64a = query_side ? c->q_k64a : c->t_k64a;
    unsigned long long *k64b = query_side ? c->q_k64b : c->t_k64b;
    uint32_t *va = query_side ? c->q_va : c->t_va, *vb = query_side ? c->q_vb : c->t_vb;
    launch_boxes_keys(b, false, c->cloud, c->dt, c->sigma_up, stats, stats, kl, key_step(b.m),
                      nullptr, k32a, k64a, va, c->d_cnt, st);
    const uint32_t *rows;
    if (!kl.wide)
        rows = radix_sort_u32(k32a, va, k32b, vb, b.n, kl.key_bits, ss, &c->d_cnt->err, st)
                   ? vb : va;
    else
        rows = radix_sort_u64(k64a, va, k64b, vb, b.n, kl.key_bits, ss, &c->d_cnt->err, st)
                   ? vb : va;
    launch_gather_rows(b, rows_rec, rows, w.soa, w.perm, st);
    return TRIL_OK;
}

int timing_pair(tril_ctx *c, hipStream_t st, std::vector<std::array<int, 2>> &dst, bool begin) {
    if (!(c->flags & TRIL_TIMING)) return TRIL_OK;
    if (begin) {
        if (c->ev_next + 2 > c->ev_pool.size()) {
            for (int k = 0; k < 64; ++k) {
                hipEvent_t e;
                HIPCHK(hipEventCreate(&e));
                c->ev_pool.push_back(e);
            }
        }
        dst.push_back({(int)c->ev_next, (int)c->ev_next + 1});
        c->ev_next += 2;
        HIPCHK(hipEventRecord(c->ev_pool[dst.back()[0]], st));
    } else {
        HIPCHK(hipEventRecord(c->ev_pool[dst.back()[1]], st));
    }
    return TRIL_OK;
}


// Steps per tree copy for a batch of m steps: window copies only in the plain regime
// (straight-line leaf boxes, query records), at most m.
// Automatic (kwin 0): 32 steps, or 16 while the descents are of 4 steps or fewer (the
// automatic descent length settles there when a target's photons move apart fast enough
// that a longer descent's hull reaches too many leaves; shorter copies then tighten the
// node boxes the same way: broadband beams 458.7 -> 444.4 ms per run, batch64 unchanged).
constexpr int32_t kDefaultWindow = 32;
constexpr int32_t kShortWindow = 16;
int32_t auto_window(const tril_ctx *c) {
    if (c->kwin > 1) return c->kwin;
    return (c->kdesc > 0 ? c->kdesc : c->kdesc_auto) <= 4 ? kShortWindow : kDefaultWindow;
}
int32_t build_window(const tril_ctx *c, int32_t m) {
    if (m < 2 || c->cloud.on != 0 || c->kwin == 1) return 1;
    const int32_t w = auto_window(c);
    return w < m ? w : m;
}

// Steps per descent over the four-child forms of copies of win steps: at most win and
// kMaxDescent; automatic (kdesc 0): the length tril_stats last chose (adapt_descent).
int32_t descent_window(const tril_ctx *c, int32_t win) {
    const int32_t d = c->kdesc > 0 ? c->kdesc : c->kdesc_auto;
    return std::min(std::min(d, win), kMaxDescent);
}

// Automatic descent length. A longer descent loads fewer nodes per step but reaches more
// leaves (its hull stretches along the motion), each tested at every step in range. From the
// leaf tests per descent L since the last adaptation: above kAdaptHigh the length halves
// and is not taken again (doubling it multiplies L by about 3 to 5), below kAdaptLow it
// doubles unless that length was given up; lengths are powers of two in 1..kMaxDescent.
constexpr double kAdaptHigh = 0.45, kAdaptLow = 0.13;
void adapt_descent(tril_ctx *c, int64_t checks, int64_t queries) {
    const int32_t d = c->kdesc_auto;
    const int64_t dq = queries - c->ad_queries0, dl = checks - c->ad_checks0;
    if (c->kdesc == 0 && c->ad_quad && dq > 0) {
        const double L = (double)dl * d / (double)dq;
        int lg = 0;
        while ((1 << lg) < d) ++lg;
        if (L > kAdaptHigh && d > 1) {
            c->kdesc_rejected |= 1u << lg;
            c->kdesc_auto = d / 2;
        } else if (L < kAdaptLow && 2 * d <= kMaxDescent && !(c->kdesc_rejected & (2u << lg))) {
            c->kdesc_auto = 2 * d;
        }
    }
    c->ad_checks0 = checks;
    c->ad_queries0 = queries;
    c->ad_quad = false;
}

// Kernels of one build on stream st (target view, with its step count m, in c->tgt;
// the target statistics c->t_stats are current): boxes of every step, one sort of the
// rows by their Morton codes at the batch's key step, the tree shape emitted from that
// order, and its copies (one per step, or one per window of steps) filled with the boxes
// of their steps.
int enqueue_build(tril_ctx *c, hipStream_t st, bool timed, bool presorted = false) {
    const BeamDev &t = c->tgt;
    const int64_t n = t.n;
    const int32_t win = build_window(c, t.m);
    const int32_t copies = window_copies(t.m, win);
    c->win_eff = win;
    const KeyLayout kl = key_layout(t.n_inst, c->morton_bits);
    if (timed) CHK(timing_pair(c, st, c->ev_build, true));
    launch_prologue(c->d_cnt, 0, t.m, st);
    // sort keys only: the refit forms every step's leaf boxes from the photons itself
    launch_boxes_keys(t, false, c->cloud, c->dt, c->sigma_up, c->t_stats, c->t_stats, kl,
                      key_step(t.m), nullptr, c->t_k32a, c->t_k64a, c->t_va, c->d_cnt, st);
    const uint32_t *rows = nullptr;
    int32_t *roots = t.n_inst > 1 ? c->inst_base : nullptr;
    // presorted: the working copy is in the order of these keys already (enqueue_order)
    if (!kl.wide) {
        const bool alt = !presorted && radix_sort_u32(c->t_k32a, c->t_va, c->t_k32b, c->t_vb, n,
                                                      kl.key_bits, c->ss, &c->d_cnt->err, st);
        const uint32_t *keys = alt ? c->t_k32b : c->t_k32a;
        rows = alt ? c->t_vb : c->t_va;
        launch_karras_u32(keys, n, kl.prefix_shift, c->prec, roots, st);
    } else {
        const bool alt = !presorted && radix_sort_u64(c->t_k64a, c->t_va, c->t_k64b, c->t_vb, n,
                                                      kl.key_bits, c->ss, &c->d_cnt->err, st);
        const unsigned long long *keys = alt ? c->t_k64b : c->t_k64a;
        rows = alt ? c->t_vb : c->t_va;
        launch_karras_u64(keys, n, kl.prefix_shift, c->prec, roots, st);
    }
    c->t_rows = rows;
    c->n_int = n > 0 ? (int64_t)copies * (n - 1) : -1;
    c->tgt_cloud = c->cloud;
    if (win > 1) launch_win_bounds(c->t_stats, t.n_inst, c->dt, c->t_wb, st);
    c->quad = win > 1 && n > 1 && (int64_t)copies * (n - 1) <= c->nodes4_cap &&
              copies <= c->frames_cap && n - 1 <= c->inside_cap;
    launch_inst_roots(t, c->cloud, c->dt, c->inst_base, rows, c->inst_root, c->root_box, c->d_cnt,
                      st, win, c->t_rec);
    int32_t *xbase = nullptr;
    bool xalt = false;
    if (refit_by_levels(n, copies)) {
        xbase = c->xlev;
        xalt = enqueue_xlevels(c->prec, n, xbase, c->ss, &c->d_cnt->err, st);
    }
    // four-child forms: the frames first; the refit forms the nodes whose descendants lie in
    // one of its chunks, the collapse the others
    if (c->quad) launch_win_frames(c->t_stats, t.n_inst, c->dt, win, t.m, c->d_cnt, c->t_frames, st);
    launch_refit(t, c->cloud, c->dt, rows, c->prec, c->nflags, c->nodes, c->refit_slots,
                 c->refit_slot_cap, xbase, xalt, c->d_cnt, &c->d_cnt->err, st, win, c->t_rec,
                 c->quad ? c->t_frames : nullptr, c->quad ? c->nodes4 : nullptr,
                 c->quad ? c->t_inside : nullptr, c->keep_nodes);
    c->nodes_partial = c->quad && !c->keep_nodes;
    if (c->quad)
        launch_collapse4(c->nodes, n, copies, c->t_frames, c->nodes4, &c->d_cnt->err, st,
                         c->t_inside);
    if (timed) CHK(timing_pair(c, st, c->ev_build, false));
    HIPCHK(hipGetLastError());
    return TRIL_OK;
}

// Query boxes of every step of the view and, when sort_queries, the order of its rows
// by their Morton codes at the batch's key step (c->q_order, q.n entries: the traversal
// repeats it for every step).
int enqueue_query_prep(tril_ctx *c, const BeamDev &q, hipStream_t st, bool sort_queries,
                       bool records = false, SortScratch *ss = nullptr) {
    SortScratch &sq = ss != nullptr ? *ss : c->ss;
    const KeyLayout kl = key_layout(q.n_inst, c->morton_bits);
    launch_boxes_keys(q, true, c->cloud, c->dt, c->sigma_up, c->t_stats, c->q_stats, kl,
                      key_step(q.m), records ? nullptr : c->q_box, c->q_k32a, c->q_k64a, c->q_va,
                      c->d_cnt, st, records ? c->q_rec : nullptr);
    if (sort_queries && q.n > 0 && q.m > 0) {
        bool alt;
        if (!kl.wide)
            alt = radix_sort_u32(c->q_k32a, c->q_va, c->q_k32b, c->q_vb, q.n, kl.key_bits, sq,
                                 &c->d_cnt->err, st);
        else
            alt = radix_sort_u64(c->q_k64a, c->q_va, c->q_k64b, c->q_vb, q.n, kl.key_bits, sq,
                                 &c->d_cnt->err, st);
        c->q_order = (q.n <= 1) ? c->q_va : (alt ? c->q_vb : c->q_va);
        c->q_order_len = q.n;
    }
    return TRIL_OK;
}

// Uniform-grid broad phase (TRIL_GRID, one step, one instance): target boxes, grid of the
// step, target rows sorted by cell, cell ranges.
int enqueue_grid_build(tril_ctx *c, hipStream_t st, bool timed) {
    const BeamDev &t = c->tgt;
    const int64_t n = t.n;
    const int64_t max_cells = std::max<int64_t>(n, 1);
    if (max_cells > c->grid_cap) {
        dev_free(c->grid_start);
        dev_free(c->grid_end);
        c->grid_cap = 0;
        CHK(dev_alloc(&c->grid_start, (size_t)max_cells));
        CHK(dev_alloc(&c->grid_end, (size_t)max_cells));
        c->grid_cap = max_cells;
    }
    if (!c->grid_dev) CHK(dev_alloc(&c->grid_dev, 1));
    if (timed) CHK(timing_pair(c, st, c->ev_build, true));
    launch_prologue(c->d_cnt, 0, 1, st);
    const KeyLayout kl = key_layout(1, c->morton_bits);
    launch_boxes_keys(t, false, c->cloud, c->dt, c->sigma_up, c->t_stats, c->t_stats, kl, 0,
                      c->t_box, nullptr, nullptr, nullptr, c->d_cnt, st);
    launch_grid_build(c->t_box, n, c->t_stats, c->d_cnt, c->dt, max_cells, c->grid_dev,
                      c->t_k32a, c->t_va, c->grid_start, c->grid_end, st);
    const uint32_t *keys = c->t_k32a;
    c->t_rows = c->t_va;
    if (n > 1) {
        const bool alt = radix_sort_u32(c->t_k32a, c->t_va, c->t_k32b, c->t_vb, n,
                                        std::max(1, bits_for((uint64_t)(max_cells - 1))), c->ss,
                                        &c->d_cnt->err, st);
        keys = alt ? c->t_k32b : c->t_k32a;
        c->t_rows = alt ? c->t_vb : c->t_va;
    }
    launch_grid_ranges(keys, n, c->grid_start, c->grid_end, st);
    c->n_int = 0;
    if (timed) CHK(timing_pair(c, st, c->ev_build, false));
    HIPCHK(hipGetLastError());
    return TRIL_OK;
}

int enqueue_grid_collide(tril_ctx *c, const BeamDev &q, const tril_pairs &out, hipStream_t st,
                         bool timed, bool sort_queries) {
    if (timed) CHK(timing_pair(c, st, c->ev_prep, true));
    launch_prologue(c->d_cnt, 1, 1, st);
    CHK(enqueue_query_prep(c, q, st, sort_queries));
    if (timed) CHK(timing_pair(c, st, c->ev_prep, false));
    if (timed) CHK(timing_pair(c, st, c->ev_trav, true));
    launch_grid_query(c->grid_dev, c->t_box, c->t_rows, c->grid_start, c->grid_end, c->q_box,
                      q.n > 0 ? c->q_order : nullptr, q.n, c->cand_i, c->cand_j, c->cand_cap,
                      c->d_cnt, st);
    if (timed) CHK(timing_pair(c, st, c->ev_trav, false));
    if (timed) CHK(timing_pair(c, st, c->ev_narrow, true));
    launch_narrow(q, c->tgt, c->dt, c->sigma_up, c->cand_i, c->cand_j, c->cand_cap, out, c->d_cnt,
                  (c->flags & TRIL_FP64_NARROW) == 0, st);
    if (timed) CHK(timing_pair(c, st, c->ev_narrow, false));
    HIPCHK(hipGetLastError());
    return TRIL_OK;
}

// The collide phase's prologue and query preparation (query boxes or records, and the Morton
// order of the query rows) on stream st.
int enqueue_collide_prep(tril_ctx *c, const BeamDev &q, hipStream_t st, bool timed,
                         bool sort_queries, SortScratch *ss = nullptr) {
    if (timed) CHK(timing_pair(c, st, c->ev_prep, true));
    launch_prologue(c->d_cnt, 1, q.m, st);
    // a batch of steps in the plain regime: one record per query row instead of a box per
    // query and step
    const bool records = q.m >= 2 && c->cloud.on == 0;
    CHK(enqueue_query_prep(c, q, st, sort_queries, records, ss));
    if (timed) CHK(timing_pair(c, st, c->ev_prep, false));
    return TRIL_OK;
}

// Collide phase on stream st: the query preparation (unless `prepped`: already enqueued,
// see enqueue_collide_prep), then the traversal and the narrow phase.
int enqueue_collide(tril_ctx *c, const BeamDev &q, const tril_pairs &out, hipStream_t st,
                    bool timed, bool sort_queries, bool prepped = false) {
    const int64_t nv = (int64_t)q.m * q.n;
    const bool records = q.m >= 2 && c->cloud.on == 0;
    if (c->win_eff > 1 && (!records || q.m != c->tgt.m)) return TRIL_E_INTERNAL;
    if (!prepped) CHK(enqueue_collide_prep(c, q, st, timed, sort_queries));
    WinArgs wa{};
    if (c->win_eff > 1) {
        wa.trec = c->t_rec;
        wa.vb = c->t_wb;
        wa.nodes4 = c->quad ? c->nodes4 : nullptr;
        wa.frames = c->t_frames;
        wa.win = c->win_eff;
        wa.m = q.m;
        wa.n = c->tgt.n;
        wa.reach = (float)((double)(q.m + c->win_eff + 8) * c->dt + 1e-6);
        wa.dwin = descent_window(c, c->win_eff);
    }
    if (timed) CHK(timing_pair(c, st, c->ev_trav, true));
    launch_traverse(c->nodes, c->n_int, c->root_box, c->q_box, c->q_order, c->q_order_len, nv, q.n,
                    c->inst_root, c->cand_i, c->cand_j, c->cand_cap, c->d_cnt, c->block, st,
                    records ? c->q_rec : nullptr, q.n_inst, c->trav_queue != 0,
                    c->win_eff > 1 ? &wa : nullptr);
    if (timed) CHK(timing_pair(c, st, c->ev_trav, false));
    if (timed) CHK(timing_pair(c, st, c->ev_narrow, true));
    launch_narrow(q, c->tgt, c->dt, c->sigma_up, c->cand_i, c->cand_j, c->cand_cap, out, c->d_cnt,
                  (c->flags & TRIL_FP64_NARROW) == 0, st);
    if (timed) CHK(timing_pair(c, st, c->ev_narrow, false));
    HIPCHK(hipGetLastError());
    return TRIL_OK;
}

bool need_query_sort(tril_ctx *c, const tril_beam *q) {
    if (!(c->flags & TRIL_SORT_QUERIES_ONCE)) return true;
    return !(c->q_order && c->q_order_key == (const void *)q->x && c->q_order_n == q->n &&
             c->q_order_len == q->n);
}

// Remember the order of a single-step query sort; with TRIL_SORT_QUERIES_ONCE it is
// copied to c->q_keep so that later batches can reuse it while overwriting the sort
// buffers.
int note_query_sorted(tril_ctx *c, const tril_beam *q, int32_t m, hipStream_t st) {
    c->q_order_key = (const void *)q->x;
    c->q_order_n = q->n;
    if ((c->flags & TRIL_SORT_QUERIES_ONCE) && m == 1 && q->n > 0) {
        HIPCHK(hipMemcpyAsync(c->q_keep, c->q_order, q->n * sizeof(uint32_t),
                              hipMemcpyDeviceToDevice, st));
        c->q_order = c->q_keep;
        c->q_order_len = q->n;
    }
    return TRIL_OK;
}

int ensure_annihilation(tril_ctx *c, int64_t n_hits, int64_t nq, int64_t nt) {
    AnnScratch &a = c->ann;
    if (n_hits > a.cap) {
        dev_free(a.ka); dev_free(a.kb); dev_free(a.va); dev_free(a.vb); dev_free(a.rank);
        dev_free(a.alive); dev_free(a.kept); dev_free(a.ti); dev_free(a.tj); dev_free(a.tk);
        a.cap = 0;
        const int64_t m = std::max<int64_t>(n_hits, 1024);
        CHK(dev_alloc(&a.ka, m)); CHK(dev_alloc(&a.kb, m));
        CHK(dev_alloc(&a.va, m)); CHK(dev_alloc(&a.vb, m)); CHK(dev_alloc(&a.rank, m));
        CHK(dev_alloc(&a.alive, m)); CHK(dev_alloc(&a.kept, m));
        CHK(dev_alloc(&a.ti, m)); CHK(dev_alloc(&a.tj, m)); CHK(dev_alloc(&a.tk, m));
        a.cap = m;
    }
    if (nq > a.cap_q) {
        dev_free(a.mq); dev_free(a.cq);
        a.cap_q = 0;
        CHK(dev_alloc(&a.mq, nq)); CHK(dev_alloc(&a.cq, nq));
        a.cap_q = nq;
    }
    if (nt > a.cap_t) {
        dev_free(a.mt); dev_free(a.ct);
        a.cap_t = 0;
        CHK(dev_alloc(&a.mt, nt)); CHK(dev_alloc(&a.ct, nt));
        a.cap_t = nt;
    }
    if (!a.counter) CHK(dev_alloc(&a.counter, 1));
    return ensure_sort_scratch(c, n_hits);
}

void free_annihilation(tril_ctx *c) {
    AnnScratch &a = c->ann;
    dev_free(a.ka); dev_free(a.kb); dev_free(a.va); dev_free(a.vb); dev_free(a.rank);
    dev_free(a.alive); dev_free(a.kept); dev_free(a.ti); dev_free(a.tj); dev_free(a.tk);
    dev_free(a.mq); dev_free(a.cq); dev_free(a.mt); dev_free(a.ct); dev_free(a.counter);
    a = AnnScratch{};
}

// Consumed-photon flags of both beams for a run with TRIL_ANNIHILATE, cleared.
int ensure_dead(tril_ctx *c, int64_t nq, int64_t nt) {
    if (nq > c->dead_cap_q) {
        ++c->alloc_gen;
        dev_free(c->dead_q);
        c->dead_cap_q = 0;
        CHK(dev_alloc(&c->dead_q, (size_t)nq));
        c->dead_cap_q = nq;
    }
    if (nt > c->dead_cap_t) {
        ++c->alloc_gen;
        dev_free(c->dead_t);
        c->dead_cap_t = 0;
        CHK(dev_alloc(&c->dead_t, (size_t)nt));
        c->dead_cap_t = nt;
    }
    if (!c->ann_count) CHK(dev_alloc(&c->ann_count, 1));
    if (nq > 0) HIPCHK(hipMemsetAsync(c->dead_q, 0, (size_t)nq, c->st));
    if (nt > 0) HIPCHK(hipMemsetAsync(c->dead_t, 0, (size_t)nt, c->st));
    return TRIL_OK;
}

int ensure_stats(tril_ctx *c, int64_t n_hits, int32_t n_steps) {
    StatsScratch &s = c->sst;
    if (n_hits > s.cap) {
        dev_free(s.keys); dev_free(s.keys_alt); dev_free(s.vals); dev_free(s.vals_alt);
        dev_free(s.flags); dev_free(s.pos); dev_free(s.block_sums);
        dev_free(s.ti); dev_free(s.tj); dev_free(s.tk);
        s.cap = 0;
        const int64_t m = std::max<int64_t>(n_hits, 1024);
        CHK(dev_alloc(&s.keys, m)); CHK(dev_alloc(&s.keys_alt, m));
        CHK(dev_alloc(&s.vals, m)); CHK(dev_alloc(&s.vals_alt, m));
        CHK(dev_alloc(&s.flags, m)); CHK(dev_alloc(&s.pos, m));
        CHK(dev_alloc(&s.block_sums, (size_t)stats_block_sums_needed(m)));
        CHK(dev_alloc(&s.ti, m)); CHK(dev_alloc(&s.tj, m)); CHK(dev_alloc(&s.tk, m));
        s.cap = m;
    }
    if (!s.acc) {
        CHK(dev_alloc(&s.acc, (size_t)c->n_bins + 1));
        CHK(dev_alloc(&s.ucount, 1));
    }
    if (n_steps > s.cap_steps) {
        dev_free(s.step_counts);
        s.cap_steps = 0;
        CHK(dev_alloc(&s.step_counts, (size_t)n_steps));
        s.cap_steps = n_steps;
    }
    return ensure_sort_scratch(c, n_hits);
}

double sum_events(tril_ctx *c, const std::vector<std::array<int, 2>> &v) {
    double tot = 0.0;
    for (const auto &p : v) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev_pool[p[0]], c->ev_pool[p[1]]) == hipSuccess) tot += ms;
    }
    return tot;
}

// Fold the recorded event pairs into running sums and recycle the events (the
// stream has been synchronised by the caller).
void fold_events(tril_ctx *c) {
    c->ms_acc[0] += sum_events(c, c->ev_build);
    c->ms_acc[1] += sum_events(c, c->ev_prep);
    c->ms_acc[2] += sum_events(c, c->ev_trav);
    c->ms_acc[3] += sum_events(c, c->ev_narrow);
    c->timed_launches += (int64_t)c->ev_trav.size();
    c->ev_build.clear();
    c->ev_prep.clear();
    c->ev_trav.clear();
    c->ev_narrow.clear();
    c->ev_next = 0;
}

// Morton bits for the batches of tril_run (both beams already in full-precision Morton
// order): the parameter if set, else as many as keep instance prefix + Morton bits
// within three 8-bit radix passes, between 18 and 30.
int run_morton_bits(const tril_ctx *c, int64_t n_inst) {
    if (c->morton_param > 0) return c->morton_param;
    const int p = bits_for((uint64_t)(n_inst > 1 ? n_inst - 1 : 0));
    return std::min(30, std::max(18, 24 - p));
}

// Steps per launch for tril_run: the parameter if set, else as many as keep the
// virtual element count of one launch within the budget (kBatchBudgetMax with window
// copies; else kBatchBudget, raised for large beams towards kBatchStepsMin steps).
int32_t pick_batch(const tril_ctx *c, const tril_beam *t, const tril_beam *q, int32_t n_steps) {
    const int64_t rows = std::max<int64_t>(std::max(t->n, q->n), 1);
    const bool windows = c->cloud.on == 0 && c->kwin != 1;
    const int64_t budget =
        windows ? kBatchBudgetMax
                : std::max(kBatchBudget, std::min(kBatchBudgetMax, kBatchStepsMin * rows));
    int64_t m = c->step_batch > 0 ? c->step_batch : std::max<int64_t>(1, budget / rows);
    if (c->step_batch <= 0 && windows && m < n_steps) {
        // a batch's last copy of fewer than w/8 steps would cost a whole copy's refit for
        // those few steps: they go to the next batch (1.6e7-photon beams: 32 steps per
        // launch rather than 33, one copy per launch instead of two)
        const int64_t w = auto_window(c);
        if (m > w && m % w < (w + 7) / 8) m -= m % w;
    }
    m = std::min<int64_t>(m, n_steps);
    m = std::min<int64_t>(m, std::max<int64_t>(1, (kMaxN - 1) / rows));
    m = std::min<int64_t>(m, std::max<int64_t>(1, kMaxComb / std::max(t->n_inst, 1)));
    return (int32_t)std::max<int64_t>(m, 1);
}

}  // namespace

namespace tril {

// Breit-Wheeler cross-section on the host (same algebraic form as the device),
// used only for the upper bound that pads query boxes.
double host_sigma(double s) {
    if (!(s > 1.0)) return 0.0;
    const double k_sig = (0.5 * M_PI) * (kRe * kRe);
    const double b2 = (s - 1.0) / s;
    const double b = std::sqrt(b2);
    const double L = 2.0 * std::log1p(b) + std::log(s);
    return (k_sig / s) * ((3.0 - b2 * b2) * L - (2.0 * b) * (2.0 - b2));
}

// Maximum over s of the cross-section: it rises from zero at threshold to one
// maximum near s = 2 and falls as ln(s)/s; golden-section search on [1, 10]
// plus a scan of the neighbourhood.
double host_sigma_max() {
    double a = 1.0, b = 10.0;
    const double g = 0.6180339887498949;
    double x1 = b - g * (b - a), x2 = a + g * (b - a);
    for (int it = 0; it < 200; ++it) {
        if (host_sigma(x1) > host_sigma(x2)) b = x2; else a = x1;
        x1 = b - g * (b - a);
        x2 = a + g * (b - a);
    }
    double m = host_sigma(0.5 * (a + b));
    for (int k = -200; k <= 200; ++k) m = std::max(m, host_sigma(0.5 * (a + b) * (1.0 + 1e-4 * k)));
    return m;
}

}  // namespace tril

// ------------------------------------------------------------------------ ABI

extern "C" {

const char *tril_strerror(int code) {
    switch (code) {
    case TRIL_OK: return "ok";
    case TRIL_E_INVAL: return "invalid argument";
    case TRIL_E_NOMEM: return "device out of memory";
    case TRIL_E_OVERFLOW: return "buffer overflow (pairs or candidates)";
    case TRIL_E_HIP: return "HIP runtime error";
    case TRIL_E_NOTIMPL: return "not implemented";
    case TRIL_E_STATE: return "call order or instance mismatch";
    case TRIL_E_DATA: return "invalid photon data (non-finite, E <= 0 or w < 0)";
    case TRIL_E_INTERNAL: return "device wait bound exceeded";
    default: return "unknown error";
    }
}

const char *tril_last_hip_error(void) { return g_last_hip.c_str(); }

int tril_create(tril_ctx **out, const tril_params *p, void *stream) {
    if (!out || !p) return TRIL_E_INVAL;
    *out = nullptr;
    if (!std::isfinite(p->dt) || !(p->dt > 0.0)) return TRIL_E_INVAL;
    if (p->n_bins < 0 || p->cand_cap < 0 || p->step_batch < 0 || p->kinetic_window < 0 ||
        p->descent_window < 0 || p->descent_window > kMaxDescent)
        return TRIL_E_INVAL;
    if (p->morton_bits != 0 && (p->morton_bits < 3 || p->morton_bits > 30)) return TRIL_E_INVAL;
    if (p->flags &
        ~(TRIL_TIMING | TRIL_SORT_QUERIES_ONCE | TRIL_FP64_NARROW | TRIL_ANNIHILATE | TRIL_GRID))
        return TRIL_E_NOTIMPL;
    if (p->n_bins > 0) {
        if (!p->bin_edges) return TRIL_E_INVAL;
        for (int32_t b = 0; b <= p->n_bins; ++b)
            if (!std::isfinite(p->bin_edges[b])) return TRIL_E_INVAL;
        for (int32_t b = 0; b < p->n_bins; ++b)
            if (!(p->bin_edges[b + 1] > p->bin_edges[b])) return TRIL_E_INVAL;
    }
    // one wave per traversal workgroup: a slot is freed as soon as its wave's queries are
    // done, not when the slowest of several waves is
    const int blk = p->block_traverse == 0 ? 64 : p->block_traverse;
    if (blk != 64 && blk != 128 && blk != 256 && blk != 512) return TRIL_E_INVAL;

    tril_ctx *c = new tril_ctx();
    c->st = reinterpret_cast<hipStream_t>(stream);
    c->dt = p->dt;
    c->flags = p->flags;
    c->n_bins = p->n_bins;
    c->cand_cap_param = p->cand_cap;
    c->block = blk;
    c->step_batch = p->step_batch;
    c->kwin = p->kinetic_window;
    c->kdesc = p->descent_window;
    c->morton_param = p->morton_bits;
    c->sigma_up = host_sigma_max() * (1.0 + 1e-6);
    int r = TRIL_OK;
    auto fail = [&](int code) {
        tril_destroy(c);
        return code;
    };
    if ((r = dev_alloc(&c->d_cnt, 1)) != TRIL_OK) return fail(r);
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&c->h_cnt), sizeof(DevCounters));
    if (e != hipSuccess) return fail(hip_fail(e));
    std::memset(c->h_cnt, 0, sizeof(DevCounters));
    e = hipMemcpy(c->d_cnt, c->h_cnt, sizeof(DevCounters), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(hip_fail(e));
    if (c->n_bins > 0) {
        if ((r = dev_alloc(&c->d_edges, (size_t)c->n_bins + 1)) != TRIL_OK) return fail(r);
        e = hipMemcpy(c->d_edges, p->bin_edges, sizeof(double) * (c->n_bins + 1),
                      hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(hip_fail(e));
    }
    e = hipStreamCreateWithFlags(&c->gst, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(hip_fail(e));
    if ((e = hipEventCreateWithFlags(&c->ev_join_a, hipEventDisableTiming)) != hipSuccess)
        return fail(hip_fail(e));
    if ((e = hipEventCreateWithFlags(&c->ev_join_b, hipEventDisableTiming)) != hipSuccess)
        return fail(hip_fail(e));
    e = hipStreamCreateWithFlags(&c->qst, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(hip_fail(e));
    if ((e = hipEventCreateWithFlags(&c->ev_qfork, hipEventDisableTiming)) != hipSuccess)
        return fail(hip_fail(e));
    if ((e = hipEventCreateWithFlags(&c->ev_qjoin, hipEventDisableTiming)) != hipSuccess)
        return fail(hip_fail(e));
    if ((e = hipEventCreateWithFlags(&c->ev_tfork, hipEventDisableTiming)) != hipSuccess)
        return fail(hip_fail(e));
    if ((e = hipEventCreateWithFlags(&c->ev_tjoin, hipEventDisableTiming)) != hipSuccess)
        return fail(hip_fail(e));
    *out = c;
    return TRIL_OK;
}

int tril_build(tril_ctx *c, const tril_beam *b, int32_t step) {
    if (!c || step < 0) return TRIL_E_INVAL;
    CHK(check_beam(b));
    if ((c->flags & TRIL_GRID) && b->n_inst > 1) return TRIL_E_NOTIMPL;
    c->morton_bits = c->morton_param > 0 ? c->morton_param : 30;
    CHK(ensure_target(c, b->n, b->n, b->n_inst, b->n_inst));
    CHK(upload_offsets(c, b, c->d_t_off, c->h_t_off));
    c->nt = b->n;
    c->tgt = view(b, c->d_t_off, 1);
    c->res_t = c->tgt;
    launch_set_step(c->d_cnt, step, c->st);
    launch_beam_stats(c->tgt, c->t_spart, c->t_stats, c->d_cnt, c->st, true);
    if (c->flags & TRIL_GRID)
        CHK(enqueue_grid_build(c, c->st, (c->flags & TRIL_TIMING) != 0));
    else
        CHK(enqueue_build(c, c->st, (c->flags & TRIL_TIMING) != 0));
    c->built = true;
    c->built_step = step;
    c->tgt_k0 = step;
    c->max_step = std::max(c->max_step, step);
    return TRIL_OK;
}

int tril_collide(tril_ctx *c, const tril_beam *q, int32_t step, tril_pairs *out) {
    if (!c) return TRIL_E_INVAL;
    CHK(check_beam(q));
    CHK(check_pairs(out));
    if (!c->built || c->tgt.m != 1 || step != c->built_step || q->n_inst != c->tgt.n_inst)
        return TRIL_E_STATE;
    c->morton_bits = c->morton_param > 0 ? c->morton_param : 30;
    CHK(ensure_query(c, q->n, q->n, q->n_inst, q->n_inst));
    CHK(upload_offsets(c, q, c->d_q_off, c->h_q_off));
    const BeamDev qv = view(q, c->d_q_off, 1);
    const bool sort = need_query_sort(c, q);
    launch_beam_stats(qv, c->q_spart, c->q_stats, c->d_cnt, c->st, true);
    if (c->flags & TRIL_GRID)
        CHK(enqueue_grid_collide(c, qv, *out, c->st, (c->flags & TRIL_TIMING) != 0, sort));
    else
        CHK(enqueue_collide(c, qv, *out, c->st, (c->flags & TRIL_TIMING) != 0, sort));
    if (sort) CHK(note_query_sorted(c, q, 1, c->st));
    c->last_q = qv;
    c->max_nq = std::max(c->max_nq, q->n);
    return TRIL_OK;
}

int tril_run(tril_ctx *c, const tril_beam *t, const tril_beam *q, int32_t k0, int32_t n_steps,
             tril_pairs *out) {
    if (!c || k0 < 0 || n_steps < 0) return TRIL_E_INVAL;
    CHK(check_beam(t));
    CHK(check_beam(q));
    CHK(check_pairs(out));
    if (q->n_inst != t->n_inst) return TRIL_E_STATE;
    if (n_steps == 0) return TRIL_OK;
    if ((int64_t)k0 + n_steps - 1 > INT32_MAX) return TRIL_E_INVAL;
    if (c->flags & TRIL_GRID) {  // the grid broad phase runs step by step
        for (int32_t k = k0; k < k0 + n_steps; ++k) {
            CHK(tril_build(c, t, k));
            CHK(tril_collide(c, q, k, out));
        }
        return TRIL_OK;
    }
    const int32_t m = pick_batch(c, t, q, n_steps);
    const int32_t bw = build_window(c, m);
    // capacities for the largest batch first, so that nothing is reallocated later: tree
    // buffers per copy (a batch's last, shorter one needs no more copies), query boxes only
    // where a batch of one step or the cloud regime writes them (else per-row records)
    const int64_t t_units = bw > 1 ? (int64_t)window_copies(m, bw) : m;
    CHK(ensure_target(c, t_units * t->n, t->n, (int64_t)m * t->n_inst, t->n_inst));
    if (bw > 1 && t->n > 1) {  // four-child forms of the window copies
        const int64_t need = (int64_t)window_copies(m, bw) * (t->n - 1);
        if (need > c->nodes4_cap) {
            ++c->alloc_gen;
            dev_free(c->nodes4);
            c->nodes4_cap = 0;
            CHK(dev_alloc(&c->nodes4, (size_t)need));
            c->nodes4_cap = need;
        }
        if (t->n - 1 > c->inside_cap) {
            ++c->alloc_gen;
            dev_free(c->t_inside);
            c->inside_cap = 0;
            CHK(dev_alloc(&c->t_inside, (size_t)(t->n - 1)));
            c->inside_cap = t->n - 1;
        }
        const int32_t nf = window_copies(m, bw);
        if (nf > c->frames_cap) {
            ++c->alloc_gen;
            dev_free(c->t_frames);
            c->frames_cap = 0;
            CHK(dev_alloc(&c->t_frames, (size_t)nf));
            c->frames_cap = nf;
        }
    }
    const bool q_records = m >= 2 && c->cloud.on == 0;
    CHK(ensure_query(c, (int64_t)m * q->n, q->n, (int64_t)m * q->n_inst, q->n_inst,
                     q_records ? q->n : (int64_t)m * q->n));
    CHK(ensure_work(c, c->wt, t->n));
    CHK(ensure_work(c, c->wq, q->n));
    CHK(upload_offsets(c, t, c->d_t_off, c->h_t_off));
    CHK(upload_offsets(c, q, c->d_q_off, c->h_q_off));
    c->nt = t->n;
    c->q_order_key = nullptr;  // the sort buffers are reused below
    const BeamDev t1 = view(t, c->d_t_off, 1), q1 = view(q, c->d_q_off, 1);
    // working copies in the caller's order; after every batch they are rewritten in the
    // Morton order of that batch's first step (a relabelling of rows: the pair set does
    // not depend on it, and the narrow phase reports caller rows)
    // first, both beams in the order the first batch's sorts would give them, which those
    // sorts then skip
    int pt = 0, pq = 0;
    c->morton_bits = run_morton_bits(c, t->n_inst);
    const int32_t m0 = std::min(m, n_steps);
    launch_set_step(c->d_cnt, k0, c->st);
    // the two beams side by side (statistics, then order): the query beam on qst with its
    // own sort scratch
    HIPCHK(hipEventRecord(c->ev_qfork, c->st));
    HIPCHK(hipStreamWaitEvent(c->qst, c->ev_qfork, 0));
    // (the statistics pass also writes each beam's rows as 64-B records into the other
    // working buffer, unused until the first batch's re-gather, for the ordering's gather)
    launch_beam_stats(t1, c->t_spart, c->t_stats, c->d_cnt, c->st, true, c->wt[1].soa);
    launch_beam_stats(q1, c->q_spart, c->q_stats, c->d_cnt, c->qst, true, c->wq[1].soa);
    CHK(enqueue_order(c, view(t, c->d_t_off, m0), false, c->wt[0], c->st, c->ss, c->wt[1].soa));
    CHK(enqueue_order(c, view(q, c->d_q_off, m0), true, c->wq[0], c->qst, c->ssq, c->wq[1].soa));
    HIPCHK(hipEventRecord(c->ev_qjoin, c->qst));
    HIPCHK(hipStreamWaitEvent(c->st, c->ev_qjoin, 0));
    const bool once = (c->flags & TRIL_SORT_QUERIES_ONCE) != 0;
    bool q_sorted = false;
    const bool timed = (c->flags & TRIL_TIMING) != 0;
    // annihilation: after every batch its hits are resolved in chronological order and the
    // photons of the kept hits are marked consumed, so that later batches leave them out of
    // their hierarchies and queries (the kept set is the same as resolving at the end)
    const bool ann = (c->flags & TRIL_ANNIHILATE) != 0;
    int64_t ann_done = 0;  // hits in the buffer that are resolved (kept hits and older hits)
    bool ann_ok = true;    // false once the pair buffer overflowed: tril_stats reports it
    if (ann) {
        CHK(ensure_annihilation(c, std::max<int64_t>(out->cap, 1), q->n, t->n));
        CHK(ensure_dead(c, q->n, t->n));
        HIPCHK(hipStreamSynchronize(c->st));
        HIPCHK(hipMemcpy(&ann_done, out->count, sizeof(ann_done), hipMemcpyDeviceToHost));
        if (ann_done > out->cap) ann_ok = false;
    }
    auto resolve = [&](hipStream_t st, int32_t last_step) -> int {
        if (!ann || !ann_ok) return TRIL_OK;
        HIPCHK(hipStreamSynchronize(st));
        int64_t cnt = 0;
        HIPCHK(hipMemcpy(&cnt, out->count, sizeof(cnt), hipMemcpyDeviceToHost));
        if (cnt > out->cap) {
            ann_ok = false;
            return TRIL_OK;
        }
        const int64_t nb = cnt - ann_done;
        if (nb <= 0) return TRIL_OK;
        const tril_pairs v{out->cap - ann_done, out->i + ann_done, out->j + ann_done,
                           out->step + ann_done, c->ann_count};
        int64_t kept = 0;
        const hipError_t e = annihilate_hits(v, nb, view(q, c->d_q_off, 1), view(t, c->d_t_off, 1),
                                             c->dt, last_step, c->ann, c->ss, &c->d_cnt->err, st,
                                             &kept);
        if (e != hipSuccess) return hip_fail(e);
        launch_ann_mark(v, kept, c->dead_q, c->dead_t, st);
        ann_done += kept;
        HIPCHK(hipMemcpyAsync(out->count, &ann_done, sizeof(ann_done), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        return TRIL_OK;
    };

    // Batch of mb steps with working buffers (pt, pq) on stream st: build, collide, and
    // (regather: another batch follows) rewrite the working copies for the next batch.
    // pre: the run's first batch, whose working copies are in its order already (no sorts;
    // sort is then false)
    auto enqueue_batch = [&](int32_t mb, bool sort, hipStream_t st, bool tm, bool regather,
                             bool pre) -> int {
        c->tgt = wview(t, c->d_t_off, mb, c->wt[pt]);
        BeamDev qv = wview(q, c->d_q_off, mb, c->wq[pq]);
        if (ann) {
            c->tgt.dead = c->dead_t;
            qv.dead = c->dead_q;
        }
        // the query preparation on qst beside the build: it reads only the query working
        // copy and the run's statistics, and writes only query buffers
        HIPCHK(hipEventRecord(c->ev_qfork, st));
        HIPCHK(hipStreamWaitEvent(c->qst, c->ev_qfork, 0));
        CHK(enqueue_build(c, st, tm, pre));
        if (!sort) {
            c->q_order = nullptr;  // the working copy is already in Morton order
            c->q_order_len = 0;
        }
        CHK(enqueue_collide_prep(c, qv, c->qst, tm, sort, &c->ssq));
        // the query working copy for the next batch in this batch's order (it writes the
        // other buffer, which this batch does not read)
        if (regather && sort)
            launch_gather_beam(wview(q, c->d_q_off, 1, c->wq[pq]), c->q_order, c->wq[pq ^ 1].soa,
                               c->wq[pq ^ 1].perm, c->qst);
        HIPCHK(hipEventRecord(c->ev_qjoin, c->qst));
        HIPCHK(hipStreamWaitEvent(st, c->ev_qjoin, 0));
        // the target working copy for the next batch in this batch's order, on qst beside the
        // traversal and narrow phase (they read the other buffer and the tree only)
        if (regather) {
            HIPCHK(hipEventRecord(c->ev_tfork, st));
            HIPCHK(hipStreamWaitEvent(c->qst, c->ev_tfork, 0));
            launch_gather_beam(wview(t, c->d_t_off, 1, c->wt[pt]), c->t_rows, c->wt[pt ^ 1].soa,
                               c->wt[pt ^ 1].perm, c->qst);
            HIPCHK(hipEventRecord(c->ev_tjoin, c->qst));
        }
        CHK(enqueue_collide(c, qv, *out, st, tm, sort, true));
        if (regather) HIPCHK(hipStreamWaitEvent(st, c->ev_tjoin, 0));
        return TRIL_OK;
    };
    int last_pq = 0;            // query working buffer of the last batch enqueued
    int32_t last_mb = 0;
    auto flip = [&](bool sort) {
        pt ^= 1;
        if (sort) pq ^= 1;
    };

    int32_t k = k0;
    int32_t left = n_steps;
    bool presorted = true;  // the first batch's working copies are in its order
    while (left > 0) {
        const int32_t mb = std::min(m, left);
        const bool pre = presorted;
        presorted = false;
        const bool sort = (!once || !q_sorted) && !pre;
        if (timed || mb != m || (!pre && sort != (!once))) {
            // eager batch (per-phase events, the shorter last batch, or the one batch that
            // orders the queries when they are ordered once)
            launch_set_step(c->d_cnt, k, c->st);
            CHK(enqueue_batch(mb, sort, c->st, timed, left > mb, pre));
            last_pq = pq;
            last_mb = mb;
            flip(sort);
            CHK(resolve(c->st, k + mb - 1));
            q_sorted = q_sorted || sort || pre;
            k += mb;
            left -= mb;
            continue;
        }
        // full batches: captured graphs (the first batch, then one per buffer parity),
        // replayed; the step index lives on the device
        const int32_t n_rep = pre ? 1 : left / m;
        q_sorted = q_sorted || pre;
        launch_set_step(c->d_cnt, k, c->st);
        HIPCHK(hipEventRecord(c->ev_join_a, c->st));
        HIPCHK(hipStreamWaitEvent(c->gst, c->ev_join_a, 0));
        for (int32_t r = 0; r < n_rep; ++r) {
            const bool regather = r + 1 < n_rep || left > n_rep * m;  // another batch follows
            std::vector<const void *> key = {
                c->wt[pt].soa, c->wq[pq].soa, c->wt[pt ^ 1].soa, c->wq[pq ^ 1].soa,
                out->i, out->j, out->step, out->count,
                (const void *)(intptr_t)t->n, (const void *)(intptr_t)q->n,
                (const void *)(intptr_t)t->n_inst, (const void *)(intptr_t)out->cap,
                (const void *)(intptr_t)sort, c->d_t_off, c->d_q_off,
                (const void *)(intptr_t)m, (const void *)(intptr_t)c->morton_bits,
                (const void *)(uintptr_t)c->alloc_gen,
                // every launch parameter read while the batch is captured
                (const void *)(intptr_t)c->block, (const void *)(uintptr_t)c->flags,
                (const void *)(intptr_t)c->trav_queue,
                (const void *)(intptr_t)c->cand_cap, (const void *)(intptr_t)c->kwin,
                (const void *)(intptr_t)c->kdesc, (const void *)(intptr_t)c->kdesc_auto,
                (const void *)(intptr_t)regather, (const void *)(intptr_t)pre};
            int slot = -1;
            for (int g = 0; g < tril_ctx::kGraphs && slot < 0; ++g)
                if (c->gexec[g] && key == c->gkey[g]) slot = g;
            if (slot < 0) {
                slot = c->g_next;
                c->g_next = (c->g_next + 1) % tril_ctx::kGraphs;
                if (c->gexec[slot]) {
                    (void)hipGraphExecDestroy(c->gexec[slot]);
                    c->gexec[slot] = nullptr;
                }
                hipGraph_t g = nullptr;
                HIPCHK(hipStreamBeginCapture(c->gst, hipStreamCaptureModeThreadLocal));
                int r1 = enqueue_batch(m, sort, c->gst, false, regather, pre);
                launch_advance_step(c->d_cnt, m, c->gst);
                hipError_t e = hipStreamEndCapture(c->gst, &g);
                if (r1 != TRIL_OK) {
                    if (g) (void)hipGraphDestroy(g);
                    return r1;
                }
                if (e != hipSuccess) return hip_fail(e);
                e = hipGraphInstantiate(&c->gexec[slot], g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) {
                    c->gexec[slot] = nullptr;
                    return hip_fail(e);
                }
                c->gkey[slot] = key;
            }
            HIPCHK(hipGraphLaunch(c->gexec[slot], c->gst));
            last_pq = pq;
            last_mb = m;
            flip(sort);
            CHK(resolve(c->gst, k + (r + 1) * m - 1));
        }
        HIPCHK(hipEventRecord(c->ev_join_b, c->gst));
        HIPCHK(hipStreamWaitEvent(c->st, c->ev_join_b, 0));
        k += n_rep * m;
        left -= n_rep * m;
    }
    // the last batch's view (its working-copy buffer: graph replays leave the host view
    // of the last capture)
    c->tgt = wview(t, c->d_t_off, c->tgt.m, c->wt[pt ^ 1]);
    if (c->quad) c->ad_quad = true;  // the counters now hold descents of kdesc_auto steps
    c->last_qrec = wview(q, c->d_q_off, last_mb, c->wq[last_pq]);
    if (!(last_mb >= 2 && c->cloud.on == 0)) c->last_qrec.m = 0;  // boxes, not records
    c->built = true;
    c->built_step = k0 + n_steps - 1;
    c->tgt_k0 = k0 + n_steps - c->tgt.m;
    c->max_step = std::max(c->max_step, c->built_step);
    c->res_t = t1;
    c->last_q = q1;
    c->max_nq = std::max(c->max_nq, q->n);
    return TRIL_OK;
}

int tril_stats(tril_ctx *c, tril_pairs *p, tril_stats_t *out) {
    if (!c || !out) return TRIL_E_INVAL;
    if (p) CHK(check_pairs(p));
    if (out->n_step_counts < 0 || (out->n_step_counts > 0 && !out->step_counts))
        return TRIL_E_INVAL;
    // host words: [0] hits, [1] unique pairs, [2] error flags, [3, 4 + n_bins) yield and
    // spectrum, then the per-step counts; the device copies go into them asynchronously, and
    // one synchronisation ends each group
    const int64_t words = 4 + (int64_t)c->n_bins + out->n_step_counts;
    if (words > c->h_pin_cap) {
        HIPCHK(hipStreamSynchronize(c->st));
        if (c->h_pin) (void)hipHostFree(c->h_pin);
        c->h_pin = nullptr;
        c->h_pin_cap = 0;
        HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&c->h_pin), (size_t)words * sizeof(*c->h_pin)));
        c->h_pin_cap = words;
    }
    unsigned long long *hp = c->h_pin;
    HIPCHK(hipMemcpyAsync(c->h_cnt, c->d_cnt, sizeof(DevCounters), hipMemcpyDeviceToHost, c->st));
    if (p) HIPCHK(hipMemcpyAsync(hp, p->count, sizeof(int64_t), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    const DevCounters &h = *c->h_cnt;
    out->n_candidates = (int64_t)h.cand_total + (int64_t)h.st_pairs;
    int64_t visits = 0, queries = 0, checks = 0;
    for (int k = 0; k < kCounterSlots; ++k) {
        visits += (int64_t)h.visits[k];
        queries += (int64_t)h.queries[k];
        checks += (int64_t)h.leaf_checks[k];
    }
    out->n_node_visits = visits;
    out->n_leaf_checks = checks;
    out->n_queries = queries;
    out->descent_window = c->ad_quad ? descent_window(c, c->win_eff) : 0;
    adapt_descent(c, checks, queries);
    out->n_sigma_evals = (int64_t)h.sigma_evals;
    out->n_fp64_rechecks = (int64_t)h.fp64_rechecks;
    out->n_builds = (int64_t)h.builds;
    out->n_collides = (int64_t)h.collides;
    const unsigned int err = h.err;
    fold_events(c);
    out->ms_build = c->ms_acc[0];
    out->ms_query_prep = c->ms_acc[1];
    out->ms_traverse = c->ms_acc[2];
    out->ms_narrow = c->ms_acc[3];
    out->n_timed_launches = c->timed_launches;
    out->n_pairs = 0;
    out->n_hits = 0;
    out->yield = 0.0;
    if (err & kErrData) return TRIL_E_DATA;
    if (err & (kErrSpin | kErrInternal)) return TRIL_E_INTERNAL;
    if (err & kErrCandOverflow) return TRIL_E_OVERFLOW;
    if (!p) return TRIL_OK;
    int64_t n_hits = (int64_t)hp[0];
    out->n_hits = n_hits;
    if (n_hits > p->cap || (err & kErrPairOverflow)) return TRIL_E_OVERFLOW;
    if (n_hits > 0 && (!c->built || c->last_q.n <= 0)) return TRIL_E_STATE;
    if ((c->flags & TRIL_ANNIHILATE) && n_hits > 0) {
        CHK(ensure_annihilation(c, n_hits, c->last_q.n, c->res_t.n));
        int64_t kept = 0;
        const hipError_t e = annihilate_hits(*p, n_hits, c->last_q, c->res_t, c->dt,
                                             std::max(c->max_step, 0), c->ann, c->ss,
                                             &c->d_cnt->err, c->st, &kept);
        if (e != hipSuccess) return hip_fail(e);
        n_hits = kept;
        out->n_hits = kept;
    }
    const int pair_bits = bits_for((uint64_t)std::max<int64_t>(c->max_nq, 1) *
                                   (uint64_t)std::max<int64_t>(c->nt, 1));
    if (pair_bits > 64) return TRIL_E_NOTIMPL;
    const int32_t nsc = out->step_counts ? out->n_step_counts : 0;
    CHK(ensure_stats(c, n_hits, std::max(nsc, 1)));
    run_union_stats(*p, n_hits, std::max<int64_t>(c->nt, 1), pair_bits,
                    c->last_q.w, c->res_t.w, c->last_q.E, c->res_t.E, c->d_edges, c->n_bins, nsc,
                    c->sst, c->ss, &c->d_cnt->err, c->st);
    HIPCHK(hipGetLastError());
    unsigned int *herr = reinterpret_cast<unsigned int *>(hp + 2);
    const double *acc = reinterpret_cast<const double *>(hp + 3);
    HIPCHK(hipMemcpyAsync(hp + 1, c->sst.ucount, sizeof(*hp), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(herr, &c->d_cnt->err, sizeof(*herr), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(hp + 3, c->sst.acc, ((size_t)c->n_bins + 1) * sizeof(double),
                          hipMemcpyDeviceToHost, c->st));
    if (nsc > 0)
        HIPCHK(hipMemcpyAsync(hp + 4 + c->n_bins, c->sst.step_counts, (size_t)nsc * sizeof(*hp),
                              hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    out->n_pairs = (int64_t)hp[1];
    out->yield = acc[0];
    if (out->spectrum)
        for (int32_t b = 0; b < c->n_bins; ++b) out->spectrum[b] = acc[1 + b];
    for (int32_t k = 0; k < nsc; ++k) out->step_counts[k] = (int64_t)hp[4 + c->n_bins + k];
    if (*herr & (kErrSpin | kErrInternal)) return TRIL_E_INTERNAL;
    return TRIL_OK;
}

int tril_pair_kinematics(tril_ctx *c, const tril_beam *q, const tril_beam *t,
                         const tril_pairs *p, int64_t n, const tril_kin_params *kp,
                         double *leptons, tril_kin_out *out) {
    if (!c || !kp || !out || n < 0) return TRIL_E_INVAL;
    CHK(check_beam(q));
    CHK(check_beam(t));
    if (n > 0) {
        CHK(check_pairs(p));
        if (n > p->cap) return TRIL_E_INVAL;
    }
    const int32_t ng = kp->n_gamma, nth = kp->n_theta;
    if (ng < 0 || ng > TRIL_KIN_MAX_BINS || nth < 0 || nth > TRIL_KIN_MAX_BINS) return TRIL_E_INVAL;
    if (ng > 0) {
        if (!kp->gamma_edges) return TRIL_E_INVAL;
        for (int32_t b = 0; b <= ng; ++b)
            if (!std::isfinite(kp->gamma_edges[b]) || (b > 0 && !(kp->gamma_edges[b] > kp->gamma_edges[b - 1])))
                return TRIL_E_INVAL;
    }
    if ((ng > 0 && !out->gamma_hist) || (nth > 0 && !out->theta_hist)) return TRIL_E_INVAL;
    out->ms_kernel = 0.0;
    constexpr int64_t kBuf = 3 * TRIL_KIN_MAX_BINS + 1;  // edges, then the histogram bins
    if (!c->kin_buf) {
        CHK(dev_alloc(&c->kin_buf, (size_t)kBuf));
        CHK(dev_alloc(&c->kin_err, 1));
        for (hipEvent_t &e : c->ev_kin) HIPCHK(hipEventCreate(&e));
    }
    double *d_edges = c->kin_buf, *d_hist = c->kin_buf + (ng + 1);
    const int32_t nb = ng + nth;
    if (ng > 0)
        HIPCHK(hipMemcpyAsync(d_edges, kp->gamma_edges, (size_t)(ng + 1) * sizeof(double),
                              hipMemcpyHostToDevice, c->st));
    if (nb > 0) HIPCHK(hipMemsetAsync(d_hist, 0, (size_t)nb * sizeof(double), c->st));
    HIPCHK(hipMemsetAsync(c->kin_err, 0, sizeof(unsigned int), c->st));
    const int64_t nrec = pair_kinematics_records(n, q->n, t->n);
    if (nrec > c->kin_rec_cap) {
        dev_free(c->kin_rec);
        c->kin_rec_cap = 0;
        CHK(dev_alloc(&c->kin_rec, (size_t)(8 * nrec)));
        c->kin_rec_cap = nrec;
    }
    HIPCHK(hipEventRecord(c->ev_kin[0], c->st));
    if (n > 0)
        launch_pair_kinematics(view(q, nullptr, 1), view(t, nullptr, 1), p->i, p->j, p->step, n,
                               kp->seed, leptons, d_edges, ng, nth, d_hist, c->kin_err,
                               nrec > 0 ? c->kin_rec : nullptr, c->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(c->ev_kin[1], c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev_kin[0], c->ev_kin[1]));
    out->ms_kernel = ms;
    std::vector<double> h((size_t)std::max(nb, 1), 0.0);
    if (nb > 0)
        HIPCHK(hipMemcpy(h.data(), d_hist, (size_t)nb * sizeof(double), hipMemcpyDeviceToHost));
    for (int32_t b = 0; b < ng; ++b) out->gamma_hist[b] = h[b];
    for (int32_t b = 0; b < nth; ++b) out->theta_hist[b] = h[ng + b];
    unsigned int err = 0;
    HIPCHK(hipMemcpy(&err, c->kin_err, sizeof(err), hipMemcpyDeviceToHost));
    return err ? TRIL_E_INVAL : TRIL_OK;
}

int tril_st_bin(const tril_beam *b, const tril_st_grid *g, int32_t *bins, double *sums,
                void *stream) {
    CHK(check_beam(b));
    if (!g || (b->n > 0 && !bins)) return TRIL_E_INVAL;
    int64_t nb = 1;
    for (int a = 0; a < 3; ++a) {
        if (g->n_pos[a] < 1 || !std::isfinite(g->lo[a]) || !std::isfinite(g->hi[a]) ||
            !(g->hi[a] > g->lo[a]))
            return TRIL_E_INVAL;
        nb *= g->n_pos[a];
    }
    if (g->n_e < 1 || g->n_th < 1 || !(g->e_lo > 0.0) || !(g->e_hi > g->e_lo) ||
        !std::isfinite(g->e_hi) || !(g->th_max > 0.0) || !std::isfinite(g->th_max) ||
        !std::isfinite(g->t_bin))
        return TRIL_E_INVAL;
    nb *= (int64_t)g->n_e * g->n_th;
    if (nb > INT32_MAX) return TRIL_E_INVAL;
    const double an = std::sqrt(g->axis[0] * g->axis[0] + g->axis[1] * g->axis[1] +
                                g->axis[2] * g->axis[2]);
    if (!(std::fabs(an - 1.0) < 1e-9)) return TRIL_E_INVAL;
    StGridDev d;
    for (int a = 0; a < 3; ++a) {
        d.lo[a] = g->lo[a];
        d.hi[a] = g->hi[a];
        d.n_pos[a] = g->n_pos[a];
        d.axis[a] = g->axis[a];
    }
    d.n_e = g->n_e; d.e_lo = g->e_lo; d.e_hi = g->e_hi;
    d.n_th = g->n_th; d.th_max = g->th_max; d.t_bin = g->t_bin;
    BeamDev v = view(b, nullptr, 1);
    v.inst_off = nullptr;
    v.n_inst = 1;
    launch_st_bin(v, d, bins, sums, reinterpret_cast<hipStream_t>(stream));
    HIPCHK(hipGetLastError());
    return TRIL_OK;
}

}  // extern "C"

namespace {

// Statistical-regime pass over steps k0 .. k0+n_steps-1 (asynchronous): clouds of edges
// `cell` in a hierarchy per step, yields (or, geometric, overlap integrals) added to the
// table under (q_bins[i], t_bins[j]); with a filter set, only its keys. Per-wave sums go
// to c->st_slots (cleared here together with the table).
int st_run(tril_ctx *c, const tril_beam *t, const int32_t *t_bins, int64_t n_t_bins,
           const tril_beam *q, const int32_t *q_bins, const double cell[3], int32_t k0,
           int32_t n_steps, int geometric, const long long *filter, int64_t filter_cap,
           long long *keys, double *vals, int64_t cap) {
    if (!c->st_slots) CHK(dev_alloc(&c->st_slots, (size_t)kCounterSlots));
    launch_st_clear(keys, vals, cap, c->st_slots, c->st);
    const int32_t m = n_steps > 0 ? pick_batch(c, t, q, n_steps) : 1;
    CHK(ensure_target(c, (int64_t)m * t->n, t->n, (int64_t)m * t->n_inst, t->n_inst));
    CHK(ensure_query(c, (int64_t)m * q->n, q->n, (int64_t)m * q->n_inst, q->n_inst));
    CHK(upload_offsets(c, t, c->d_t_off, c->h_t_off));
    CHK(upload_offsets(c, q, c->d_q_off, c->h_q_off));
    c->nt = t->n;
    c->q_order_key = nullptr;
    const BeamDev t1 = view(t, c->d_t_off, 1), q1 = view(q, c->d_q_off, 1);
    // caller photons must be light-like; the bin clouds of the surrogate's geometric pass
    // (mode 1) carry mean directions
    launch_beam_stats(t1, c->t_spart, c->t_stats, c->d_cnt, c->st, geometric != 1);
    launch_beam_stats(q1, c->q_spart, c->q_stats, c->d_cnt, c->st, geometric != 1);
    const StCell sc{{cell[0], cell[1], cell[2]}};
    // clouds at mid-step; swarms (geometric 3): clouds swept over the step
    c->cloud = CloudBox{geometric == 3 ? 2 : 1, {0.5 * cell[0], 0.5 * cell[1], 0.5 * cell[2]}};
    c->morton_bits = c->morton_param > 0 ? c->morton_param : 30;
    int rc = TRIL_OK;
    for (int32_t k = k0, left = n_steps; left > 0 && rc == TRIL_OK;) {
        const int32_t mb = std::min(m, left);
        c->tgt = view(t, c->d_t_off, mb);
        const BeamDev qv = view(q, c->d_q_off, mb);
        launch_set_step(c->d_cnt, k, c->st);
        c->tgt_k0 = k;
        if ((rc = enqueue_build(c, c->st, false)) != TRIL_OK) break;
        launch_prologue(c->d_cnt, 1, mb, c->st);
        if ((rc = enqueue_query_prep(c, qv, c->st, true)) != TRIL_OK) break;
        const int64_t nqv = (int64_t)mb * q->n;
        launch_st_traverse(c->nodes, c->n_int, c->root_box, c->q_box, nqv > 0 ? c->q_order : nullptr,
                           c->q_order_len, nqv, q->n, c->inst_root, qv, c->tgt, q_bins, t_bins,
                           n_t_bins, c->dt, sc, geometric, filter, filter_cap, keys, vals, cap,
                           c->st_slots, c->d_cnt, c->st);
        k += mb;
        left -= mb;
    }
    c->cloud.on = 0;
    CHK(rc);
    HIPCHK(hipGetLastError());
    c->built = true;
    c->built_step = k0 + std::max(n_steps, 1) - 1;
    c->res_t = t1;
    c->last_q = q1;
    return TRIL_OK;
}

// Sum of the per-wave slots and the device error flags after a pass (synchronises).
int st_finish(tril_ctx *c, double *total) {
    HIPCHK(hipStreamSynchronize(c->st));
    double slots[kCounterSlots];
    HIPCHK(hipMemcpy(slots, c->st_slots, sizeof(slots), hipMemcpyDeviceToHost));
    double tot = 0.0;
    for (double v : slots) tot += v;
    if (total) *total = tot;
    unsigned int err = 0;
    HIPCHK(hipMemcpy(&err, &c->d_cnt->err, sizeof(err), hipMemcpyDeviceToHost));
    if (err & kErrData) return TRIL_E_DATA;
    if (err & kErrSpin) return TRIL_E_INTERNAL;
    if (err & kErrTableFull) return TRIL_E_OVERFLOW;
    return TRIL_OK;
}

int check_cell(const double cell[3]) {
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(cell[a]) || !(cell[a] > 0.0)) return TRIL_E_INVAL;
    return TRIL_OK;
}

int64_t pow2_at_least(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

int64_t grid_bins(const tril_st_grid *g) {
    return (int64_t)g->n_pos[0] * g->n_pos[1] * g->n_pos[2] * g->n_e * g->n_th;
}

void grid_cell(const tril_st_grid *g, double cell[3]) {
    for (int a = 0; a < 3; ++a) cell[a] = (g->hi[a] - g->lo[a]) / g->n_pos[a];
}

int check_grid(const tril_st_grid *g) {
    if (!g) return TRIL_E_INVAL;
    for (int a = 0; a < 3; ++a)
        if (g->n_pos[a] < 1 || !std::isfinite(g->lo[a]) || !std::isfinite(g->hi[a]) ||
            !(g->hi[a] > g->lo[a]))
            return TRIL_E_INVAL;
    if (g->n_e < 1 || g->n_th < 1) return TRIL_E_INVAL;
    const int64_t nb = grid_bins(g);
    return (nb > 0 && nb <= INT32_MAX) ? TRIL_OK : TRIL_E_INVAL;
}

// Bin clouds of one beam from its per-bin sums: records in the scratch beam w (SoA of
// 8 x cap doubles), their bins in rec_bin; returns the record count in *n.
int st_records(tril_ctx *c, const double *sums, const tril_st_grid *g, WorkBeam &w,
               int32_t *&rec_bin, int64_t &rec_cap, int64_t *n) {
    unsigned long long *cnt = nullptr;
    CHK(dev_alloc(&cnt, 1));
    int rc = TRIL_OK;
    for (int pass = 0; pass < 2; ++pass) {
        if (hipMemsetAsync(cnt, 0, sizeof(*cnt), c->st) != hipSuccess) {
            rc = TRIL_E_HIP;
            break;
        }
        launch_st_records(sums, grid_bins(g), g->t_bin, w.soa, w.cap, rec_bin, cnt, c->st);
        unsigned long long h = 0;
        if (hipMemcpy(&h, cnt, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) {
            rc = TRIL_E_HIP;
            break;
        }
        *n = (int64_t)h;
        if ((int64_t)h <= w.cap) break;
        free_work(w);
        dev_free(rec_bin);
        if ((rc = dev_alloc(&w.soa, (size_t)(8 * h))) != TRIL_OK) break;
        if ((rc = dev_alloc(&w.perm, 1)) != TRIL_OK) break;
        if ((rc = dev_alloc(&rec_bin, (size_t)h)) != TRIL_OK) break;
        w.cap = (int64_t)h;
        rec_cap = (int64_t)h;
    }
    dev_free(cnt);
    return rc;
}

tril_beam soa_beam(const double *soa, int64_t cap, int64_t n) {
    tril_beam b;
    std::memset(&b, 0, sizeof(b));
    b.n = n;
    b.x = soa; b.y = soa + cap; b.z = soa + 2 * cap;
    b.px = soa + 3 * cap; b.py = soa + 4 * cap; b.pz = soa + 5 * cap;
    b.E = soa + 6 * cap; b.w = soa + 7 * cap;
    b.n_inst = 1;
    b.inst_off = nullptr;
    return b;
}

tril_beam record_beam(const WorkBeam &w, int64_t n) { return soa_beam(w.soa, w.cap, n); }

// Feature rows of every candidate bin pair into the context's surrogate buffers (c->sf_*),
// growing them until the rows fit; *nrow receives the row count.
int sur_features(tril_ctx *c, const double *q_sums, const tril_st_grid *gq, const double *t_sums,
                 const tril_st_grid *gt, int32_t k0, int32_t n_steps, const tril_st_sur_params *p,
                 int64_t *nrow);

// Sum of the per-wave slots (synchronises the stream).
int slot_sum(tril_ctx *c, double *out) {
    HIPCHK(hipStreamSynchronize(c->st));
    double sl[kCounterSlots];
    HIPCHK(hipMemcpy(sl, c->st_slots, sizeof(sl), hipMemcpyDeviceToHost));
    double t = 0.0;
    for (double v : sl) t += v;
    *out = t;
    return TRIL_OK;
}

int clear_slots(tril_ctx *c) {
    if (!c->st_slots) CHK(dev_alloc(&c->st_slots, (size_t)kCounterSlots));
    launch_au_zero(c->st_slots, kCounterSlots, c->st);
    return TRIL_OK;
}

int sur_features(tril_ctx *c, const double *q_sums, const tril_st_grid *gq, const double *t_sums,
                 const tril_st_grid *gt, int32_t k0, int32_t n_steps, const tril_st_sur_params *p,
                 int64_t *nrow) {
    int64_t cap = std::max<int64_t>(c->sf_cap, 1 << 16);
    *nrow = 0;
    for (int attempt = 0;; ++attempt) {
        if (cap > c->sf_cap) {
            dev_free(c->sf_x); dev_free(c->sf_y0); dev_free(c->sf_key);
            dev_free(c->sf_mean); dev_free(c->sf_sd);
            c->sf_cap = 0;
            CHK(dev_alloc(&c->sf_x, (size_t)(kMlpIn * cap)));
            CHK(dev_alloc(&c->sf_y0, (size_t)cap));
            CHK(dev_alloc(&c->sf_key, (size_t)cap));
            CHK(dev_alloc(&c->sf_mean, (size_t)cap));
            CHK(dev_alloc(&c->sf_sd, (size_t)cap));
            c->sf_cap = cap;
        }
        const int r = tril_st_features(c, q_sums, gq, t_sums, gt, k0, n_steps, p, c->sf_x, c->sf_y0,
                                       c->sf_key, c->sf_cap, nrow);
        if (r == TRIL_OK) return TRIL_OK;
        if (r != TRIL_E_OVERFLOW || attempt >= 2) return r;
        cap = pow2_at_least(*nrow + 1);
    }
}

// Two-sided 95% quantile of Student's t with nu degrees of freedom.
double t975(int nu) {
    static const double tab[31] = {0.0,    12.706, 4.303, 3.182, 2.776, 2.571, 2.447, 2.365,
                                   2.306,  2.262,  2.228, 2.201, 2.179, 2.160, 2.145, 2.131,
                                   2.120,  2.110,  2.101, 2.093, 2.086, 2.080, 2.074, 2.069,
                                   2.064,  2.060,  2.056, 2.052, 2.048, 2.045, 2.042};
    if (nu < 1) return 0.0;
    if (nu <= 30) return tab[nu];
    // Cornish-Fisher expansion about the normal quantile (error below 1e-3 from nu = 31)
    const double z = 1.959963984540054, z3 = z * z * z, z5 = z3 * z * z;
    const double v = (double)nu;
    return z + (z3 + z) / (4.0 * v) + (5.0 * z5 + 16.0 * z3 + 3.0 * z) / (96.0 * v * v);
}

// Sampled estimate of the exact total of the candidate rows (key, control per row from y0 and
// the ensemble mean by mode, see tril_st_audit_params), over steps k0 .. k0+n_steps-1.
int st_audit_rows(tril_ctx *c, const tril_beam *t, const int32_t *t_bins, const double *t_sums,
                  const tril_st_grid *gt, const tril_beam *q, const int32_t *q_bins,
                  const double *q_sums, const tril_st_grid *gq, int32_t k0, int32_t n_steps,
                  const long long *key, const double *y0, const float *mean, int64_t nrow,
                  int mode, double eps, double scale, const tril_st_audit_params *ap,
                  tril_st_audit_result *out) {
    const double lambda = (ap && ap->n_sample > 0) ? (double)ap->n_sample : 32768.0;
    const int G = (ap && ap->n_rep > 0) ? ap->n_rep : 8;
    const double mix = (ap && ap->mix > 0.0) ? ap->mix : 0.9;
    const uint64_t seed = ap ? ap->seed : 0ull;
    if (G < 2 || G > 64 || !(mix >= 0.0 && mix < 1.0)) return TRIL_E_INVAL;
    const int64_t nbq = grid_bins(gq), nbt = grid_bins(gt);
    const int64_t ncell = 2 * (nbq + nbt);
    if (ncell > c->au_cell_cap) {
        dev_free(c->au_cell);
        c->au_cell_cap = 0;
        CHK(dev_alloc(&c->au_cell, (size_t)ncell));
        c->au_cell_cap = ncell;
    }
    if (nrow > c->au_ctl_cap) {
        dev_free(c->au_ctl);
        c->au_ctl_cap = 0;
        CHK(dev_alloc(&c->au_ctl, (size_t)std::max<int64_t>(nrow, 1)));
        c->au_ctl_cap = std::max<int64_t>(nrow, 1);
    }
    if (!c->au_count) CHK(dev_alloc(&c->au_count, 2));
    double *pa = c->au_cell, *pb = pa + nbq, *Rq = pb + nbt, *Rt = Rq + nbq;
    // control per row, per cell, in total; total weights of the two beams
    launch_au_zero(pa, nbq + nbt, c->st);
    CHK(clear_slots(c));
    launch_au_control(key, y0, mean, nrow, mode, eps, scale, nbt, c->au_ctl, pa, pb, c->st_slots,
                      c->st);
    HIPCHK(hipGetLastError());
    double c_tot = 0.0, w_q = 0.0, w_t = 0.0;
    CHK(slot_sum(c, &c_tot));
    CHK(clear_slots(c));
    launch_au_weight(q_sums, nbq, c->st_slots, c->st);
    CHK(slot_sum(c, &w_q));
    CHK(clear_slots(c));
    launch_au_weight(t_sums, nbt, c->st_slots, c->st);
    CHK(slot_sum(c, &w_t));
    out->control_total = c_tot;
    out->control_scale = 1.0;
    out->n_bin_pairs = nrow;
    if (!(w_q > 0.0) || !(w_t > 0.0)) {  // an empty beam: nothing collides
        out->n_rep = G;
        return TRIL_OK;
    }
    double cell[3];
    grid_cell(gq, cell);
    const BeamDev qv = view(q, nullptr, 1), tv = view(t, nullptr, 1);
    int64_t cap = std::max<int64_t>(c->au_cap, (int64_t)(lambda + 8.0 * std::sqrt(lambda)) + 1024);
    // one replicate: thin both beams (draw index g), exact pass over the thinned beams (ys),
    // and the thinned beams' estimate of the control total (cs)
    auto replicate = [&](int g, double &ys, double &cs) -> int {
        int64_t n_s[2] = {0, 0};
        for (int attempt = 0;; ++attempt) {
            if (cap > c->au_cap) {
                for (int p = 0; p < 2; ++p) {
                    dev_free(c->au_soa[p]); dev_free(c->au_bin[p]); dev_free(c->au_row[p]);
                    dev_free(c->au_pi[p]);
                }
                c->au_cap = 0;
                for (int p = 0; p < 2; ++p) {
                    CHK(dev_alloc(&c->au_soa[p], (size_t)(8 * cap)));
                    CHK(dev_alloc(&c->au_bin[p], (size_t)cap));
                    CHK(dev_alloc(&c->au_row[p], (size_t)cap));
                    CHK(dev_alloc(&c->au_pi[p], (size_t)cap));
                }
                c->au_cap = cap;
            }
            launch_au_zero(Rq, nbq + nbt, c->st);
            HIPCHK(hipMemsetAsync(c->au_count, 0, 2 * sizeof(unsigned long long), c->st));
            launch_au_sample(qv, q_bins, q_sums, pa, c_tot, w_q, lambda, mix, seed, (uint32_t)g, 0u,
                             c->au_soa[0], c->au_cap, c->au_bin[0], c->au_row[0], c->au_pi[0],
                             c->au_count, Rq, c->st);
            launch_au_sample(tv, t_bins, t_sums, pb, c_tot, w_t, lambda, mix, seed, (uint32_t)g, 1u,
                             c->au_soa[1], c->au_cap, c->au_bin[1], c->au_row[1], c->au_pi[1],
                             c->au_count + 1, Rt, c->st);
            HIPCHK(hipGetLastError());
            unsigned long long h[2] = {0, 0};
            HIPCHK(hipStreamSynchronize(c->st));
            HIPCHK(hipMemcpy(h, c->au_count, sizeof(h), hipMemcpyDeviceToHost));
            n_s[0] = (int64_t)h[0];
            n_s[1] = (int64_t)h[1];
            if (n_s[0] <= c->au_cap && n_s[1] <= c->au_cap) break;
            if (attempt >= 2) return TRIL_E_NOMEM;
            cap = pow2_at_least(std::max(n_s[0], n_s[1]) + (std::max(n_s[0], n_s[1]) >> 2));
        }
        c->au_n[0] = n_s[0];
        c->au_n[1] = n_s[1];
        out->n_sampled[0] += n_s[0];
        out->n_sampled[1] += n_s[1];
        const tril_beam qs = soa_beam(c->au_soa[0], c->au_cap, n_s[0]);
        const tril_beam ts = soa_beam(c->au_soa[1], c->au_cap, n_s[1]);
        int64_t ecap = std::max<int64_t>(c->se_cap, pow2_at_least(8 * (n_s[0] + n_s[1]) + (1 << 16)));
        for (int attempt = 0;; ++attempt) {
            if (ecap > c->se_cap) {
                dev_free(c->se_key);
                dev_free(c->se_val);
                c->se_cap = 0;
                CHK(dev_alloc(&c->se_key, (size_t)ecap));
                CHK(dev_alloc(&c->se_val, (size_t)ecap));
                c->se_cap = ecap;
            }
            HIPCHK(hipMemsetAsync(&c->d_cnt->err, 0, sizeof(unsigned int), c->st));
            CHK(st_run(c, &ts, c->au_bin[1], nbt, &qs, c->au_bin[0], cell, k0, n_steps, 0, nullptr,
                       0, c->se_key, c->se_val, c->se_cap));
            const int r = st_finish(c, &ys);
            if (r == TRIL_OK) break;
            if (r != TRIL_E_OVERFLOW || attempt >= 3) return r;
            ecap = c->se_cap * 4;
        }
        cs = 0.0;
        if (c_tot > 0.0) {
            CHK(clear_slots(c));
            launch_au_ctl_sample(key, c->au_ctl, nrow, nbt, Rq, Rt, q_sums, t_sums, c->st_slots,
                                 c->st);
            HIPCHK(hipGetLastError());
            CHK(slot_sum(c, &cs));
        }
        return TRIL_OK;
    };
    // the control's scale from a pilot replicate with draws of its own (index G): the
    // bin-level yield has no absolute scale, and a network's shared bias shows here; being
    // independent of the replicates below, the scale leaves each of them unbiased
    double kappa = 1.0;
    if (c_tot > 0.0) {
        double ys = 0.0, cs = 0.0;
        CHK(replicate(G, ys, cs));
        if (cs > 0.0) kappa = ys / cs;
    }
    out->control_scale = kappa;
    out->control_total = kappa * c_tot;
    for (int g = 0; g < G; ++g) {
        double ys = 0.0, cs = 0.0;
        CHK(replicate(g, ys, cs));
        out->rep[g] = kappa * c_tot + ys - kappa * cs;
    }
    out->n_rep = G;
    double mean_t = 0.0;
    for (int g = 0; g < G; ++g) mean_t += out->rep[g];
    mean_t /= G;
    double ss = 0.0;
    for (int g = 0; g < G; ++g) ss += (out->rep[g] - mean_t) * (out->rep[g] - mean_t);
    out->estimate = mean_t;
    out->half_width = t975(G - 1) * std::sqrt(ss / (G - 1) / G);
    return TRIL_OK;
}

}  // namespace

extern "C" {

int tril_st_exact(tril_ctx *c, const tril_beam *t, const int32_t *t_bins, int64_t n_t_bins,
                  const tril_beam *q, const int32_t *q_bins, const double cell[3], int32_t k0,
                  int32_t n_steps, tril_st_table *tab, double *total) {
    if (!c || !cell || !tab || !total || k0 < 0 || n_steps < 0) return TRIL_E_INVAL;
    CHK(check_beam(t));
    CHK(check_beam(q));
    if ((t->n > 0 && !t_bins) || (q->n > 0 && !q_bins)) return TRIL_E_INVAL;
    if (n_t_bins < 1 || n_t_bins > INT32_MAX) return TRIL_E_INVAL;
    CHK(check_cell(cell));
    if (tab->cap < 1 || (tab->cap & (tab->cap - 1)) != 0 || !tab->key || !tab->yield)
        return TRIL_E_INVAL;
    if (q->n_inst != t->n_inst) return TRIL_E_STATE;
    if ((int64_t)k0 + n_steps - 1 > INT32_MAX) return TRIL_E_INVAL;
    *total = 0.0;
    CHK(st_run(c, t, t_bins, n_t_bins, q, q_bins, cell, k0, n_steps, 0, nullptr, 0,
               reinterpret_cast<long long *>(tab->key), tab->yield, tab->cap));
    return st_finish(c, total);
}

int tril_st_exact_depleted(tril_ctx *c, const tril_beam *t, const int32_t *t_bins,
                           int64_t n_t_bins, const tril_beam *q, const int32_t *q_bins,
                           const double cell[3], int32_t k0, int32_t n_steps,
                           tril_st_table *pair_tab, tril_st_table *tab, double *total) {
    if (!c || !cell || !tab || !pair_tab || !total || k0 < 0 || n_steps < 0) return TRIL_E_INVAL;
    CHK(check_beam(t));
    CHK(check_beam(q));
    if ((t->n > 0 && !t_bins) || (q->n > 0 && !q_bins)) return TRIL_E_INVAL;
    if (n_t_bins < 1 || n_t_bins > INT32_MAX) return TRIL_E_INVAL;
    CHK(check_cell(cell));
    for (const tril_st_table *tb : {tab, pair_tab})
        if (tb->cap < 1 || (tb->cap & (tb->cap - 1)) != 0 || !tb->key || !tb->yield)
            return TRIL_E_INVAL;
    if (q->n_inst != t->n_inst) return TRIL_E_STATE;
    if ((int64_t)k0 + n_steps - 1 > INT32_MAX) return TRIL_E_INVAL;
    *total = 0.0;
    long long *pkeys = reinterpret_cast<long long *>(pair_tab->key);
    CHK(st_run(c, t, t_bins, n_t_bins, q, q_bins, cell, k0, n_steps, 2, nullptr, 0, pkeys,
               pair_tab->yield, pair_tab->cap));
    long long *keys = reinterpret_cast<long long *>(tab->key);
    launch_st_clear(keys, tab->yield, tab->cap, c->st_slots, c->st);
    const StCell sc{{cell[0], cell[1], cell[2]}};
    launch_st_deplete(pkeys, pair_tab->yield, pair_tab->cap, view(q, c->d_q_off, 1),
                      view(t, c->d_t_off, 1), q_bins, t_bins, n_t_bins, sc, keys, tab->yield,
                      tab->cap, c->st_slots, c->d_cnt, c->st);
    HIPCHK(hipGetLastError());
    return st_finish(c, total);
}

int tril_ip_swarm(tril_ctx *c, const tril_beam *t, const int32_t *t_bins, int64_t n_t_bins,
                  const tril_beam *q, const int32_t *q_bins, const double cell[3], int32_t k0,
                  int32_t n_steps, tril_st_table *pair_tab, tril_st_table *tab, int64_t *total) {
    if (!c || !cell || !tab || !pair_tab || !total || k0 < 0 || n_steps < 0) return TRIL_E_INVAL;
    CHK(check_beam(t));
    CHK(check_beam(q));
    if ((t->n > 0 && !t_bins) || (q->n > 0 && !q_bins)) return TRIL_E_INVAL;
    if (n_t_bins < 1 || n_t_bins > INT32_MAX) return TRIL_E_INVAL;
    CHK(check_cell(cell));
    for (const tril_st_table *tb : {tab, pair_tab})
        if (tb->cap < 1 || (tb->cap & (tb->cap - 1)) != 0 || !tb->key || !tb->yield)
            return TRIL_E_INVAL;
    if (q->n_inst != t->n_inst) return TRIL_E_STATE;
    if ((int64_t)k0 + n_steps - 1 > INT32_MAX) return TRIL_E_INVAL;
    *total = 0;
    if (!c->swarm_total) CHK(dev_alloc(&c->swarm_total, 1));
    long long *pkeys = reinterpret_cast<long long *>(pair_tab->key);
    CHK(st_run(c, t, t_bins, n_t_bins, q, q_bins, cell, k0, n_steps, 3, nullptr, 0, pkeys,
               pair_tab->yield, pair_tab->cap));
    long long *keys = reinterpret_cast<long long *>(tab->key);
    launch_st_clear(keys, tab->yield, tab->cap, c->st_slots, c->st);
    HIPCHK(hipMemsetAsync(c->swarm_total, 0, sizeof(unsigned long long), c->st));
    const StCell sc{{cell[0], cell[1], cell[2]}};
    launch_swarm(pkeys, pair_tab->yield, pair_tab->cap, view(q, c->d_q_off, 1),
                 view(t, c->d_t_off, 1), q_bins, t_bins, n_t_bins, sc, (double)k0 * c->dt,
                 (double)n_steps * c->dt, keys, tab->yield, tab->cap, c->swarm_total, c->d_cnt,
                 c->st);
    HIPCHK(hipGetLastError());
    CHK(st_finish(c, nullptr));
    unsigned long long tot = 0;
    HIPCHK(hipMemcpy(&tot, c->swarm_total, sizeof(tot), hipMemcpyDeviceToHost));
    *total = (int64_t)tot;
    return TRIL_OK;
}

int tril_st_features(tril_ctx *c, const double *q_sums, const tril_st_grid *gq,
                     const double *t_sums, const tril_st_grid *gt, int32_t k0, int32_t n_steps,
                     const tril_st_sur_params *p, float *x, double *y0, int64_t *key, int64_t cap,
                     int64_t *n) {
    if (!c || !q_sums || !t_sums || !n || cap < 0 || (cap > 0 && (!x || !y0 || !key)) || k0 < 0 ||
        n_steps < 0)
        return TRIL_E_INVAL;
    CHK(check_grid(gq));
    CHK(check_grid(gt));
    const double factor = (p && p->cloud_factor > 0.0) ? p->cloud_factor : 3.5;
    if (!(factor >= 1.0) || !std::isfinite(factor)) return TRIL_E_INVAL;
    double cq[3], ct[3];
    grid_cell(gq, cq);
    grid_cell(gt, ct);
    for (int a = 0; a < 3; ++a)
        if (!(std::fabs(cq[a] - ct[a]) <= 1e-12 * cq[a])) return TRIL_E_INVAL;
    *n = 0;
    // bin clouds of both beams
    CHK(st_records(c, q_sums, gq, c->sr_q, c->sr_q_bin, c->sr_q_cap, &c->sr_nq));
    CHK(st_records(c, t_sums, gt, c->sr_t, c->sr_t_bin, c->sr_t_cap, &c->sr_nt));
    const tril_beam bq = record_beam(c->sr_q, c->sr_nq), bt = record_beam(c->sr_t, c->sr_nt);
    const double big[3] = {factor * cq[0], factor * cq[1], factor * cq[2]};
    // geometric overlap of the bin clouds; the table grows until it holds every pair
    const double vol_ratio = factor * factor * factor;
    int64_t tcap = std::max<int64_t>(
        c->sg_cap,
        pow2_at_least((int64_t)(64.0 * vol_ratio) * std::max(c->sr_nq, c->sr_nt) + ((int64_t)1 << 20)));
    for (int attempt = 0;; ++attempt) {
        if (tcap > c->sg_cap) {
            dev_free(c->sg_key);
            dev_free(c->sg_val);
            c->sg_cap = 0;
            CHK(dev_alloc(&c->sg_key, (size_t)tcap));
            CHK(dev_alloc(&c->sg_val, (size_t)tcap));
            c->sg_cap = tcap;
        }
        HIPCHK(hipMemsetAsync(&c->d_cnt->err, 0, sizeof(unsigned int), c->st));
        CHK(st_run(c, &bt, c->sr_t_bin, grid_bins(gt), &bq, c->sr_q_bin, big, k0, n_steps, 1,
                   nullptr, 0, c->sg_key, c->sg_val, c->sg_cap));
        const int r = st_finish(c, nullptr);
        if (r == TRIL_OK) break;
        if (r != TRIL_E_OVERFLOW) return r;
        if (attempt >= 3) return TRIL_E_NOMEM;  // the pair table did not fit the scratch it may take
        tcap = c->sg_cap * 4;
    }
    // one feature row per occupied slot
    unsigned long long *cnt = nullptr;
    CHK(dev_alloc(&cnt, 1));
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(*cnt), c->st);
    const double vol = (cq[0] * cq[1]) * cq[2];
    launch_st_features(c->sg_key, c->sg_val, c->sg_cap, grid_bins(gt), q_sums, t_sums, vol, x, y0,
                       reinterpret_cast<long long *>(key), cap, cnt, c->st);
    unsigned long long h = 0;
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(&h, cnt, sizeof(h), hipMemcpyDeviceToHost);
    dev_free(cnt);
    if (e != hipSuccess) return hip_fail(e);
    *n = (int64_t)h;
    if ((int64_t)h > cap) return TRIL_E_OVERFLOW;
    // rows in ascending key order: threads claimed their slots in no fixed order, and the
    // rows feed training, whose minibatches index them
    const int64_t nr = (int64_t)h;
    if (nr < 2) return TRIL_OK;
    if (nr >= ((int64_t)1 << 32)) return TRIL_E_INVAL;
    const uint64_t max_key = (uint64_t)grid_bins(gq) * (uint64_t)grid_bins(gt) - 1;
    const int key_bits = std::max(1, bits_for(max_key));
    CHK(ensure_sort_scratch(c, nr));
    unsigned long long *ka = nullptr, *kb = nullptr;
    uint32_t *va = nullptr, *vb = nullptr;
    float *xt = nullptr;
    double *yt = nullptr;
    long long *kt = nullptr;
    int rc = TRIL_OK;
    if ((rc = dev_alloc(&ka, (size_t)nr)) == TRIL_OK && (rc = dev_alloc(&kb, (size_t)nr)) == TRIL_OK &&
        (rc = dev_alloc(&va, (size_t)nr)) == TRIL_OK && (rc = dev_alloc(&vb, (size_t)nr)) == TRIL_OK &&
        (rc = dev_alloc(&xt, (size_t)(kMlpIn * nr))) == TRIL_OK &&
        (rc = dev_alloc(&yt, (size_t)nr)) == TRIL_OK && (rc = dev_alloc(&kt, (size_t)nr)) == TRIL_OK) {
        long long *key_ll = reinterpret_cast<long long *>(key);
        launch_st_keys_iota(key_ll, nr, ka, va, c->st);
        const bool alt = radix_sort_u64(ka, va, kb, vb, nr, key_bits, c->ss, &c->d_cnt->err, c->st);
        launch_st_permute_rows(x, y0, key_ll, alt ? vb : va, nr, xt, yt, kt, c->st);
        e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(x, xt, (size_t)(kMlpIn * nr) * sizeof(float), hipMemcpyDeviceToDevice, c->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(y0, yt, (size_t)nr * sizeof(double), hipMemcpyDeviceToDevice, c->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(key_ll, kt, (size_t)nr * sizeof(long long), hipMemcpyDeviceToDevice, c->st);
        if (e == hipSuccess) e = hipStreamSynchronize(c->st);
        if (e != hipSuccess) rc = hip_fail(e);
    }
    dev_free(ka); dev_free(kb); dev_free(va); dev_free(vb);
    dev_free(xt); dev_free(yt); dev_free(kt);
    return rc;
}

int tril_st_targets(const int64_t *key, const double *y0, int64_t n, const tril_st_table *exact,
                    double eps, float *target, double *y_exact, void *stream) {
    if (n < 0 || !exact || !(eps > 0.0) || (n > 0 && (!key || !y0 || !target))) return TRIL_E_INVAL;
    if (exact->cap < 1 || (exact->cap & (exact->cap - 1)) != 0 || !exact->key || !exact->yield)
        return TRIL_E_INVAL;
    launch_st_targets(reinterpret_cast<const long long *>(key), y0, n,
                      reinterpret_cast<const long long *>(exact->key), exact->yield, exact->cap, eps,
                      target, y_exact, reinterpret_cast<hipStream_t>(stream));
    HIPCHK(hipGetLastError());
    return TRIL_OK;
}

int tril_st_surrogate(tril_ctx *c, tril_mlp *mlp, const tril_beam *t, const int32_t *t_bins,
                      const double *t_sums, const tril_st_grid *gt, const tril_beam *q,
                      const int32_t *q_bins, const double *q_sums, const tril_st_grid *gq,
                      int32_t k0, int32_t n_steps, const tril_st_sur_params *p,
                      tril_st_sur_result *out) {
    if (!c || !mlp || !out) return TRIL_E_INVAL;
    CHK(check_beam(t));
    CHK(check_beam(q));
    if ((t->n > 0 && !t_bins) || (q->n > 0 && !q_bins)) return TRIL_E_INVAL;
    if (q->n_inst != 1 || t->n_inst != 1) return TRIL_E_NOTIMPL;
    const double eps = (p && p->eps > 0.0) ? p->eps : 1e-3;
    const double gate = (p && p->gate > 0.0) ? p->gate : 0.01;
    const double scale = (p && p->scale > 0.0) ? p->scale : 1.0;
    if (p && (p->gate_mode < 0 || p->gate_mode > 2)) return TRIL_E_INVAL;
    std::memset(out, 0, sizeof(*out));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, c->st));
    // features of every candidate bin pair
    int64_t nrow = 0;
    CHK(sur_features(c, q_sums, gq, t_sums, gt, k0, n_steps, p, &nrow));
    out->n_bin_pairs = nrow;
    // ensemble prediction on the same stream
    if (mlp->m.st != c->st) HIPCHK(hipStreamSynchronize(c->st));
    CHK(tril_mlp_predict(mlp, c->sf_x, nrow, c->sf_mean, c->sf_sd));
    if (mlp->m.st != c->st) HIPCHK(hipStreamSynchronize(mlp->m.st));
    if (p && p->gate_mode == 2) {
        // audit: the predictions are the control of a sampled estimate of the exact total
        tril_st_audit_params ap{};
        ap.n_sample = p->audit_sample;
        ap.n_rep = p->audit_reps;
        ap.control = 0;
        ap.seed = p->audit_seed;
        ap.mix = 0.0;
        tril_st_audit_result ar;
        std::memset(&ar, 0, sizeof(ar));
        const int r = st_audit_rows(c, t, t_bins, t_sums, gt, q, q_bins, q_sums, gq, k0, n_steps,
                                    reinterpret_cast<const long long *>(c->sf_key), c->sf_y0,
                                    c->sf_mean, nrow, 0, eps, scale, &ap, &ar);
        if (r != TRIL_OK) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return r;
        }
        // the network's own total, and the audit's correction of it
        out->surrogate_part = ar.control_scale > 0.0 ? ar.control_total / ar.control_scale : 0.0;
        out->exact_part = ar.estimate - out->surrogate_part;
        out->total = ar.estimate;
        out->audit_half_width = ar.half_width;
        out->audit_sampled = ar.n_sampled[0] + ar.n_sampled[1];
        out->predicted_spread = ar.estimate > 0.0 ? ar.half_width / ar.estimate : 0.0;
        float ms = 0.f;
        if (hipEventRecord(e1, c->st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            out->ms = ms;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return TRIL_OK;
    }
    // gate: surrogate yields for confident rows; the rest to an exact pass
    const int64_t nbq = grid_bins(gq), nbt = grid_bins(gt);
    const int64_t fcap = pow2_at_least(2 * nrow + 16);
    long long *filter = nullptr;
    uint8_t *qmark = nullptr, *tmark = nullptr;
    int32_t *qb2 = nullptr, *tb2 = nullptr;
    unsigned long long *nflag = nullptr;
    int rc = TRIL_OK;
    auto cleanup = [&]() {
        dev_free(filter); dev_free(qmark); dev_free(tmark); dev_free(qb2); dev_free(tb2);
        dev_free(nflag);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    };
    if ((rc = dev_alloc(&filter, (size_t)fcap)) || (rc = dev_alloc(&qmark, (size_t)nbq)) ||
        (rc = dev_alloc(&tmark, (size_t)nbt)) || (rc = dev_alloc(&qb2, (size_t)std::max<int64_t>(q->n, 1))) ||
        (rc = dev_alloc(&tb2, (size_t)std::max<int64_t>(t->n, 1))) || (rc = dev_alloc(&nflag, 1))) {
        cleanup();
        return rc;
    }
    launch_fill_keys(filter, fcap, c->st);
    hipError_t he = hipMemsetAsync(qmark, 0, (size_t)nbq, c->st);
    if (he == hipSuccess) he = hipMemsetAsync(tmark, 0, (size_t)nbt, c->st);
    if (he == hipSuccess) he = hipMemsetAsync(nflag, 0, sizeof(*nflag), c->st);
    if (he == hipSuccess) he = hipMemsetAsync(c->st_slots, 0, kCounterSlots * sizeof(double), c->st);
    if (he != hipSuccess) {
        cleanup();
        return hip_fail(he);
    }
    int cut = -1;  // per-pair mode
    if (!(p && p->gate_mode == 1)) {
        // budget mode: pairs with the largest uncertainty contributions go exact until the
        // remaining ensemble spread of the total is within gate x the predicted total
        double *hist = nullptr;
        if ((rc = dev_alloc(&hist, kUncBuckets)) != TRIL_OK) {
            cleanup();
            return rc;
        }
        he = hipMemsetAsync(hist, 0, kUncBuckets * sizeof(double), c->st);
        if (he == hipSuccess)
            launch_st_unc(c->sf_y0, c->sf_mean, c->sf_sd, nrow, eps, scale, hist, c->st_slots, c->st);
        std::vector<double> h((size_t)kUncBuckets);
        double pred_total = 0.0;
        if (he == hipSuccess) he = hipGetLastError();
        if (he == hipSuccess) he = hipStreamSynchronize(c->st);
        if (he == hipSuccess) he = hipMemcpy(h.data(), hist, kUncBuckets * sizeof(double), hipMemcpyDeviceToHost);
        if (he == hipSuccess) {
            double sl[kCounterSlots];
            he = hipMemcpy(sl, c->st_slots, sizeof(sl), hipMemcpyDeviceToHost);
            for (double v : sl) pred_total += v;
        }
        dev_free(hist);
        if (he == hipSuccess) he = hipMemsetAsync(c->st_slots, 0, kCounterSlots * sizeof(double), c->st);
        if (he != hipSuccess) {
            cleanup();
            return hip_fail(he);
        }
        const double budget = (gate * pred_total) * (gate * pred_total);
        double acc = 0.0;
        cut = kUncBuckets - 1;
        for (int b = 0; b < kUncBuckets; ++b) {
            if (acc + h[(size_t)b] > budget) {
                cut = b - 1;
                break;
            }
            acc += h[(size_t)b];
        }
        if (cut < 0) cut = 0;
        out->predicted_spread = pred_total > 0.0 ? std::sqrt(acc) / pred_total : 0.0;
    }
    launch_st_gate(reinterpret_cast<const long long *>(c->sf_key), c->sf_y0, c->sf_mean, c->sf_sd,
                   nrow, eps, gate, scale, cut, nbt, filter, fcap, qmark, tmark, c->st_slots, nflag,
                   &c->d_cnt->err, c->st);
    double sur = 0.0;
    if ((rc = st_finish(c, &sur)) != TRIL_OK) {
        cleanup();
        return rc;
    }
    unsigned long long hf = 0;
    if ((he = hipMemcpy(&hf, nflag, sizeof(hf), hipMemcpyDeviceToHost)) != hipSuccess) {
        cleanup();
        return hip_fail(he);
    }
    out->surrogate_part = sur;
    out->n_gated = (int64_t)hf;
    double exact = 0.0;
    if (hf > 0) {
        launch_st_mask_bins(q_bins, q->n, qmark, qb2, c->st);
        launch_st_mask_bins(t_bins, t->n, tmark, tb2, c->st);
        double cell[3];
        grid_cell(gq, cell);
        const int64_t ecap = pow2_at_least(4 * (int64_t)hf + 1024);
        if (ecap > c->se_cap) {
            dev_free(c->se_key);
            dev_free(c->se_val);
            c->se_cap = 0;
            if ((rc = dev_alloc(&c->se_key, (size_t)ecap)) || (rc = dev_alloc(&c->se_val, (size_t)ecap))) {
                cleanup();
                return rc;
            }
            c->se_cap = ecap;
        }
        if ((rc = st_run(c, t, tb2, nbt, q, qb2, cell, k0, n_steps, 0, filter, fcap, c->se_key,
                         c->se_val, c->se_cap)) != TRIL_OK ||
            (rc = st_finish(c, &exact)) != TRIL_OK) {
            cleanup();
            return rc;
        }
    }
    out->exact_part = exact;
    out->total = sur + exact;
    float ms = 0.f;
    if (hipEventRecord(e1, c->st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
        hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
        out->ms = ms;
    cleanup();
    return TRIL_OK;
}

// ------------------------------------------------------------ surrogate network

int tril_st_audit(tril_ctx *c, tril_mlp *mlp, const tril_beam *t, const int32_t *t_bins,
                  const double *t_sums, const tril_st_grid *gt, const tril_beam *q,
                  const int32_t *q_bins, const double *q_sums, const tril_st_grid *gq, int32_t k0,
                  int32_t n_steps, const tril_st_sur_params *sp, const tril_st_audit_params *ap,
                  tril_st_audit_result *out) {
    if (!c || !out || !ap || !t_sums || !q_sums || k0 < 0 || n_steps < 0) return TRIL_E_INVAL;
    CHK(check_beam(t));
    CHK(check_beam(q));
    CHK(check_grid(gq));
    CHK(check_grid(gt));
    if ((t->n > 0 && !t_bins) || (q->n > 0 && !q_bins)) return TRIL_E_INVAL;
    if (q->n_inst != 1 || t->n_inst != 1) return TRIL_E_NOTIMPL;
    if (ap->control < 0 || ap->control > 2 || (ap->control == 0 && !mlp)) return TRIL_E_INVAL;
    const double eps = (sp && sp->eps > 0.0) ? sp->eps : 1e-3;
    const double scale = (sp && sp->scale > 0.0) ? sp->scale : 1.0;
    std::memset(out, 0, sizeof(*out));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int rc = TRIL_OK;
    int64_t nrow = 0;
    if (hipEventRecord(e0, c->st) != hipSuccess) rc = TRIL_E_HIP;
    if (rc == TRIL_OK) rc = sur_features(c, q_sums, gq, t_sums, gt, k0, n_steps, sp, &nrow);
    if (rc == TRIL_OK && ap->control == 0) {
        if (mlp->m.st != c->st && hipStreamSynchronize(c->st) != hipSuccess) rc = TRIL_E_HIP;
        if (rc == TRIL_OK) rc = tril_mlp_predict(mlp, c->sf_x, nrow, c->sf_mean, c->sf_sd);
        if (rc == TRIL_OK && mlp->m.st != c->st && hipStreamSynchronize(mlp->m.st) != hipSuccess)
            rc = TRIL_E_HIP;
    }
    if (rc == TRIL_OK)
        rc = st_audit_rows(c, t, t_bins, t_sums, gt, q, q_bins, q_sums, gq, k0, n_steps,
                           reinterpret_cast<const long long *>(c->sf_key), c->sf_y0,
                           ap->control == 0 ? c->sf_mean : nullptr, nrow, ap->control, eps, scale,
                           ap, out);
    float ms = 0.f;
    if (rc == TRIL_OK && hipEventRecord(e1, c->st) == hipSuccess &&
        hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
        out->ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int tril_st_calibrate(tril_mlp *mlp, const float *x, const double *y0, const double *y_exact,
                      int64_t n, double eps, double *scale) {
    if (!mlp || !scale || n < 0 || !(eps > 0.0) || (n > 0 && (!x || !y0 || !y_exact)))
        return TRIL_E_INVAL;
    *scale = 1.0;
    if (n == 0) return TRIL_OK;
    const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
    float *mean = nullptr, *sd = nullptr;
    double *part = nullptr;
    int rc = TRIL_OK;
    if ((rc = dev_alloc(&mean, (size_t)n)) == TRIL_OK && (rc = dev_alloc(&sd, (size_t)n)) == TRIL_OK &&
        (rc = dev_alloc(&part, (size_t)(2 * blocks))) == TRIL_OK)
        rc = tril_mlp_predict(mlp, x, n, mean, sd);
    std::vector<double> h((size_t)(2 * blocks), 0.0);
    if (rc == TRIL_OK) {
        launch_au_calib(y0, mean, y_exact, n, eps, part, blocks, mlp->m.st);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(mlp->m.st);
        if (e == hipSuccess)
            e = hipMemcpy(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = hip_fail(e);
    }
    dev_free(mean);
    dev_free(sd);
    dev_free(part);
    if (rc != TRIL_OK) return rc;
    double se = 0.0, sp = 0.0;
    for (int b = 0; b < blocks; ++b) {
        se += h[(size_t)(2 * b)];
        sp += h[(size_t)(2 * b + 1)];
    }
    if (!(sp > 0.0)) return TRIL_E_INVAL;  // nothing predicted: no ratio
    *scale = se / sp;
    return TRIL_OK;
}

int tril_mlp_create(tril_mlp **out, int32_t n_members, uint64_t seed, void *stream) {
    if (!out || n_members < 1 || n_members > 64) return TRIL_E_INVAL;
    *out = nullptr;
    tril_mlp *p = new tril_mlp();
    const int r = mlp_init(&p->m, n_members, seed, reinterpret_cast<hipStream_t>(stream));
    if (r != TRIL_OK) {
        delete p;
        return r;
    }
    *out = p;
    return TRIL_OK;
}

void tril_mlp_destroy(tril_mlp *p) {
    if (!p) return;
    (void)hipStreamSynchronize(p->m.st);
    delete p;
}

int tril_mlp_set_params(tril_mlp *p, int32_t member, const float *host, int64_t n) {
    if (!p || !host || member < 0 || member >= p->m.K || n != kMlpParams) return TRIL_E_INVAL;
    HIPCHK(hipStreamSynchronize(p->m.st));
    HIPCHK(hipMemcpy(p->m.w + (int64_t)member * kMlpParams, host, kMlpParams * sizeof(float),
                     hipMemcpyHostToDevice));
    mlp_cast(&p->m);
    HIPCHK(hipGetLastError());
    return TRIL_OK;
}

int tril_mlp_get_params(tril_mlp *p, int32_t member, float *host, int64_t n) {
    if (!p || !host || member < 0 || member >= p->m.K || n != kMlpParams) return TRIL_E_INVAL;
    HIPCHK(hipStreamSynchronize(p->m.st));
    HIPCHK(hipMemcpy(host, p->m.w + (int64_t)member * kMlpParams, kMlpParams * sizeof(float),
                     hipMemcpyDeviceToHost));
    return TRIL_OK;
}

int tril_mlp_set_norm(tril_mlp *p, const float *mu_x, const float *sd_x, float mu_y, float sd_y) {
    if (!p || !mu_x || !sd_x || !std::isfinite(mu_y) || !(sd_y > 0.0f) || !std::isfinite(sd_y))
        return TRIL_E_INVAL;
    float h[2 * kMlpIn];
    for (int c = 0; c < kMlpIn; ++c) {
        if (!std::isfinite(mu_x[c]) || !(sd_x[c] > 0.0f) || !std::isfinite(sd_x[c])) return TRIL_E_INVAL;
        h[c] = mu_x[c];
        h[kMlpIn + c] = sd_x[c];
    }
    HIPCHK(hipStreamSynchronize(p->m.st));
    HIPCHK(hipMemcpy(p->m.norm, h, sizeof(h), hipMemcpyHostToDevice));
    p->m.mu_y = mu_y;
    p->m.sd_y = sd_y;
    return TRIL_OK;
}

int tril_mlp_fit_norm(tril_mlp *p, const float *x, const float *y, int64_t n) {
    if (!p || !x || !y || n < 2) return TRIL_E_INVAL;
    double *mom = nullptr, *part = nullptr;
    CHK(dev_alloc(&mom, 2 * (kMlpIn + 1)));
    if (dev_alloc(&part, (size_t)(2 * (kMlpIn + 1) * kMomentSlices)) != TRIL_OK) {
        dev_free(mom);
        return TRIL_E_NOMEM;
    }
    mlp_moments(x, n, kMlpIn, mom, part, p->m.st);
    mlp_moments(y, n, 1, mom + 2 * kMlpIn, part + 2 * kMlpIn * kMomentSlices, p->m.st);
    double h[2 * (kMlpIn + 1)];
    hipError_t e = hipStreamSynchronize(p->m.st);
    if (e == hipSuccess) e = hipMemcpy(h, mom, sizeof(h), hipMemcpyDeviceToHost);
    dev_free(mom);
    dev_free(part);
    if (e != hipSuccess) return hip_fail(e);
    float mu[kMlpIn], sd[kMlpIn];
    for (int c = 0; c <= kMlpIn; ++c) {
        const double m1 = h[2 * c] / n;
        const double var = std::max(h[2 * c + 1] / n - m1 * m1, 0.0);
        const double sdv = var > 1e-30 ? std::sqrt(var) : 1.0;
        if (c < kMlpIn) {
            mu[c] = (float)m1;
            sd[c] = (float)sdv;
        } else {
            return tril_mlp_set_norm(p, mu, sd, (float)m1, (float)sdv);
        }
    }
    return TRIL_OK;
}

int tril_mlp_grad(tril_mlp *p, int32_t member, const float *x, const float *y, int64_t n,
                  float *host_grad, double *host_loss) {
    if (!p || !x || !y || !host_grad || !host_loss || member < 0 || member >= p->m.K || n < 1 ||
        n > INT32_MAX)
        return TRIL_E_INVAL;
    MlpModel &m = p->m;
    CHK(mlp_scratch(&m, n));
    HIPCHK(hipMemsetAsync(m.loss, 0, sizeof(float), m.st));
    mlp_input(&m, x, nullptr, n);
    mlp_forward(&m, member, n, m.yhat);
    mlp_loss(&m, y, nullptr, n);
    mlp_backward(&m, member, n);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(m.st));
    HIPCHK(hipMemcpy(host_grad, m.g, kMlpParams * sizeof(float), hipMemcpyDeviceToHost));
    float l = 0.f;
    HIPCHK(hipMemcpy(&l, m.loss, sizeof(float), hipMemcpyDeviceToHost));
    *host_loss = (double)l / (double)n;
    return TRIL_OK;
}

int tril_mlp_train(tril_mlp *p, const float *x, const float *y, int64_t n, int32_t n_steps,
                   int32_t batch, float lr, uint64_t seed, double *host_loss) {
    if (!p || !x || !y || n < 1 || n > INT32_MAX || n_steps < 0 || batch < 1 || !(lr > 0.0f))
        return TRIL_E_INVAL;
    MlpModel &m = p->m;
    CHK(mlp_scratch(&m, batch));
    const int32_t tail = std::max(1, n_steps / 10);
    std::vector<double> acc((size_t)m.K, 0.0);
    for (int k = 0; k < m.K; ++k) {
        HIPCHK(hipMemsetAsync(m.loss, 0, sizeof(float), m.st));
        for (int32_t s = 0; s < n_steps; ++s) {
            mlp_batch_idx(&m, seed, k, m.adam_t + s, n, batch);
            mlp_input(&m, x, m.idx, batch);
            mlp_forward(&m, k, batch, m.yhat);
            if (s == n_steps - tail) HIPCHK(hipMemsetAsync(m.loss, 0, sizeof(float), m.st));
            mlp_loss(&m, y, m.idx, batch);
            mlp_backward(&m, k, batch);
            mlp_adam(&m, k, lr, m.adam_t + s + 1);
        }
        HIPCHK(hipGetLastError());
        if (host_loss && n_steps > 0) {
            float l = 0.f;
            HIPCHK(hipStreamSynchronize(m.st));
            HIPCHK(hipMemcpy(&l, m.loss, sizeof(float), hipMemcpyDeviceToHost));
            acc[(size_t)k] = (double)l / ((double)tail * batch);
        }
    }
    m.adam_t += n_steps;
    HIPCHK(hipStreamSynchronize(m.st));
    if (host_loss)
        for (int k = 0; k < m.K; ++k) host_loss[k] = acc[(size_t)k];
    return TRIL_OK;
}

int tril_mlp_predict(tril_mlp *p, const float *x, int64_t n, float *mean, float *sdev) {
    if (!p || n < 0 || (n > 0 && (!x || !mean || !sdev))) return TRIL_E_INVAL;
    if (n == 0) return TRIL_OK;
    MlpModel &m = p->m;
    const int64_t chunk = std::min<int64_t>(n, (int64_t)1 << 20);
    float *outs = nullptr;
    CHK(dev_alloc(&outs, (size_t)(m.K * chunk)));
    mlp_pack_inference(&m);
    for (int64_t a = 0; a < n; a += chunk) {
        const int64_t c = std::min(chunk, n - a);
        for (int k = 0; k < m.K; ++k) mlp_fused_forward(&m, k, x + a * kMlpIn, c, outs + (int64_t)k * c);
        mlp_reduce(&m, outs, c, mean + a, sdev + a);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(m.st);
    dev_free(outs);
    if (e != hipSuccess) return hip_fail(e);
    return TRIL_OK;
}

int tril_dbg_gemm_bf16(const uint16_t *A, int64_t sam, int64_t sak, const uint16_t *B, int64_t sbk,
                       int64_t sbn, int32_t M, int32_t N, int32_t K, float *C, void *stream) {
    if (!A || !B || !C || M < 1 || N < 1 || K < 0) return TRIL_E_INVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    mlp_gemm(A, sam, sak, B, sbk, sbn, M, N, K, 0, nullptr, nullptr, C, nullptr, nullptr, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return TRIL_OK;
}

int tril_set_tune(tril_ctx *c, const tril_tune *tu) {
    if (!c || !tu) return TRIL_E_INVAL;
    const int blk = tu->block_traverse;
    if (blk != 64 && blk != 128 && blk != 256 && blk != 512) return TRIL_E_INVAL;
    if (tu->step_batch < 0) return TRIL_E_INVAL;
    if (tu->morton_bits != 0 && (tu->morton_bits < 3 || tu->morton_bits > 30)) return TRIL_E_INVAL;
    if (tu->traverse_queue != 0 && tu->traverse_queue != 1) return TRIL_E_INVAL;
    if (tu->kinetic_window < 0) return TRIL_E_INVAL;
    if (tu->descent_window < 0 || tu->descent_window > kMaxDescent) return TRIL_E_INVAL;
    c->block = blk;
    c->trav_queue = tu->traverse_queue;
    c->kwin = tu->kinetic_window;
    c->kdesc = tu->descent_window;
    c->step_batch = tu->step_batch;
    c->morton_param = tu->morton_bits;
    return TRIL_OK;
}

int tril_autotune(tril_ctx *c, const tril_beam *t, const tril_beam *q, int32_t k0, int32_t n_probe,
                  tril_tune *best) {
    if (!c || !best || k0 < 0 || n_probe < 1) return TRIL_E_INVAL;
    CHK(check_beam(t));
    CHK(check_beam(q));
    if (q->n_inst != t->n_inst) return TRIL_E_STATE;
    if ((int64_t)k0 + n_probe - 1 > INT32_MAX) return TRIL_E_INVAL;
    const int64_t cap = (int64_t)1 << 22;
    tril_pairs pr{cap, nullptr, nullptr, nullptr, nullptr};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const uint32_t save_flags = c->flags;
    int rc = TRIL_OK;
    auto cleanup = [&]() {
        dev_free(pr.i); dev_free(pr.j); dev_free(pr.step); dev_free(pr.count);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        c->flags = save_flags;
    };
    if ((rc = dev_alloc(&pr.i, cap)) != TRIL_OK || (rc = dev_alloc(&pr.j, cap)) != TRIL_OK ||
        (rc = dev_alloc(&pr.step, cap)) != TRIL_OK || (rc = dev_alloc(&pr.count, 1)) != TRIL_OK) {
        cleanup();
        return rc;
    }
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        cleanup();
        return hip_fail(he);
    }
    c->flags &= ~TRIL_TIMING;  // time graph replays, as a run without per-phase events
    const int64_t rows = std::max<int64_t>(std::max(t->n, q->n), 1);
    int cur_queue = 0, cur_win = 0, cur_desc = 0;
    auto probe = [&](int blk, int sb, int mb, double &ms) -> int {
        c->block = blk;
        c->step_batch = sb;
        c->morton_param = mb;
        c->trav_queue = cur_queue;
        c->kwin = cur_win;
        c->kdesc = cur_desc;
        for (int rep = 0; rep < 2; ++rep) {
            HIPCHK(hipMemsetAsync(pr.count, 0, sizeof(int64_t), c->st));
            HIPCHK(hipEventRecord(e0, c->st));
            CHK(tril_run(c, t, q, k0, n_probe, &pr));
            HIPCHK(hipEventRecord(e1, c->st));
        }
        HIPCHK(hipEventSynchronize(e1));
        float f = 0.f;
        HIPCHK(hipEventElapsedTime(&f, e0, e1));
        ms = (double)f / n_probe;
        return TRIL_OK;
    };
    tril_tune cur{64, 0, 0, 0, 0, 0, 0.0};
    cur.step_batch = pick_batch(c, t, q, n_probe);
    cur_queue = 0;
    double best_ms = 0.0;
    if ((rc = probe(cur.block_traverse, cur.step_batch, cur.morton_bits, best_ms)) != TRIL_OK) {
        cleanup();
        return rc;
    }
    for (int sb : {1, 2, 4, 8, 16, 32, 64, 128}) {
        const int64_t lim = std::max<int64_t>((int64_t)1 << 27,
                                              std::min(kBatchBudgetMax, kBatchStepsMin * rows));
        if (sb == cur.step_batch || sb > n_probe || (int64_t)sb * rows > lim) continue;
        double ms = 0.0;
        if ((rc = probe(cur.block_traverse, sb, cur.morton_bits, ms)) != TRIL_OK) break;
        if (ms < best_ms) {
            best_ms = ms;
            cur.step_batch = sb;
        }
    }
    for (int w : {1, 4, 8, 16}) {  // steps per tree copy (0: the default, 32)
        if (rc != TRIL_OK || cur.step_batch == 1) break;
        double ms = 0.0;
        cur_win = w;
        if ((rc = probe(cur.block_traverse, cur.step_batch, cur.morton_bits, ms)) != TRIL_OK) break;
        if (ms < best_ms) {
            best_ms = ms;
            cur.kinetic_window = w;
        }
        cur_win = cur.kinetic_window;
    }
    for (int d : {4, 16, 32}) {  // steps per four-child descent (0: the default, 8)
        if (rc != TRIL_OK || cur.step_batch == 1 || cur.kinetic_window == 1) break;
        double ms = 0.0;
        cur_desc = d;
        if ((rc = probe(cur.block_traverse, cur.step_batch, cur.morton_bits, ms)) != TRIL_OK) break;
        if (ms < best_ms) {
            best_ms = ms;
            cur.descent_window = d;
        }
        cur_desc = cur.descent_window;
    }
    for (int blk : {64, 128, 512}) {
        if (rc != TRIL_OK) break;
        double ms = 0.0;
        if ((rc = probe(blk, cur.step_batch, cur.morton_bits, ms)) != TRIL_OK) break;
        if (ms < best_ms) {
            best_ms = ms;
            cur.block_traverse = blk;
        }
    }
    if (rc == TRIL_OK) {
        double ms = 0.0;
        if ((rc = probe(cur.block_traverse, cur.step_batch, 30, ms)) == TRIL_OK && ms < best_ms) {
            best_ms = ms;
            cur.morton_bits = 30;
        }
    }
    if (rc == TRIL_OK) {  // the persistent work-queue traversal against the flat grid
        double ms = 0.0;
        cur_queue = 1;
        if ((rc = probe(cur.block_traverse, cur.step_batch, cur.morton_bits, ms)) == TRIL_OK &&
            ms < best_ms) {
            best_ms = ms;
            cur.traverse_queue = 1;
        }
        cur_queue = cur.traverse_queue;
    }
    cleanup();
    if (rc != TRIL_OK) return rc;
    cur.ms_per_step = best_ms;
    c->block = cur.block_traverse;
    c->step_batch = cur.step_batch;
    c->morton_param = cur.morton_bits;
    c->trav_queue = cur.traverse_queue;
    c->kwin = cur.kinetic_window;
    c->kdesc = cur.descent_window;
    *best = cur;
    return tril_reset_counters(c);
}

int tril_reset_counters(tril_ctx *c) {
    if (!c) return TRIL_E_INVAL;
    HIPCHK(hipStreamSynchronize(c->st));
    HIPCHK(hipMemcpy(c->h_cnt, c->d_cnt, sizeof(DevCounters), hipMemcpyDeviceToHost));
    // a launch stopped by a device error may have left refit arrival flags set
    if (c->h_cnt->err != 0u && c->nflags != nullptr)
        HIPCHK(hipMemset(c->nflags, 0, (size_t)c->t_cap * sizeof(int32_t)));
    std::memset(c->h_cnt, 0, sizeof(DevCounters));
    HIPCHK(hipMemcpy(c->d_cnt, c->h_cnt, sizeof(DevCounters), hipMemcpyHostToDevice));
    c->ev_build.clear(); c->ev_prep.clear(); c->ev_trav.clear(); c->ev_narrow.clear();
    c->ev_next = 0;
    for (double &m : c->ms_acc) m = 0.0;
    c->timed_launches = 0;
    c->max_step = c->built ? c->built_step : -1;
    c->ad_checks0 = c->ad_queries0 = 0;
    c->ad_quad = false;
    return TRIL_OK;
}

void tril_destroy(tril_ctx *c) {
    if (!c) return;
    if (c->st) (void)hipStreamSynchronize(c->st);
    if (c->gst) (void)hipStreamSynchronize(c->gst);
    if (c->qst) (void)hipStreamSynchronize(c->qst);
    for (hipGraphExec_t &g : c->gexec)
        if (g) (void)hipGraphExecDestroy(g);
    free_target(c);
    free_target_rows(c);
    free_annihilation(c);
    dev_free(c->dead_q);
    dev_free(c->dead_t);
    dev_free(c->ann_count);
    dev_free(c->kin_buf);
    dev_free(c->kin_rec);
    dev_free(c->swarm_total);
    dev_free(c->grid_dev);
    dev_free(c->grid_start);
    dev_free(c->grid_end);
    dev_free(c->kin_err);
    for (hipEvent_t e : c->ev_kin)
        if (e) (void)hipEventDestroy(e);
    for (int p = 0; p < 2; ++p) {
        free_work(c->wt[p]);
        free_work(c->wq[p]);
    }
    dev_free(c->st_slots);
    free_work(c->sr_q); free_work(c->sr_t);
    dev_free(c->sr_q_bin); dev_free(c->sr_t_bin);
    dev_free(c->sg_key); dev_free(c->sg_val);
    dev_free(c->sf_x); dev_free(c->sf_mean); dev_free(c->sf_sd); dev_free(c->sf_y0);
    dev_free(c->sf_key); dev_free(c->se_key); dev_free(c->se_val);
    for (int p = 0; p < 2; ++p) {
        dev_free(c->au_soa[p]); dev_free(c->au_bin[p]); dev_free(c->au_row[p]);
        dev_free(c->au_pi[p]);
    }
    dev_free(c->au_cell); dev_free(c->au_ctl); dev_free(c->au_count);
    dev_free(c->d_t_off); dev_free(c->t_stats); dev_free(c->t_wb); dev_free(c->inst_root); dev_free(c->inst_base); dev_free(c->root_box);
    dev_free(c->nodes4); dev_free(c->t_frames); dev_free(c->t_inside);
    dev_free(c->q_box); dev_free(c->q_spart); dev_free(c->q_k32a); dev_free(c->q_k32b);
    dev_free(c->q_k64a); dev_free(c->q_k64b); dev_free(c->q_va); dev_free(c->q_vb);
    dev_free(c->q_keep); dev_free(c->q_rec); dev_free(c->d_q_off); dev_free(c->q_stats); dev_free(c->cand_i);
    dev_free(c->cand_j);
    dev_free(c->ss.hist); dev_free(c->ss.tile_ctr); dev_free(c->ss.status);
    dev_free(c->ssq.hist); dev_free(c->ssq.tile_ctr); dev_free(c->ssq.status);
    StatsScratch &s = c->sst;
    dev_free(s.keys); dev_free(s.keys_alt); dev_free(s.vals); dev_free(s.vals_alt);
    dev_free(s.flags); dev_free(s.pos); dev_free(s.block_sums); dev_free(s.ti); dev_free(s.tj);
    dev_free(s.tk); dev_free(s.acc); dev_free(s.ucount); dev_free(s.step_counts);
    dev_free(c->d_edges);
    dev_free(c->d_cnt);
    if (c->h_cnt) (void)hipHostFree(c->h_cnt);
    if (c->h_pin) (void)hipHostFree(c->h_pin);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->ev_join_a) (void)hipEventDestroy(c->ev_join_a);
    if (c->ev_join_b) (void)hipEventDestroy(c->ev_join_b);
    if (c->gst) (void)hipStreamDestroy(c->gst);
    if (c->ev_qfork) (void)hipEventDestroy(c->ev_qfork);
    if (c->ev_qjoin) (void)hipEventDestroy(c->ev_qjoin);
    if (c->ev_tfork) (void)hipEventDestroy(c->ev_tfork);
    if (c->ev_tjoin) (void)hipEventDestroy(c->ev_tjoin);
    if (c->qst) (void)hipStreamDestroy(c->qst);
    delete c;
}

}  // extern "C"

// ------------------------------------------------------------- inspection ABI

namespace {
template <typename K, typename Sorter>
int dbg_sort(K *keys, uint32_t *vals, int64_t n, hipStream_t st, Sorter sorter) {
    SortScratch ss;
    K *ka = nullptr;
    uint32_t *va = nullptr;
    unsigned int *err = nullptr;
    int r = TRIL_OK;
    if ((r = dev_alloc(&ss.hist, 8 * 256)) == TRIL_OK && (r = dev_alloc(&ss.tile_ctr, 8)) == TRIL_OK &&
        (r = dev_alloc(&ss.status, sort_status_words(n, 8))) == TRIL_OK &&
        (r = dev_alloc(&ka, (size_t)n)) == TRIL_OK && (r = dev_alloc(&va, (size_t)n)) == TRIL_OK &&
        (r = dev_alloc(&err, 1)) == TRIL_OK) {
        hipError_t e = hipMemsetAsync(err, 0, sizeof(unsigned int), st);
        if (e == hipSuccess) {
            const bool alt = sorter(keys, vals, ka, va, ss, err);
            if (alt) {
                e = hipMemcpyAsync(keys, ka, n * sizeof(K), hipMemcpyDeviceToDevice, st);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
            }
        }
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        unsigned int h_err = 0;
        if (e == hipSuccess) e = hipMemcpy(&h_err, err, sizeof(h_err), hipMemcpyDeviceToHost);
        r = e != hipSuccess ? hip_fail(e) : (h_err ? TRIL_E_INTERNAL : TRIL_OK);
    }
    dev_free(ss.hist); dev_free(ss.tile_ctr); dev_free(ss.status);
    dev_free(ka); dev_free(va); dev_free(err);
    return r;
}
}  // namespace

extern "C" {

int tril_dbg_sort_u32(uint32_t *keys, uint32_t *vals, int64_t n, int key_bits, void *stream) {
    if (n < 0 || n >= kMaxN || key_bits < 1 || key_bits > 32) return TRIL_E_INVAL;
    if (n > 0 && (!keys || !vals)) return TRIL_E_INVAL;
    if (n <= 1) return TRIL_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return dbg_sort(keys, vals, n, st,
                    [&](uint32_t *k, uint32_t *v, uint32_t *ka, uint32_t *va, SortScratch &ss,
                        unsigned int *err) {
                        return radix_sort_u32(k, v, ka, va, n, key_bits, ss, err, st);
                    });
}

int tril_dbg_sort_u64(uint64_t *keys, uint32_t *vals, int64_t n, int key_bits, void *stream) {
    if (n < 0 || n >= kMaxN || key_bits < 1 || key_bits > 64) return TRIL_E_INVAL;
    if (n > 0 && (!keys || !vals)) return TRIL_E_INVAL;
    if (n <= 1) return TRIL_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    unsigned long long *k64 = reinterpret_cast<unsigned long long *>(keys);
    return dbg_sort(k64, vals, n, st,
                    [&](unsigned long long *k, uint32_t *v, unsigned long long *ka, uint32_t *va,
                        SortScratch &ss, unsigned int *err) {
                        return radix_sort_u64(k, v, ka, va, n, key_bits, ss, err, st);
                    });
}

int tril_dbg_morton(const float *boxes, int64_t n, const float *bounds, uint32_t *keys,
                    void *stream) {
    if (n < 0 || n >= kMaxN || !bounds) return TRIL_E_INVAL;
    if (n > 0 && (!boxes || !keys)) return TRIL_E_INVAL;
    if (n == 0) return TRIL_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint32_t hb[6];
    for (int a = 0; a < 6; ++a) {
        uint32_t u;
        std::memcpy(&u, bounds + a, 4);
        hb[a] = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    }
    uint32_t *db = nullptr, *dv = nullptr;
    int r = dev_alloc(&db, 6);
    if (r == TRIL_OK) r = dev_alloc(&dv, (size_t)n);
    if (r == TRIL_OK) {
        hipError_t e = hipMemcpy(db, hb, sizeof(hb), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            launch_morton_u32(reinterpret_cast<const PBox *>(boxes), n, db, keys, dv, st);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) r = hip_fail(e);
    }
    dev_free(db);
    dev_free(dv);
    return r;
}

int tril_dbg_pair_eval(int64_t n, const double *in, double *out, void *stream) {
    if (n < 0 || (n > 0 && (!in || !out))) return TRIL_E_INVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    launch_pair_eval(n, in, out, st);
    HIPCHK(hipGetLastError());
    return TRIL_OK;
}

int tril_dbg_math(int which, int64_t n, const double *a, const double *b, double *out,
                  void *stream) {
    if (which < 0 || which > 5 || n < 0 || (n > 0 && (!a || !out)) ||
        (n > 0 && (which == 0 || which == 2) && !b))
        return TRIL_E_INVAL;
    launch_math_sweep(which, n, a, b, out, reinterpret_cast<hipStream_t>(stream));
    HIPCHK(hipGetLastError());
    return TRIL_OK;
}

int tril_dbg_pair_eval32(int64_t n, const double *in, double *out, void *stream) {
    if (n < 0 || (n > 0 && (!in || !out))) return TRIL_E_INVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    launch_pair_eval32(n, in, host_sigma_max() * (1.0 + 1e-6), out, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return TRIL_OK;
}

int tril_dbg_tree(tril_ctx *c, void *nodes, int64_t cap_nodes, int64_t *n_nodes, int32_t *roots) {
    if (!c || !n_nodes) return TRIL_E_INVAL;
    if (!c->built || c->nodes_partial) return TRIL_E_STATE;
    HIPCHK(hipStreamSynchronize(c->st));
    const int32_t copies = window_copies(c->tgt.m, c->win_eff);
    const int64_t nn = c->tgt.n > 1 ? (int64_t)copies * (c->tgt.n - 1) : 0;
    *n_nodes = nn;
    if (nn > cap_nodes) return TRIL_E_OVERFLOW;
    if (nn > 0) {
        if (!nodes) return TRIL_E_INVAL;
        HIPCHK(hipMemcpy(nodes, c->nodes, nn * sizeof(Node), hipMemcpyDeviceToHost));
    }
    const size_t n_comb = (size_t)copies * c->tgt.n_inst;
    if (roots) HIPCHK(hipMemcpy(roots, c->inst_root, n_comb * sizeof(int32_t), hipMemcpyDeviceToHost));
    return TRIL_OK;
}

int tril_dbg_keep_nodes(tril_ctx *c, int32_t on) {
    if (!c || on < 0 || on > 1) return TRIL_E_INVAL;
    c->keep_nodes = on != 0;
    return TRIL_OK;
}

int tril_dbg_target_records(tril_ctx *c, void *recs, int64_t cap, int64_t *n, int32_t *win) {
    if (!c || !n || !win) return TRIL_E_INVAL;
    if (!c->built) return TRIL_E_STATE;
    HIPCHK(hipStreamSynchronize(c->st));
    *win = c->win_eff;
    const int64_t nn = c->win_eff > 1 ? c->tgt.n : 0;
    *n = nn;
    if (nn > cap) return TRIL_E_OVERFLOW;
    if (nn > 0) {
        if (!recs) return TRIL_E_INVAL;
        HIPCHK(hipMemcpy(recs, c->t_rec, nn * sizeof(TRec), hipMemcpyDeviceToHost));
    }
    return TRIL_OK;
}

int tril_dbg_quad_nodes(tril_ctx *c, void *nodes, int64_t cap, int64_t *n, float *frames,
                        int32_t *n_copies) {
    if (!c || !n || !n_copies) return TRIL_E_INVAL;
    if (!c->built) return TRIL_E_STATE;
    HIPCHK(hipStreamSynchronize(c->st));
    const int32_t copies = c->quad ? window_copies(c->tgt.m, c->win_eff) : 0;
    const int64_t nn = copies > 0 ? (int64_t)copies * (c->tgt.n - 1) : 0;
    *n = nn;
    *n_copies = copies;
    if (nn > cap) return TRIL_E_OVERFLOW;
    if (nn > 0) {
        if (!nodes || !frames) return TRIL_E_INVAL;
        HIPCHK(hipMemcpy(nodes, c->nodes4, nn * sizeof(CNode4), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(frames, c->t_frames, copies * sizeof(WinFrame), hipMemcpyDeviceToHost));
    }
    return TRIL_OK;
}

int tril_dbg_boxes(tril_ctx *c, int which, void *boxes, int64_t cap, int64_t *n) {
    if (!c || !n || (which != 0 && which != 1)) return TRIL_E_INVAL;
    HIPCHK(hipStreamSynchronize(c->st));
    const int64_t nn = which == 0 ? (int64_t)c->tgt.m * c->tgt.n : c->last_q.n;
    *n = nn;
    if (nn > cap) return TRIL_E_OVERFLOW;
    if (nn > 0) {
        if (!boxes) return TRIL_E_INVAL;
        PBox *src = which == 0 ? c->t_box : c->q_box, *tmp = nullptr;
        if (which == 0) {
            // the refit forms the target's leaf boxes itself: recompute them as it did (into
            // a buffer of its own where the tree buffers hold copies, not steps)
            if (!c->built) return TRIL_E_STATE;
            if (nn > c->t_cap) {
                CHK(dev_alloc(&tmp, (size_t)nn));
                src = tmp;
            }
            launch_set_step(c->d_cnt, c->tgt_k0, c->st);
            launch_leaf_boxes(c->tgt, c->tgt_cloud, c->dt, c->d_cnt, src, c->st);
            const hipError_t e = hipGetLastError();
            const hipError_t e2 = hipStreamSynchronize(c->st);
            if (e != hipSuccess || e2 != hipSuccess) {
                dev_free(tmp);
                HIPCHK(e != hipSuccess ? e : e2);
            }
        }
        const hipError_t e = hipMemcpy(boxes, src, nn * sizeof(PBox), hipMemcpyDeviceToHost);
        dev_free(tmp);
        HIPCHK(e);
    }
    return TRIL_OK;
}

int tril_dbg_target_rows(tril_ctx *c, int32_t *rows, int64_t cap, int64_t *n) {
    if (!c || !n) return TRIL_E_INVAL;
    HIPCHK(hipStreamSynchronize(c->st));
    if (!c->built) return TRIL_E_STATE;
    const BeamDev &t = c->tgt;
    *n = t.n;
    if (t.n > cap) return TRIL_E_OVERFLOW;
    if (t.n == 0) return TRIL_OK;
    if (!rows) return TRIL_E_INVAL;
    if (t.perm) {
        HIPCHK(hipMemcpy(rows, t.perm, t.n * sizeof(int32_t), hipMemcpyDeviceToHost));
    } else {
        for (int64_t r = 0; r < t.n; ++r) rows[r] = (int32_t)r;
    }
    return TRIL_OK;
}

int tril_dbg_query_records(tril_ctx *c, int32_t s, void *boxes, int64_t cap, int64_t *n) {
    if (!c || !n) return TRIL_E_INVAL;
    HIPCHK(hipStreamSynchronize(c->st));
    const BeamDev &v = c->last_qrec;
    if (v.m < 2 || c->q_rec == nullptr) return TRIL_E_STATE;
    if (s < 0 || s >= v.m) return TRIL_E_INVAL;
    *n = v.n;
    if (v.n > cap) return TRIL_E_OVERFLOW;
    if (v.n == 0) return TRIL_OK;
    if (!boxes) return TRIL_E_INVAL;
    PBox *tmp = nullptr;
    CHK(dev_alloc(&tmp, (size_t)v.n));
    launch_record_boxes(c->q_rec, v.n, v.perm, s, tmp, c->st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e == hipSuccess) e = hipMemcpy(boxes, tmp, v.n * sizeof(PBox), hipMemcpyDeviceToHost);
    dev_free(tmp);
    if (e != hipSuccess) return hip_fail(e);
    return TRIL_OK;
}

int tril_dbg_st_audit_sample(tril_ctx *c, int side, int32_t *rows, double *pis, int64_t cap,
                             int64_t *n) {
    if (!c || !n || (side != 0 && side != 1)) return TRIL_E_INVAL;
    HIPCHK(hipStreamSynchronize(c->st));
    const int64_t nn = c->au_row[side] ? c->au_n[side] : 0;
    *n = nn;
    if (nn > cap) return TRIL_E_OVERFLOW;
    if (nn > 0) {
        if (!rows || !pis) return TRIL_E_INVAL;
        HIPCHK(hipMemcpy(rows, c->au_row[side], nn * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(pis, c->au_pi[side], nn * sizeof(double), hipMemcpyDeviceToHost));
    }
    return TRIL_OK;
}

int tril_dbg_candidates(tril_ctx *c, int32_t *ci, int32_t *cj, int64_t cap, int64_t *count) {
    if (!c || !count || cap < 0) return TRIL_E_INVAL;
    HIPCHK(hipStreamSynchronize(c->st));
    HIPCHK(hipMemcpy(c->h_cnt, c->d_cnt, sizeof(DevCounters), hipMemcpyDeviceToHost));
    const int64_t nc = (int64_t)c->h_cnt->cand_step;
    *count = nc;
    const int64_t m = std::min<int64_t>(std::min<int64_t>(nc, cap), c->cand_cap);
    if (m > 0) {
        if (!ci || !cj) return TRIL_E_INVAL;
        HIPCHK(hipMemcpy(ci, c->cand_i, m * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(cj, c->cand_j, m * sizeof(int32_t), hipMemcpyDeviceToHost));
    }
    return TRIL_OK;
}

}  // extern "C"
