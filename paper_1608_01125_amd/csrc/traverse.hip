#include <algorithm>

// Broad phase: every query photon's swept, radius-padded box descends the
// target hierarchy depth-first (Sec. 2.2): a node whose box fails the overlap
// test (Eq. 5) has its whole subtree skipped; a leaf whose box passes yields a
// candidate pair. A node holds its two children's boxes, so one 64-byte load tests
// both: a child that fails is never loaded, and the descent costs one dependent load
// per internal node whose box the query overlaps (a scalar load when every active lane of
// the wave is at the same node). When both children are internal and
// overlap, the right one waits on a per-lane stack (four entries in registers, the
// rest in a private spill array).
//
// Threshold prune (Eq. 2): a node's child half also holds the largest photon energy of
// its subtree, rounded up, and a query box its photon's energy, rounded up. Since
// s = E_i E_j (1 - u_i.u_j) / (2 m_e^2) <= E_i E_j / m_e^2, a child whose bound gives
// E_q E_max < m_e^2 (1 - 1e-5) holds no photon above threshold with the query and is
// skipped (the FP32 product's rounding is far inside the margin).
//
// The overlap test is closed (<=) on both sides, so touching boxes stay
// candidates; boxes are rounded outward, so the candidate set contains every
// pair the exact narrow phase can accept.
//
// Candidates are compacted per wave: a 64-lane ballot of the lanes that found
// one, a single atomicAdd by the first such lane, and each lane's slot from the
// count of set ballot bits below it.
//
// Window copies: when one copy of the target hierarchy serves W consecutive steps (its
// boxes those of the window's middle step r), a query of step s tests internal nodes
// with its box widened by the target instance's motion over s - r plus a rounding slack
// (wslack), and a leaf that passes against the leaf's own box at step s, formed from the
// leaf's record as the per-step refit would form it: the candidates are those of per-step
// copies.
//
// With four-child forms a query descends each window copy once for all the window's steps:
// its box is the hull of the widened boxes of the window's first and last steps, which
// holds the widened box of every step between them (below), and a leaf that passes is
// tested against the query's exact box at every step of the window, each hit a candidate
// of that step. The candidates are again those of per-step copies, found with one descent
// and one query record read per window instead of one per step.
#include "tril_internal.h"

namespace tril {

namespace {

__device__ __forceinline__ uint32_t count_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Wave-compacted append of the candidates (qi, j) of the lanes with emit set; called by
// every active lane of the wave.
__device__ __forceinline__ void emit_candidate(bool emit, int32_t qi, int64_t j,
                                               int32_t *__restrict__ cand_i,
                                               int32_t *__restrict__ cand_j, int64_t cand_cap,
                                               DevCounters *c) {
    const unsigned long long m = __ballot(emit);
    if (m == 0ull) return;
    const int leader = __ffsll((long long)m) - 1;
    unsigned long long base = 0;
    if (emit && count_below(m) == 0) {
        const unsigned long long cnt = (unsigned long long)__popcll(m);
        base = atomicAdd(&c->cand_step, cnt);
        if (base + cnt > (unsigned long long)cand_cap) atomicOr(&c->err, kErrCandOverflow);
    }
    base = __shfl(base, leader);
    if (emit) {
        const unsigned long long pos = base + count_below(m);
        if (pos < (unsigned long long)cand_cap) {
            cand_i[pos] = qi;
            cand_j[pos] = (int32_t)j;
        }
    }
}

__device__ __forceinline__ bool box_overlap(const float q[6], float4 lo, float4 hi) {
    return (q[0] <= hi.x) & (q[3] >= lo.x) & (q[1] <= hi.y) & (q[4] >= lo.y) & (q[2] <= hi.z) &
           (q[5] >= lo.z);
}

constexpr float kPruneProduct = (float)(kMe * kMe * (1.0 - 1e-5));

constexpr int kStackRegs = 4;
constexpr int kStackSpill = 124;  // deeper than any radix tree over (key, index) pairs
// four-child descent: at most three pushes per level of a tree at most 48 levels deep
constexpr int kStackSpill4 = 144;
// four-child descent: leaf slots queued per lane (in LDS) and tested together, when a lane's
// queue would overflow and at the end of the descent
constexpr int kLeafQ = 16;

// Box of a query of step offset s from the row's record for the batch (moved_box).
__device__ __forceinline__ void record_box(const float4 a, const float4 d, const float4 w,
                                           float s, float qb[6]) {
    moved_box(a.x, a.y, a.z, d.x, d.y, d.z, w.x, w.y, w.z, s, qb, qb + 3);
}

// Window copies: the box of target leaf j (sorted position) at step offset s tested
// against the query's box at s (closed test and the threshold prune); elem receives the
// element s n + row.
__device__ __forceinline__ bool leaf_exact(const WinArgs &wa, int64_t j, int32_t s,
                                           const float qb[6], float qe, int64_t &elem) {
    const float4 *tp = reinterpret_cast<const float4 *>(wa.trec + j);
    const float4 a = tp[0], d = tp[1], w = tp[2];
    float lo[3], hi[3];
    moved_box(a.x, a.y, a.z, d.x, d.y, d.z, w.x, w.y, w.z, (float)s, lo, hi);
    elem = (int64_t)s * wa.n + __float_as_int(a.w);
    return (qb[0] <= hi[0]) & (qb[3] >= lo[0]) & (qb[1] <= hi[1]) & (qb[4] >= lo[1]) &
           (qb[2] <= hi[2]) & (qb[5] >= lo[2]) & (qe * d.w >= kPruneProduct);
}

// One descent per window: the steps s0 + t (t < len, bit t of the result) at which target
// leaf j's box meets the box of query row `row` (both formed from their records as the
// per-step paths form them; closed test), and the threshold prune, which does not depend on
// the step; trow receives the leaf's target row.
//
// Only the steps of an interval are tested. On each axis the two boxes at step s are the
// offset-0 boxes moved by s v (v: each one's motion per step), each widened by its rounding
// bound, at most 2^-19 (|lo| + w + s |v|) (moved_box), so they can meet only where
// s (vq - vl) lies in [(ll - lq) - wq - g, (ll - lq) + wl + g] with g = 2^-17 (|lq| + |ll| +
// wq + wl + s1 (|vq| + |vl|)), more than twice the sum of the two bounds and the FP32 error
// of forming the interval ends. Solving for s, each end moved outward by a step past its
// FP32 quotient, gives a range of steps that holds every step the exact test can accept.
__device__ __forceinline__ uint32_t leaf_steps(const WinArgs &wa, int64_t j,
                                               const QRec *__restrict__ qrec, int32_t row,
                                               int32_t s0, int32_t len, float qe, int32_t &trow) {
    // the step range from both records in one round of loads; the exact test one axis at a
    // time from single-word loads again (the records' words x, y, z of lo, d and w sit at
    // 4 k, 16 + 4 k and 32 + 4 k bytes), so that few registers are live beside the descent's
    const float *tf = reinterpret_cast<const float *>(wa.trec + j);
    const float *qf = reinterpret_cast<const float *>(qrec + row);
    const float4 ta = reinterpret_cast<const float4 *>(tf)[0];
    const float4 td = reinterpret_cast<const float4 *>(tf)[1];
    const float4 tw = reinterpret_cast<const float4 *>(tf)[2];
    const float4 qa = reinterpret_cast<const float4 *>(qf)[0];
    const float4 qd = reinterpret_cast<const float4 *>(qf)[1];
    const float4 qw = reinterpret_cast<const float4 *>(qf)[2];
    trow = __float_as_int(ta.w);
    if (!(qe * td.w >= kPruneProduct)) return 0u;
    const float s1 = (float)(s0 + len - 1);
    float tlo = (float)s0, thi = s1;
    const float lqs[3] = {qa.x, qa.y, qa.z}, vqs[3] = {qd.x, qd.y, qd.z};
    const float wqs[3] = {qw.x, qw.y, qw.z}, lls[3] = {ta.x, ta.y, ta.z};
    const float vls[3] = {td.x, td.y, td.z}, wls[3] = {tw.x, tw.y, tw.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float lq = lqs[k], vq = vqs[k], wq = wqs[k];
        const float ll = lls[k], vl = vls[k], wl = wls[k];
        const float g = (((fabsf(lq) + fabsf(ll)) + (wq + wl)) + s1 * (fabsf(vq) + fabsf(vl))) *
                        0x1p-17f;
        const float dd = ll - lq;
        const float lo = (dd - wq) - g, hi = (dd + wl) + g;
        const float rel = vq - vl;
        if (rel == 0.0f) {
            if (!((lo <= 0.0f) & (hi >= 0.0f))) thi = -1.0f;
        } else {
            const float a1 = lo / rel, a2 = hi / rel;
            // infinite quotients clamp to the window; the comparisons keep it otherwise
            tlo = fmaxf(tlo, floorf(fminf(a1, a2)) - 1.0f);
            thi = fminf(thi, ceilf(fmaxf(a1, a2)) + 1.0f);
        }
    }
    if (!(tlo <= thi)) return 0u;
    // the exact test of every step of the range: the steps at which every axis meets
    const int32_t t0 = (int32_t)tlo - s0, t1 = (int32_t)thi - s0;
    uint32_t mask = (t1 >= 31 ? 0xFFFFFFFFu : (2u << t1) - 1u) & ~((1u << t0) - 1u);
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
        const float lq = qf[k], vq = qf[4 + k], wq = qf[8 + k];
        const float ll = tf[k], vl = tf[4 + k], wl = tf[8 + k];
        for (int32_t t = t0; t <= t1; ++t) {
            const float s = (float)(s0 + t);
            float ql, qh, tl, th;
            moved_axis(lq, vq, wq, s, ql, qh);
            moved_axis(ll, vl, wl, s, tl, th);
            if (!((ql <= th) & (qh >= tl))) mask &= ~(1u << t);
        }
    }
    return mask;
}

// Appends one candidate per set bit t of mask: query row `row` and target row trow at step
// s0 + t (elements s nq_base + row and s n + trow). Called by every active lane of the wave.
__device__ __forceinline__ void emit_steps(uint32_t mask, int32_t row, int32_t trow, int32_t s0,
                                           int64_t nq_base, int64_t n,
                                           int32_t *__restrict__ cand_i,
                                           int32_t *__restrict__ cand_j, int64_t cand_cap,
                                           DevCounters *c) {
    for (;;) {
        const bool has = mask != 0u;
        if (__ballot(has) == 0ull) break;
        const int32_t s = s0 + (has ? __builtin_ctz(mask) : 0);
        mask &= mask - 1u;
        emit_candidate(has, (int32_t)(s * nq_base + row), (int64_t)s * n + trow, cand_i, cand_j,
                       cand_cap, c);
    }
}

// The descent of virtual query q (q >= nq: an idle lane that still takes part in the
// wave's ballots); adds its node loads to visits (and, over window copies, its leaf
// record loads to checks) and returns the number of query steps it stood for: 0 without a
// root, else 1, or with four-child forms the steps of its window.
template <bool kRec, bool kWin, bool kQuad>
__device__ __forceinline__ int32_t traverse_query(int64_t q, const Node *__restrict__ nodes,
                                               int32_t n_int, const PBox *__restrict__ root_box,
                                               const PBox *__restrict__ qbox,
                                               const QRec *__restrict__ qrec, int32_t n_inst,
                                               const uint32_t *__restrict__ qorder,
                                               int64_t order_len, int64_t nq, int64_t nq_base,
                                               const int32_t *__restrict__ inst_root,
                                               int32_t *__restrict__ cand_i,
                                               int32_t *__restrict__ cand_j, int64_t cand_cap,
                                               DevCounters *c, uint32_t &visits,
                                               const WinArgs &wa, uint32_t &checks,
                                               uint32_t *__restrict__ lq, int32_t lq_stride) {
    int32_t node = -1, qi = 0, tag = -1, qs = 0;
    float qb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float qw[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // window copies: the widened box
    int32_t qc[6] = {0, 0, 0, 0, 0, 0};  // four-child forms: the widened box in frame cells
    int32_t cbase = 0;                   // four-child forms: first node of the query's copy
    int32_t qn = 1;                      // four-child forms: the steps of the query's window
    float qe = 0.f;
    if (kQuad && q < nq) {
        // virtual query q: descent k = q / nq_base (steps qs .. qs + qn - 1, part sub of
        // copy cp, whose descents are nd each but for the last copy's) and the row at
        // position q - k nq_base of the step order; qi holds the row
        const int64_t kd = q / nq_base;
        const int64_t t = q - kd * nq_base;
        const int32_t nd = (wa.win + wa.dwin - 1) / wa.dwin;
        const int32_t cp = (int32_t)(kd / nd);
        const int32_t sub = (int32_t)(kd - (int64_t)cp * nd);
        qi = (int32_t)(qorder == nullptr ? t : qorder[t]);
        const float4 *rp = reinterpret_cast<const float4 *>(qrec + qi);
        const float4 a = rp[0], d = rp[1], w = rp[2];
        const int32_t inst = __float_as_int(a.w);
        if (inst >= 0) {
            qs = cp * wa.win + sub * wa.dwin;
            qn = min(wa.dwin, min(wa.win, wa.m - cp * wa.win) - sub * wa.dwin);
            const int32_t r = window_ref_step(cp, wa.win, wa.m);
            // the widened boxes of the first and last steps (box at the step, less the
            // instance's motion over s - r, less the slack). In exact arithmetic the low side
            // of a step's box less the motion is concave in the step (a line, less the
            // rounding bound's |lo| + |hi| and the motion's max(d lo, d hi), both convex) and
            // the high side convex, so the hull of the two ends holds every step's. The slack
            // is taken with the larger coordinates of the two boxes, which bound those of
            // every step between them: it is twice the rounding bound of any step of the
            // window, and the half to spare exceeds the FP32 error of the two ends' boxes.
            float qa[6], qz[6];
            record_box(a, d, w, (float)qs, qa);
            record_box(a, d, w, (float)(qs + qn - 1), qz);
            qe = d.w;
            const float da = (float)(qs - r), dz = (float)(qs + qn - 1 - r);
            float4 vlo, vhi;
            const int32_t iu = __builtin_amdgcn_readfirstlane(inst);
            if (__ballot(inst == iu) == __ballot(1)) {
                typedef int v8i __attribute__((ext_vector_type(8)));
                v8i rv;
                const WinBound *p = wa.vb + iu;
                asm volatile("s_load_dwordx8 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)"
                             : "=s"(rv)
                             : "s"(p));
                vlo = make_float4(__int_as_float(rv[0]), __int_as_float(rv[1]),
                                  __int_as_float(rv[2]), __int_as_float(rv[3]));
                vhi = make_float4(__int_as_float(rv[4]), __int_as_float(rv[5]),
                                  __int_as_float(rv[6]), __int_as_float(rv[7]));
            } else {
                const float4 *vp = reinterpret_cast<const float4 *>(wa.vb + inst);
                vlo = vp[0];
                vhi = vp[1];
            }
            float4 fb, fi;
            const int32_t cu = __builtin_amdgcn_readfirstlane(cp);
            if (__ballot(cp == cu) == __ballot(1)) {
                typedef int v8i __attribute__((ext_vector_type(8)));
                v8i rf;
                const WinFrame *p = wa.frames + cu;
                asm volatile("s_load_dwordx8 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)"
                             : "=s"(rf)
                             : "s"(p));
                fb = make_float4(__int_as_float(rf[0]), __int_as_float(rf[1]),
                                 __int_as_float(rf[2]), 0.0f);
                fi = make_float4(__int_as_float(rf[4]), __int_as_float(rf[5]),
                                 __int_as_float(rf[6]), 0.0f);
            } else {
                const float4 *fp = reinterpret_cast<const float4 *>(wa.frames + cp);
                fb = fp[0];
                fi = fp[1];
            }
            const float lo3[3] = {vlo.x, vlo.y, vlo.z}, hi3[3] = {vhi.x, vhi.y, vhi.z};
            const float b3[3] = {fb.x, fb.y, fb.z}, i3[3] = {fi.x, fi.y, fi.z};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float e1 = da * lo3[k], e2 = da * hi3[k];
                const float f1 = dz * lo3[k], f2 = dz * hi3[k];
                const float sl =
                    wslack(fminf(qa[k], qz[k]), fmaxf(qa[k + 3], qz[k + 3]), wa.reach);
                const float wl = fminf((qa[k] - fmaxf(e1, e2)) - sl, (qz[k] - fmaxf(f1, f2)) - sl);
                const float wh = fmaxf((qa[k + 3] - fminf(e1, e2)) + sl,
                                       (qz[k + 3] - fminf(f1, f2)) + sl);
                // in the copy's frame cells (floor - 1, ceil + 1: the one-cell margins cover
                // the FP32 rounding), kept within [-1, 65536]
                const float lo = (wl - b3[k]) * i3[k];
                const float hi = (wh - b3[k]) * i3[k];
                qc[k] = (int32_t)fminf(fmaxf(floorf(lo) - 1.0f, -1.0f), 65536.0f);
                qc[k + 3] = (int32_t)fminf(fmaxf(ceilf(hi) + 1.0f, -1.0f), 65536.0f);
            }
            cbase = cp * (int32_t)(wa.n - 1);
            tag = cp * n_inst + inst;
        }
    } else if (q < nq) {
        if (qorder == nullptr) {
            qi = (int32_t)q;
        } else if (order_len == nq) {
            qi = (int32_t)qorder[q];
        } else {  // one step's order, repeated for every step of the launch
            const int64_t s = q / nq_base;
            qi = (int32_t)(s * nq_base + qorder[q - s * nq_base]);
        }
        if (kRec) {
            const int64_t s = qi / nq_base;
            const float4 *rp = reinterpret_cast<const float4 *>(qrec + (qi - s * nq_base));
            const float4 a = rp[0], d = rp[1], w = rp[2];
            const int32_t inst = __float_as_int(a.w);
            if (inst >= 0) {
                record_box(a, d, w, (float)s, qb);
                qe = d.w;
                if (kWin) {
                    qs = (int32_t)s;
                    const int32_t cp = qs / wa.win;
                    const float delta = (float)(qs - window_ref_step(cp, wa.win, wa.m));
                    // the instance's motion bounds: one scalar load when the wave's queries
                    // share their instance (nearly always: queries run in instance order),
                    // keeping two vector loads per query off the texture path
                    float4 vlo, vhi;
                    const int32_t iu = __builtin_amdgcn_readfirstlane(inst);
                    if (__ballot(inst == iu) == __ballot(1)) {
                        typedef int v8i __attribute__((ext_vector_type(8)));
                        v8i r;
                        const WinBound *p = wa.vb + iu;
                        asm volatile("s_load_dwordx8 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)"
                                     : "=s"(r)
                                     : "s"(p));
                        vlo = make_float4(__int_as_float(r[0]), __int_as_float(r[1]),
                                          __int_as_float(r[2]), __int_as_float(r[3]));
                        vhi = make_float4(__int_as_float(r[4]), __int_as_float(r[5]),
                                          __int_as_float(r[6]), __int_as_float(r[7]));
                    } else {
                        const float4 *vp = reinterpret_cast<const float4 *>(wa.vb + inst);
                        vlo = vp[0];
                        vhi = vp[1];
                    }
                    const float lo3[3] = {vlo.x, vlo.y, vlo.z}, hi3[3] = {vhi.x, vhi.y, vhi.z};
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const float e1 = delta * lo3[k], e2 = delta * hi3[k];
                        const float sl = wslack(qb[k], qb[k + 3], wa.reach);
                        qw[k] = (qb[k] - fmaxf(e1, e2)) - sl;
                        qw[k + 3] = (qb[k + 3] - fminf(e1, e2)) + sl;
                    }
                    tag = cp * n_inst + inst;
                } else {
                    tag = (int32_t)(s * n_inst + inst);
                }
            }
        } else {
            const float4 *bp = reinterpret_cast<const float4 *>(qbox + qi);
            const float4 a = bp[0], b = bp[1];
            qb[0] = a.x; qb[1] = a.y; qb[2] = a.z;
            qb[3] = b.x; qb[4] = b.y; qb[5] = b.z;
            qe = b.w;
            tag = __float_as_int(a.w);
        }
    }
    if (tag >= 0) {
        // the root of the query's (step or copy, instance) tree: a scalar load when the
        // wave's queries share it (they nearly always do), else a vector load
        const int32_t tu = __builtin_amdgcn_readfirstlane(tag);
        if (__ballot(tag == tu) == __ballot(1)) {
            int32_t r;
            const int32_t *p = inst_root + tu;
            asm volatile("s_load_dword %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(p));
            node = r;
        } else {
            node = inst_root[tag];
        }
    }
    const bool active = node != -1;
    if (kQuad) {
        // an instance of one row: its root is that leaf
        uint32_t mask = 0u;
        int32_t trow = 0;
        if (node <= -2) {
            mask = leaf_steps(wa, link_elem(node), qrec, qi, qs, qn, qe, trow);
            ++checks;
            ++visits;
            node = -1;
        }
        emit_steps(mask, qi, trow, qs, nq_base, wa.n, cand_i, cand_j, cand_cap, c);
    } else {
        // an instance of one row: its root is that leaf
        bool hit = false;
        int64_t e = 0;
        if (node <= -2) {
            e = link_elem(node);
            if (kWin) {
                hit = leaf_exact(wa, e, qs, qb, qe, e);
                ++checks;
            } else {
                const float4 *lp = reinterpret_cast<const float4 *>(root_box + tag);
                hit = box_overlap(qb, lp[0], lp[1]);
            }
            ++visits;
            node = -1;
        }
        emit_candidate(hit, qi, e, cand_i, cand_j, cand_cap, c);
    }
    int32_t st0 = -1, st1 = -1, st2 = -1, st3 = -1;
    int32_t spill[kQuad ? kStackSpill4 : kStackSpill];
    int32_t depth = 0;
    // every internal node is loaded at most once per query in a well-formed tree
    const uint32_t max_visits = (uint32_t)n_int + 2u;
    if (kQuad) {
        // four-child descent: every load brings the boxes of the node's grandchildren, so the
        // chain of dependent loads is half as long; up to three overlapping internal
        // children wait on the stack
        uint32_t qlen = 0u;  // leaf slots queued in lq (sorted leaf positions)
        auto flush = [&]() {
            for (;;) {
                const bool has = qlen != 0u;
                if (__ballot(has) == 0ull) break;
                // the query's exact boxes at the descent's steps are formed again from its
                // record (kept out of the registers the descent holds)
                uint32_t mask = 0u;
                int32_t trow = 0;
                if (has) {
                    --qlen;
                    mask = leaf_steps(wa, (int64_t)lq[qlen * lq_stride], qrec, qi, qs, qn, qe, trow);
                    ++checks;
                }
                emit_steps(mask, qi, trow, qs, nq_base, wa.n, cand_i, cand_j, cand_cap, c);
            }
        };
        while (node >= 0) {
            if (visits > max_visits) {
                atomicOr(&c->err, kErrSpin);
                break;
            }
            uint32_t w[16];
            const int32_t first = __builtin_amdgcn_readfirstlane(node);
            if (__ballot(node == first) == __ballot(1)) {
                typedef int v16i __attribute__((ext_vector_type(16)));
                v16i r;
                const CNode4 *p = wa.nodes4 + first;
                asm volatile("s_load_dwordx16 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(p));
#pragma unroll
                for (int k = 0; k < 16; ++k) w[k] = (uint32_t)r[k];
            } else {
                const uint4 *np = reinterpret_cast<const uint4 *>(wa.nodes4 + node);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint4 v = np[k];
                    w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
                }
            }
            ++visits;
            int32_t lk[4];
            bool ov[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t a0 = w[3 * k], a1 = w[3 * k + 1], a2 = w[3 * k + 2];
                const uint32_t eh = (k & 1) ? (w[14 + (k >> 1)] >> 16) : (w[14 + (k >> 1)] & 0xFFFFu);
                const float e = __uint_as_float((eh & 0x7FFFu) << 16);
                ov[k] = ((int32_t)(a0 & 0xFFFFu) <= qc[3]) & ((int32_t)(a1 >> 16) >= qc[0]) &
                        ((int32_t)(a0 >> 16) <= qc[4]) & ((int32_t)(a2 & 0xFFFFu) >= qc[1]) &
                        ((int32_t)(a1 & 0xFFFFu) <= qc[5]) & ((int32_t)(a2 >> 16) >= qc[2]) &
                        (qe * e >= kPruneProduct);
                const int32_t g = (int32_t)w[12 + (k >> 1)] + (k & 1);
                lk[k] = (eh & 0x8000u) ? leaf_link(g) : cbase + g;
            }
            // the next node and the pushes first, so that only the leaf slots' ids stay live
            // through the leaf tests
            uint32_t pend = 0u;
#pragma unroll
            for (int k = 0; k < 4; ++k) pend |= (uint32_t)(ov[k] & (lk[k] <= -2)) << k;
            const uint32_t g0 = w[12], g2 = w[13];
            int32_t nxt = -1;
            bool full = false;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!(ov[k] & (lk[k] >= 0))) continue;
                if (nxt < 0) {
                    nxt = lk[k];
                    continue;
                }
                if (depth >= kStackRegs) {
                    if (depth - kStackRegs >= kStackSpill4) {
                        full = true;
                        continue;
                    }
                    spill[depth - kStackRegs] = st3;
                }
                st3 = st2; st2 = st1; st1 = st0; st0 = lk[k];
                ++depth;
            }
            if (full) {
                atomicOr(&c->err, kErrSpin);
                break;
            }
            if (nxt >= 0) {
                node = nxt;
            } else if (depth > 0) {  // pop
                node = st0;
                st0 = st1; st1 = st2; st2 = st3;
                --depth;
                if (depth >= kStackRegs) st3 = spill[depth - kStackRegs];
            } else {
                node = -1;
            }
            // leaf slots: queued, and tested in rounds in which every lane with a queued leaf
            // tests one, once a lane's queue would overflow (and at the end of the descent),
            // so that a round finds many lanes busy rather than the one or two of a visit
            if (__ballot(pend != 0u) != 0ull) {
                if (__ballot(qlen + (uint32_t)__popc(pend) > (uint32_t)kLeafQ) != 0ull) flush();
                while (pend != 0u) {
                    const uint32_t k = (uint32_t)__builtin_ctz(pend);
                    pend &= pend - 1u;
                    lq[qlen * lq_stride] = ((k & 2u) ? g2 : g0) + (k & 1u);
                    ++qlen;
                }
            }
        }
        flush();
        return active ? qn : 0;
    }
    while (node >= 0) {
        if (visits > max_visits) {
            atomicOr(&c->err, kErrSpin);
            break;
        }
        float4 l0, l1, r0, r1;
        const int32_t first = __builtin_amdgcn_readfirstlane(node);
        if (__ballot(node == first) == __ballot(1)) {
            // every active lane descends the same node (common in the upper levels, whose
            // boxes a wave's neighbouring queries share): one scalar load for the wave
            // instead of four vector loads that each take an L1 lookup
            typedef int v16i __attribute__((ext_vector_type(16)));
            v16i r;
            const Node *p = nodes + first;
            asm volatile("s_load_dwordx16 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(p));
            l0 = make_float4(__int_as_float(r[0]), __int_as_float(r[1]), __int_as_float(r[2]),
                             __int_as_float(r[3]));
            l1 = make_float4(__int_as_float(r[4]), __int_as_float(r[5]), __int_as_float(r[6]),
                             __int_as_float(r[7]));
            r0 = make_float4(__int_as_float(r[8]), __int_as_float(r[9]), __int_as_float(r[10]),
                             __int_as_float(r[11]));
            r1 = make_float4(__int_as_float(r[12]), __int_as_float(r[13]), __int_as_float(r[14]),
                             __int_as_float(r[15]));
        } else {
            const float4 *np = reinterpret_cast<const float4 *>(nodes + node);
            l0 = np[0];
            l1 = np[1];
            r0 = np[2];
            r1 = np[3];
        }
        ++visits;
        const int32_t lc = __float_as_int(l0.w), rc = __float_as_int(r0.w);
        const bool ovl = box_overlap(kWin ? qw : qb, l0, l1) & (qe * l1.w >= kPruneProduct);
        const bool ovr = box_overlap(kWin ? qw : qb, r0, r1) & (qe * r1.w >= kPruneProduct);
        const bool leafl = lc < 0, leafr = rc < 0;
        bool el = ovl & leafl, er = ovr & leafr;
        // leaves: nothing to do in most visits of most waves (one ballot decides)
        if (__ballot(el | er) != 0ull) {
            int64_t jl = link_elem(lc), jr = link_elem(rc);
            if (kWin) {
                if (el) {
                    el = leaf_exact(wa, jl, qs, qb, qe, jl);
                    ++checks;
                }
                if (er) {
                    er = leaf_exact(wa, jr, qs, qb, qe, jr);
                    ++checks;
                }
            }
            emit_candidate(el, qi, jl, cand_i, cand_j, cand_cap, c);
            emit_candidate(er, qi, jr, cand_i, cand_j, cand_cap, c);
        }
        const bool gol = ovl & !leafl, gor = ovr & !leafr;
        if (gol) {
            if (gor) {  // push the right child
                if (depth >= kStackRegs) {
                    if (depth - kStackRegs >= kStackSpill) {
                        atomicOr(&c->err, kErrSpin);
                        break;
                    }
                    spill[depth - kStackRegs] = st3;
                }
                st3 = st2; st2 = st1; st1 = st0; st0 = rc;
                ++depth;
            }
            node = lc;
        } else if (gor) {
            node = rc;
        } else if (depth > 0) {  // pop
            node = st0;
            st0 = st1; st1 = st2; st2 = st3;
            --depth;
            if (depth >= kStackRegs) st3 = spill[depth - kStackRegs];
        } else {
            node = -1;
        }
    }
    return active ? 1 : 0;
}

// Per-wave counter updates of a traversal workgroup's wave (lane 0 adds): node loads, leaf
// record loads and query steps of the wave's lanes.
__device__ __forceinline__ void add_counts(uint32_t visits, uint32_t checks, uint32_t qsteps,
                                           DevCounters *c) {
    unsigned long long v = visits, k = checks, n_active = qsteps;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        v += __shfl_xor(v, off);
        k += __shfl_xor(k, off);
        n_active += __shfl_xor(n_active, off);
    }
    if ((threadIdx.x & 63) == 0) {
        const int slot = blockIdx.x & (kCounterSlots - 1);
        if (v) atomicAdd(&c->visits[slot], v);
        if (k) atomicAdd(&c->leaf_checks[slot], k);
        if (n_active) atomicAdd(&c->queries[slot], n_active);
    }
}

// One virtual query per lane over a flat grid.
constexpr int kXcdRun = 16;

template <int BLOCK, bool kRec, bool kWin, bool kQuad>
__global__ void __launch_bounds__(BLOCK, kQuad ? 8 : 1) k_traverse(const Node *__restrict__ nodes, int32_t n_int,
                                                    const PBox *__restrict__ root_box,
                                                    const PBox *__restrict__ qbox,
                                                    const QRec *__restrict__ qrec, int32_t n_inst,
                                                    const uint32_t *__restrict__ qorder,
                                                    int64_t order_len, int64_t nq, int64_t nq_base,
                                                    const int32_t *__restrict__ inst_root,
                                                    int32_t *__restrict__ cand_i,
                                                    int32_t *__restrict__ cand_j, int64_t cand_cap,
                                                    DevCounters *c, WinArgs wa) {
    __shared__ uint32_t s_lq[kQuad ? kLeafQ * BLOCK : 1];
    // the dispatcher deals workgroups to the 8 XCDs in turn: runs of kXcdRun consecutive
    // workgroups (neighbouring queries, which descend the same subtrees) go to one XCD and
    // share its L2, while the runs still spread the dense part of the beam over all XCDs
    int64_t b = blockIdx.x;
    if (kQuad) {
        const int64_t span = 8 * (int64_t)kXcdRun;
        if (b < ((int64_t)gridDim.x / span) * span) {
            const int64_t slot = b >> 3;
            b = ((slot / kXcdRun) * 8 + (b & 7)) * kXcdRun + slot % kXcdRun;
        }
    }
    const int64_t q = b * BLOCK + threadIdx.x;
    uint32_t visits = 0, checks = 0;
    const int32_t qsteps = traverse_query<kRec, kWin, kQuad>(
        q, nodes, n_int, root_box, qbox, qrec, n_inst, qorder, order_len, nq, nq_base, inst_root,
        cand_i, cand_j, cand_cap, c, visits, wa, checks, kQuad ? s_lq + threadIdx.x : nullptr, BLOCK);
    add_counts(visits, checks, (uint32_t)qsteps, c);
}


// Persistent form: a fixed grid whose waves take chunks of kQueueChunk consecutive virtual
// queries from device-wide cursors until the chunks run out; every wave leaves its loop once
// its cursor passes the last chunk. Workgroup b uses cursor b mod 8 (one per XCD, as the
// dispatcher deals workgroups out round-robin), which hands out chunks x, x + 8, x + 16, ...
// (the cursors are cleared by the batch's prologue): one device atomic per chunk, spread
// over eight addresses, instead of one per wave of queries at one address.
constexpr int kQueueChunk = 1024;

template <int BLOCK, bool kRec, bool kWin, bool kQuad>
__global__ void __launch_bounds__(BLOCK) k_traverse_queue(const Node *__restrict__ nodes,
                                                          int32_t n_int,
                                                          const PBox *__restrict__ root_box,
                                                          const PBox *__restrict__ qbox,
                                                          const QRec *__restrict__ qrec,
                                                          int32_t n_inst,
                                                          const uint32_t *__restrict__ qorder,
                                                          int64_t order_len, int64_t nq,
                                                          int64_t nq_base,
                                                          const int32_t *__restrict__ inst_root,
                                                          int32_t *__restrict__ cand_i,
                                                          int32_t *__restrict__ cand_j,
                                                          int64_t cand_cap, DevCounters *c,
                                                          WinArgs wa) {
    __shared__ uint32_t s_lq[kQuad ? kLeafQ * BLOCK : 1];
    const int lane = threadIdx.x & 63;
    const int x = blockIdx.x & (kTravCursors - 1);
    uint32_t visits = 0, checks = 0, qsteps = 0;
    for (;;) {
        unsigned long long k = 0;
        if (lane == 0) k = atomicAdd(&c->trav_next[x], 1ull);
        k = __shfl(k, 0);
        const int64_t base = ((int64_t)k * kTravCursors + x) * kQueueChunk;
        if (base >= nq) break;
        for (int sub = 0; sub < kQueueChunk; sub += 64) {
            if (base + sub >= nq) break;
            qsteps += (uint32_t)traverse_query<kRec, kWin, kQuad>(
                base + sub + lane, nodes, n_int, root_box, qbox, qrec, n_inst, qorder, order_len,
                nq, nq_base, inst_root, cand_i, cand_j, cand_cap, c, visits, wa, checks,
                kQuad ? s_lq + threadIdx.x : nullptr, BLOCK);
        }
    }
    add_counts(visits, checks, qsteps, c);
}

template <int BLOCK, bool kRec, bool kWin, bool kQuad>
void launch_traverse_k(const Node *nodes, int32_t n_int, const PBox *root_box, const PBox *qbox,
                       const QRec *qrec, int32_t n_inst, const uint32_t *qorder, int64_t order_len,
                       int64_t nq, int64_t nq_base, const int32_t *inst_root, int32_t *cand_i,
                       int32_t *cand_j, int64_t cand_cap, DevCounters *c, bool queue,
                       const WinArgs &wa, hipStream_t st) {
    const int64_t want = (nq + BLOCK - 1) / BLOCK;
    if (queue) {
        // as many workgroups as keep 32 waves on each of the 256 CUs
        const unsigned grid = (unsigned)std::min<int64_t>(want, 8192 * 64 / BLOCK);
        hipLaunchKernelGGL((k_traverse_queue<BLOCK, kRec, kWin, kQuad>), dim3(grid), dim3(BLOCK), 0, st,
                           nodes, n_int, root_box, qbox, qrec, n_inst, qorder, order_len, nq,
                           nq_base, inst_root, cand_i, cand_j, cand_cap, c, wa);
        return;
    }
    hipLaunchKernelGGL((k_traverse<BLOCK, kRec, kWin, kQuad>), dim3((unsigned)want), dim3(BLOCK), 0, st,
                       nodes, n_int, root_box, qbox, qrec, n_inst, qorder, order_len, nq, nq_base,
                       inst_root, cand_i, cand_j, cand_cap, c, wa);
}

template <int BLOCK>
void launch_traverse_b(const Node *nodes, int32_t n_int, const PBox *root_box, const PBox *qbox,
                       const QRec *qrec, int32_t n_inst, const uint32_t *qorder, int64_t order_len,
                       int64_t nq, int64_t nq_base, const int32_t *inst_root, int32_t *cand_i,
                       int32_t *cand_j, int64_t cand_cap, DevCounters *c, bool queue,
                       const WinArgs *win, hipStream_t st) {
    WinArgs wa = {};
    if (qrec != nullptr && win != nullptr && win->nodes4 != nullptr && win->dwin >= 1 &&
        win->dwin <= kMaxDescent && win->dwin <= win->win &&
        (qorder == nullptr || order_len == nq_base)) {
        // one virtual query per (descent, row) of the one step order
        wa = *win;
        const int64_t nq_win = descent_count(wa.m, wa.win, wa.dwin) * nq_base;
        launch_traverse_k<BLOCK, true, true, true>(nodes, n_int, root_box, qbox, qrec, n_inst,
                                                   qorder, order_len, nq_win, nq_base, inst_root,
                                                   cand_i, cand_j, cand_cap, c, queue, wa, st);
    } else if (qrec != nullptr && win != nullptr) {
        wa = *win;
        launch_traverse_k<BLOCK, true, true, false>(nodes, n_int, root_box, qbox, qrec, n_inst,
                                                    qorder, order_len, nq, nq_base, inst_root,
                                                    cand_i, cand_j, cand_cap, c, queue, wa, st);
    } else if (qrec != nullptr) {
        launch_traverse_k<BLOCK, true, false, false>(nodes, n_int, root_box, qbox, qrec, n_inst,
                                                     qorder, order_len, nq, nq_base, inst_root,
                                                     cand_i, cand_j, cand_cap, c, queue, wa, st);
    } else {
        launch_traverse_k<BLOCK, false, false, false>(nodes, n_int, root_box, qbox, qrec, n_inst,
                                                      qorder, order_len, nq, nq_base, inst_root,
                                                      cand_i, cand_j, cand_cap, c, queue, wa, st);
    }
}

__global__ void k_record_boxes(const QRec *__restrict__ qrec, int64_t n,
                               const int32_t *__restrict__ perm, float s, PBox *__restrict__ out) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const float4 *rp = reinterpret_cast<const float4 *>(qrec + r);
    const float4 a = rp[0], d = rp[1], w = rp[2];
    float qb[6];
    record_box(a, d, w, s, qb);
    PBox b;
    b.lox = qb[0]; b.loy = qb[1]; b.loz = qb[2];
    b.hix = qb[3]; b.hiy = qb[4]; b.hiz = qb[5];
    b.tag = __float_as_int(a.w);
    b.pad = (int32_t)r;
    out[perm ? perm[r] : r] = b;
}

}  // namespace

void launch_record_boxes(const QRec *qrec, int64_t n, const int32_t *perm, int32_t s, PBox *out,
                         hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_record_boxes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, qrec, n,
                       perm, (float)s, out);
}

void launch_traverse(const Node *nodes, int64_t n_int64, const PBox *root_box, const PBox *qbox,
                     const uint32_t *qorder, int64_t order_len, int64_t nq, int64_t nq_base,
                     const int32_t *inst_root, int32_t *cand_i, int32_t *cand_j,
                     int64_t cand_cap, DevCounters *c, int block, hipStream_t st,
                     const QRec *qrec, int32_t n_inst, bool queue, const WinArgs *win) {
    if (nq <= 0 || n_int64 < 0) return;
    const int32_t n_int = (int32_t)n_int64;
    switch (block) {
    case 64:
        launch_traverse_b<64>(nodes, n_int, root_box, qbox, qrec, n_inst, qorder, order_len, nq,
                              nq_base, inst_root, cand_i, cand_j, cand_cap, c, queue, win, st);
        break;
    case 128:
        launch_traverse_b<128>(nodes, n_int, root_box, qbox, qrec, n_inst, qorder, order_len, nq,
                               nq_base, inst_root, cand_i, cand_j, cand_cap, c, queue, win, st);
        break;
    case 512:
        launch_traverse_b<512>(nodes, n_int, root_box, qbox, qrec, n_inst, qorder, order_len, nq,
                               nq_base, inst_root, cand_i, cand_j, cand_cap, c, queue, win, st);
        break;
    default:
        launch_traverse_b<256>(nodes, n_int, root_box, qbox, qrec, n_inst, qorder, order_len, nq,
                               nq_base, inst_root, cand_i, cand_j, cand_cap, c, queue, win, st);
        break;
    }
}

}  // namespace tril
