// Broad phase: every query photon's swept, radius-padded box descends the
// target hierarchy depth-first (Sec. 2.2): a node whose box fails the overlap
// test (Eq. 5) has its whole subtree skipped; a leaf whose box passes yields a
// candidate pair. The descent follows ropes (next node in depth-first order),
// so a lane needs no stack: overlap -> left child, otherwise -> rope.
//
// The overlap test is closed (<=) on both sides, so touching boxes stay
// candidates; boxes are rounded outward, so the candidate set contains every
// pair the exact narrow phase can accept.
//
// Candidates are compacted per wave: a 64-lane ballot of the lanes that found
// one, a single atomicAdd by the first such lane, and each lane's slot from the
// count of set ballot bits below it.
#include "tril_internal.h"

namespace tril {

namespace {

__device__ __forceinline__ uint32_t count_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_traverse(const Node *__restrict__ nodes, int32_t n_int,
                                                    const PBox *__restrict__ qbox,
                                                    const uint32_t *__restrict__ qorder,
                                                    int64_t order_len, int64_t nq, int64_t nq_base,
                                                    const int32_t *__restrict__ inst_root,
                                                    const int32_t *__restrict__ inst_stop,
                                                    int32_t *__restrict__ cand_i,
                                                    int32_t *__restrict__ cand_j, int64_t cand_cap,
                                                    DevCounters *c) {
    const int64_t q = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    int32_t node = -1, stop = -1, qi = 0;
    float lx = 0.f, ly = 0.f, lz = 0.f, hx = 0.f, hy = 0.f, hz = 0.f;
    if (q < nq) {
        if (qorder == nullptr) {
            qi = (int32_t)q;
        } else if (order_len == nq) {
            qi = (int32_t)qorder[q];
        } else {  // one step's order, repeated for every step of the launch
            const int64_t s = q / nq_base;
            qi = (int32_t)(s * nq_base + qorder[q - s * nq_base]);
        }
        const float4 *bp = reinterpret_cast<const float4 *>(qbox + qi);
        const float4 a = bp[0], b = bp[1];
        lx = a.x; ly = a.y; lz = a.z;
        hx = b.x; hy = b.y; hz = b.z;
        const int32_t tag = __float_as_int(a.w);
        if (tag >= 0) {
            node = inst_root[tag];
            stop = inst_stop[tag];
        }
    }
    const unsigned long long active_q = __ballot(node >= 0);
    uint32_t visits = 0;
    // every node is visited at most once per query in a well-formed tree
    const uint32_t max_visits = 2u * (uint32_t)n_int + 2u;
    while (node >= 0 && node != stop) {
        if (visits > max_visits) {
            atomicOr(&c->err, kErrSpin);
            break;
        }
        const float4 *np = reinterpret_cast<const float4 *>(nodes + node);
        const float4 a = np[0], b = np[1];
        ++visits;
        const bool ov = (lx <= b.x) & (hx >= a.x) & (ly <= b.y) & (hy >= a.y) & (lz <= b.z) &
                        (hz >= a.z);
        const bool leaf = node >= n_int;
        const bool emit = ov & leaf;
        const unsigned long long m = __ballot(emit);
        if (m) {
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
                    cand_j[pos] = __float_as_int(a.w);
                }
            }
        }
        node = (ov && !leaf) ? __float_as_int(a.w) : __float_as_int(b.w);
    }
    // per-wave counter updates
    unsigned long long v = visits;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) {
        const int slot = blockIdx.x & (kCounterSlots - 1);
        if (v) atomicAdd(&c->visits[slot], v);
        if (active_q) atomicAdd(&c->queries[slot], (unsigned long long)__popcll(active_q));
    }
}

}  // namespace

void launch_traverse(const Node *nodes, int64_t n_int64, const PBox *qbox, const uint32_t *qorder,
                     int64_t order_len, int64_t nq, int64_t nq_base,
                     const int32_t *inst_root, const int32_t *inst_stop,
                     int32_t *cand_i, int32_t *cand_j, int64_t cand_cap, DevCounters *c, int block,
                     hipStream_t st) {
    if (nq <= 0 || n_int64 < 0) return;
    const int32_t n_int = (int32_t)n_int64;
    const unsigned grid = (unsigned)((nq + block - 1) / block);
    switch (block) {
    case 64:
        hipLaunchKernelGGL(k_traverse<64>, dim3(grid), dim3(64), 0, st, nodes, n_int, qbox, qorder,
                           order_len, nq, nq_base, inst_root, inst_stop, cand_i, cand_j, cand_cap, c);
        break;
    case 128:
        hipLaunchKernelGGL(k_traverse<128>, dim3(grid), dim3(128), 0, st, nodes, n_int, qbox,
                           qorder, order_len, nq, nq_base, inst_root, inst_stop, cand_i, cand_j, cand_cap, c);
        break;
    case 512:
        hipLaunchKernelGGL(k_traverse<512>, dim3(grid), dim3(512), 0, st, nodes, n_int, qbox,
                           qorder, order_len, nq, nq_base, inst_root, inst_stop, cand_i, cand_j, cand_cap, c);
        break;
    default:
        hipLaunchKernelGGL(k_traverse<256>, dim3(grid), dim3(256), 0, st, nodes, n_int, qbox,
                           qorder, order_len, nq, nq_base, inst_root, inst_stop, cand_i, cand_j, cand_cap, c);
        break;
    }
}

}  // namespace tril
