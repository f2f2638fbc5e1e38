/*
 * tril_debug.h -- inspection entry points of libtril for tests and tools.
 *
 * Applications do not need these. They expose single stages of the pipeline
 * (radix sort, Morton keys, the FP64 pair evaluation of the narrow phase) and
 * copies of a context's internal state (hierarchy nodes, swept boxes, the
 * candidate pairs of the last step) so each stage can be checked on its own.
 * Same conventions as tril.h: device pointers unless marked host, asynchronous
 * on the given stream unless stated, TRIL_OK or a negative TRIL_E_* code.
 */
#ifndef TRIL_DEBUG_H
#define TRIL_DEBUG_H

#include <stdint.h>

#include "tril.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Stable sort of (keys, vals) by the low key_bits bits of the keys, in place.
 * n in [0, 2^30); key_bits in [1, 32] resp. [1, 64]. Synchronises the stream. */
int tril_dbg_sort_u32(uint32_t *keys, uint32_t *vals, int64_t n, int key_bits, void *stream);
int tril_dbg_sort_u64(uint64_t *keys, uint32_t *vals, int64_t n, int key_bits, void *stream);

/* Morton keys of box centroids. boxes: device, n x 8 floats laid out as
 * (lox, loy, loz, tag, hix, hiy, hiz, pad); bounds: host, 6 floats (min xyz, max xyz)
 * of the quantisation box; keys: device, n. Each axis maps [min, max] to 0..1023,
 * clamped, then bits interleave as x2 y1 z0 per level (x most significant). */
int tril_dbg_morton(const float *boxes, int64_t n, const float *bounds, uint32_t *keys,
                    void *stream);

/* FP64 evaluation of the narrow-phase quantities for n photon pairs.
 * in: device, n x 18 doubles per row:
 *   E_i px_i py_i pz_i x_i y_i z_i w_i  E_j px_j py_j pz_j x_j y_j z_j w_j  t  dt
 * out: device, n x 4 doubles per row: s, sigma(s) [um^2], d^2 (smallest squared
 * distance over [t, t + dt]) and r^2 = sqrt(w_i w_j) sigma / pi. */
int tril_dbg_pair_eval(int64_t n, const double *in, double *out, void *stream);

/* The FP32 stage of the narrow phase on the same n x 18 input rows (sigma bound of the
 * library): out, device, n x 8 doubles per row: s, bound on |s - s_exact|, d^2, its
 * bound, r^2, its bound (r^2 and its bound are 0 when the stage stopped at the threshold,
 * and the radius upper bound when it stopped there), decision (0 no pair, 1 pair,
 * 2 left to FP64), 0. Bounds are relative to exact arithmetic on the FP64 inputs.
 * Synchronises the stream. */
int tril_dbg_pair_eval32(int64_t n, const double *in, double *out, void *stream);

/* The device arithmetic the narrow phase relies on, one operation per element, compiled
 * with the narrow phase's flags (no contraction, no fast math): which = 0: FP64 a / b;
 * 1: FP64 sqrt(a); on the arguments rounded to FP32: 2: a / b, 3: sqrtf(a), 4: logf(a),
 * 5: log1pf(a), results widened to FP64. a, b (b for 0 and 2 only), out: device, n
 * doubles. Asynchronous on the stream. */
int tril_dbg_math(int which, int64_t n, const double *a, const double *b, double *out,
                  void *stream);

/* The surrogate's matrix-core product C = A B: A(m, k) = A[m sam + k sak] and
 * B(k, n) = B[k sbk + n sbn] as BF16 bit patterns (device), C [M][N] row-major FP32
 * (device). Synchronises the stream. */
int tril_dbg_gemm_bf16(const uint16_t *A, int64_t sam, int64_t sak, const uint16_t *B, int64_t sbk,
                       int64_t sbn, int32_t M, int32_t N, int32_t K, float *C, void *stream);

/* Copy the last built hierarchy to host memory (synchronises the context stream).
 * nodes: host, cap_nodes x 16 words, one internal node each: its left child's box and
 * link (lox loy loz link hix hiy hiz pad), then its right child's, as float/int32; a
 * link >= 0 is an internal node, a link <= -2 a leaf: with one copy per step the leaf
 * holding target element -2 - link, with window copies (tril_params.kinetic_window)
 * the leaf at sorted position -2 - link (tril_dbg_target_records). *n_nodes receives
 * c (n-1) for the c copies of the last build (c = m, the build's steps, or ceil(m / W)
 * for windows of W steps; 0 below two rows). roots: host, c n_inst root links (same
 * encoding; -1: empty instance), or NULL. TRIL_E_OVERFLOW if cap_nodes < *n_nodes;
 * TRIL_E_STATE before a build, or after a build with window copies of several steps that
 * left the binary nodes below the refit's chunk tops unstored (tril_dbg_keep_nodes). */
int tril_dbg_tree(tril_ctx *ctx, void *nodes, int64_t cap_nodes, int64_t *n_nodes,
                  int32_t *roots);

/* With window copies of several steps the traversal descends the four-child forms, and the
 * refit stores the binary node of an internal node only where another build step reads it:
 * the crossing nodes (those whose leaves span two 512-leaf chunks) and the chunks' top
 * nodes. on = 1 makes later builds of ctx store every binary node as well, so that
 * tril_dbg_tree can return the whole tree (same forms, candidates and pairs); on = 0
 * restores the default. TRIL_E_INVAL for a NULL ctx or another value of on. */
int tril_dbg_keep_nodes(tril_ctx *ctx, int32_t on);

/* Window copies of the last build: *win receives its steps per copy (1: a copy per
 * step, and *n = 0); otherwise *n receives the target rows n and recs (host, n x 12
 * words) the record of each sorted position: lox loy loz row, dx dy dz e, wx wy wz 0 as
 * float/int32, the leaf's box at step offset 0 (low corner, widths) and its motion per
 * step, from which every step's leaf box is formed as the refit forms it (copy k holds
 * the boxes of step offset k W + (min(W, m - k W) - 1) / 2). Synchronises the stream;
 * TRIL_E_OVERFLOW if cap < *n. */
int tril_dbg_target_records(tril_ctx *ctx, void *recs, int64_t cap, int64_t *n, int32_t *win);

/* Four-child forms of the window copies of the last build, which the traversal descends:
 * *n_copies receives the copies (0 without them, and *n = 0), *n their count (copies x
 * (n - 1), one per internal node in the order of tril_dbg_tree); nodes (host, cap x 16
 * words): slot k's box in words 3k..3k+2 as 16-bit frame cells (lo x | lo y << 16,
 * lo z | hi x << 16, hi y | hi z << 16; lo > hi: empty), word 12 the first child g0 of the
 * node's left child (slots 0 and 1 are g0 and g0 + 1: internal nodes of the same copy, or
 * sorted leaf positions; a leaf left child is slot 0 itself), word 13 likewise g2 for slots
 * 2 and 3, words 14 and 15 the slots' energy bounds (bits 0-14 and 16-30: the top 15 bits of
 * the FP32 bound, rounded up) and leaf flags (bits 15 and 31) for slots 0, 1 and 2, 3;
 * frames (host, 8 floats per copy): base x y z, 0, cells per unit x y z, 0 (cell k of an axis
 * spans [base + k / inv, base + (k + 1) / inv]). Synchronises the stream; TRIL_E_OVERFLOW if
 * cap < *n. */
int tril_dbg_quad_nodes(tril_ctx *ctx, void *nodes, int64_t cap, int64_t *n, float *frames,
                        int32_t *n_copies);

/* Copy the swept boxes of the last target (which = 0: all m n of the last build's m
 * steps, formed again here exactly as the build's refit formed them) or query
 * (which = 1) beam to host memory as n x 8 words (lox loy loz tag hix hiy hiz
 * instance). Synchronises the context stream. */
int tril_dbg_boxes(tril_ctx *ctx, int which, void *boxes, int64_t cap, int64_t *n);

/* Caller row of each row of the last build's target view (host, n entries): the element
 * s n + r of tril_dbg_boxes (which = 0) and of the hierarchy's leaves is the photon of
 * caller row rows[r] at step offset s (tril_run builds over Morton-ordered working
 * copies; tril_build over the caller's rows, rows[r] = r). Synchronises the stream. */
int tril_dbg_target_rows(tril_ctx *ctx, int32_t *rows, int64_t cap, int64_t *n);

/* Query boxes of step offset s (0 <= s < m) of the last step batch of tril_run, formed
 * from the batch's per-row query records exactly as the traversal forms them, in the
 * caller's row order: host, n x 8 words (lox loy loz tag hix hiy hiz working-row) as in
 * tril_dbg_boxes; tag -1 marks a row that can collide with nothing. *n receives the
 * query rows. TRIL_E_STATE when the last batch had no records (one step per launch).
 * Synchronises the context stream. */
int tril_dbg_query_records(tril_ctx *ctx, int32_t s, void *boxes, int64_t cap, int64_t *n);

/* Thinned beam of the last replicate of the last tril_st_audit (side 0: query, 1: target)
 * in kept order: host arrays of the source rows and of their inclusion probabilities.
 * *n receives the kept rows (0 before any audit). Synchronises the context stream. */
int tril_dbg_st_audit_sample(tril_ctx *ctx, int side, int32_t *rows, double *pis, int64_t cap,
                             int64_t *n);

/* Copy the candidate pairs of the last tril_collide to host memory. *count gets the
 * number found (may exceed cap; only min(count, cap) are written). */
int tril_dbg_candidates(tril_ctx *ctx, int32_t *ci, int32_t *cj, int64_t cap, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif /* TRIL_DEBUG_H */
