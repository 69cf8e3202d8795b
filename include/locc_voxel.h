/* C-ABI of the voxel-embedding LOCC variant: the paper's own design (Sec.
 * III, appendix "Architecture Details"), beside the crop-point path of
 * locc.h.  Shares locc.h's status codes and object record.
 *
 * Shape encoder, once per shape, on the device at upload (float32):
 *   a per-point MLP 3 -> 256 -> 256 -> 256 (ReLU) on the stored xyz; a 6x6x6
 *   grid on the shape's box [lo, hi] (component-wise min / max of the stored
 *   xyz), point p in cell i_k = min(5, floor(((p_k - lo_k) * 6) / (hi_k -
 *   lo_k))) per axis (float64; 0 on an axis of zero extent), flat index
 *   (i_0 * 6 + i_1) * 6 + i_2, channel-wise max per cell (empty cell: 0); a 3D
 *   U-Net: conv 256 -> 128 without padding (6^3 -> 4^3), three convs 128 ->
 *   128 with padding 1, a global feature [max, mean] over the 64 bottleneck
 *   cells (256 values), four transposed convs 128 -> 128 (on the bottleneck)
 *   then 256 -> 128 on [previous, matching conv output] with padding 1, the
 *   last one without padding (4^3 -> 6^3), ReLU after every conv; per cell a
 *   linear map of [last transposed conv output, global feature] (384) to the
 *   embedding E (16 floats).  conv: y[o][x] = b[o] + sum_c sum_u
 *   W[o][c][u] in[c][x + u - pad]; transposed: in[c][x - u + pad]; u in
 *   {0,1,2}^3, zero outside the input.
 *
 * Collision predictor, per pair (canonical order a = min(i, j), float64
 * relative pose T_ab = (R_ab, t_ab) as in locc.h):
 *   cell centres c = lo + (i + 1/2) s, s = (hi - lo) / 6, margin eps =
 *   sqrt((s_0^2 + s_1^2) + s_2^2) / 2 of the cell under test (its
 *   centre-to-vertex distance); a's cell is selected when R_ab^T (c - t_ab)
 *   lies in b's box widened by eps_a on every axis (closed), b's cell when
 *   R_ab c + t_ab lies in a's box widened by eps_b (float64, fixed order, no
 *   fused multiply-add); per object the mean embedding of its selected cells
 *   (0 if none) and its pose in the other object's frame (t then R
 *   row-major: (-R_ab^T t_ab, R_ab^T) for a, (t_ab, R_ab) for b); a shared
 *   MLP 28 -> 128 -> 128 -> 128 (ReLU) per object, the element-wise max over
 *   the two, an MLP 128 -> 128 -> 128 -> 128 (ReLU), a linear 128 -> 1 (the
 *   logit) and the sigmoid.  The result does not depend on the order the
 *   caller gives a pair in.
 *
 * Weights: float32, flat, W row-major [out][in...]: P1 [256][3], p1, P2
 * [256][256], p2, P3 [256][256], p3, C1 [128][256][3][3][3], k1, C2..C4
 * [128][128][3][3][3], k2..k4, D1 [128][128][3][3][3], e1, D2..D4
 * [128][256][3][3][3], e2..e4, L [16][384], l, A1 [128][28], a1, A2, a2, A3,
 * a3 ([128][128]), B1, b1, B2, b2, B3, b3 ([128][128]), B4 [1][128], b4. */
#ifndef LOCC_VOXEL_H
#define LOCC_VOXEL_H

#include "locc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct locc_voxel_ctx locc_voxel_ctx;

/* Number of float32 weights (5,534,609). */
LOCC_API size_t locc_voxel_weight_count(void);

/* Context on HIP device `device`.  Errors: INVALID_ARG, HIP. */
LOCC_API locc_status locc_voxel_create(int device, locc_voxel_ctx** out);
LOCC_API void locc_voxel_destroy(locc_voxel_ctx* ctx);

/* Host weights (copied; synchronous).  If shapes are resident their
 * embeddings are recomputed.  Errors: INVALID_ARG (null, wrong count,
 * non-finite value), OOM, HIP. */
LOCC_API locc_status locc_voxel_upload_weights(locc_voxel_ctx* ctx, const float* h_weights, size_t n);

/* Host shape library in locc_upload_shapes' format (offsets int64 [S + 1],
 * points float32 [N][6]; only xyz is used), copied; if weights are resident
 * the embeddings of every shape are computed on the device (synchronous).
 * Errors: INVALID_ARG (empty shape, non-finite value), RANGE (more than
 * 65,536 points in a shape), OOM, HIP. */
LOCC_API locc_status locc_voxel_upload_shapes(locc_voxel_ctx* ctx, int32_t n_shapes, const int64_t* h_offsets,
                                              const float* h_points);

/* Copies the shape embeddings E, float32 [S][216][16] (cell-major, flat cell
 * index as above), into d_out (device, caller-owned), asynchronously on
 * `stream`.  Errors: INVALID_ARG, NOT_READY (no weights or shapes), HIP. */
LOCC_API locc_status locc_voxel_embeddings(locc_voxel_ctx* ctx, float* d_out, void* stream);

/* Collision prediction for n_pairs pairs, asynchronous on `stream`.
 *   d_objs    [n_objs] locc_object, device
 *   d_pairs   int32 [n_pairs][2], device
 *   d_out     float32 [n_pairs][2], device: logit, probability
 *   d_counts  int32 [n_pairs][2] selected cells per object in the caller's
 *             order, or NULL
 *   d_pooled  float32 [n_pairs][2][16] mean embeddings in the caller's
 *             order, or NULL
 * An invalid pair (index out of range, i == j, shape id out of range) gets
 * NaN outputs, counts -1 and one increment of the device error counter.
 * Errors: INVALID_ARG, NOT_READY, HIP. */
LOCC_API locc_status locc_voxel_detect(locc_voxel_ctx* ctx, const locc_object* d_objs, int32_t n_objs,
                                       const int32_t* d_pairs, int32_t n_pairs, float* d_out, int32_t* d_counts,
                                       float* d_pooled, void* stream);

/* Invalid pairs seen since the last reset (synchronises `stream`). */
LOCC_API locc_status locc_voxel_device_errors(locc_voxel_ctx* ctx, void* stream, int64_t* n_bad, int reset);

#ifdef __cplusplus
}
#endif

#endif /* LOCC_VOXEL_H */
