/*
 * locc.h - C-ABI of the LOCC crop-collision library for AMD MI355X (gfx950).
 *
 * The library evaluates, for many pairs of rigid objects at once, the local
 * object crop collision network of Son & Kim (arXiv 2304.09439).  The paper
 * poses the problem as evaluating the collision between two objects directly
 * from their shapes and poses (Sec. III), with an Object Collision Net that
 * takes the shapes and poses of the two objects (Sec. II) and a dataset of
 * tuples (shape 1, shape 2, pose 1, pose 2, label) (Sec. III-A).  Here the
 * shapes are uploaded once as surface point clouds with normals and each
 * call passes poses and object pairs.
 *
 * Per pair (i, j) the library computes, in the frame of a = min(i, j):
 *   - the relative pose of b = max(i, j) and a crop box: a's axis-aligned box
 *     intersected with the axis-aligned hull of b's transformed box, widened
 *     by a margin on every face (the paper pads the colliding region so that
 *     nothing in contact is missed; Sec. III, appendix "Architecture
 *     Details").  Pose composition and the membership test run in float64,
 *     with no fused multiply-add, so crop sets are reproducible bit for bit;
 *   - the first K stored points of each object inside the box (count before
 *     the cap is returned), as (xyz, normal) rows in a's frame;
 *   - a per-point MLP 6 -> h1 -> h2 (ReLU) max-pooled per object, and a head
 *     MLP 2*h2 -> hh -> hh -> 8 (ReLU on hidden layers, last layer linear;
 *     the appendix applies ReLU across all layers and ends in a linear layer);
 *   - the contact record below, mapped to the world by a's pose.
 *
 * Pointers named h_* are host memory, d_* are device memory of the context's
 * device.  `stream` is a hipStream_t (NULL = the default stream).  Every call
 * returns a locc_status; on failure locc_last_error() describes it.  Calls on
 * one context must not overlap in time (one context per host thread).
 */
#ifndef LOCC_H
#define LOCC_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define LOCC_API __attribute__((visibility("default")))
#else
#define LOCC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LOCC_OK = 0,
  LOCC_ERR_INVALID_ARG = -1, /* null pointer, negative size, bad layout: nothing was touched */
  LOCC_ERR_OOM = -2,         /* device allocation failed */
  LOCC_ERR_HIP = -3,         /* a HIP runtime call failed (message has the HIP error) */
  LOCC_ERR_NOT_READY = -4,   /* detect before shapes and weights were uploaded */
  LOCC_ERR_RANGE = -5,       /* a size exceeds a library limit */
  LOCC_ERR_BUSY = -6,        /* serving: request does not fit the memory budget now (retry); or a captured
                                graph still holds what the call would change (see locc_graph_capture) */
  LOCC_ERR_UNSUPPORTED = -7  /* widths / K / precision combination not compiled in */
} locc_status;

typedef enum { LOCC_FP32 = 0, LOCC_BF16 = 1, LOCC_FP8 = 2, LOCC_FP8_ENCODER = 3 } locc_precision;

/* Network and crop configuration, fixed for the life of a context.
 *   K       crop cap per object, multiple of 32, 32..256
 *   enc_h1  encoder hidden width, enc_h2 encoder output width (per object)
 *   head_h  head hidden width; the head input is 2 * enc_h2
 *   pad_m   crop margin added to every face of the box, metres (>= 0)
 *   precision  arithmetic of the encoder and head (locc_precision);
 *              the crop geometry is float64 in every precision.
 *              LOCC_FP32 runs the per-step path (crop, encoder, head
 *              kernels); LOCC_BF16 runs one fused persistent kernel or
 *              a crop kernel plus a persistent network kernel (see
 *              locc_schedule); LOCC_FP8 runs the crop kernel plus a
 *              persistent network kernel whose encoder layer 2 and head
 *              layers 1-2 multiply OCP e4m3 operands (encoder layer 1 and
 *              head layer 3 stay bf16) and needs activation maxima
 *              (locc_calibrate or locc_set_activation_amax) first;
 *              LOCC_FP8_ENCODER is LOCC_FP8 with e4m3 on encoder layer 2
 *              only and the whole head in bf16 as in LOCC_BF16 (about
 *              half of LOCC_FP8's error against full precision; the same
 *              calls, of which only the first activation maximum is used)
 * Compiled width sets: (h1, h2, hh) = (64, 128, 256) and (128, 256, 512). */
typedef struct {
  int32_t K;
  int32_t enc_h1;
  int32_t enc_h2;
  int32_t head_h;
  double pad_m;
  int32_t precision;
  int32_t reserved; /* must be 0 */
} locc_config;

/* One rigid object: position of its frame origin, shape id, and orientation
 * as a Hamilton quaternion (w, x, y, z) rotating object-frame vectors into
 * the world.  The quaternion is used as given (not renormalised).  32 bytes. */
typedef struct {
  float p[3];
  int32_t shape;
  float q[4];
} locc_object;

/* Result per pair, 32 bytes:
 *   logit   collision logit; flag = logit > 0 (sigmoid(logit) > 0.5)
 *   point   contact point, world frame
 *   normal  contact normal in the world frame, from the caller's first object
 *           towards its second; not normalised
 *   depth   penetration depth (positive = overlapping)
 * An invalid pair (index out of range, i == j, shape id out of range) gets
 * all-NaN fields, counts of -1, and increments the device error counter. */
typedef struct {
  float logit;
  float point[3];
  float normal[3];
  float depth;
} locc_contact;

typedef struct locc_ctx locc_ctx;

/* Library version string, e.g. "locc 0.1.0 gfx950". Static storage. */
LOCC_API const char* locc_version(void);

/* Message of the last failed call on this host thread (static thread-local
 * storage, valid until the next failing call). */
LOCC_API const char* locc_last_error(void);

/* Create a context on HIP device `device` with configuration `cfg` (copied).
 * Allocates nothing large; uploads and the first detect allocate.
 * Errors: INVALID_ARG (null, bad K/pad), UNSUPPORTED (widths/precision), HIP. */
LOCC_API locc_status locc_create(const locc_config* cfg, int device, locc_ctx** out);

/* Free every device buffer of the context and the context itself. NULL is a no-op. */
LOCC_API void locc_destroy(locc_ctx* ctx);

/* Network weights, float32, host memory, copied synchronously (the caller may
 * free h_weights on return).  Order W1, b1, W2, b2, H1, c1, H2, c2, H3, c3;
 * each W row-major [out][in]:
 *   W1 [h1][6]  W2 [h2][h1]  H1 [hh][2 h2]  H2 [hh][hh]  H3 [8][hh].
 * n_floats must equal the total.  The encoder input row is
 * (x, y, z, nx, ny, nz) in a's frame; the head input is [f_a, f_b].
 * Low precisions quantise from these values (per-layer scales for FP8).
 * Errors: INVALID_ARG (null, wrong n_floats, non-finite value), BUSY (FP8
 * context with a captured graph alive, see locc_graph_capture), OOM, HIP. */
LOCC_API locc_status locc_upload_weights(locc_ctx* ctx, const float* h_weights, size_t n_floats);

/* FP8 contexts (LOCC_FP8 and LOCC_FP8_ENCODER): activation scales of the
 * quantised encoder and head layers
 * (Sec. III and appendix "Architecture Details" define the layers; the
 * quantisation is this library's).  Each e4m3 layer input x enters as
 * e4m3(min(x / s, 448)) with s = amax / 448, a static per-layer scale; the
 * weights carry their own per-layer scale (amax|W| / 448) set at upload.
 * amax[0]: encoder layer-1 output (after ReLU), amax[1]: pooled encoder
 * features [f_a, f_b], amax[2]: head layer-1 output (after ReLU).
 * LOCC_FP8_ENCODER quantises only encoder layer 2's input and uses amax[0];
 * the other two are measured and kept all the same.
 *
 * locc_calibrate measures them: it runs the crop step on the given workload
 * (valid input for locc_detect, device buffers as there) and a float32
 * forward pass of the uploaded (unquantised) weights over the valid pairs,
 * takes the maxima, installs them and, if h_amax_out is not NULL, copies them
 * to host memory.  It synchronises `stream` and may grow the workspace.
 * locc_set_activation_amax installs given maxima (host memory, finite,
 * >= 0; 0 means the activation is always 0).  locc_upload_weights clears
 * them: calibrate again after new weights.
 * Errors: INVALID_ARG (null, bad values), UNSUPPORTED (not an FP8 context),
 * NOT_READY (no shapes or weights), RANGE (during graph capture), BUSY (a
 * captured graph alive, see locc_graph_capture), OOM, HIP. */
LOCC_API locc_status locc_calibrate(locc_ctx* ctx, const locc_object* d_objs, int32_t n_objs, const int32_t* d_pairs,
                           int32_t n_pairs, void* stream, float* h_amax_out);
LOCC_API locc_status locc_set_activation_amax(locc_ctx* ctx, const float* h_amax);

/* Shape library: n_shapes point clouds in their own frames, host memory,
 * copied synchronously; replaces any previous library.  Shape s owns rows
 * h_offsets[s] .. h_offsets[s+1]-1 of h_points, each row
 * (x, y, z, nx, ny, nz) float32.  Offsets start at 0 and never decrease;
 * every shape has at least one point; total < 2^31.  The per-shape
 * axis-aligned box is the min/max of the stored xyz.  Shape ids are 0..n-1.
 * Errors: INVALID_ARG (null, bad offsets, empty shape, non-finite value),
 * RANGE (too many points), BUSY (a captured graph alive, see
 * locc_graph_capture), OOM, HIP. */
LOCC_API locc_status locc_upload_shapes(locc_ctx* ctx, int32_t n_shapes, const int64_t* h_offsets,
                               const float* h_points);

/* The whole path for n_pairs pairs, asynchronous on `stream`.
 *   d_objs    [n_objs] locc_object, device
 *   d_pairs   [n_pairs][2] int32 object indices (i, j), device
 *   d_out     [n_pairs] locc_contact, device, written
 *   d_counts  [n_pairs][2] int32, device, or NULL: members of object i and of
 *             object j inside the crop box before the cap at K (-1 if invalid).
 *             Without it each object's scan stops once its first K members
 *             in stored order are known; the contacts are the same.
 * Device buffers belong to the caller and must stay valid until the stream
 * has run the work.  n_pairs == 0 is a no-op.  The library's own workspace
 * grows on demand (this may allocate; the call then synchronises the
 * device once).
 * Errors (nothing enqueued): INVALID_ARG, NOT_READY, RANGE, OOM, HIP. */
LOCC_API locc_status locc_detect(locc_ctx* ctx, const locc_object* d_objs, int32_t n_objs, const int32_t* d_pairs,
                        int32_t n_pairs, locc_contact* d_out, int32_t* d_counts, void* stream);

/* Crop step only (parity hook).  Same inputs as locc_detect; writes
 *   d_idx     [n_pairs][2][K] int32: the selected point indices of object i
 *             and of object j in stored order, -1 padded (-1 everywhere for
 *             invalid pairs)
 *   d_counts  [n_pairs][2] int32 as in locc_detect (required here). */
LOCC_API locc_status locc_debug_crop(locc_ctx* ctx, const locc_object* d_objs, int32_t n_objs, const int32_t* d_pairs,
                            int32_t n_pairs, int32_t* d_idx, int32_t* d_counts, void* stream);

/* Network intermediates (parity hook).  Runs the whole path and also writes
 *   d_z  [n_pairs][2 h2] float32 pooled features [f_a, f_b] (a = min(i, j))
 *   d_y  [n_pairs][8] float32 raw head output in a's frame
 * Either may be NULL. */
LOCC_API locc_status locc_debug_forward(locc_ctx* ctx, const locc_object* d_objs, int32_t n_objs, const int32_t* d_pairs,
                               int32_t n_pairs, locc_contact* d_out, int32_t* d_counts, float* d_z, float* d_y,
                               void* stream);

/* Work schedule of the BF16 path:
 *   wg_per_cu  workgroups per compute unit of the persistent network kernel
 *              (1 .. 2); grid = CUs x wg_per_cu.  With split = 1 and
 *              wg_per_cu = 1 the encoder+head kernel is a different one: a
 *              workgroup of eight waves per CU with layer 2's weights in LDS,
 *              taking groups of 64 pairs (w, w + CUs, ...), each wave
 *              encoding whole objects; claim and dynamic do not apply to it
 *   claim      pairs a workgroup takes from the queue at a time (1 .. 64)
 *   dynamic    1: pairs are claimed from a device-side atomic queue;
 *              0: static round robin (workgroup w takes claims w, w + grid, ...)
 *   split      0: one persistent kernel does crop, encoder and head;
 *              1: a crop kernel writes bf16 encoder rows to a library
 *              workspace, then the persistent kernel runs encoder and head
 *   crop_unroll  also used by the FP32 path's crop kernel
 *   chunks     split schedule and FP8 (1, 2, 4 or 8): the step is cut into
 *              that many runs of pairs; the crop of run k + 1 runs on a
 *              second stream of the context while the network of run k runs
 *              on the caller's stream (halved while a run would hold fewer
 *              than 256 pairs; always 1 for serving slots)
 * Results do not depend on the schedule: every pair is computed on its own.
 * Errors: INVALID_ARG (null, out of range). */
typedef struct {
  int32_t wg_per_cu;
  int32_t claim;
  int32_t dynamic;
  int32_t split;
  int32_t crop_unroll; /* 2, 4 or 8: a crop wave issues the loads of max(1, crop_unroll / 4)
                          blocks of 256 stored points together (2 and 4 run the same kernel) */
  int32_t chunks;
  int32_t reserved[2]; /* must be 0 */
} locc_schedule;

LOCC_API locc_status locc_set_schedule(locc_ctx* ctx, const locc_schedule* sched);
LOCC_API locc_status locc_get_schedule(const locc_ctx* ctx, locc_schedule* sched);

/* Picks the fastest schedule for this context on the given workload (which
 * must be valid input for locc_detect): every candidate (split or fused,
 * workgroups per CU, claim size, queue kind, crop unroll) is timed with HIP
 * events on `stream` (one warm-up and three timed launches each), the best
 * is installed with locc_set_schedule and returned.  With cache_path set, a
 * text file of earlier results keyed by device, configuration and the
 * power-of-two bucket of n_pairs is read first (a hit skips the timing) and
 * appended to after a miss.  d_out / d_counts receive the outputs of the
 * timed runs; d_counts may be NULL (the candidates are then timed as
 * locc_detect runs without counts, whose scans stop once K members are
 * known).  Synchronises `stream`.  *h_best_ms may be NULL.
 * Errors: as locc_detect, plus HIP. */
LOCC_API locc_status locc_autotune(locc_ctx* ctx, const locc_object* d_objs, int32_t n_objs, const int32_t* d_pairs,
                                   int32_t n_pairs, locc_contact* d_out, int32_t* d_counts, void* stream,
                                   const char* cache_path, locc_schedule* h_best, double* h_best_ms);

/* Grows the library workspace to hold max_pairs pairs (synchronous; may
 * allocate).  Needed before graph capture, which must not allocate.
 * Errors: INVALID_ARG, OOM, HIP. */
LOCC_API locc_status locc_reserve(locc_ctx* ctx, int32_t max_pairs);

/* locc_detect with the pair count read from device memory at run time:
 * *d_n_pairs (int32, device) pairs of d_pairs are processed, clamped to
 * [0, max_pairs]; buffers are sized for max_pairs.  Every kernel of the step
 * is launched for the capacity and idles past the actual count, so the same
 * launch sequence (or captured graph) serves steps whose pair counts differ.
 * The workspace must already hold max_pairs (locc_reserve), else RANGE. */
LOCC_API locc_status locc_detect_device_count(locc_ctx* ctx, const locc_object* d_objs, int32_t n_objs,
                                              const int32_t* d_pairs, const int32_t* d_n_pairs, int32_t max_pairs,
                                              locc_contact* d_out, int32_t* d_counts, void* stream);

/* One simulation step's detect captured once as a HIP graph and replayed.
 * The graph keeps the device pointers given here: the caller updates the
 * objects, pairs and *d_n_pairs in place between launches (for example with
 * asynchronous copies on the launch stream before locc_graph_launch).
 * Capture uses a stream of the library's own, reserves the workspace first,
 * and records no memset node.  The schedule in force at capture time is the
 * one replayed.
 * Lifetime: a graph holds the context's workspace, broad-phase scratch,
 * shape library and (FP8) scales as they were at capture.  While any graph
 * of a context exists, calls that would move or change them are refused and
 * touch nothing: a detect, broad phase, pose-gradient or training call that
 * needs more workspace or scratch (RANGE: reserve enough before capturing),
 * locc_upload_shapes, and on FP8 contexts locc_upload_weights,
 * locc_set_activation_amax and locc_calibrate (BUSY).  FP32 and BF16 weights
 * are rewritten in place, and replays after an upload use the new weights.
 * Destroy every graph of a context before the context.
 * Errors: INVALID_ARG, NOT_READY, OOM, HIP. */
typedef struct locc_graph locc_graph;
LOCC_API locc_status locc_graph_capture(locc_ctx* ctx, const locc_object* d_objs, int32_t n_objs,
                                        const int32_t* d_pairs, const int32_t* d_n_pairs, int32_t max_pairs,
                                        locc_contact* d_out, int32_t* d_counts, locc_graph** out);
LOCC_API locc_status locc_graph_launch(locc_graph* graph, void* stream);
LOCC_API void locc_graph_destroy(locc_graph* graph);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the path of
 * locc_detect (same arguments, same results bit for bit) with its workspace
 * in a fixed 32 MiB device array of the library instead of the context's
 * workspace.  The call allocates nothing and frees nothing; it runs one run
 * of pairs in the static claim order and records no event timing, whatever
 * the context's schedule says.  Largest batch: the workspace per pair is
 * about 16 + 320 + 2K * 32 + 8 h2 bytes (FP32 contexts; 10.6 KB at K = 128,
 * h2 = 256: about 3,100 pairs) or 16 + 320 + 2K * 16 (BF16 split schedule and
 * FP8: 4.4 KB, about 7,500 pairs); the BF16 fused schedule needs none.
 * Every context on a device shares that device's array, and it keeps the
 * last call's contents: calls on one device whose GPU work overlaps in time
 * (other streams, other contexts, other host threads) race on it.  The array
 * is looked up when the context is created (locc_create fails with HIP if
 * that fails).
 * Errors: as locc_detect, and RANGE (more pairs than the array holds; the
 * message gives the largest count for the context), NOT_READY (no array on
 * the context's device). */
LOCC_API locc_status locc_detect_noalloc(locc_ctx* ctx, const locc_object* d_objs, int32_t n_objs,
                                         const int32_t* d_pairs, int32_t n_pairs, locc_contact* d_out,
                                         int32_t* d_counts, void* stream);

/* Pose gradients of the collision logit (Sec. II, collision resolution with
 * an object collision network: contact force and torque directions come from
 * the gradient of the network's output with respect to the poses).  FP32
 * and BF16 contexts.  Runs the crop and the FP32 encoder (recording per object
 * and channel the row of the largest raw second-layer sum, the first on
 * ties), the head backward and the encoder backward at those rows of the
 * second object (the first object's rows are its own stored points and do
 * not depend on the poses), then the chain rule through R_ab = R_a^T R_b,
 * t_ab = R_a^T (p_b - p_a) and the rotation polynomial of the quaternion as
 * given (not renormalised).  The crop selection is piecewise constant in
 * the poses and contributes nothing.
 * BF16 contexts run the encoder in BF16 (the split schedule's kernel,
 * recording the argmax rows and the pooled features) and the rest in FP32
 * as above; d_out then holds the FP32 head's outputs on those pooled
 * features.
 *   d_grad  float32 [n_pairs][14], device, out: d logit / d (p (3), q (4)) of
 *           the caller's first object, then of its second; NaN for an
 *           invalid pair
 *   d_out   [n_pairs] locc_contact (as locc_detect), or NULL
 *   d_argmax_b  uint8 [n_pairs][enc_h2], or NULL: the argmax row (index in
 *           the object's crop) of each channel of the canonical second
 *           object (b = max(i, j)), 255 where it has no rows or the pair
 *           is invalid; a parity hook for ties
 * Asynchronous on `stream`; the workspace grows on demand (synchronous).
 * Errors: INVALID_ARG, NOT_READY, UNSUPPORTED (FP8 contexts), OOM, HIP. */
LOCC_API locc_status locc_pose_gradients(locc_ctx* ctx, const locc_object* d_objs, int32_t n_objs,
                                         const int32_t* d_pairs, int32_t n_pairs, float* d_grad,
                                         locc_contact* d_out, uint8_t* d_argmax_b, void* stream);

/* One training step of an FP32 context on a labelled batch (Sec. III-A: the
 * network is fitted to collision labels of pairs placed by distance
 * manipulation, with binary cross-entropy plus alpha times the squared norm
 * of the shape features, and Adam; the appendix gives alpha = 0.5, lr 1e-3,
 * beta1 0.9, beta2 0.999, eps 1e-8).  Here the shape features are the two
 * pooled crop features of a pair and only the logit output is trained:
 *   loss = (1/B) sum_p [BCE(logit_p, y_p) + alpha ||[f_a, f_b]||^2],
 * B = n_pairs (an invalid pair contributes nothing), then one Adam step on
 * every weight (t counts the steps since the last locc_upload_weights).
 * Runs the crop and the FP32 encoder (argmax rows), the head forward and
 * backward, the weight gradients (every reduction in a fixed order: a step
 * is reproducible bit for bit), Adam, and the repacking of the updated
 * weights; later detect calls use them.
 *   d_labels  float32 [n_pairs], device: 1 for a collision, 0 otherwise
 *   d_loss    float32 [2], device, out: mean cross-entropy, alpha x mean
 *             squared feature norm (of the weights before the step)
 *   d_argmax  uint8 [n_pairs][2][enc_h2], device, or NULL: the argmax rows
 *             used (canonical order; undefined for invalid pairs), a parity
 *             hook for ties
 * Asynchronous on `stream`; workspace and optimiser state grow on demand.
 * Errors: INVALID_ARG (empty batch, null pointers, alpha < 0, lr <= 0, beta
 * outside [0, 1), eps <= 0), NOT_READY, UNSUPPORTED (not FP32), OOM, HIP. */
LOCC_API locc_status locc_train_step(locc_ctx* ctx, const locc_object* d_objs, int32_t n_objs, const int32_t* d_pairs,
                                     const float* d_labels, int32_t n_pairs, float alpha, float lr, float beta1,
                                     float beta2, float eps, float* d_loss, uint8_t* d_argmax, void* stream);

/* Copies the FP32 context's flat weights (which = 0, in the locc_upload_weights
 * order), the last step's gradient (1) or the Adam moments (2: first, 3:
 * second) to host memory (n floats, synchronous).  Errors: INVALID_ARG,
 * NOT_READY, UNSUPPORTED, HIP. */
LOCC_API locc_status locc_get_weights(locc_ctx* ctx, int which, float* h_out, size_t n);

/* Broad phase over environments (Sec. II, footnote on the broad phase:
 * pairs that are far apart are ruled out before the narrow phase; the
 * paper's simulations step many environments at once, and an object pairs
 * only with objects of its own environment).
 *
 *   d_objs         [n_objs] locc_object, device
 *   d_env_offsets  int32 [n_envs + 1], device: environment e holds objects
 *                  d_env_offsets[e] .. d_env_offsets[e + 1] - 1, both
 *                  bounds clamped to [0, n_objs]; an empty or reversed range
 *                  holds none
 *   d_pairs        int32 [capacity][2], device, out: pairs (i, j), i < j,
 *                  listed by environment, then i, then j; may be NULL when
 *                  capacity is 0
 *   d_count        int32 [2], device, out: [0] pairs written =
 *                  min(total, capacity), [1] total (saturated at INT32_MAX)
 *
 * The world box of an object is the axis-aligned hull of its shape's box
 * (component-wise min and max of the stored xyz) after its rotation and
 * translation, computed in float64 as
 *   c_w[i] = ((R[i][0] c0 + R[i][1] c1) + R[i][2] c2) + p_i,
 *   e_w[i] = (|R[i][0]| e0 + |R[i][1]| e1) + |R[i][2]| e2,
 *   lo = c_w - e_w, hi = c_w + e_w
 * with c, e the centre and half extent of the shape box and R the rotation
 * of the quaternion as given; two boxes overlap when their closed intervals
 * meet on all three axes.  An object whose shape id is out of range (or
 * whose pose holds a NaN) is in no pair.  Each environment is tested pair by
 * pair (n (n - 1) / 2 tests for n objects).
 *
 * Asynchronous on `stream`.  The scratch (48 bytes per object, 16 per
 * environment) grows synchronously on first use; under graph capture it
 * must already be large enough (locc_reserve_broad_phase), else RANGE.
 * Errors: INVALID_ARG (negative sizes, null pointers), NOT_READY (no shape
 * library), RANGE, OOM, HIP. */
LOCC_API locc_status locc_broad_phase(locc_ctx* ctx, const locc_object* d_objs, int32_t n_objs,
                                      const int32_t* d_env_offsets, int32_t n_envs, int32_t* d_pairs,
                                      int32_t capacity, int32_t* d_count, void* stream);

/* Grows the broad-phase scratch for n_objs objects and n_envs environments
 * (synchronous; may allocate).  Errors: INVALID_ARG, OOM, HIP. */
LOCC_API locc_status locc_reserve_broad_phase(locc_ctx* ctx, int32_t n_objs, int32_t n_envs);

/* One whole simulation step captured as a HIP graph: locc_broad_phase into
 * d_pairs / d_count, then locc_detect_device_count on those pairs with the
 * device count d_count[0] (results in d_out[0 .. d_count[0]), counts in
 * d_counts, which may be NULL).  The caller updates the objects in place
 * between launches.  Reserves the workspace and the scratch first; records
 * no memset node.  Errors: as locc_broad_phase and locc_graph_capture
 * (capacity must be positive, d_out non-NULL). */
LOCC_API locc_status locc_step_graph_capture(locc_ctx* ctx, const locc_object* d_objs, int32_t n_objs,
                                             const int32_t* d_env_offsets, int32_t n_envs, int32_t* d_pairs,
                                             int32_t capacity, int32_t* d_count, locc_contact* d_out,
                                             int32_t* d_counts, locc_graph** out);

/* Serving.  A server keeps an object table (poses) and the context's shape
 * library and weights resident on the device, and runs a worker thread that
 * batches collision-detection requests continuously: each request brings
 * pose updates for some objects and a list of pairs; requests that arrive
 * while earlier ones are on the GPU join the next batch as soon as a slot
 * (device buffers sized from the memory budget) is free, and up to `slots`
 * batches are in flight at once on separate streams.
 *
 * Batches are formed by scanning the queue in submission order: a request
 * joins the batch if it fits the slot and conflicts (updates an object
 * another one reads or updates, or reads one another updates) with no
 * request in flight, in the batch, or still waiting ahead of it; otherwise
 * it waits, and the objects it touches are closed to the requests behind it
 * for this batch.  A request's pairs therefore see the object table after
 * its own updates and after those of every earlier request that touches
 * the same objects, as in submission order, and its result is the same
 * whether it runs alone or in a mix; requests on disjoint objects may
 * complete out of order.  While a server runs, no other call may use its
 * context.
 *
 *   max_objects        size of the resident object table
 *   max_batch_pairs    pairs per batch; 0 = as many as the budget allows
 *   max_batch_updates  pose updates per batch (>= the largest request's)
 *   slots              batches in flight at once (1 .. 4)
 *   batching           1: continuous batching; 0: one request per launch
 *                      and one slot (the plain per-request path)
 *   max_queued_pairs   host queue limit in pairs (0 = none); submit
 *                      returns BUSY beyond it
 *   hbm_budget_bytes   device memory the server may allocate (object
 *                      table + every slot's buffers and scratch) */
typedef struct {
  int32_t max_objects;
  int32_t max_batch_pairs;
  int32_t max_batch_updates;
  int32_t slots;
  int32_t batching;
  int32_t max_queued_pairs;
  size_t hbm_budget_bytes;
} locc_serve_config;

typedef struct {
  int64_t submitted, completed, batches, pairs_done;
  int64_t max_batch_pairs; /* pairs per batch the budget allowed */
  double busy_ms;          /* wall time with at least one batch in flight */
} locc_serve_stats;

typedef struct locc_server locc_server;

/* Starts a server on ctx with the initial object table h_objects [n_objects]
 * (host, copied).  Errors: INVALID_ARG, NOT_READY (no shapes / weights),
 * OOM (budget too small for one slot of the given sizes), HIP. */
LOCC_API locc_status locc_serve_start(locc_ctx* ctx, const locc_serve_config* cfg, const locc_object* h_objects,
                                      int32_t n_objects, locc_server** out);

/* Queues one request (host arrays, copied): n_upd pose updates
 * (h_upd_ids[k] gets pose h_upd[k]) and n_pairs pairs of object indices.
 * Returns its id.  Errors: INVALID_ARG (null, index out of the table),
 * RANGE (larger than one batch), BUSY (queue full: retry later). */
LOCC_API locc_status locc_serve_submit(locc_server* srv, const int32_t* h_upd_ids, const locc_object* h_upd,
                                       int32_t n_upd, const int32_t* h_pairs, int32_t n_pairs, uint64_t* h_req_id);

/* Queues n_req requests in order under one lock (host arrays, copied):
 * request k holds the updates h_upd_offsets[k] .. h_upd_offsets[k + 1] - 1
 * of h_upd_ids / h_upd and the pairs h_pair_offsets[k] .. h_pair_offsets[k +
 * 1] - 1 of h_pairs (offsets [n_req + 1], non-decreasing, from 0); ids go to
 * h_req_ids [n_req].  For callers that submit many requests at once (and
 * for measuring the server without a per-request call): each request is
 * checked as by locc_serve_submit, and the first one refused stops the call
 * with its status; *h_n_accepted is the number queued before it.
 * Errors: as locc_serve_submit; INVALID_ARG for negative or decreasing
 * offsets. */
LOCC_API locc_status locc_serve_submit_many(locc_server* srv, int32_t n_req, const int32_t* h_upd_offsets,
                                            const int32_t* h_upd_ids, const locc_object* h_upd,
                                            const int32_t* h_pair_offsets, const int32_t* h_pairs,
                                            uint64_t* h_req_ids, int32_t* h_n_accepted);

/* *h_done = 1 once the request has completed; then its contacts and counts
 * are copied to h_out [n_pairs] / h_counts [n_pairs][2] (either may be NULL),
 * *h_latency_ms (may be NULL) is completion minus submission on the host's
 * steady clock, and the request is forgotten.  *h_done = 0 otherwise.
 * Errors: INVALID_ARG (unknown id). */
LOCC_API locc_status locc_serve_poll(locc_server* srv, uint64_t req_id, locc_contact* h_out, int32_t* h_counts,
                                     int32_t* h_done, double* h_latency_ms);

LOCC_API locc_status locc_serve_get_stats(locc_server* srv, locc_serve_stats* h_stats);

/* Finishes every queued request, joins the worker and frees the server's
 * device memory.  Unpolled results are dropped.  NULL is a no-op. */
LOCC_API locc_status locc_serve_stop(locc_server* srv);

/* Per-kernel timing.  While enabled, every kernel the context launches is
 * bracketed by two HIP events recorded on its launch stream; reading
 * synchronises on the recorded events and returns, per kernel name, the
 * number of launches and their summed duration in milliseconds (the same
 * per-dispatch durations a kernel-trace profiler reports, plus event
 * overhead).  locc_profile(ctx, 1) clears the totals and starts recording,
 * locc_profile(ctx, 0) stops.  Kernel names: "crop", "encoder_fp32",
 * "head_fp32" (FP32 per-step path), "fused_bf16" (BF16, one launch),
 * "crop" and "encoder_head_bf16" (BF16 split schedule; "encoder_head_bf16_lds"
 * for its one-workgroup-per-CU kernel), "crop" and
 * "encoder_head_fp8" (LOCC_FP8) or "encoder_fp8_head_bf16"
 * (LOCC_FP8_ENCODER). */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
} locc_kernel_time;

LOCC_API locc_status locc_profile(locc_ctx* ctx, int enable);

/* Copies up to `capacity` entries into h_out (host) and sets *h_count to the
 * number of kernels seen.  Errors: INVALID_ARG, HIP. */
LOCC_API locc_status locc_profile_read(locc_ctx* ctx, locc_kernel_time* h_out, int32_t capacity, int32_t* h_count);

/* Number of invalid pairs seen by all detect calls since the last reset;
 * synchronises `stream`.  reset != 0 clears the counter afterwards. */
LOCC_API locc_status locc_device_errors(locc_ctx* ctx, void* stream, int64_t* h_n_bad, int reset);

#ifdef __cplusplus
}
#endif

#endif /* LOCC_H */
