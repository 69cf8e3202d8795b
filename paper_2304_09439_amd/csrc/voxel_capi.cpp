// C-ABI of the voxel-embedding variant: resident shapes and weights, the
// shape encoder at upload, and the per-pair predictor launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "context.h"
#include "voxel.h"

using namespace locc;
using namespace locc::vox;

struct locc_voxel_ctx {
  int device = 0;
  bool have_weights = false;
  // shapes (resident; new weights re-encode them)
  int32_t n_shapes = 0;
  int max_points = 0;
  int64_t n_points = 0;
  Shape* d_shapes = nullptr;
  float* d_xyz = nullptr;
  // weights
  float* d_raw = nullptr;
  float* d_packed = nullptr;
  // per-shape results of the encoder
  float* d_emb = nullptr;       // [S][216][16]
  double* d_consts = nullptr;   // [S][4] cell size and margin
  bool have_embeddings = false;
  unsigned long long* d_err = nullptr;
  // predictor workspace (grown on demand)
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
};

namespace {

void free_shapes(locc_voxel_ctx* c) {
  (void)hipFree(c->d_shapes);
  (void)hipFree(c->d_xyz);
  (void)hipFree(c->d_emb);
  (void)hipFree(c->d_consts);
  c->d_shapes = nullptr;
  c->d_xyz = nullptr;
  c->d_emb = nullptr;
  c->d_consts = nullptr;
  c->have_embeddings = false;
}

// Runs the shape encoder over every resident shape (synchronous).
locc_status encode(locc_voxel_ctx* c) {
  c->have_embeddings = false;
  if (!c->have_weights || c->n_shapes == 0) return LOCC_OK;
  const int S = c->n_shapes;
  float* scratch = nullptr;
  const size_t n = encoder_scratch_floats(S, c->n_points);
  HIP_TRY(hipMalloc(&scratch, n * sizeof(float)));
  const EncoderBuffers b = encoder_carve(scratch, S, c->n_points);
  hipError_t e = hipMemset(b.grid, 0, (size_t)S * kH * kCells * sizeof(float));
  if (e == hipSuccess)
    e = launch_encoder(packed_view(c->d_raw, c->d_packed), c->d_shapes, S, c->max_points, c->d_xyz, c->n_points, b,
                       c->d_emb, c->d_consts, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  (void)hipFree(scratch);
  if (e != hipSuccess) return fail(LOCC_ERR_HIP, "shape encoder: %s", hipGetErrorString(e));
  c->have_embeddings = true;
  return LOCC_OK;
}

}  // namespace

extern "C" {

size_t locc_voxel_weight_count(void) { return kWeightCount; }

locc_status locc_voxel_create(int device, locc_voxel_ctx** out) {
  if (!out) return fail(LOCC_ERR_INVALID_ARG, "null output");
  *out = nullptr;
  int n_dev = 0;
  HIP_TRY(hipGetDeviceCount(&n_dev));
  if (device < 0 || device >= n_dev) return fail(LOCC_ERR_INVALID_ARG, "device %d of %d", device, n_dev);
  HIP_TRY(hipSetDevice(device));
  locc_voxel_ctx* c = new locc_voxel_ctx();
  c->device = device;
  hipError_t e = hipMalloc(&c->d_err, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(c->d_err, 0, sizeof(unsigned long long));
  if (e != hipSuccess) {
    locc_voxel_destroy(c);
    return fail(LOCC_ERR_HIP, "error counter: %s", hipGetErrorString(e));
  }
  *out = c;
  return LOCC_OK;
}

void locc_voxel_destroy(locc_voxel_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  free_shapes(c);
  (void)hipFree(c->d_raw);
  (void)hipFree(c->d_packed);
  (void)hipFree(c->d_err);
  (void)hipFree(c->d_ws);
  delete c;
}

locc_status locc_voxel_upload_weights(locc_voxel_ctx* c, const float* h, size_t n) {
  if (!c || !h) return fail(LOCC_ERR_INVALID_ARG, "null context or weights");
  if (n != kWeightCount) return fail(LOCC_ERR_INVALID_ARG, "expected %zu weights, got %zu", kWeightCount, n);
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(h[i])) return fail(LOCC_ERR_INVALID_ARG, "weight %zu is not finite", i);
  std::vector<float> packed(packed_floats());
  pack_transposed(h, packed.data());
  HIP_TRY(hipSetDevice(c->device));
  c->have_weights = false;
  if (!c->d_raw) HIP_TRY(hipMalloc(&c->d_raw, n * sizeof(float)));
  if (!c->d_packed) HIP_TRY(hipMalloc(&c->d_packed, packed.size() * sizeof(float)));
  HIP_TRY(hipMemcpy(c->d_raw, h, n * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->d_packed, packed.data(), packed.size() * sizeof(float), hipMemcpyHostToDevice));
  c->have_weights = true;
  return encode(c);
}

locc_status locc_voxel_upload_shapes(locc_voxel_ctx* c, int32_t n_shapes, const int64_t* off, const float* pts) {
  if (!c || !off || !pts) return fail(LOCC_ERR_INVALID_ARG, "null context, offsets or points");
  if (n_shapes <= 0) return fail(LOCC_ERR_INVALID_ARG, "n_shapes=%d", n_shapes);
  if (off[0] != 0) return fail(LOCC_ERR_INVALID_ARG, "offsets[0]=%lld, must be 0", (long long)off[0]);
  int max_points = 0;
  for (int s = 0; s < n_shapes; ++s) {
    const int64_t n = off[s + 1] - off[s];
    if (n <= 0) return fail(LOCC_ERR_INVALID_ARG, "shape %d has %lld points", s, (long long)n);
    if (n > kMaxPoints) return fail(LOCC_ERR_RANGE, "shape %d has %lld points (max %d)", s, (long long)n, kMaxPoints);
    max_points = n > max_points ? (int)n : max_points;
  }
  const int64_t total = off[n_shapes];
  if (total >= (int64_t)INT32_MAX) return fail(LOCC_ERR_RANGE, "%lld points in total", (long long)total);
  std::vector<float> xyz((size_t)total * 3);
  std::vector<Shape> shapes(n_shapes);
  for (int s = 0; s < n_shapes; ++s) {
    Shape d{};
    d.off = (int32_t)off[s];
    d.n = (int32_t)(off[s + 1] - off[s]);
    for (int k = 0; k < 3; ++k) {
      d.lo[k] = INFINITY;
      d.hi[k] = -INFINITY;
    }
    for (int64_t r = off[s]; r < off[s + 1]; ++r) {
      const float* row = pts + r * 6;
      for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(row[k]))
          return fail(LOCC_ERR_INVALID_ARG, "shape %d point %lld: non-finite value", s, (long long)(r - off[s]));
        xyz[(size_t)k * total + r] = row[k];
        d.lo[k] = row[k] < d.lo[k] ? row[k] : d.lo[k];
        d.hi[k] = row[k] > d.hi[k] ? row[k] : d.hi[k];
      }
    }
    shapes[s] = d;
  }
  HIP_TRY(hipSetDevice(c->device));
  free_shapes(c);
  c->n_shapes = 0;
  HIP_TRY(hipMalloc(&c->d_shapes, sizeof(Shape) * n_shapes));
  HIP_TRY(hipMalloc(&c->d_xyz, sizeof(float) * xyz.size()));
  HIP_TRY(hipMalloc(&c->d_emb, sizeof(float) * (size_t)n_shapes * kCells * kF));
  HIP_TRY(hipMalloc(&c->d_consts, sizeof(double) * (size_t)n_shapes * 4));
  HIP_TRY(hipMemcpy(c->d_shapes, shapes.data(), sizeof(Shape) * n_shapes, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->d_xyz, xyz.data(), sizeof(float) * xyz.size(), hipMemcpyHostToDevice));
  c->n_shapes = n_shapes;
  c->max_points = max_points;
  c->n_points = total;
  return encode(c);
}

locc_status locc_voxel_embeddings(locc_voxel_ctx* c, float* d_out, void* stream) {
  if (!c || !d_out) return fail(LOCC_ERR_INVALID_ARG, "null context or output");
  if (!c->have_embeddings) return fail(LOCC_ERR_NOT_READY, "no weights or no shapes uploaded");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipMemcpyAsync(d_out, c->d_emb, sizeof(float) * (size_t)c->n_shapes * kCells * kF,
                         hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  return LOCC_OK;
}

locc_status locc_voxel_detect(locc_voxel_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs,
                              int32_t n_pairs, float* out, int32_t* counts, float* pooled, void* stream) {
  if (!c) return fail(LOCC_ERR_INVALID_ARG, "null context");
  if (n_objs < 0 || n_pairs < 0)
    return fail(LOCC_ERR_INVALID_ARG, "negative count (n_objs=%d, n_pairs=%d)", n_objs, n_pairs);
  if (n_pairs > 0 && (!objs || !pairs || !out)) return fail(LOCC_ERR_INVALID_ARG, "null objects, pairs or output");
  if (!c->have_embeddings) return fail(LOCC_ERR_NOT_READY, "no weights or no shapes uploaded");
  if (n_pairs == 0) return LOCC_OK;
  HIP_TRY(hipSetDevice(c->device));
  PairArgs a{};
  a.objs = objs;
  a.n_objs = n_objs;
  a.pairs = pairs;
  a.n_pairs = n_pairs;
  a.shapes = c->d_shapes;
  a.n_shapes = c->n_shapes;
  a.consts = c->d_consts;
  a.emb = c->d_emb;
  a.w = packed_view(c->d_raw, c->d_packed);
  a.out = out;
  a.counts = counts;
  a.pooled = pooled;
  a.err = c->d_err;
  const size_t need = pair_workspace_bytes(n_pairs);
  if (need > c->ws_bytes) {  // synchronous growth
    if (c->d_ws) HIP_TRY(hipFree(c->d_ws));
    c->d_ws = nullptr;
    c->ws_bytes = 0;
    HIP_TRY(hipMalloc(&c->d_ws, need + need / 4));
    c->ws_bytes = need + need / 4;
  }
  pair_workspace_carve(c->d_ws, n_pairs, a);
  HIP_TRY(launch_pairs(a, static_cast<hipStream_t>(stream)));
  return LOCC_OK;
}

locc_status locc_voxel_device_errors(locc_voxel_ctx* c, void* stream, int64_t* n_bad, int reset) {
  if (!c || !n_bad) return fail(LOCC_ERR_INVALID_ARG, "null context or output");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  unsigned long long v = 0;
  HIP_TRY(hipMemcpy(&v, c->d_err, sizeof v, hipMemcpyDeviceToHost));
  *n_bad = (int64_t)v;
  if (reset) HIP_TRY(hipMemset(c->d_err, 0, sizeof(unsigned long long)));
  return LOCC_OK;
}

}  // extern "C"
