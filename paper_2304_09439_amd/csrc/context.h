// Library-internal view of a context, shared by the C-ABI and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "fused.h"
#include "locc_internal.h"

struct locc_ctx {
  locc_config cfg{};
  int device = 0;
  int n_cu = 0;
  // shape library
  int32_t n_shapes = 0;
  int64_t n_points = 0;
  locc::ShapeDesc* d_shapes = nullptr;
  float* d_points = nullptr;  // SoA: x, y, z, nx, ny, nz, each n_points floats
  // weights
  float* d_wfp32 = nullptr;
  unsigned char* d_wbf16 = nullptr;
  unsigned char* d_wfp8 = nullptr;
  float* d_wraw = nullptr;         // FP8 and FP32: the flat FP32 weights (calibration, pose gradients)
  float* d_wgrad = nullptr;        // FP32: H1^T [2 h2][hh], H2^T [hh][hh], W2^T [h1][h2], for the pose gradients
  // FP32 training: source index of every packed weight (d_wfp32, d_wgrad) in the flat vector (-1: zero),
  // the gradient and the two Adam moments [3][n], and the step count
  int32_t* d_pack_idx = nullptr;
  int32_t* d_tr_idx = nullptr;
  float* d_train = nullptr;
  int64_t train_t = 0;
  std::vector<float> h_w1b1;       // FP8: W1 then b1 (host), repacked when the activation scale changes
  float fp8_wscale[3] = {1, 1, 1}; // FP8: s_w2, s_h1, s_h2
  float fp8_amax[3] = {0, 0, 0};   // FP8: activation maxima (layer-1 output, pooled z, head layer 1)
  bool have_act_scales = false;
  unsigned int* d_amax = nullptr;  // FP8 calibration accumulator [3]
  bool have_weights = false;
  // fused-kernel schedule and its self-resetting queue (two uint32, zero between launches)
  locc_schedule sched{locc::kFusedWgPerCu, 4, 1, 1, 8, 1, {0, 0}};  // split, claim 4
  unsigned int* d_queue = nullptr;
  // chunked schedules: the crop's stream and the fork / per-run events
  static constexpr int kMaxChunks = 8;
  hipStream_t crop_stream = nullptr;
  hipEvent_t chunk_ev[kMaxChunks + 1] = {};
  hipStream_t capture_stream = nullptr;  // created on first graph capture
  bool capturing = false;
  // graphs captured on this context and not yet destroyed: they hold raw pointers to the workspace, the
  // broad-phase scratch, the shape library and (FP8) scales taken at capture, so nothing of these may move
  // or change while any exists
  int live_graphs = 0;
  // workspace
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
  unsigned long long* d_err = nullptr;
  // broad-phase scratch (world boxes, per-environment counts and starts)
  void* d_bp = nullptr;
  size_t bp_bytes = 0;
  // event timing of each launch (locc_profile)
  struct Pending {
    std::string name;
    hipEvent_t start, stop;
  };
  bool profiling = false;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  std::map<std::string, std::pair<int64_t, double>> totals;

  // the FP8 network kernel: e4m3 on encoder layer 2 (both FP8 precisions), and on head layers 1-2 (LOCC_FP8)
  bool fp8() const { return cfg.precision == LOCC_FP8 || cfg.precision == LOCC_FP8_ENCODER; }
  bool fp8_head() const { return cfg.precision == LOCC_FP8; }

  locc::DeviceLibrary lib() const {
    const float* b = d_points;
    const size_t n = (size_t)n_points;
    return locc::DeviceLibrary{d_shapes, n_shapes, b, b + n, b + 2 * n, b + 3 * n, b + 4 * n, b + 5 * n};
  }
};


namespace locc {

// Records a formatted message for locc_last_error() and returns st.
locc_status fail(locc_status st, const char* fmt, ...);

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return ::locc::fail(e_ == hipErrorOutOfMemory ? LOCC_ERR_OOM : LOCC_ERR_HIP,          \
                          "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
  } while (0)

// Scratch a launch uses: the context's own (grown on demand), or a caller's
// region of at least workspace_bytes() plus its own queue (serving slots).
struct Scratch {
  void* base = nullptr;
  size_t bytes = 0;
  unsigned int* queue = nullptr;
};

// Workspace bytes one launch of n_pairs needs under the current schedule.
size_t workspace_bytes(const locc_ctx* c, int n_pairs);

// Argument checks shared by the detect entry points.
locc_status check_call(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs, int32_t n_pairs);

// The no-allocation entry point's device array: looked up once per device
// (that device current) at context creation; its size in bytes.
locc_status noalloc_setup(int device);
size_t noalloc_scratch_bytes();

// One step of the path for n_pairs pairs (the capacity when n_dev is set),
// enqueued on stream s.
locc_status run_path(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs, int32_t n_pairs,
                     const int32_t* n_dev, locc_contact* out, int32_t* counts, float* z_out, float* y_out,
                     hipStream_t s, const Scratch* own = nullptr);

}  // namespace locc
