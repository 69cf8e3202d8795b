// C-ABI of the LOCC library: argument checks, resident shape library and
// weights, workspace, and the launch sequence of the path.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "context.h"
#include "grad.h"

using namespace locc;

namespace locc {

thread_local std::string g_last_error;
thread_local LaunchTiming g_launch_timing;

locc_status fail(locc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

}  // namespace locc

namespace {

bool widths_supported(int h1, int h2, int hh) {
  return (h1 == 64 && h2 == 128 && hh == 256) || (h1 == 128 && h2 == 256 && hh == 512);
}

size_t weight_floats(int h1, int h2, int hh) {
  return (size_t)h1 * 6 + h1 + (size_t)h2 * h1 + h2 + (size_t)hh * 2 * h2 + hh + (size_t)hh * hh + hh +
         (size_t)8 * hh + 8;
}

}  // namespace


namespace {

hipError_t take_event(locc_ctx* c, hipEvent_t* e) {
  if (!c->event_pool.empty()) {
    *e = c->event_pool.back();
    c->event_pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Launch `launch()` on stream s; while profiling is on, its kernels carry a
// start and a stop event (from the start of the first to the end of the last).
template <class F>
hipError_t timed(locc_ctx* c, const char* name, hipStream_t s, F&& launch) {
  if (!c->profiling) return launch();
  locc_ctx::Pending pd{name, nullptr, nullptr};
  hipError_t e = take_event(c, &pd.start);
  if (e == hipSuccess) e = take_event(c, &pd.stop);
  if (e != hipSuccess) return e;
  g_launch_timing = LaunchTiming{pd.start, pd.stop};
  e = launch();
  const bool launched = g_launch_timing.start == nullptr;
  g_launch_timing = LaunchTiming{};
  if (e != hipSuccess) return e;
  if (!launched) {  // nothing to run: an empty interval
    e = hipEventRecord(pd.start, s);
    if (e == hipSuccess) e = hipEventRecord(pd.stop, s);
    if (e != hipSuccess) return e;
  }
  c->pending.push_back(pd);
  return hipSuccess;
}

hipError_t drain_profile(locc_ctx* c) {
  for (auto& pd : c->pending) {
    hipError_t e = hipEventSynchronize(pd.stop);
    if (e != hipSuccess) return e;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, pd.start, pd.stop);
    if (e != hipSuccess) return e;
    auto& t = c->totals[pd.name];
    t.first += 1;
    t.second += ms;
    c->event_pool.push_back(pd.start);
    c->event_pool.push_back(pd.stop);
  }
  c->pending.clear();
  return hipSuccess;
}

locc_status ensure_workspace(locc_ctx* c, size_t bytes) {
  if (bytes <= c->ws_bytes) return LOCC_OK;
  if (c->capturing)
    return fail(LOCC_ERR_RANGE, "workspace of %zu bytes too small for %zu during graph capture", c->ws_bytes, bytes);
  if (c->live_graphs > 0)
    return fail(LOCC_ERR_RANGE, "workspace of %zu bytes too small for %zu while %d captured graph(s) use it: "
                "reserve before capturing, or destroy the graphs first", c->ws_bytes, bytes, c->live_graphs);
  if (c->d_ws) HIP_TRY(hipFree(c->d_ws));  // implicit device synchronisation
  c->d_ws = nullptr;
  c->ws_bytes = 0;
  size_t want = bytes + bytes / 4;
  HIP_TRY(hipMalloc(&c->d_ws, want));
  c->ws_bytes = want;
  return LOCC_OK;
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// Workspace of one launch, carved from the context's buffer:
//   FP32 path: PairMeta [P], float rows [P][2K][8], pooled features z [P][2 h2]
//   BF16 split and FP8: PairMeta [P], bf16 rows [P][2K][8]
//   BF16 fused: nothing
// followed, for every path that runs the crop kernel, by the pair set-up
// records [P].
struct Workspace {
  PairMeta* meta = nullptr;
  float* rows = nullptr;
  float* z = nullptr;
  unsigned short* rows_bf16 = nullptr;
  void* setup = nullptr;  // pair set-up records of the crop kernel
};

}  // namespace

size_t locc::workspace_bytes(const locc_ctx* c, int n_pairs) {
  const size_t P = (size_t)n_pairs;
  const size_t meta = align256(P * sizeof(PairMeta));
  const size_t setup = align256(P * kPairSetupBytes);
  if (c->cfg.precision == LOCC_FP32)
    return meta + align256(P * 2 * c->cfg.K * kRowFloats * sizeof(float)) +
           align256(P * 2 * c->cfg.enc_h2 * sizeof(float)) + setup;
  if (c->sched.split || c->fp8())
    return meta + align256(P * 2 * c->cfg.K * 8 * sizeof(unsigned short)) + setup;
  return 0;
}

namespace {

locc_status carve(locc_ctx* c, int n_pairs, Workspace* w, const Scratch* own) {
  const size_t bytes = workspace_bytes(c, n_pairs);
  if (bytes == 0) return LOCC_OK;
  char* b = nullptr;
  if (own) {
    if (own->bytes < bytes) return fail(LOCC_ERR_RANGE, "scratch of %zu bytes, %zu needed", own->bytes, bytes);
    b = static_cast<char*>(own->base);
  } else {
    locc_status st = ensure_workspace(c, bytes);
    if (st != LOCC_OK) return st;
    b = static_cast<char*>(c->d_ws);
  }
  const size_t P = (size_t)n_pairs;
  w->meta = reinterpret_cast<PairMeta*>(b);
  b += align256(P * sizeof(PairMeta));
  if (c->cfg.precision == LOCC_FP32) {
    w->rows = reinterpret_cast<float*>(b);
    b += align256(P * 2 * c->cfg.K * kRowFloats * sizeof(float));
    w->z = reinterpret_cast<float*>(b);
    b += align256(P * 2 * c->cfg.enc_h2 * sizeof(float));
  } else {
    w->rows_bf16 = reinterpret_cast<unsigned short*>(b);
    b += align256(P * 2 * c->cfg.K * 8 * sizeof(unsigned short));
  }
  w->setup = b;
  return LOCC_OK;
}

}  // namespace

locc_status locc::check_call(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs,
                             int32_t n_pairs) {
  if (!c) return fail(LOCC_ERR_INVALID_ARG, "null context");
  if (n_objs < 0 || n_pairs < 0) return fail(LOCC_ERR_INVALID_ARG, "negative count (n_objs=%d, n_pairs=%d)",
                                             n_objs, n_pairs);
  if (n_pairs > 0 && (!objs || !pairs)) return fail(LOCC_ERR_INVALID_ARG, "null objects or pairs");
  if (!c->d_shapes) return fail(LOCC_ERR_NOT_READY, "no shape library uploaded");
  if (!c->have_weights) return fail(LOCC_ERR_NOT_READY, "no weights uploaded");
  if (c->fp8() && !c->have_act_scales)
    return fail(LOCC_ERR_NOT_READY, "FP8: no activation scales (locc_calibrate or locc_set_activation_amax)");
  return LOCC_OK;
}

namespace {

// Scale of an fp8 activation with maximum amax (448 is e4m3's largest finite value).
float fp8_scale(float amax) { return amax > 0.f ? amax / 448.f : 1.f; }

int fused_grid(const locc_ctx* c, int n_pairs) {
  const int claim = c->sched.claim;
  const int tiles = (n_pairs + claim - 1) / claim;
  const int grid = c->n_cu * c->sched.wg_per_cu;
  return tiles < grid ? tiles : grid;
}

}  // namespace

locc_status locc::run_path(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs,
                           int32_t n_pairs, const int32_t* n_dev, locc_contact* out, int32_t* counts, float* z_out,
                           float* y_out, hipStream_t s, const Scratch* own) {
  if (n_pairs == 0) return LOCC_OK;
  Workspace w{};
  locc_status st = carve(c, n_pairs, &w, own);
  if (st != LOCC_OK) return st;
  HIP_TRY(hipSetDevice(c->device));
  const int unroll = c->sched.crop_unroll;
  if (c->cfg.precision == LOCC_FP32) {
    CropArgs ca{objs, n_objs, pairs, n_pairs, n_dev, c->lib(), c->cfg.K, c->cfg.pad_m,
                nullptr, counts, w.meta, w.rows, nullptr, c->d_err, w.setup};
    HIP_TRY(timed(c, "crop", s, [&] { return launch_crop(ca, s, unroll); }));
    const Fp32Net net = fp32_view(c->d_wfp32, c->cfg.enc_h1, c->cfg.enc_h2, c->cfg.head_h);
    NetArgs na{w.rows, w.meta, objs, n_pairs, n_dev, c->cfg.K, z_out ? z_out : w.z, y_out, out};
    HIP_TRY(timed(c, "encoder_fp32", s, [&] { return launch_encoder_fp32(net, na, c->n_cu, s); }));
    HIP_TRY(timed(c, "head_fp32", s, [&] { return launch_head_fp32(net, na, s); }));
    return LOCC_OK;
  }
  const int h1 = c->cfg.enc_h1, h2 = c->cfg.enc_h2, hh = c->cfg.head_h;
  const int K = c->cfg.K;
  if (c->fp8() || c->sched.split) {
    // Crop kernel, then the persistent encoder + head kernel.  With chunks > 1
    // the step is cut into that many runs of pairs: the crop of run k + 1 (on
    // the context's second stream) overlaps the network of run k (on s).
    int C = own ? 1 : c->sched.chunks;
    while (C > 1 && n_pairs / C < 256) C >>= 1;
    const int L = (n_pairs + C - 1) / C;
    hipStream_t cs = C > 1 ? c->crop_stream : s;
    if (C > 1) {
      HIP_TRY(hipEventRecord(c->chunk_ev[0], s));
      HIP_TRY(hipStreamWaitEvent(cs, c->chunk_ev[0], 0));
    }
    for (int k = 0; k < C; ++k) {
      const int s0 = k * L;
      const int len = n_pairs - s0 < L ? n_pairs - s0 : L;
      if (len <= 0) break;
      PairMeta* meta = w.meta + s0;
      unsigned short* rows = w.rows_bf16 + (size_t)s0 * 2 * K * 8;
      CropArgs ca{objs, n_objs, pairs + 2 * (size_t)s0, len, n_dev, c->lib(), K, c->cfg.pad_m,
                  nullptr, counts ? counts + 2 * (size_t)s0 : nullptr, meta, nullptr, rows, c->d_err,
                  static_cast<char*>(w.setup) + (size_t)s0 * kPairSetupBytes, s0};
      HIP_TRY(timed(c, "crop", cs, [&] { return launch_crop(ca, cs, unroll); }));
      if (C > 1) {
        HIP_TRY(hipEventRecord(c->chunk_ev[k + 1], cs));
        HIP_TRY(hipStreamWaitEvent(s, c->chunk_ev[k + 1], 0));
      }
      const int grid = fused_grid(c, len);
      if (c->fp8()) {
        Fp8Args fa{};
        fa.objs = objs;
        fa.n_pairs = len;
        fa.n_pairs_dev = n_dev;
        fa.dev_base = s0;
        fa.K = K;
        fp8_bind(fa, c->d_wfp8, h1, h2, hh, c->fp8_head());
        fa.s_w2 = c->fp8_wscale[0];
        fa.s_h1 = c->fp8_wscale[1];
        fa.s_h2 = c->fp8_wscale[2];
        fa.s_h1in = fp8_scale(c->fp8_amax[0]);
        fa.s_z = fp8_scale(c->fp8_amax[1]);
        fa.s_g1 = fp8_scale(c->fp8_amax[2]);
        fa.rows_bf16 = rows;
        fa.meta = meta;
        fa.out = out + s0;
        fa.z_dbg = z_out ? z_out + (size_t)s0 * 2 * h2 : nullptr;
        fa.y_dbg = y_out ? y_out + (size_t)s0 * 8 : nullptr;
        fa.queue = own ? own->queue : c->d_queue;
        fa.claim = c->sched.claim;
        fa.dynamic = c->sched.dynamic;
        const bool h8 = c->fp8_head();
        HIP_TRY(timed(c, h8 ? "encoder_head_fp8" : "encoder_fp8_head_bf16", s,
                      [&] { return launch_encoder_head_fp8(fa, h1, h2, hh, h8, grid, s); }));
      } else {
        FusedArgs fa{};
        fa.objs = objs;
        fa.n_objs = n_objs;
        fa.n_pairs = len;
        fa.n_pairs_dev = n_dev;
        fa.dev_base = s0;
        fa.lib = c->lib();
        fa.K = K;
        fa.pad = c->cfg.pad_m;
        bf16_bind(fa, c->d_wbf16, h1, h2, hh);
        fa.out = out + s0;
        fa.z_dbg = z_out ? z_out + (size_t)s0 * 2 * h2 : nullptr;
        fa.y_dbg = y_out ? y_out + (size_t)s0 * 8 : nullptr;
        fa.rows_bf16 = rows;
        fa.meta = meta;
        fa.queue = own ? own->queue : c->d_queue;
        fa.claim = c->sched.claim;
        fa.dynamic = c->sched.dynamic;
        if (c->sched.wg_per_cu == 1) {  // one workgroup of eight waves per CU, W2 in LDS
          const int groups = (len + 63) / 64;
          const int g8 = groups < c->n_cu ? groups : c->n_cu;
          HIP_TRY(timed(c, "encoder_head_bf16_lds", s,
                        [&] { return launch_encoder_head_bf16_lds(fa, h1, h2, hh, g8, false, s); }));
        } else {
          HIP_TRY(timed(c, "encoder_head_bf16", s,
                        [&] { return launch_fused_bf16(fa, h1, h2, hh, grid, true, s); }));
        }
      }
    }
    return LOCC_OK;
  }
  FusedArgs fa{};
  fa.objs = objs;
  fa.n_objs = n_objs;
  fa.pairs = pairs;
  fa.n_pairs = n_pairs;
  fa.n_pairs_dev = n_dev;
  fa.lib = c->lib();
  fa.K = K;
  fa.pad = c->cfg.pad_m;
  bf16_bind(fa, c->d_wbf16, h1, h2, hh);
  fa.out = out;
  fa.counts = counts;
  fa.z_dbg = z_out;
  fa.y_dbg = y_out;
  fa.err_counter = c->d_err;
  fa.queue = own ? own->queue : c->d_queue;
  fa.claim = c->sched.claim;
  fa.dynamic = c->sched.dynamic;
  const int grid = fused_grid(c, n_pairs);
  HIP_TRY(timed(c, "fused_bf16", s, [&] { return launch_fused_bf16(fa, h1, h2, hh, grid, false, s); }));
  return LOCC_OK;
}

namespace {

locc_status check_schedule(const locc_schedule* sc) {
  if (sc->wg_per_cu < 1 || sc->wg_per_cu > kFusedWgPerCu)
    return fail(LOCC_ERR_INVALID_ARG, "wg_per_cu=%d: must be 1..%d", sc->wg_per_cu, kFusedWgPerCu);
  if (sc->claim < 1 || sc->claim > 64) return fail(LOCC_ERR_INVALID_ARG, "claim=%d: must be 1..64", sc->claim);
  if (sc->dynamic != 0 && sc->dynamic != 1) return fail(LOCC_ERR_INVALID_ARG, "dynamic must be 0 or 1");
  if (sc->split != 0 && sc->split != 1) return fail(LOCC_ERR_INVALID_ARG, "split must be 0 or 1");
  if (sc->crop_unroll != 2 && sc->crop_unroll != 4 && sc->crop_unroll != 8)
    return fail(LOCC_ERR_INVALID_ARG, "crop_unroll=%d: must be 2, 4 or 8", sc->crop_unroll);
  if (sc->chunks != 1 && sc->chunks != 2 && sc->chunks != 4 && sc->chunks != 8)
    return fail(LOCC_ERR_INVALID_ARG, "chunks=%d: must be 1, 2, 4 or 8", sc->chunks);
  if (sc->reserved[0] || sc->reserved[1])
    return fail(LOCC_ERR_INVALID_ARG, "reserved fields must be 0");
  return LOCC_OK;
}

// ------------------------------------------------------------------ autotuner
std::string tune_key(const locc_ctx* c, int n_pairs) {
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, c->device);
  int bucket = 0;
  while ((1 << (bucket + 1)) <= n_pairs) ++bucket;
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s/cu%d/K%d/h%d-%d-%d/p%d/pairs2^%d", prop.gcnArchName, c->n_cu, c->cfg.K,
                c->cfg.enc_h1, c->cfg.enc_h2, c->cfg.head_h, c->cfg.precision, bucket);
  for (char* q = buf; *q; ++q)
    if (*q == ' ') *q = '_';
  return buf;
}

bool tune_cache_lookup(const char* path, const std::string& key, locc_schedule* sc, double* ms) {
  if (!path) return false;
  std::FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char k[256];
  locc_schedule t{};
  double m = 0;
  bool hit = false;
  while (std::fscanf(f, "%255s %d %d %d %d %d %d %lf", k, &t.wg_per_cu, &t.claim, &t.dynamic, &t.split,
                     &t.crop_unroll, &t.chunks, &m) == 8) {
    if (key == k && check_schedule(&t) == LOCC_OK) {
      *sc = t;
      *ms = m;
      hit = true;
    }
  }
  std::fclose(f);
  return hit;
}

void tune_cache_store(const char* path, const std::string& key, const locc_schedule& sc, double ms) {
  if (!path) return;
  std::FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d %d %d %.6f\n", key.c_str(), sc.wg_per_cu, sc.claim, sc.dynamic, sc.split,
               sc.crop_unroll, sc.chunks, ms);
  std::fclose(f);
}

std::vector<locc_schedule> tune_candidates(const locc_ctx* c) {
  std::vector<locc_schedule> out;
  if (c->cfg.precision == LOCC_FP32) {
    for (int u : {2, 4, 8}) out.push_back(locc_schedule{kFusedWgPerCu, 4, 1, 0, u, 1, {0, 0}});
    return out;
  }
  for (int split : {1, 0})
    for (int wg : {2, 1})
      for (int claim : {4, 16})
        for (int dyn : {1, 0})
          for (int u : {4, 8})
            for (int chunks : {1, 2, 4}) {
              if (!split && (u != 8 || chunks != 1)) continue;  // the fused kernel: fixed scan unroll, no chunks
              if (!split && c->fp8()) continue;  // FP8 runs split only
              out.push_back(locc_schedule{wg, claim, dyn, split, u, chunks, {0, 0}});
            }
  return out;
}

}  // namespace

struct locc_graph {
  locc_ctx* ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

const char* locc_version(void) { return "locc 0.1.0 gfx950"; }

const char* locc_last_error(void) { return g_last_error.c_str(); }

locc_status locc_create(const locc_config* cfg, int device, locc_ctx** out) {
  if (!cfg || !out) return fail(LOCC_ERR_INVALID_ARG, "null cfg or out");
  *out = nullptr;
  if (cfg->K < 32 || cfg->K > kMaxK || cfg->K % 32 != 0)
    return fail(LOCC_ERR_INVALID_ARG, "K=%d: must be a multiple of 32 in [32, %d]", cfg->K, kMaxK);
  if (!(cfg->pad_m >= 0.0) || !std::isfinite(cfg->pad_m))
    return fail(LOCC_ERR_INVALID_ARG, "pad_m must be finite and >= 0");
  if (cfg->reserved != 0) return fail(LOCC_ERR_INVALID_ARG, "reserved field must be 0");
  if (cfg->precision < LOCC_FP32 || cfg->precision > LOCC_FP8_ENCODER)
    return fail(LOCC_ERR_INVALID_ARG, "unknown precision %d", cfg->precision);
  if (!widths_supported(cfg->enc_h1, cfg->enc_h2, cfg->head_h))
    return fail(LOCC_ERR_UNSUPPORTED, "widths (%d, %d, %d) not compiled in", cfg->enc_h1, cfg->enc_h2,
                cfg->head_h);
  if (device < 0) return fail(LOCC_ERR_INVALID_ARG, "device %d", device);
  int n_dev = 0;
  HIP_TRY(hipGetDeviceCount(&n_dev));
  if (device >= n_dev) return fail(LOCC_ERR_INVALID_ARG, "device %d of %d", device, n_dev);
  HIP_TRY(hipSetDevice(device));
  int n_cu = 0;
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device));
  locc_ctx* c = new locc_ctx();
  c->cfg = *cfg;
  c->device = device;
  c->n_cu = n_cu;
  hipError_t e = hipMalloc(&c->d_err, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(c->d_err, 0, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMalloc(&c->d_queue, 2 * sizeof(unsigned int));
  if (e == hipSuccess) e = hipMemset(c->d_queue, 0, 2 * sizeof(unsigned int));
  if (e == hipSuccess && (cfg->precision == LOCC_FP8 || cfg->precision == LOCC_FP8_ENCODER))
    e = hipMalloc(&c->d_amax, 3 * sizeof(unsigned int));
  if (e == hipSuccess && cfg->precision != LOCC_FP32) {
    e = hipStreamCreateWithFlags(&c->crop_stream, hipStreamNonBlocking);
    for (int k = 0; e == hipSuccess && k <= locc_ctx::kMaxChunks; ++k)
      e = hipEventCreateWithFlags(&c->chunk_ev[k], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    locc_destroy(c);
    return fail(LOCC_ERR_HIP, "error counter: %s", hipGetErrorString(e));
  }
  const locc_status ns = noalloc_setup(device);   // this device's copy of the no-allocation scratch
  if (ns != LOCC_OK) {
    locc_destroy(c);
    return ns;
  }
  *out = c;
  return LOCC_OK;
}

void locc_destroy(locc_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)drain_profile(c);
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  (void)hipFree(c->d_shapes);
  (void)hipFree(c->d_points);
  (void)hipFree(c->d_wfp32);
  (void)hipFree(c->d_wbf16);
  (void)hipFree(c->d_wfp8);
  (void)hipFree(c->d_wraw);
  (void)hipFree(c->d_wgrad);
  (void)hipFree(c->d_pack_idx);
  (void)hipFree(c->d_tr_idx);
  (void)hipFree(c->d_train);
  (void)hipFree(c->d_amax);
  (void)hipFree(c->d_queue);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  if (c->crop_stream) (void)hipStreamDestroy(c->crop_stream);
  for (hipEvent_t e : c->chunk_ev)
    if (e) (void)hipEventDestroy(e);
  (void)hipFree(c->d_ws);
  (void)hipFree(c->d_bp);
  (void)hipFree(c->d_err);
  delete c;
}

locc_status locc_upload_weights(locc_ctx* c, const float* h, size_t n) {
  if (!c || !h) return fail(LOCC_ERR_INVALID_ARG, "null context or weights");
  const int h1 = c->cfg.enc_h1, h2 = c->cfg.enc_h2, hh = c->cfg.head_h;
  const size_t want = weight_floats(h1, h2, hh);
  if (n != want) return fail(LOCC_ERR_INVALID_ARG, "weights: %zu floats given, %zu expected", n, want);
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(h[k])) return fail(LOCC_ERR_INVALID_ARG, "weights: non-finite value at %zu", k);
  if (c->fp8() && c->live_graphs > 0)
    return fail(LOCC_ERR_BUSY, "FP8 weights: %d captured graph(s) hold the current scales; destroy them first",
                c->live_graphs);
  const float* W1 = h;
  const float* b1 = W1 + (size_t)h1 * 6;
  const float* W2 = b1 + h1;
  const float* b2 = W2 + (size_t)h2 * h1;
  const float* H1 = b2 + h2;
  const float* c1 = H1 + (size_t)hh * 2 * h2;
  const float* H2 = c1 + hh;
  const float* c2 = H2 + (size_t)hh * hh;
  const float* H3 = c2 + hh;
  const float* c3 = H3 + (size_t)8 * hh;
  std::vector<float> pack(fp32_pack_floats(h1, h2, hh));
  fp32_pack(W1, b1, W2, b2, H1, c1, H2, c2, H3, c3, h1, h2, hh, pack.data());
  HIP_TRY(hipSetDevice(c->device));
  if (!c->d_wfp32) HIP_TRY(hipMalloc(&c->d_wfp32, pack.size() * sizeof(float)));
  HIP_TRY(hipMemcpy(c->d_wfp32, pack.data(), pack.size() * sizeof(float), hipMemcpyHostToDevice));
  if (c->cfg.precision == LOCC_FP32 || c->cfg.precision == LOCC_BF16) {
    // the pose gradients read the plain weights, the two head matrices transposed and W2 transposed
    std::vector<float> t((size_t)2 * h2 * hh + (size_t)hh * hh + (size_t)h1 * h2);
    for (int o = 0; o < hh; ++o)
      for (int k = 0; k < 2 * h2; ++k) t[(size_t)k * hh + o] = H1[(size_t)o * 2 * h2 + k];
    float* t2 = t.data() + (size_t)2 * h2 * hh;
    for (int o = 0; o < hh; ++o)
      for (int k = 0; k < hh; ++k) t2[(size_t)k * hh + o] = H2[(size_t)o * hh + k];
    float* t3 = t2 + (size_t)hh * hh;
    for (int c = 0; c < h2; ++c)
      for (int k = 0; k < h1; ++k) t3[(size_t)k * h2 + c] = W2[(size_t)c * h1 + k];
    if (!c->d_wraw) HIP_TRY(hipMalloc(&c->d_wraw, n * sizeof(float)));
    if (!c->d_wgrad) HIP_TRY(hipMalloc(&c->d_wgrad, t.size() * sizeof(float)));
    HIP_TRY(hipMemcpy(c->d_wraw, h, n * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d_wgrad, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice));
  }
  if (c->cfg.precision == LOCC_FP32) {
    // training: where each packed value comes from (the packing is positional, so packing the
    // vector of indices + 1 gives the map; floats hold these integers exactly)
    std::vector<float> ix(n);
    for (size_t k = 0; k < n; ++k) ix[k] = (float)(k + 1);
    const float* X = ix.data();
    const float* xb1 = X + (b1 - W1);
    std::vector<float> pk(pack.size());
    fp32_pack(X, xb1, X + (W2 - W1), X + (b2 - W1), X + (H1 - W1), X + (c1 - W1), X + (H2 - W1),
              X + (c2 - W1), X + (H3 - W1), X + (c3 - W1), h1, h2, hh, pk.data());
    std::vector<int32_t> pidx(pk.size()), tidx((size_t)2 * h2 * hh + (size_t)hh * hh + (size_t)h1 * h2);
    for (size_t k = 0; k < pk.size(); ++k) pidx[k] = (int32_t)pk[k] - 1;
    const size_t oH1 = (size_t)(H1 - W1), oH2 = (size_t)(H2 - W1), oW2 = (size_t)(W2 - W1);
    for (int o = 0; o < hh; ++o)
      for (int k = 0; k < 2 * h2; ++k) tidx[(size_t)k * hh + o] = (int32_t)(oH1 + (size_t)o * 2 * h2 + k);
    int32_t* ti2 = tidx.data() + (size_t)2 * h2 * hh;
    for (int o = 0; o < hh; ++o)
      for (int k = 0; k < hh; ++k) ti2[(size_t)k * hh + o] = (int32_t)(oH2 + (size_t)o * hh + k);
    int32_t* ti3 = ti2 + (size_t)hh * hh;
    for (int cc = 0; cc < h2; ++cc)
      for (int k = 0; k < h1; ++k) ti3[(size_t)k * h2 + cc] = (int32_t)(oW2 + (size_t)cc * h1 + k);
    if (!c->d_pack_idx) HIP_TRY(hipMalloc(&c->d_pack_idx, pidx.size() * sizeof(int32_t)));
    if (!c->d_tr_idx) HIP_TRY(hipMalloc(&c->d_tr_idx, tidx.size() * sizeof(int32_t)));
    HIP_TRY(hipMemcpy(c->d_pack_idx, pidx.data(), pidx.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d_tr_idx, tidx.data(), tidx.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    c->train_t = 0;  // new weights start a new optimisation
    if (c->d_train) HIP_TRY(hipMemset(c->d_train, 0, 3 * n * sizeof(float)));
  }
  if (c->cfg.precision == LOCC_BF16) {
    const Bf16Layout L = bf16_layout(h1, h2, hh);
    std::vector<unsigned char> bpack(L.total);
    bf16_pack(W1, b1, W2, b2, H1, c1, H2, c2, H3, c3, h1, h2, hh, bpack.data());
    if (!c->d_wbf16) HIP_TRY(hipMalloc(&c->d_wbf16, L.total));
    HIP_TRY(hipMemcpy(c->d_wbf16, bpack.data(), L.total, hipMemcpyHostToDevice));
  }
  if (c->fp8()) {
    const Fp8Layout L = fp8_layout(h1, h2, hh, c->fp8_head());
    std::vector<unsigned char> fpack(L.total);
    float sc[3];
    fp8_pack(W1, b1, W2, b2, H1, c1, H2, c2, H3, c3, h1, h2, hh, c->fp8_head(), fpack.data(), sc);
    if (!c->d_wfp8) HIP_TRY(hipMalloc(&c->d_wfp8, L.total));
    HIP_TRY(hipMemcpy(c->d_wfp8, fpack.data(), L.total, hipMemcpyHostToDevice));
    if (!c->d_wraw) HIP_TRY(hipMalloc(&c->d_wraw, n * sizeof(float)));
    HIP_TRY(hipMemcpy(c->d_wraw, h, n * sizeof(float), hipMemcpyHostToDevice));
    for (int k = 0; k < 3; ++k) c->fp8_wscale[k] = sc[k];
    c->h_w1b1.assign(W1, W1 + (size_t)h1 * 6);
    c->h_w1b1.insert(c->h_w1b1.end(), b1, b1 + h1);
    c->have_act_scales = false;  // activation maxima belong to the previous weights
  }
  c->have_weights = true;
  return LOCC_OK;
}

namespace {

// Installs FP8 activation maxima and repacks encoder layer 1 in units of the
// scale of its output (so the kernel converts without a multiply).
locc_status fp8_install_amax(locc_ctx* c, const float* amax) {
  const int h1 = c->cfg.enc_h1;
  const float inv = 1.f / fp8_scale(amax[0]);
  std::vector<unsigned short> w1((size_t)h1 * 8);
  fp8_pack_w1(c->h_w1b1.data(), c->h_w1b1.data() + (size_t)h1 * 6, h1, inv, w1.data());
  const Fp8Layout L = fp8_layout(h1, c->cfg.enc_h2, c->cfg.head_h, c->fp8_head());
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipMemcpy(c->d_wfp8 + L.w1, w1.data(), w1.size() * sizeof(unsigned short), hipMemcpyHostToDevice));
  for (int k = 0; k < 3; ++k) c->fp8_amax[k] = amax[k];
  c->have_act_scales = true;
  return LOCC_OK;
}

}  // namespace

locc_status locc_set_activation_amax(locc_ctx* c, const float* amax) {
  if (!c || !amax) return fail(LOCC_ERR_INVALID_ARG, "null context or maxima");
  if (!c->fp8()) return fail(LOCC_ERR_UNSUPPORTED, "activation maxima: not an FP8 context");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(amax[k]) || amax[k] < 0.f)
      return fail(LOCC_ERR_INVALID_ARG, "activation maximum %d = %g: must be finite and >= 0", k, amax[k]);
  if (!c->have_weights) return fail(LOCC_ERR_NOT_READY, "no weights uploaded");
  if (c->capturing) return fail(LOCC_ERR_RANGE, "activation maxima during graph capture");
  if (c->live_graphs > 0)
    return fail(LOCC_ERR_BUSY, "activation maxima: %d captured graph(s) hold the current scales; destroy them first",
                c->live_graphs);
  return fp8_install_amax(c, amax);
}

locc_status locc_calibrate(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs,
                           int32_t n_pairs, void* stream, float* amax_out) {
  if (!c) return fail(LOCC_ERR_INVALID_ARG, "null context");
  if (!c->fp8()) return fail(LOCC_ERR_UNSUPPORTED, "calibration: not an FP8 context");
  if (n_objs < 0 || n_pairs < 0) return fail(LOCC_ERR_INVALID_ARG, "negative count");
  if (n_pairs > 0 && (!objs || !pairs)) return fail(LOCC_ERR_INVALID_ARG, "null objects or pairs");
  if (!c->d_shapes) return fail(LOCC_ERR_NOT_READY, "no shape library uploaded");
  if (!c->have_weights) return fail(LOCC_ERR_NOT_READY, "no weights uploaded");
  if (c->capturing) return fail(LOCC_ERR_RANGE, "calibration during graph capture");
  if (c->live_graphs > 0)
    return fail(LOCC_ERR_BUSY, "calibration: %d captured graph(s) hold the current scales; destroy them first",
                c->live_graphs);
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(c->device));
  float amax[3] = {0.f, 0.f, 0.f};
  if (n_pairs > 0) {
    Workspace w{};
    locc_status st = carve(c, n_pairs, &w, nullptr);
    if (st != LOCC_OK) return st;
    PairMeta* meta = w.meta;
    unsigned short* rows = w.rows_bf16;
    CropArgs ca{objs, n_objs, pairs, n_pairs, nullptr, c->lib(), c->cfg.K, c->cfg.pad_m,
                nullptr, nullptr, meta, nullptr, rows, c->d_err, w.setup};
    HIP_TRY(launch_crop(ca, s, c->sched.crop_unroll));
    HIP_TRY(hipMemsetAsync(c->d_amax, 0, 3 * sizeof(unsigned int), s));
    CalibArgs ka{c->d_wraw, c->cfg.enc_h1, c->cfg.enc_h2, c->cfg.head_h, n_pairs, c->cfg.K, rows, meta, c->d_amax};
    const int grid = n_pairs < 8 * c->n_cu ? n_pairs : 8 * c->n_cu;
    HIP_TRY(launch_calibrate_fp8(ka, grid, s));
    unsigned int bits[3];
    HIP_TRY(hipMemcpyAsync(bits, c->d_amax, sizeof bits, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(amax, bits, sizeof amax);
  }
  const locc_status ist = fp8_install_amax(c, amax);
  if (ist != LOCC_OK) return ist;
  if (amax_out) std::memcpy(amax_out, amax, sizeof amax);
  return LOCC_OK;
}

locc_status locc_upload_shapes(locc_ctx* c, int32_t n_shapes, const int64_t* off, const float* pts) {
  if (!c || !off || !pts) return fail(LOCC_ERR_INVALID_ARG, "null context, offsets or points");
  if (n_shapes <= 0) return fail(LOCC_ERR_INVALID_ARG, "n_shapes=%d", n_shapes);
  if (off[0] != 0) return fail(LOCC_ERR_INVALID_ARG, "offsets[0]=%lld, must be 0", (long long)off[0]);
  for (int s = 0; s < n_shapes; ++s) {
    const int64_t n = off[s + 1] - off[s];
    if (n <= 0) return fail(LOCC_ERR_INVALID_ARG, "shape %d has %lld points", s, (long long)n);
    if (n > kMaxShapePoints)
      return fail(LOCC_ERR_RANGE, "shape %d has %lld points (max %d)", s, (long long)n, kMaxShapePoints);
  }
  const int64_t total = off[n_shapes];
  if (total >= (int64_t)INT32_MAX) return fail(LOCC_ERR_RANGE, "%lld points in total", (long long)total);
  if (c->live_graphs > 0)
    return fail(LOCC_ERR_BUSY, "shape library: %d captured graph(s) read the current one; destroy them first",
                c->live_graphs);
  std::vector<float> soa((size_t)total * 6);
  std::vector<ShapeDesc> desc(n_shapes);
  for (int s = 0; s < n_shapes; ++s) {
    ShapeDesc d{};
    d.off = (int32_t)off[s];
    d.n = (int32_t)(off[s + 1] - off[s]);
    for (int k = 0; k < 3; ++k) {
      d.lo[k] = INFINITY;
      d.hi[k] = -INFINITY;
    }
    for (int64_t r = off[s]; r < off[s + 1]; ++r) {
      const float* row = pts + r * 6;
      for (int k = 0; k < 6; ++k) {
        if (!std::isfinite(row[k]))
          return fail(LOCC_ERR_INVALID_ARG, "shape %d point %lld: non-finite value", s, (long long)(r - off[s]));
        soa[(size_t)k * total + r] = row[k];
      }
      for (int k = 0; k < 3; ++k) {
        d.lo[k] = row[k] < d.lo[k] ? row[k] : d.lo[k];
        d.hi[k] = row[k] > d.hi[k] ? row[k] : d.hi[k];
      }
    }
    desc[s] = d;
  }
  HIP_TRY(hipSetDevice(c->device));
  (void)hipFree(c->d_shapes);
  (void)hipFree(c->d_points);
  c->d_shapes = nullptr;
  c->d_points = nullptr;
  c->n_shapes = 0;
  c->n_points = 0;
  HIP_TRY(hipMalloc(&c->d_shapes, sizeof(ShapeDesc) * n_shapes));
  HIP_TRY(hipMalloc(&c->d_points, sizeof(float) * soa.size()));
  HIP_TRY(hipMemcpy(c->d_shapes, desc.data(), sizeof(ShapeDesc) * n_shapes, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->d_points, soa.data(), sizeof(float) * soa.size(), hipMemcpyHostToDevice));
  c->n_shapes = n_shapes;
  c->n_points = total;
  return LOCC_OK;
}

locc_status locc_detect(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs,
                        int32_t n_pairs, locc_contact* out, int32_t* counts, void* stream) {
  locc_status st = check_call(c, objs, n_objs, pairs, n_pairs);
  if (st != LOCC_OK) return st;
  if (n_pairs > 0 && !out) return fail(LOCC_ERR_INVALID_ARG, "null output");
  return run_path(c, objs, n_objs, pairs, n_pairs, nullptr, out, counts, nullptr, nullptr,
                  static_cast<hipStream_t>(stream));
}

locc_status locc_debug_forward(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs,
                               int32_t n_pairs, locc_contact* out, int32_t* counts, float* z, float* y,
                               void* stream) {
  locc_status st = check_call(c, objs, n_objs, pairs, n_pairs);
  if (st != LOCC_OK) return st;
  if (n_pairs > 0 && !out) return fail(LOCC_ERR_INVALID_ARG, "null output");
  return run_path(c, objs, n_objs, pairs, n_pairs, nullptr, out, counts, z, y, static_cast<hipStream_t>(stream));
}

locc_status locc_debug_crop(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs,
                            int32_t n_pairs, int32_t* idx, int32_t* counts, void* stream) {
  if (!c) return fail(LOCC_ERR_INVALID_ARG, "null context");
  if (n_objs < 0 || n_pairs < 0) return fail(LOCC_ERR_INVALID_ARG, "negative count");
  if (n_pairs > 0 && (!objs || !pairs || !idx || !counts))
    return fail(LOCC_ERR_INVALID_ARG, "null objects, pairs, idx or counts");
  if (!c->d_shapes) return fail(LOCC_ERR_NOT_READY, "no shape library uploaded");
  if (n_pairs == 0) return LOCC_OK;
  HIP_TRY(hipSetDevice(c->device));
  locc_status st = ensure_workspace(c, align256((size_t)n_pairs * kPairSetupBytes));
  if (st != LOCC_OK) return st;
  CropArgs ca{objs, n_objs, pairs, n_pairs, nullptr, c->lib(), c->cfg.K, c->cfg.pad_m,
              idx, counts, nullptr, nullptr, nullptr, c->d_err, c->d_ws};
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(timed(c, "crop", s, [&] { return launch_crop(ca, s, c->sched.crop_unroll); }));
  return LOCC_OK;
}

locc_status locc_set_schedule(locc_ctx* c, const locc_schedule* sc) {
  if (!c || !sc) return fail(LOCC_ERR_INVALID_ARG, "null context or schedule");
  locc_status st = check_schedule(sc);
  if (st != LOCC_OK) return st;
  c->sched = *sc;
  return LOCC_OK;
}

locc_status locc_get_schedule(const locc_ctx* c, locc_schedule* sc) {
  if (!c || !sc) return fail(LOCC_ERR_INVALID_ARG, "null context or schedule");
  *sc = c->sched;
  return LOCC_OK;
}

locc_status locc_profile(locc_ctx* c, int enable) {
  if (!c) return fail(LOCC_ERR_INVALID_ARG, "null context");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(drain_profile(c));
  if (enable) c->totals.clear();
  c->profiling = enable != 0;
  return LOCC_OK;
}

locc_status locc_profile_read(locc_ctx* c, locc_kernel_time* out, int32_t capacity, int32_t* count) {
  if (!c || !count || capacity < 0 || (capacity > 0 && !out))
    return fail(LOCC_ERR_INVALID_ARG, "null context, output or count");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(drain_profile(c));
  int32_t n = 0;
  for (const auto& kv : c->totals) {
    if (n < capacity) {
      locc_kernel_time& t = out[n];
      std::memset(&t, 0, sizeof t);
      std::snprintf(t.name, sizeof t.name, "%s", kv.first.c_str());
      t.launches = kv.second.first;
      t.total_ms = kv.second.second;
    }
    ++n;
  }
  *count = n;
  return LOCC_OK;
}

locc_status locc_reserve(locc_ctx* c, int32_t max_pairs) {
  if (!c || max_pairs < 0) return fail(LOCC_ERR_INVALID_ARG, "null context or negative size");
  HIP_TRY(hipSetDevice(c->device));
  // the largest workspace any schedule of this context could need
  const locc_schedule keep = c->sched;
  c->sched.split = 1;
  const size_t bytes = workspace_bytes(c, max_pairs);
  c->sched = keep;
  return ensure_workspace(c, bytes);
}

locc_status locc_detect_device_count(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs,
                                     const int32_t* n_dev, int32_t max_pairs, locc_contact* out, int32_t* counts,
                                     void* stream) {
  locc_status st = check_call(c, objs, n_objs, pairs, max_pairs);
  if (st != LOCC_OK) return st;
  if (!n_dev) return fail(LOCC_ERR_INVALID_ARG, "null device pair count");
  if (max_pairs > 0 && !out) return fail(LOCC_ERR_INVALID_ARG, "null output");
  if (workspace_bytes(c, max_pairs) > c->ws_bytes)
    return fail(LOCC_ERR_RANGE, "workspace holds fewer than %d pairs: call locc_reserve first", max_pairs);
  return run_path(c, objs, n_objs, pairs, max_pairs, n_dev, out, counts, nullptr, nullptr,
                  static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

// Captures body(stream) on the context's capture stream as a HIP graph.
template <class F>
locc_status capture_graph(locc_ctx* c, locc_graph** graph, F&& body) {
  if (!c->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
  HIP_TRY(hipDeviceSynchronize());
  const bool prof = c->profiling;
  c->profiling = false;  // no event nodes in the graph
  c->capturing = true;
  HIP_TRY(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeRelaxed));
  locc_status st = body(c->capture_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
  c->capturing = false;
  c->profiling = prof;
  if (st != LOCC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(LOCC_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  locc_graph* G = new locc_graph();
  G->ctx = c;
  G->graph = g;
  ++c->live_graphs;  // counted down by locc_graph_destroy, on the failure path below too
  const hipError_t e2 = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    locc_graph_destroy(G);
    return fail(LOCC_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
  }
  *graph = G;
  return LOCC_OK;
}

locc_status ensure_broad_scratch(locc_ctx* c, int n_objs, int n_envs) {
  const size_t bytes = broad_phase_scratch_bytes(n_objs, n_envs);
  if (bytes <= c->bp_bytes) return LOCC_OK;
  if (c->capturing)
    return fail(LOCC_ERR_RANGE, "broad-phase scratch of %zu bytes too small for %zu during graph capture",
                c->bp_bytes, bytes);
  if (c->live_graphs > 0)
    return fail(LOCC_ERR_RANGE, "broad-phase scratch of %zu bytes too small for %zu while %d captured graph(s) "
                "use it: reserve before capturing, or destroy the graphs first", c->bp_bytes, bytes, c->live_graphs);
  if (c->d_bp) HIP_TRY(hipFree(c->d_bp));
  c->d_bp = nullptr;
  c->bp_bytes = 0;
  HIP_TRY(hipMalloc(&c->d_bp, bytes));
  c->bp_bytes = bytes;
  return LOCC_OK;
}

locc_status check_broad(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* env_offsets,
                        int32_t n_envs, const int32_t* pairs, int32_t capacity, const int32_t* count) {
  if (!c) return fail(LOCC_ERR_INVALID_ARG, "null context");
  if (n_objs < 0 || n_envs < 0 || capacity < 0)
    return fail(LOCC_ERR_INVALID_ARG, "negative size (n_objs=%d, n_envs=%d, capacity=%d)", n_objs, n_envs,
                capacity);
  if (!count) return fail(LOCC_ERR_INVALID_ARG, "null pair count");
  if (n_objs > 0 && !objs) return fail(LOCC_ERR_INVALID_ARG, "null objects");
  if (n_envs > 0 && !env_offsets) return fail(LOCC_ERR_INVALID_ARG, "null environment offsets");
  if (capacity > 0 && !pairs) return fail(LOCC_ERR_INVALID_ARG, "null pair output");
  if (!c->d_shapes) return fail(LOCC_ERR_NOT_READY, "no shape library uploaded");
  return LOCC_OK;
}

locc_status run_broad(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* env_offsets,
                      int32_t n_envs, int32_t* pairs, int32_t capacity, int32_t* count, hipStream_t s) {
  locc_status st = ensure_broad_scratch(c, n_objs, n_envs);
  if (st != LOCC_OK) return st;
  BroadArgs a{};
  a.objs = objs;
  a.n_objs = n_objs;
  a.env_offsets = env_offsets;
  a.n_envs = n_envs;
  a.lib = c->lib();
  broad_phase_carve(c->d_bp, n_objs, n_envs, a);
  a.pairs = pairs;
  a.capacity = capacity;
  a.count = count;
  HIP_TRY(timed(c, "broad_phase", s, [&] { return launch_broad_phase(a, s); }));
  return LOCC_OK;
}

}  // namespace

extern "C" {

locc_status locc_graph_capture(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs,
                               const int32_t* n_dev, int32_t max_pairs, locc_contact* out, int32_t* counts,
                               locc_graph** graph) {
  if (!graph) return fail(LOCC_ERR_INVALID_ARG, "null graph output");
  *graph = nullptr;
  locc_status st = check_call(c, objs, n_objs, pairs, max_pairs);
  if (st != LOCC_OK) return st;
  if (!n_dev || max_pairs <= 0 || !out) return fail(LOCC_ERR_INVALID_ARG, "null count or output, or no capacity");
  st = locc_reserve(c, max_pairs);
  if (st != LOCC_OK) return st;
  return capture_graph(c, graph, [&](hipStream_t s) {
    return run_path(c, objs, n_objs, pairs, max_pairs, n_dev, out, counts, nullptr, nullptr, s);
  });
}

locc_status locc_broad_phase(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* env_offsets,
                             int32_t n_envs, int32_t* pairs, int32_t capacity, int32_t* count, void* stream) {
  locc_status st = check_broad(c, objs, n_objs, env_offsets, n_envs, pairs, capacity, count);
  if (st != LOCC_OK) return st;
  HIP_TRY(hipSetDevice(c->device));
  return run_broad(c, objs, n_objs, env_offsets, n_envs, pairs, capacity, count, static_cast<hipStream_t>(stream));
}

locc_status locc_reserve_broad_phase(locc_ctx* c, int32_t n_objs, int32_t n_envs) {
  if (!c || n_objs < 0 || n_envs < 0) return fail(LOCC_ERR_INVALID_ARG, "null context or negative size");
  HIP_TRY(hipSetDevice(c->device));
  return ensure_broad_scratch(c, n_objs, n_envs);
}

locc_status locc_step_graph_capture(locc_ctx* c, const locc_object* objs, int32_t n_objs,
                                    const int32_t* env_offsets, int32_t n_envs, int32_t* pairs, int32_t capacity,
                                    int32_t* count, locc_contact* out, int32_t* counts, locc_graph** graph) {
  if (!graph) return fail(LOCC_ERR_INVALID_ARG, "null graph output");
  *graph = nullptr;
  locc_status st = check_broad(c, objs, n_objs, env_offsets, n_envs, pairs, capacity, count);
  if (st != LOCC_OK) return st;
  st = check_call(c, objs, n_objs, pairs, capacity);
  if (st != LOCC_OK) return st;
  if (capacity <= 0 || !out) return fail(LOCC_ERR_INVALID_ARG, "null output or no capacity");
  HIP_TRY(hipSetDevice(c->device));
  st = locc_reserve(c, capacity);
  if (st == LOCC_OK) st = ensure_broad_scratch(c, n_objs, n_envs);
  if (st != LOCC_OK) return st;
  return capture_graph(c, graph, [&](hipStream_t s) {
    locc_status r = run_broad(c, objs, n_objs, env_offsets, n_envs, pairs, capacity, count, s);
    if (r != LOCC_OK) return r;
    return run_path(c, objs, n_objs, pairs, capacity, count, out, counts, nullptr, nullptr, s);
  });
}

locc_status locc_graph_launch(locc_graph* G, void* stream) {
  if (!G || !G->exec) return fail(LOCC_ERR_INVALID_ARG, "null graph");
  HIP_TRY(hipSetDevice(G->ctx->device));
  HIP_TRY(hipGraphLaunch(G->exec, static_cast<hipStream_t>(stream)));
  return LOCC_OK;
}

void locc_graph_destroy(locc_graph* G) {
  if (!G) return;
  if (G->ctx) --G->ctx->live_graphs;
  if (G->exec) (void)hipGraphExecDestroy(G->exec);
  if (G->graph) (void)hipGraphDestroy(G->graph);
  delete G;
}

locc_status locc_autotune(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs,
                          int32_t n_pairs, locc_contact* out, int32_t* counts, void* stream, const char* cache_path,
                          locc_schedule* best, double* best_ms) {
  locc_status st = check_call(c, objs, n_objs, pairs, n_pairs);
  if (st != LOCC_OK) return st;
  if (!best || (n_pairs > 0 && !out)) return fail(LOCC_ERR_INVALID_ARG, "null output or result");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const std::string key = tune_key(c, n_pairs);
  locc_schedule pick = c->sched;
  double pick_ms = 0.0;
  if (!tune_cache_lookup(cache_path, key, &pick, &pick_ms)) {
    st = locc_reserve(c, n_pairs);
    if (st != LOCC_OK) return st;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const bool prof = c->profiling;
    c->profiling = false;
    pick_ms = 1e30;
    for (const locc_schedule& cand : tune_candidates(c)) {
      c->sched = cand;
      st = run_path(c, objs, n_objs, pairs, n_pairs, nullptr, out, counts, nullptr, nullptr, s);
      if (st != LOCC_OK) break;
      HIP_TRY(hipEventRecord(e0, s));
      for (int r = 0; r < 3 && st == LOCC_OK; ++r)
        st = run_path(c, objs, n_objs, pairs, n_pairs, nullptr, out, counts, nullptr, nullptr, s);
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (st != LOCC_OK) break;
      if (ms / 3.0 < pick_ms) {
        pick_ms = ms / 3.0;
        pick = cand;
      }
    }
    c->profiling = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != LOCC_OK) return st;
    tune_cache_store(cache_path, key, pick, pick_ms);
  }
  c->sched = pick;
  *best = pick;
  if (best_ms) *best_ms = pick_ms;
  return LOCC_OK;
}

locc_status locc_pose_gradients(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs,
                                int32_t n_pairs, float* grad, locc_contact* out, uint8_t* argmax_b, void* stream) {
  locc_status st = check_call(c, objs, n_objs, pairs, n_pairs);
  if (st != LOCC_OK) return st;
  const bool bf16 = c->cfg.precision == LOCC_BF16;
  if (c->cfg.precision != LOCC_FP32 && !bf16)
    return fail(LOCC_ERR_UNSUPPORTED, "pose gradients need an FP32 or BF16 context");
  if (n_pairs > 0 && !grad) return fail(LOCC_ERR_INVALID_ARG, "null gradient output");
  if (n_pairs == 0) return LOCC_OK;
  HIP_TRY(hipSetDevice(c->device));
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int h1 = c->cfg.enc_h1, h2 = c->cfg.enc_h2, hh = c->cfg.head_h, K = c->cfg.K;
  const size_t P = (size_t)n_pairs;
  // workspace: pair records, set-up records, float32 rows (the gradient reads them), pooled features, then
  // the selected indices, the argmax rows and the gradient scratch; BF16 adds the bf16 rows of its encoder
  const size_t b_meta = align256(P * sizeof(PairMeta)), b_setup = align256(P * kPairSetupBytes);
  const size_t b_rows = align256(P * 2 * K * kRowFloats * sizeof(float)), b_z = align256(P * 2 * h2 * sizeof(float));
  const size_t b_rows16 = bf16 ? align256(P * 2 * K * 8 * sizeof(unsigned short)) : 0;
  const size_t b_idx = align256(P * 2 * K * sizeof(int32_t)), b_amax = align256(P * 2 * h2);
  const size_t b_dm = align256(P * h2 * sizeof(float));
  st = ensure_workspace(c, b_meta + b_setup + b_rows + b_z + b_rows16 + b_idx + b_amax + b_dm);
  if (st != LOCC_OK) return st;
  char* b = static_cast<char*>(c->d_ws);
  PairMeta* meta = reinterpret_cast<PairMeta*>(b);
  b += b_meta;
  void* setup = b;
  b += b_setup;
  float* rows = reinterpret_cast<float*>(b);
  b += b_rows;
  float* z = reinterpret_cast<float*>(b);
  b += b_z;
  unsigned short* rows16 = bf16 ? reinterpret_cast<unsigned short*>(b) : nullptr;
  b += b_rows16;
  int32_t* idx = reinterpret_cast<int32_t*>(b);
  b += b_idx;
  uint8_t* amax = reinterpret_cast<uint8_t*>(b);
  b += b_amax;
  float* dm = reinterpret_cast<float*>(b);
  CropArgs ca{objs, n_objs, pairs, n_pairs, nullptr, c->lib(), K, c->cfg.pad_m,
              idx, nullptr, meta, rows, rows16, c->d_err, setup};
  HIP_TRY(timed(c, "crop", s, [&] { return launch_crop(ca, s, c->sched.crop_unroll); }));
  const Fp32Net net = fp32_view(c->d_wfp32, h1, h2, hh);
  NetArgs na{rows, meta, objs, n_pairs, nullptr, K, z, nullptr, out, amax};
  if (bf16) {
    // the BF16 encoder of the split schedule, recording the pooled features and the argmax rows
    FusedArgs fa{};
    fa.objs = objs;
    fa.n_objs = n_objs;
    fa.n_pairs = n_pairs;
    fa.lib = c->lib();
    fa.K = K;
    fa.pad = c->cfg.pad_m;
    bf16_bind(fa, c->d_wbf16, h1, h2, hh);
    fa.z_dbg = z;
    fa.amax = amax;
    fa.rows_bf16 = rows16;
    fa.meta = meta;
    fa.queue = c->d_queue;
    fa.claim = c->sched.claim;
    fa.dynamic = c->sched.dynamic;
    if (c->sched.wg_per_cu == 1) {  // one workgroup of eight waves per CU, W2 in LDS
      const int groups = (n_pairs + 63) / 64;
      const int g8 = groups < c->n_cu ? groups : c->n_cu;
      HIP_TRY(timed(c, "encoder_bf16_argmax", s,
                    [&] { return launch_encoder_head_bf16_lds(fa, h1, h2, hh, g8, true, s); }));
    } else {
      const int grid = fused_grid(c, n_pairs);
      HIP_TRY(timed(c, "encoder_bf16_argmax", s,
                    [&] { return launch_encoder_bf16_argmax(fa, h1, h2, hh, grid, s); }));
    }
  } else {
    HIP_TRY(timed(c, "encoder_fp32", s, [&] { return launch_encoder_fp32(net, na, c->n_cu, s); }));
  }
  if (out) HIP_TRY(timed(c, "head_fp32", s, [&] { return launch_head_fp32(net, na, s); }));
  GradArgs ga{};
  ga.objs = objs;
  ga.n_objs = n_objs;
  ga.pairs = pairs;
  ga.n_pairs = n_pairs;
  ga.meta = meta;
  ga.rows = rows;
  ga.idx = idx;
  ga.z = z;
  ga.amax = amax;
  ga.dm = dm;
  ga.grad = grad;
  ga.K = K;
  ga.lib = c->lib();
  ga.raw = c->d_wraw;
  size_t o = 0;
  ga.off.W1 = o;
  o += (size_t)h1 * 6;
  ga.off.b1 = o;
  o += h1;
  ga.off.W2 = o;
  o += (size_t)h2 * h1;
  ga.off.b2 = o;
  o += h2;
  ga.off.H1 = o;
  o += (size_t)hh * 2 * h2;
  ga.off.c1 = o;
  o += hh;
  ga.off.H2 = o;
  o += (size_t)hh * hh;
  ga.off.c2 = o;
  o += hh;
  ga.off.H3 = o;
  o += (size_t)8 * hh;
  ga.off.c3 = o;
  ga.H1t = c->d_wgrad;
  ga.H2t = c->d_wgrad + (size_t)2 * h2 * hh;
  ga.W2t = ga.H2t + (size_t)hh * hh;
  ga.argmax_b = argmax_b;
  HIP_TRY(timed(c, "pose_grad", s, [&] { return launch_pose_gradients(ga, h1, h2, hh, s); }));
  return LOCC_OK;
}

locc_status locc_train_step(locc_ctx* c, const locc_object* objs, int32_t n_objs, const int32_t* pairs,
                            const float* labels, int32_t n_pairs, float alpha, float lr, float beta1, float beta2,
                            float eps, float* loss, uint8_t* argmax, void* stream) {
  locc_status st = check_call(c, objs, n_objs, pairs, n_pairs);
  if (st != LOCC_OK) return st;
  if (c->cfg.precision != LOCC_FP32) return fail(LOCC_ERR_UNSUPPORTED, "training needs an FP32 context");
  if (n_pairs <= 0 || !labels || !loss) return fail(LOCC_ERR_INVALID_ARG, "empty batch, null labels or loss");
  if (!(alpha >= 0.f) || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return fail(LOCC_ERR_INVALID_ARG, "alpha >= 0, lr > 0, 0 <= beta < 1 and eps > 0 are required");
  HIP_TRY(hipSetDevice(c->device));
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int h1 = c->cfg.enc_h1, h2 = c->cfg.enc_h2, hh = c->cfg.head_h, K = c->cfg.K;
  const size_t n = weight_floats(h1, h2, hh);
  if (!c->d_train) {
    HIP_TRY(hipMalloc(&c->d_train, 3 * n * sizeof(float)));
    HIP_TRY(hipMemset(c->d_train, 0, 3 * n * sizeof(float)));
    c->train_t = 0;
  }
  const size_t P = (size_t)n_pairs;
  const size_t base = workspace_bytes(c, n_pairs);
  const size_t b_amax = align256(P * 2 * h2), b_act = align256(P * hh * sizeof(float));
  const size_t b_dm = align256(P * 2 * h2 * sizeof(float)), b_p = align256(P * 3 * sizeof(float));
  const size_t b_w1 = align256((size_t)kEncSplit * h2 * h1 * 7 * sizeof(float));
  const size_t b_w2 = align256((size_t)kEncSplit * h2 * (h1 + 1) * sizeof(float));
  const size_t nk = (size_t)(hh > 2 * h2 ? hh : 2 * h2) + 1;
  const size_t b_op = align256((size_t)kOuterSplit * hh * nk * sizeof(float));
  st = ensure_workspace(c, base + b_amax + 4 * b_act + b_dm + b_p + b_w1 + b_w2 + b_op);
  if (st != LOCC_OK) return st;
  Workspace w{};
  st = carve(c, n_pairs, &w, nullptr);
  if (st != LOCC_OK) return st;
  char* e = static_cast<char*>(c->d_ws) + base;
  uint8_t* amax = reinterpret_cast<uint8_t*>(e);
  e += b_amax;
  TrainArgs ta{};
  float* act[4];
  for (int k = 0; k < 4; ++k) {
    act[k] = reinterpret_cast<float*>(e);
    e += b_act;
  }
  ta.g1 = act[0];
  ta.g2 = act[1];
  ta.du2 = act[2];
  ta.du1 = act[3];
  ta.dmv = reinterpret_cast<float*>(e);
  e += b_dm;
  ta.dx = reinterpret_cast<float*>(e);
  ta.lossp = ta.dx + P;
  e += b_p;
  ta.w1part = reinterpret_cast<float*>(e);
  e += b_w1;
  ta.w2part = reinterpret_cast<float*>(e);
  e += b_w2;
  ta.opart = reinterpret_cast<float*>(e);
  CropArgs ca{objs, n_objs, pairs, n_pairs, nullptr, c->lib(), K, c->cfg.pad_m,
              nullptr, nullptr, w.meta, w.rows, nullptr, c->d_err, w.setup};
  HIP_TRY(timed(c, "crop", s, [&] { return launch_crop(ca, s, c->sched.crop_unroll); }));
  const Fp32Net net = fp32_view(c->d_wfp32, h1, h2, hh);
  NetArgs na{w.rows, w.meta, objs, n_pairs, nullptr, K, w.z, nullptr, nullptr, amax};
  HIP_TRY(timed(c, "encoder_fp32", s, [&] { return launch_encoder_fp32(net, na, c->n_cu, s); }));
  ta.n_pairs = n_pairs;
  ta.meta = w.meta;
  ta.rows = w.rows;
  ta.z = w.z;
  ta.amax = amax;
  ta.labels = labels;
  ta.K = K;
  ta.alpha = alpha;
  ta.raw = c->d_wraw;
  size_t o = 0;
  ta.off.W1 = o;
  o += (size_t)h1 * 6;
  ta.off.b1 = o;
  o += h1;
  ta.off.W2 = o;
  o += (size_t)h2 * h1;
  ta.off.b2 = o;
  o += h2;
  ta.off.H1 = o;
  o += (size_t)hh * 2 * h2;
  ta.off.c1 = o;
  o += hh;
  ta.off.H2 = o;
  o += (size_t)hh * hh;
  ta.off.c2 = o;
  o += hh;
  ta.off.H3 = o;
  o += (size_t)8 * hh;
  ta.off.c3 = o;
  ta.H1t = c->d_wgrad;
  ta.H2t = c->d_wgrad + (size_t)2 * h2 * hh;
  ta.grad = c->d_train;
  ta.m = c->d_train + n;
  ta.v = c->d_train + 2 * n;
  ta.n = n;
  const int64_t t_next = c->train_t + 1;
  ta.lr = lr;
  ta.beta1 = beta1;
  ta.beta2 = beta2;
  ta.eps = eps;
  ta.corr1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)t_next)));
  ta.corr2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)t_next)));
  ta.loss = loss;
  ta.pack_dst = c->d_wfp32;
  ta.pack_idx = c->d_pack_idx;
  ta.pack_n = fp32_pack_floats(h1, h2, hh);
  ta.tr_dst = c->d_wgrad;
  ta.tr_idx = c->d_tr_idx;
  ta.tr_n = (size_t)2 * h2 * hh + (size_t)hh * hh + (size_t)h1 * h2;
  if (argmax) HIP_TRY(hipMemcpyAsync(argmax, amax, P * 2 * h2, hipMemcpyDeviceToDevice, s));
  HIP_TRY(timed(c, "train", s, [&] { return launch_train_step(ta, h1, h2, hh, s); }));
  c->train_t = t_next;
  return LOCC_OK;
}

locc_status locc_get_weights(locc_ctx* c, int which, float* h_out, size_t n) {
  if (!c || !h_out) return fail(LOCC_ERR_INVALID_ARG, "null context or output");
  if (c->cfg.precision != LOCC_FP32) return fail(LOCC_ERR_UNSUPPORTED, "FP32 contexts keep the flat weights");
  if (!c->have_weights) return fail(LOCC_ERR_NOT_READY, "no weights uploaded");
  if (which < 0 || which > 3) return fail(LOCC_ERR_INVALID_ARG, "which=%d (0 weights, 1 gradient, 2-3 moments)", which);
  if (which > 0 && !c->d_train) return fail(LOCC_ERR_NOT_READY, "no training step run yet");
  const size_t want = weight_floats(c->cfg.enc_h1, c->cfg.enc_h2, c->cfg.head_h);
  if (n != want) return fail(LOCC_ERR_INVALID_ARG, "weights: %zu floats asked, %zu held", n, want);
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipDeviceSynchronize());
  const float* src = which == 0 ? c->d_wraw : c->d_train + (size_t)(which - 1) * n;
  HIP_TRY(hipMemcpy(h_out, src, n * sizeof(float), hipMemcpyDeviceToHost));
  return LOCC_OK;
}

locc_status locc_device_errors(locc_ctx* c, void* stream, int64_t* n_bad, int reset) {
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
