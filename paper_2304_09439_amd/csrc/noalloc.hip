// locc_detect_noalloc: the path of locc_detect with its workspace in a fixed
// device array of the library instead of memory the context allocates, for
// callers that cannot allocate (code under HIP graph capture, serving loops,
// harnesses that forbid allocation).
//
// The array below is file scope and static; each device that runs the library
// holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel or a copy: in host code that name is a host-side
// stand-in, not a device address.  locc_create calls noalloc_setup on its
// device (that device current), which looks the device address up once per
// device with hipGetSymbolAddress and keeps it; the entry point hands that
// address to the kernels as their workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "context.h"

namespace locc {

constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;

namespace {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` on each device, once looked up

}  // namespace

size_t noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

// Once per device, with that device current: the device address of this
// device's copy of the array.
locc_status noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(LOCC_ERR_RANGE, "device %d: at most %d devices", device,
                                                       kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return LOCC_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(LOCC_ERR_HIP, "no-allocation scratch on device %d: hipGetSymbolAddress: %s", device,
                hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  return LOCC_OK;
}

}  // namespace locc

using namespace locc;

extern "C" LOCC_API locc_status locc_detect_noalloc(locc_ctx* c, const locc_object* objs, int32_t n_objs,
                                                    const int32_t* pairs, int32_t n_pairs, locc_contact* out,
                                                    int32_t* counts, void* stream) {
  locc_status st = check_call(c, objs, n_objs, pairs, n_pairs);
  if (st != LOCC_OK) return st;
  if (n_pairs > 0 && !out) return fail(LOCC_ERR_INVALID_ARG, "null output");
  if (n_pairs == 0) return LOCC_OK;
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = c->device < kMaxDevices ? g_scratch_ptr[c->device] : nullptr;
  }
  if (!base) return fail(LOCC_ERR_NOT_READY, "no-allocation scratch not set up on device %d", c->device);
  const size_t need = workspace_bytes(c, n_pairs);
  if (need > kNoAllocScratchBytes) {
    int max_pairs = 0;   // the largest batch this context's configuration fits (workspace grows with the count)
    for (int step = 1 << 20; step > 0; step >>= 1)
      if (workspace_bytes(c, max_pairs + step) <= kNoAllocScratchBytes) max_pairs += step;
    return fail(LOCC_ERR_RANGE, "%d pairs need %zu bytes of workspace; the no-allocation scratch holds %zu (at most "
                "%d pairs in this configuration)", n_pairs, need, kNoAllocScratchBytes, max_pairs);
  }
  // One run of pairs, the static claim order (no queue) and no event timing: nothing here allocates.
  const locc_schedule saved = c->sched;
  const bool prof = c->profiling;
  c->sched.dynamic = 0;
  c->sched.chunks = 1;
  c->profiling = false;
  const Scratch own{base, kNoAllocScratchBytes, nullptr};
  st = run_path(c, objs, n_objs, pairs, n_pairs, nullptr, out, counts, nullptr, nullptr,
                static_cast<hipStream_t>(stream), &own);
  c->sched = saved;
  c->profiling = prof;
  return st;
}
