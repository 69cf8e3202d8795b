// Final step of the head: the network predicts the contact point and normal
// in the frame of the canonical first object (Sec. III, appendix
// "Architecture Details"); map them to the world frame with that object's
// pose and flip the normal when the pair was given in the other order.
// Device code shared by the BF16 and FP8 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "locc_internal.h"

namespace locc {

// y: the 8 network outputs (logit, point, normal, depth) of pair p; a < 0
// marks an invalid pair (every output NaN).
__device__ __forceinline__ void post_contact(const locc_object* __restrict__ objs, int a, int swapped,
                                             const float* y, locc_contact* out, float* y_dbg, int p) {
  float o8[8];
  if (a < 0) {
    for (int k = 0; k < 8; ++k) o8[k] = __builtin_nanf("");
  } else {
    const locc_object o = objs[a];
    const double w = o.q[0], x = o.q[1], yq = o.q[2], zq = o.q[3];
    const double R[9] = {1.0 - 2.0 * (yq * yq + zq * zq), 2.0 * (x * yq - w * zq), 2.0 * (x * zq + w * yq),
                         2.0 * (x * yq + w * zq), 1.0 - 2.0 * (x * x + zq * zq), 2.0 * (yq * zq - w * x),
                         2.0 * (x * zq - w * yq), 2.0 * (yq * zq + w * x), 1.0 - 2.0 * (x * x + yq * yq)};
    const double sg = swapped ? -1.0 : 1.0;
    o8[0] = y[0];
    for (int r = 0; r < 3; ++r) {
      o8[1 + r] = (float)(R[3 * r] * y[1] + R[3 * r + 1] * y[2] + R[3 * r + 2] * y[3] + (double)o.p[r]);
      o8[4 + r] = (float)(sg * (R[3 * r] * y[4] + R[3 * r + 1] * y[5] + R[3 * r + 2] * y[6]));
    }
    o8[7] = y[7];
  }
  float4* dst = reinterpret_cast<float4*>(out + p);
  dst[0] = make_float4(o8[0], o8[1], o8[2], o8[3]);
  dst[1] = make_float4(o8[4], o8[5], o8[6], o8[7]);
  if (y_dbg) {
    float4* yd = reinterpret_cast<float4*>(y_dbg + (size_t)p * 8);
    const float nan = __builtin_nanf("");
    yd[0] = a < 0 ? make_float4(nan, nan, nan, nan) : make_float4(y[0], y[1], y[2], y[3]);
    yd[1] = a < 0 ? make_float4(nan, nan, nan, nan) : make_float4(y[4], y[5], y[6], y[7]);
  }
}

}  // namespace locc
