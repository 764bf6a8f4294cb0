// Adam (the optimiser of Alg. 1), one parameter array per call, in place. HBM
// bound: 28 bytes per value (p, m, v read and written, g read).
#include <algorithm>
#include <math.h>

#include "gs_internal.h"

namespace gs {

struct AdamArgs {
  float step;     // lr / (1 - beta1^t)
  float c2;       // 1 / (1 - beta2^t)
  float b1, b2, eps;
};

__device__ __forceinline__ void adam1(float& p, float g, float& m, float& v, const AdamArgs& a) {
  m = a.b1 * m + (1.0f - a.b1) * g;
  v = a.b2 * v + (1.0f - a.b2) * (g * g);
  p = p - a.step * m / (sqrtf(v * a.c2) + a.eps);
}

// ALIGNED: all four arrays 16-byte aligned, float4 accesses plus a scalar tail;
// otherwise scalar accesses throughout.
template <bool ALIGNED>
__global__ void __launch_bounds__(256)
adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
            float* __restrict__ v, int64_t n, AdamArgs a) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t first = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if constexpr (ALIGNED) {
    const int64_t n4 = n / 4;
    float4* p4 = reinterpret_cast<float4*>(p);
    const float4* g4 = reinterpret_cast<const float4*>(g);
    float4* m4 = reinterpret_cast<float4*>(m);
    float4* v4 = reinterpret_cast<float4*>(v);
    for (int64_t i = first; i < n4; i += stride) {
      float4 pp = p4[i], mm = m4[i], vv = v4[i];
      const float4 gg = g4[i];
      adam1(pp.x, gg.x, mm.x, vv.x, a);
      adam1(pp.y, gg.y, mm.y, vv.y, a);
      adam1(pp.z, gg.z, mm.z, vv.z, a);
      adam1(pp.w, gg.w, mm.w, vv.w, a);
      p4[i] = pp;
      m4[i] = mm;
      v4[i] = vv;
    }
    // the tail of fewer than four values
    if (first < n - 4 * n4) {
      const int64_t i = 4 * n4 + first;
      adam1(p[i], g[i], m[i], v[i], a);
    }
  } else {
    for (int64_t i = first; i < n; i += stride) adam1(p[i], g[i], m[i], v[i], a);
  }
}

}  // namespace gs

using namespace gs;

extern "C" int gs_adam_step(float* param, const float* grad, float* m, float* v, int64_t n,
                            float lr, float beta1, float beta2, float eps, int32_t t,
                            gs_stream_t stream) {
  if (n < 0 || t < 1) return GS_ERR_ARG;
  if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f) ||
      !isfinite(lr))
    return GS_ERR_ARG;
  if (n == 0) return GS_OK;
  if (!param || !grad || !m || !v) return GS_ERR_ARG;
  AdamArgs a;
  a.step = (float)((double)lr / (1.0 - pow((double)beta1, (double)t)));
  a.c2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)t)));
  a.b1 = beta1;
  a.b2 = beta2;
  a.eps = eps;
  const bool aligned =
      (((uintptr_t)param | (uintptr_t)grad | (uintptr_t)m | (uintptr_t)v) & 15u) == 0;
  const int64_t items = aligned ? n / 4 : n;
  const unsigned blocks =
      (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, 8192));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (aligned)
    adam_kernel<true><<<blocks, 256, 0, s>>>(param, grad, m, v, n, a);
  else
    adam_kernel<false><<<blocks, 256, 0, s>>>(param, grad, m, v, n, a);
  return launch_status();
}
