// Adaptive density control (Sec. 5.2 and Alg. 1): positional-gradient statistics,
// the remove / keep / clone / split plan with its output offsets, the new parameter
// arrays, and the periodic opacity reset. All HBM-bound streaming kernels over N.
#include <algorithm>
#include <math.h>

#include "gs_device_math.h"

namespace gs {

constexpr int kDenBlock = 256;
constexpr int kDenItems = 16;
constexpr int kDenTile = kDenBlock * kDenItems;   // Gaussians per scan block
enum : uint8_t { kRemove = 0, kKeep = 1, kClone = 2, kSplit = 3 };

struct DensifyRules {
  float grad_threshold, min_opacity, split_scale, max_world_scale, max_screen_radius,
      log_split_factor;
};

// Per Gaussian, over the views where it is visible: the norm of the gradient of its
// projected mean in normalised device coordinates, the view count and the largest
// pixel-box half-extent.
__global__ void __launch_bounds__(256)
densify_accumulate_kernel(const int32_t* __restrict__ tiles_touched,
                          const float* __restrict__ record, const float* __restrict__ grad2d,
                          TileViews tv, int64_t n, float* __restrict__ grad_sum,
                          int32_t* __restrict__ view_count, float* __restrict__ max_radius) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= n) return;
  float sum = 0.0f, rad = 0.0f;
  int cnt = 0;
  for (int v = 0; v < tv.n_views; ++v) {
    const int64_t idx = (int64_t)v * n + g;
    if (tiles_touched[idx] <= 0) continue;
    const float du = grad2d[idx * GS_GRAD2D_FLOATS + 0] * (0.5f * (float)tv.W[v]);
    const float dv = grad2d[idx * GS_GRAD2D_FLOATS + 1] * (0.5f * (float)tv.H[v]);
    sum += sqrtf(du * du + dv * dv);
    cnt += 1;
    const int2 lohi = *reinterpret_cast<const int2*>(record + idx * GS_RECORD_FLOATS);
    const int wx = (lohi.y & 0xFFFF) - (lohi.x & 0xFFFF) + 1;
    const int wy = ((lohi.y >> 16) & 0xFFFF) - ((lohi.x >> 16) & 0xFFFF) + 1;
    rad = fmaxf(rad, 0.5f * (float)max(wx, wy));
  }
  if (cnt > 0) {
    grad_sum[g] += sum;
    view_count[g] += cnt;
    max_radius[g] = fmaxf(max_radius[g], rad);
  }
}

__device__ __forceinline__ uint8_t densify_action(const float* __restrict__ log_scales,
                                                  const float* __restrict__ logits,
                                                  const float* __restrict__ grad_sum,
                                                  const int32_t* __restrict__ view_count,
                                                  const float* __restrict__ max_radius,
                                                  int64_t n, int64_t g, const DensifyRules& r) {
  const float o = 1.0f / (1.0f + expf(-logits[g]));
  const float smax = expf(fmaxf(fmaxf(log_scales[g], log_scales[n + g]), log_scales[2 * n + g]));
  const int c = view_count[g];
  const float avg = c > 0 ? grad_sum[g] / (float)c : 0.0f;
  bool remove = !(o >= r.min_opacity);
  if (r.max_world_scale > 0.0f) remove = remove || smax > r.max_world_scale;
  if (r.max_screen_radius > 0.0f) remove = remove || max_radius[g] > r.max_screen_radius;
  if (remove) return kRemove;
  if (!(avg > r.grad_threshold)) return kKeep;
  return smax > r.split_scale ? kSplit : kClone;
}

__device__ __forceinline__ uint32_t outputs_of(uint8_t a) { return a == kRemove ? 0u : (a == kKeep ? 1u : 2u); }

__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t x, uint32_t* s4, uint32_t* total) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  uint32_t incl = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += y;
  }
  if (lane == kWave - 1) s4[wave] = incl;
  __syncthreads();
  uint32_t base = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kDenBlock / kWave; ++w) {
    base += (w < wave) ? s4[w] : 0u;
    all += s4[w];
  }
  __syncthreads();
  *total = all;
  return base + incl - x;
}

// Plan, pass 1: the action of every Gaussian and the output count of each block.
__global__ void __launch_bounds__(kDenBlock)
densify_plan_kernel(const float* __restrict__ log_scales, const float* __restrict__ logits,
                    const float* __restrict__ grad_sum, const int32_t* __restrict__ view_count,
                    const float* __restrict__ max_radius, int64_t n, DensifyRules r,
                    uint8_t* __restrict__ action, uint32_t* __restrict__ block_sums) {
  __shared__ uint32_t s4[kDenBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kDenTile;
  uint32_t acc = 0;
#pragma unroll 4
  for (int j = 0; j < kDenItems; ++j) {
    const int64_t g = base + (int64_t)j * kDenBlock + threadIdx.x;
    if (g < n) {
      const uint8_t a = densify_action(log_scales, logits, grad_sum, view_count, max_radius, n, g, r);
      action[g] = a;
      acc += outputs_of(a);
    }
  }
  uint32_t tot;
  block_excl_scan256(acc, s4, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Plan, pass 2 (one block): exclusive scan of the block sums; the new count.
__global__ void __launch_bounds__(1024)
densify_scan_kernel(uint32_t* __restrict__ block_sums, int64_t n_blocks, uint32_t* __restrict__ n_out) {
  __shared__ uint64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n_blocks + 1023) / 1024;
  const int64_t lo = (int64_t)t * per, hi = min(lo + per, n_blocks);
  uint64_t acc = 0;
  for (int64_t i = lo; i < hi; ++i) acc += block_sums[i];
  part[t] = acc;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const uint64_t y = (t >= d) ? part[t - d] : 0;
    __syncthreads();
    part[t] += y;
    __syncthreads();
  }
  uint64_t run = part[t] - acc;
  for (int64_t i = lo; i < hi; ++i) {
    const uint32_t s = block_sums[i];
    block_sums[i] = (uint32_t)run;
    run += s;
  }
  if (t == 1023) n_out[0] = (uint32_t)part[1023];
}

// Plan, pass 3: per-Gaussian output offsets (thread t owns 16 consecutive Gaussians).
__global__ void __launch_bounds__(kDenBlock)
densify_offsets_kernel(const uint8_t* __restrict__ action, int64_t n,
                       const uint32_t* __restrict__ block_sums, uint32_t* __restrict__ offsets) {
  __shared__ uint32_t s4[kDenBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kDenTile + (int64_t)threadIdx.x * kDenItems;
  uint32_t c[kDenItems], local = 0;
#pragma unroll
  for (int j = 0; j < kDenItems; ++j) {
    c[j] = (base + j < n) ? outputs_of(action[base + j]) : 0u;
    local += c[j];
  }
  uint32_t tot;
  uint32_t run = block_sums[blockIdx.x] + block_excl_scan256(local, s4, &tot);
#pragma unroll
  for (int j = 0; j < kDenItems; ++j) {
    if (base + j < n) offsets[base + j] = run;
    run += c[j];
  }
}

// The new parameter arrays: kept Gaussians copied once, clones twice, and each split
// Gaussian replaced by two children mu + R diag(s) z (z from `normals`, [N][2][3]) with
// log-scales lowered by log(split factor).
template <int K>
__global__ void __launch_bounds__(256)
densify_apply_kernel(gs_params in, const uint8_t* __restrict__ action,
                     const uint32_t* __restrict__ offsets, const float* __restrict__ normals,
                     float log_split, int64_t n_out, float* __restrict__ o_means,
                     float* __restrict__ o_log_scales, float* __restrict__ o_quats,
                     float* __restrict__ o_logits, float* __restrict__ o_sh,
                     uint32_t* __restrict__ src_index) {
  const int64_t n = in.n;
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= n) return;
  const uint8_t a = action[g];
  if (a == kRemove) return;
  const int64_t j0 = offsets[g];
  const int copies = a == kKeep ? 1 : 2;
  if (j0 + copies > n_out) return;   // defensive: outputs were sized from the plan
  const float q0 = in.quats[g], q1 = in.quats[n + g], q2 = in.quats[2 * n + g], q3 = in.quats[3 * n + g];
  const float l0 = in.log_scales[g], l1 = in.log_scales[n + g], l2 = in.log_scales[2 * n + g];
  double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  if (a == kSplit) {
    const double qn = sqrt((double)q0 * q0 + (double)q1 * q1 + (double)q2 * q2 + (double)q3 * q3);
    const double iq = qn > 0.0 ? 1.0 / qn : 0.0;
    quat_to_rot(q0 * iq, q1 * iq, q2 * iq, q3 * iq, R);
  }
  for (int c = 0; c < copies; ++c) {
    const int64_t j = j0 + c;
    float m[3] = {in.means[g], in.means[n + g], in.means[2 * n + g]};
    float ls[3] = {l0, l1, l2};
    if (a == kSplit) {
      const float* z = normals + (g * 2 + c) * 3;
      const double sz[3] = {exp((double)l0) * z[0], exp((double)l1) * z[1], exp((double)l2) * z[2]};
      for (int r = 0; r < 3; ++r)
        m[r] = (float)((double)m[r] + R[r * 3 + 0] * sz[0] + R[r * 3 + 1] * sz[1] + R[r * 3 + 2] * sz[2]);
      for (int r = 0; r < 3; ++r) ls[r] = ls[r] - log_split;
    }
    for (int r = 0; r < 3; ++r) {
      o_means[r * n_out + j] = m[r];
      o_log_scales[r * n_out + j] = ls[r];
    }
    o_quats[j] = q0;
    o_quats[n_out + j] = q1;
    o_quats[2 * n_out + j] = q2;
    o_quats[3 * n_out + j] = q3;
    o_logits[j] = in.opacity_logits[g];
#pragma unroll
    for (int k = 0; k < K * 3; ++k) o_sh[(int64_t)k * n_out + j] = in.sh[(int64_t)k * n + g];
    if (src_index) src_index[j] = (uint32_t)g;
  }
}

// Per-Gaussian state laid out like the parameters (e.g. optimiser moments) carried
// through a densification: every output takes its source's values, or zeros for the
// Gaussians a clone or split created when zero_created is set.
template <int K>
__global__ void __launch_bounds__(256)
densify_gather_kernel(gs_params in, const uint8_t* __restrict__ action,
                      const uint32_t* __restrict__ offsets, int zero_created, int64_t n_out,
                      float* __restrict__ o_means, float* __restrict__ o_log_scales,
                      float* __restrict__ o_quats, float* __restrict__ o_logits,
                      float* __restrict__ o_sh) {
  const int64_t n = in.n;
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= n) return;
  const uint8_t a = action[g];
  if (a == kRemove) return;
  const int64_t j0 = offsets[g];
  const int copies = a == kKeep ? 1 : 2;
  if (j0 + copies > n_out) return;   // defensive: outputs were sized from the plan
  const float keep = (a == kKeep || !zero_created) ? 1.0f : 0.0f;
  for (int c = 0; c < copies; ++c) {
    const int64_t j = j0 + c;
    for (int r = 0; r < 3; ++r) {
      o_means[r * n_out + j] = keep * in.means[r * n + g];
      o_log_scales[r * n_out + j] = keep * in.log_scales[r * n + g];
    }
    for (int r = 0; r < 4; ++r) o_quats[r * n_out + j] = keep * in.quats[r * n + g];
    o_logits[j] = keep * in.opacity_logits[g];
#pragma unroll
    for (int k = 0; k < K * 3; ++k) o_sh[(int64_t)k * n_out + j] = keep * in.sh[(int64_t)k * n + g];
  }
}

__global__ void __launch_bounds__(256)
reset_opacity_kernel(float* __restrict__ logits, int64_t n, float cap) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < n; g += stride)
    logits[g] = fminf(logits[g], cap);
}

static int check_densify_config(const gs_densify_config* c, DensifyRules* r) {
  if (!c) return GS_ERR_ARG;
  if (!(c->grad_threshold >= 0.0f) || !(c->min_opacity >= 0.0f) || !(c->split_scale > 0.0f) ||
      !(c->split_factor > 1.0f) || !isfinite(c->max_world_scale) || !isfinite(c->max_screen_radius))
    return GS_ERR_ARG;
  r->grad_threshold = c->grad_threshold;
  r->min_opacity = c->min_opacity;
  r->split_scale = c->split_scale;
  r->max_world_scale = c->max_world_scale;
  r->max_screen_radius = c->max_screen_radius;
  r->log_split_factor = logf(c->split_factor);
  return GS_OK;
}

}  // namespace gs

using namespace gs;

extern "C" void gs_default_densify_config(gs_densify_config* c) {
  if (!c) return;
  c->grad_threshold = 0.0002f;
  c->min_opacity = 0.005f;
  c->split_scale = 0.01f;
  c->max_world_scale = 0.0f;
  c->max_screen_radius = 0.0f;
  c->split_factor = 1.6f;
}

extern "C" int gs_densify_accumulate(const gs_projected* proj, const float* grad2d,
                                     const gs_camera* cams, int32_t n_views, int64_t n,
                                     float* grad_sum, int32_t* view_count, float* max_radius,
                                     gs_stream_t stream) {
  if (!proj || !grad2d || !grad_sum || !view_count || !max_radius || n < 0) return GS_ERR_ARG;
  TileViews tv;
  int rc = fill_tile_views(cams, n_views, 16, &tv);
  if (rc != GS_OK) return rc;
  if (n == 0) return GS_OK;
  if (!proj->tiles_touched || !proj->record) return GS_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  densify_accumulate_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(
      proj->tiles_touched, proj->record, grad2d, tv, n, grad_sum, view_count, max_radius);
  return launch_status();
}

extern "C" size_t gs_densify_workspace_bytes(int64_t n) {
  if (n < 0) return 0;
  return (size_t)((n + kDenTile - 1) / kDenTile + 1) * sizeof(uint32_t);
}

extern "C" int gs_densify_plan(const gs_params* params, const float* grad_sum,
                               const int32_t* view_count, const float* max_radius,
                               const gs_densify_config* cfg, uint8_t* action, uint32_t* offsets,
                               uint32_t* n_out, void* workspace, size_t workspace_bytes,
                               gs_stream_t stream) {
  DensifyRules r;
  if (!params || params->n < 0 || !n_out) return GS_ERR_ARG;
  int rc = check_densify_config(cfg, &r);
  if (rc != GS_OK) return rc;
  const int64_t n = params->n;
  if (n >= ((int64_t)1 << 31)) return GS_ERR_UNSUPPORTED;
  if (n > 0 && (!params->log_scales || !params->opacity_logits || !grad_sum || !view_count ||
                !max_radius || !action || !offsets))
    return GS_ERR_ARG;
  if (workspace_bytes < gs_densify_workspace_bytes(n) || !workspace) return GS_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t nb = (n + kDenTile - 1) / kDenTile;
  uint32_t* sums = static_cast<uint32_t*>(workspace);
  if (nb > 0)
    densify_plan_kernel<<<dim3((unsigned)nb), kDenBlock, 0, s>>>(
        params->log_scales, params->opacity_logits, grad_sum, view_count, max_radius, n, r,
        action, sums);
  densify_scan_kernel<<<1, 1024, 0, s>>>(sums, nb, n_out);
  if (nb > 0)
    densify_offsets_kernel<<<dim3((unsigned)nb), kDenBlock, 0, s>>>(action, n, sums, offsets);
  return launch_status();
}

extern "C" int gs_densify_apply(const gs_params* params, int32_t sh_degree, const uint8_t* action,
                                const uint32_t* offsets, const float* normals,
                                const gs_densify_config* cfg, const gs_params_grad* out,
                                int64_t n_out, uint32_t* src_index, gs_stream_t stream) {
  DensifyRules r;
  if (!params || !out || params->n < 0 || n_out < 0) return GS_ERR_ARG;
  int rc = check_densify_config(cfg, &r);
  if (rc != GS_OK) return rc;
  if (sh_degree < 0 || sh_degree > 3) return GS_ERR_ARG;
  const int64_t n = params->n;
  if (n == 0 || n_out == 0) return GS_OK;
  if (!params->means || !params->log_scales || !params->quats || !params->opacity_logits ||
      !params->sh || !action || !offsets || !normals || !out->means || !out->log_scales ||
      !out->quats || !out->opacity_logits || !out->sh)
    return GS_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const dim3 grid((unsigned)((n + 255) / 256));
#define GS_APPLY(K)                                                                             \
  densify_apply_kernel<K><<<grid, 256, 0, s>>>(*params, action, offsets, normals,              \
                                               r.log_split_factor, n_out, out->means,          \
                                               out->log_scales, out->quats,                   \
                                               out->opacity_logits, out->sh, src_index)
  switch (sh_degree) {
    case 0: GS_APPLY(1); break;
    case 1: GS_APPLY(4); break;
    case 2: GS_APPLY(9); break;
    default: GS_APPLY(16); break;
  }
#undef GS_APPLY
  return launch_status();
}

extern "C" int gs_densify_gather(const gs_params* state, int32_t sh_degree, const uint8_t* action,
                                 const uint32_t* offsets, int32_t zero_created,
                                 const gs_params_grad* out, int64_t n_out, gs_stream_t stream) {
  if (!state || !out || state->n < 0 || n_out < 0) return GS_ERR_ARG;
  if (sh_degree < 0 || sh_degree > 3) return GS_ERR_ARG;
  const int64_t n = state->n;
  if (n == 0 || n_out == 0) return GS_OK;
  if (!state->means || !state->log_scales || !state->quats || !state->opacity_logits ||
      !state->sh || !action || !offsets || !out->means || !out->log_scales || !out->quats ||
      !out->opacity_logits || !out->sh)
    return GS_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const dim3 grid((unsigned)((n + 255) / 256));
#define GS_GATHER(K)                                                                            \
  densify_gather_kernel<K><<<grid, 256, 0, s>>>(*state, action, offsets, zero_created, n_out,   \
                                                out->means, out->log_scales, out->quats,      \
                                                out->opacity_logits, out->sh)
  switch (sh_degree) {
    case 0: GS_GATHER(1); break;
    case 1: GS_GATHER(4); break;
    case 2: GS_GATHER(9); break;
    default: GS_GATHER(16); break;
  }
#undef GS_GATHER
  return launch_status();
}

extern "C" int gs_reset_opacity(float* opacity_logits, int64_t n, float max_opacity,
                                gs_stream_t stream) {
  if (n < 0 || !(max_opacity > 0.0f && max_opacity < 1.0f)) return GS_ERR_ARG;
  if (n == 0) return GS_OK;
  if (!opacity_logits) return GS_ERR_ARG;
  const float cap = (float)log((double)max_opacity / (1.0 - (double)max_opacity));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  reset_opacity_kernel<<<dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), 256, 0, s>>>(
      opacity_logits, n, cap);
  return launch_status();
}
