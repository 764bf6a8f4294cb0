// Photometric loss of Sec. 5.1, L = (1 - lambda) L1 + lambda (1 - SSIM), and its
// gradient with respect to the rendered image, as two stencil passes over 32 x 32
// output tiles (one workgroup per tile and colour channel):
//   pass 1: the five windowed moments of (x, y) -> SSIM, the loss, and the three
//           partial derivatives of SSIM with respect to mu_x, E[x^2], E[xy];
//   pass 2: the window sums of those partials -> dL/dx.
// The 11 x 11 Gaussian window (sigma 1.5) is separable, so each window sum is a
// horizontal 11-tap pass into LDS followed by a vertical one. Values outside the
// image are zero (the window is not renormalised at the borders).
#include <algorithm>
#include <math.h>

#include "gs_internal.h"

namespace gs {

constexpr int kLT = 32;                 // output tile edge
constexpr int kLR = 5;                  // window radius
constexpr int kLI = kLT + 2 * kLR;      // staged input edge (42)
constexpr int kLThreads = 256;
constexpr float kC1 = 0.0001f;          // (0.01 * dynamic range 1)^2
constexpr float kC2 = 0.0009f;          // (0.03 * dynamic range 1)^2

struct LossArgs {
  float g[2 * kLR + 1];   // normalised 1D window
  float lambda;
};

__device__ __forceinline__ int tile_view(const TileViews& tv, int tile) {
  int v = 0;
  while (v + 1 < tv.n_views && tile >= tv.tile_offset[v + 1]) ++v;
  return v;
}

// Stage a (32 + 10)^2 window of one channel plane (zero outside the image).
template <int NM>
__device__ __forceinline__ void stage_planes(const float* const (&src)[NM], int W, int H, int x0,
                                             int y0, float (*dst)[kLI][kLI + 1]) {
  for (int k = threadIdx.x; k < kLI * kLI; k += kLThreads) {
    const int r = k / kLI, q = k - r * kLI;
    const int gy = y0 - kLR + r, gx = x0 - kLR + q;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    const int64_t off = in ? (int64_t)gy * W + gx : 0;
#pragma unroll
    for (int m = 0; m < NM; ++m) dst[m][r][q] = in ? src[m][off] : 0.0f;
  }
}

// Both passes are register blocked: in the horizontal pass a thread produces four
// neighbouring columns of a row from 14 staged values, in the vertical pass four
// neighbouring rows of a column, so each staged value is read from LDS about 3.5
// times instead of 11. Lanes walk rows (horizontal) or columns (vertical), which keeps
// the LDS accesses free of bank conflicts (odd row strides).
constexpr int kLB = 4;                          // outputs per thread along the pass
constexpr int kLW = kLB + 2 * kLR;              // staged values per thread (14)

__global__ void __launch_bounds__(kLThreads)
ssim_moments_kernel(const float* __restrict__ image, const float* __restrict__ target,
                    TileViews tv, LossArgs la, float* __restrict__ partials,
                    float* __restrict__ loss) {
  __shared__ float s_in[2][kLI][kLI + 1];
  __shared__ float s_h[5][kLI][kLT + 1];
  __shared__ float s_part[kLThreads / kWave];
  const int tile = blockIdx.x, c = blockIdx.y;
  const int v = tile_view(tv, tile);
  const int W = tv.W[v], H = tv.H[v];
  const int64_t HW = (int64_t)W * H;
  const int local = tile - tv.tile_offset[v];
  const int x0 = (local % tv.tiles_x[v]) * kLT, y0 = (local / tv.tiles_x[v]) * kLT;
  const int64_t plane = 3 * tv.pix_offset[v] + c * HW;
  const float* const src[2] = {image + plane, target + plane};
  stage_planes<2>(src, W, H, x0, y0, s_in);
  __syncthreads();

  // horizontal pass: 42 rows x 32 columns of the five moments, four columns per item
  for (int k = threadIdx.x; k < kLI * (kLT / kLB); k += kLThreads) {
    const int r = k % kLI, q0 = (k / kLI) * kLB;
    float xv[kLW], yv[kLW];
#pragma unroll
    for (int j = 0; j < kLW; ++j) {
      xv[j] = s_in[0][r][q0 + j];
      yv[j] = s_in[1][r][q0 + j];
    }
#pragma unroll
    for (int o = 0; o < kLB; ++o) {
      float mx = 0.0f, my = 0.0f, xx = 0.0f, yy = 0.0f, xy = 0.0f;
#pragma unroll
      for (int b = 0; b <= 2 * kLR; ++b) {
        const float w = la.g[b], wx = w * xv[o + b], wy = w * yv[o + b];
        mx += wx;
        my += wy;
        xx = fmaf(wx, xv[o + b], xx);
        yy = fmaf(wy, yv[o + b], yy);
        xy = fmaf(wx, yv[o + b], xy);
      }
      s_h[0][r][q0 + o] = mx;
      s_h[1][r][q0 + o] = my;
      s_h[2][r][q0 + o] = xx;
      s_h[3][r][q0 + o] = yy;
      s_h[4][r][q0 + o] = xy;
    }
  }
  __syncthreads();

  const float inv = 1.0f / (3.0f * (float)HW);
  const float* X = src[0];
  const float* Y = src[1];
  float part = 0.0f;
  const int64_t P = 3 * tv.pix_offset[tv.n_views];   // values per partial map
  // vertical pass: 32 columns x 8 groups of four rows, one item per thread
  {
    const int q = threadIdx.x % kLT, r0 = (threadIdx.x / kLT) * kLB;
    float m[5][kLB];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      float col[kLW];
#pragma unroll
      for (int a = 0; a < kLW; ++a) col[a] = s_h[j][r0 + a][q];
#pragma unroll
      for (int o = 0; o < kLB; ++o) {
        float acc = 0.0f;
#pragma unroll
        for (int a = 0; a <= 2 * kLR; ++a) acc = fmaf(la.g[a], col[o + a], acc);
        m[j][o] = acc;
      }
    }
    const int gx = x0 + q;
#pragma unroll
    for (int o = 0; o < kLB; ++o) {
      const int gy = y0 + r0 + o;
      if (gy >= H || gx >= W) continue;
      const float mx = m[0][o], my = m[1][o];
      const float a1 = 2.0f * mx * my + kC1;
      const float a2 = 2.0f * (m[4][o] - mx * my) + kC2;
      const float b1 = mx * mx + my * my + kC1;
      const float b2 = (m[2][o] - mx * mx) + (m[3][o] - my * my) + kC2;
      const float den = b1 * b2;
      const float iden = 1.0f / den;
      const float S = a1 * a2 * iden;
      // dS/dmu_x, dS/dE[x^2], dS/dE[xy]
      const float d_mx = 2.0f * my * (a2 - a1) * iden - 2.0f * mx * S * (b2 - b1) * iden;
      const float d_xx = -S / b2;
      const float d_xy = 2.0f * a1 * iden;
      const int64_t o_ = plane + (int64_t)gy * W + gx;
      partials[o_] = d_mx;
      partials[P + o_] = d_xx;
      partials[2 * P + o_] = d_xy;
      const float d = X[(int64_t)gy * W + gx] - Y[(int64_t)gy * W + gx];
      part += ((1.0f - la.lambda) * fabsf(d) + la.lambda * (1.0f - S)) * inv;
    }
  }
  if (loss) {
    part = wave_sum_to_lane63(part);
    if (__lane_id() == kWave - 1) s_part[threadIdx.x / kWave] = part;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss + v, s_part[0] + s_part[1] + s_part[2] + s_part[3]);
  }
}

__global__ void __launch_bounds__(kLThreads)
ssim_grad_kernel(const float* __restrict__ image, const float* __restrict__ target,
                 TileViews tv, LossArgs la, const float* __restrict__ partials,
                 float* __restrict__ dL) {
  __shared__ float s_in[3][kLI][kLI + 1];
  __shared__ float s_h[3][kLI][kLT + 1];
  const int tile = blockIdx.x, c = blockIdx.y;
  const int v = tile_view(tv, tile);
  const int W = tv.W[v], H = tv.H[v];
  const int64_t HW = (int64_t)W * H;
  const int local = tile - tv.tile_offset[v];
  const int x0 = (local % tv.tiles_x[v]) * kLT, y0 = (local / tv.tiles_x[v]) * kLT;
  const int64_t plane = 3 * tv.pix_offset[v] + c * HW;
  const int64_t P = 3 * tv.pix_offset[tv.n_views];
  const float* const src[3] = {partials + plane, partials + P + plane, partials + 2 * P + plane};
  stage_planes<3>(src, W, H, x0, y0, s_in);
  __syncthreads();
  for (int k = threadIdx.x; k < kLI * (kLT / kLB); k += kLThreads) {
    const int r = k % kLI, q0 = (k / kLI) * kLB;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      float row[kLW];
#pragma unroll
      for (int b = 0; b < kLW; ++b) row[b] = s_in[j][r][q0 + b];
#pragma unroll
      for (int o = 0; o < kLB; ++o) {
        float acc = 0.0f;
#pragma unroll
        for (int b = 0; b <= 2 * kLR; ++b) acc = fmaf(la.g[b], row[o + b], acc);
        s_h[j][r][q0 + o] = acc;
      }
    }
  }
  __syncthreads();
  const float inv = 1.0f / (3.0f * (float)HW);
  const float l1w = (1.0f - la.lambda) * inv, sw = -la.lambda * inv;
  const int q = threadIdx.x % kLT, r0 = (threadIdx.x / kLT) * kLB;
  float f[3][kLB];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    float col[kLW];
#pragma unroll
    for (int a = 0; a < kLW; ++a) col[a] = s_h[j][r0 + a][q];
#pragma unroll
    for (int o = 0; o < kLB; ++o) {
      float acc = 0.0f;
#pragma unroll
      for (int a = 0; a <= 2 * kLR; ++a) acc = fmaf(la.g[a], col[o + a], acc);
      f[j][o] = acc;
    }
  }
  const int gx = x0 + q;
#pragma unroll
  for (int o = 0; o < kLB; ++o) {
    const int gy = y0 + r0 + o;
    if (gy >= H || gx >= W) continue;
    const int64_t o_ = plane + (int64_t)gy * W + gx;
    const float x = image[o_], y = target[o_];
    const float d = x - y;
    const float sg = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
    dL[o_] = l1w * sg + sw * (f[0][o] + 2.0f * x * f[1][o] + y * f[2][o]);
  }
}

}  // namespace gs

using namespace gs;

extern "C" size_t gs_loss_workspace_bytes(const gs_camera* cams, int32_t n_views) {
  TileViews tv;
  if (fill_tile_views(cams, n_views, kLT, &tv) != GS_OK) return 0;
  return (size_t)9 * (size_t)tv.pix_offset[n_views] * sizeof(float);
}

extern "C" int gs_loss_photometric(const float* image, const float* target, const gs_camera* cams,
                                   int32_t n_views, float lambda, float* dL_dimage, float* loss,
                                   void* workspace, size_t workspace_bytes, gs_stream_t stream) {
  if (!image || !target || !dL_dimage) return GS_ERR_ARG;
  if (!(lambda >= 0.0f && lambda <= 1.0f)) return GS_ERR_ARG;
  TileViews tv;
  int rc = fill_tile_views(cams, n_views, kLT, &tv);
  if (rc != GS_OK) return rc;
  if (!workspace || workspace_bytes < gs_loss_workspace_bytes(cams, n_views)) return GS_ERR_ARG;
  LossArgs la;
  double g[2 * kLR + 1], sum = 0.0;
  for (int k = 0; k <= 2 * kLR; ++k) {
    const double r = (double)(k - kLR);
    g[k] = exp(-r * r / (2.0 * 1.5 * 1.5));
    sum += g[k];
  }
  for (int k = 0; k <= 2 * kLR; ++k) la.g[k] = (float)(g[k] / sum);
  la.lambda = lambda;
  const unsigned tiles = (unsigned)tv.tile_offset[n_views];
  if (tiles == 0) return GS_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float* part = static_cast<float*>(workspace);
  ssim_moments_kernel<<<dim3(tiles, 3), kLThreads, 0, s>>>(image, target, tv, la, part, loss);
  ssim_grad_kernel<<<dim3(tiles, 3), kLThreads, 0, s>>>(image, target, tv, la, part, dL_dimage);
  return launch_status();
}
