// FP64 per-Gaussian math shared by the projection forward and backward kernels, so
// that both take every discrete decision (culls, colour clamp) from identical
// instruction sequences. The library is built with -ffp-contract=off; fused
// multiply-adds appear only where written.
#pragma once

#include "gs_internal.h"

namespace gs {

// Real SH basis, degree <= 3, as polynomials of the unit direction (x, y, z);
// coefficient index k = l^2 + l + m, no Condon-Shortley phase.
constexpr double kY0 = 0.28209479177387814;   // 1 / (2 sqrt(pi))
constexpr double kY1 = 0.4886025119029199;    // sqrt(3 / (4 pi))
constexpr double kY2a = 1.0925484305920792;   // sqrt(15 / (4 pi))
constexpr double kY2b = 0.31539156525252005;  // sqrt(5 / (16 pi))
constexpr double kY2c = 0.5462742152960396;   // sqrt(15 / (16 pi))
constexpr double kY3a = 0.5900435899266435;   // sqrt(35 / (32 pi))
constexpr double kY3b = 2.890611442640554;    // sqrt(105 / (4 pi))
constexpr double kY3c = 0.4570457994644658;   // sqrt(21 / (32 pi))
constexpr double kY3d = 0.3731763325901154;   // sqrt(7 / (16 pi))
constexpr double kY3e = 1.445305721320277;    // sqrt(105 / (16 pi))

// FP32 evaluation (the colour's error, ~1e-7, is far below the image tolerance):
// Y[k] for the unit direction (x, y, z).
template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = (float)kY0;
  if constexpr (DEG >= 1) {
    Y[1] = (float)kY1 * y;
    Y[2] = (float)kY1 * z;
    Y[3] = (float)kY1 * x;
  }
  if constexpr (DEG >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = (float)kY2a * x * y;
    Y[5] = (float)kY2a * y * z;
    Y[6] = (float)kY2b * (3.0f * zz - 1.0f);
    Y[7] = (float)kY2a * x * z;
    Y[8] = (float)kY2c * (xx - yy);
    if constexpr (DEG >= 3) {
      Y[9] = (float)kY3a * y * (3.0f * xx - yy);
      Y[10] = (float)kY3b * x * y * z;
      Y[11] = (float)kY3c * y * (5.0f * zz - 1.0f);
      Y[12] = (float)kY3d * z * (5.0f * zz - 3.0f);
      Y[13] = (float)kY3c * x * (5.0f * zz - 1.0f);
      Y[14] = (float)kY3e * z * (xx - yy);
      Y[15] = (float)kY3a * x * (xx - 3.0f * yy);
    }
  }
}

// g = sum_k w[k] grad Y_k(x, y, z): the gradient of each basis polynomial with
// respect to (x, y, z), weighted and summed without storing it.
template <int DEG>
__device__ __forceinline__ void sh_weighted_grad(float x, float y, float z, const float* w, float* g) {
  g[0] = g[1] = g[2] = 0.0f;
  if constexpr (DEG >= 1) {
    g[0] += (float)kY1 * w[3];
    g[1] += (float)kY1 * w[1];
    g[2] += (float)kY1 * w[2];
  }
  if constexpr (DEG >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    const float a = (float)kY2a, b = (float)kY2b, c = (float)kY2c;
    g[0] += a * (y * w[4] + z * w[7]) + c * 2.0f * x * w[8];
    g[1] += a * (x * w[4] + z * w[5]) - c * 2.0f * y * w[8];
    g[2] += a * (y * w[5] + x * w[7]) + b * 6.0f * z * w[6];
    if constexpr (DEG >= 3) {
      const float A = (float)kY3a, B = (float)kY3b, C = (float)kY3c, D = (float)kY3d,
                  E = (float)kY3e;
      g[0] += A * 6.0f * x * y * w[9] + B * y * z * w[10] + C * (5.0f * zz - 1.0f) * w[13] +
              E * 2.0f * x * z * w[14] + A * (3.0f * xx - 3.0f * yy) * w[15];
      g[1] += A * (3.0f * xx - 3.0f * yy) * w[9] + B * x * z * w[10] +
              C * (5.0f * zz - 1.0f) * w[11] - E * 2.0f * y * z * w[14] - A * 6.0f * x * y * w[15];
      g[2] += B * x * y * w[10] + C * 10.0f * y * z * w[11] + D * (15.0f * zz - 3.0f) * w[12] +
              C * 10.0f * x * z * w[13] + E * (xx - yy) * w[14];
    }
  }
}

// 1/x, 1/sqrt(x) and sqrt(x) for finite x > 0: the hardware estimates (v_rcp_f64,
// v_rsq_f64) refined by two Newton steps, within an ulp or two of the correctly rounded
// value at a fraction of the IEEE sequences' cost. Every decision taken from these
// values (pixel-box bounds, culls) has a margin many orders of magnitude wider. x = 0
// gives inf or NaN, which the callers' culls reject as before.
__device__ __forceinline__ double rcp_d(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ double rsqrt_d(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  return y * fma(-hx * y, y, 1.5);
}

__device__ __forceinline__ double sqrt_d(double x) {
  const double y = rsqrt_d(x);
  const double s = x * y;
  return fma(fma(-s, s, x), 0.5 * y, s);
}

// Unit view direction from the camera centre to the mean: the difference in FP64
// (the mean and the centre may be far apart and close in value), rounded once to FP32,
// then normalised in FP32 (the SH colour is evaluated in FP32 anyway; the direction
// is within a few FP32 ulps). Returns the distance.
__device__ __forceinline__ float view_dir(const Cam& cam, double x, double y, double z, float* d) {
  const float ex = (float)(x - cam.C[0]), ey = (float)(y - cam.C[1]), ez = (float)(z - cam.C[2]);
  const float r2 = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
  const float inv = __builtin_amdgcn_rsqf(r2);
  d[0] = ex * inv;
  d[1] = ey * inv;
  d[2] = ez * inv;
  return r2 * inv;
}

// Colour before the clamp, per channel: sum_k sh[k][ch] Y[k] + 0.5, in a fixed
// order so the forward and backward passes take the same clamp decision.
template <int K>
__device__ __forceinline__ float sh_colour_raw(const float (*shc)[3], const float* Y, int ch) {
  float acc = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) acc = fmaf(shc[k][ch], Y[k], acc);
  return acc + 0.5f;
}

// Rotation of a unit quaternion (r, i, j, k): App. A, Eq. (quat).
__device__ __forceinline__ void quat_to_rot(double r, double i, double j, double k, double* R) {
  R[0] = 1.0 - 2.0 * (j * j + k * k);
  R[1] = 2.0 * (i * j - r * k);
  R[2] = 2.0 * (i * k + r * j);
  R[3] = 2.0 * (i * j + r * k);
  R[4] = 1.0 - 2.0 * (i * i + k * k);
  R[5] = 2.0 * (j * k - r * i);
  R[6] = 2.0 * (i * k - r * j);
  R[7] = 2.0 * (j * k + r * i);
  R[8] = 1.0 - 2.0 * (i * i + j * j);
}

// Camera-space position: each row evaluated as ((R0 x + R1 y) + R2 z) + t in FP64,
// in this order and unfused, so the FP32 rounding of the depth is reproducible.
__device__ __forceinline__ double cam_row(const float* Rrow, float t, double x, double y, double z) {
  return __dadd_rn(__dadd_rn(__dadd_rn(__dmul_rn((double)Rrow[0], x), __dmul_rn((double)Rrow[1], y)),
                             __dmul_rn((double)Rrow[2], z)),
                   (double)t);
}

// Everything the forward and backward projection derive from one (Gaussian, view).
struct ProjGeom {
  double tx, ty, tz, iz;    // camera-space mean and 1 / tz
  double WM[9];             // W * M, row-major
  double A0[3], A1[3];      // rows of A = J W M (Sigma' = A A^T)
  double a, b, c, det;      // Sigma' = [[a, b], [b, c]], det by Cauchy-Binet
  double sa, isa;           // sqrt(a) and 1 / sqrt(a) (forward only)
  double u, v;              // projected mean
  int32_t i_lo, i_hi, j_lo, j_hi;
  bool ok;
};

__device__ __forceinline__ double ceil_clamped(double x, double lo, double hi) {
  return fmin(fmax(ceil(x), lo), hi);
}

__device__ __forceinline__ double floor_clamped(double x, double lo, double hi) {
  return fmin(fmax(floor(x), lo), hi);
}

// Camera transform, near cull and the 2D covariance Sigma' = A A^T with A = J W M
// (Sec. 4, Eq. volume-render; J the pinhole Jacobian at the camera-space mean).
// Shared by both passes; returns false when the Gaussian is culled here.
__device__ __forceinline__ bool project_covariance(const Cam& cam, const Rules& rules, double x,
                                                   double y, double z, const double* M,
                                                   ProjGeom& p) {
  p.tx = cam_row(cam.R + 0, cam.t[0], x, y, z);
  p.ty = cam_row(cam.R + 3, cam.t[1], x, y, z);
  p.tz = cam_row(cam.R + 6, cam.t[2], x, y, z);
  if (!((float)p.tz >= rules.near_z)) return false;  // near cull on the FP32 depth
  // fused multiply-adds throughout (written out: the library is built without
  // contraction); the backward recomputes this with the same instructions
  for (int r = 0; r < 3; ++r)
    for (int c2 = 0; c2 < 3; ++c2)
      p.WM[r * 3 + c2] = fma((double)cam.R[r * 3 + 0], M[0 * 3 + c2],
                             fma((double)cam.R[r * 3 + 1], M[1 * 3 + c2],
                                 (double)cam.R[r * 3 + 2] * M[2 * 3 + c2]));
  const double fx = cam.fx, fy = cam.fy;
  p.iz = rcp_d(p.tz);
  const double J00 = fx * p.iz, J02 = -fx * p.tx * p.iz * p.iz;
  const double J11 = fy * p.iz, J12 = -fy * p.ty * p.iz * p.iz;
  for (int c2 = 0; c2 < 3; ++c2) {
    p.A0[c2] = fma(J00, p.WM[0 * 3 + c2], J02 * p.WM[2 * 3 + c2]);
    p.A1[c2] = fma(J11, p.WM[1 * 3 + c2], J12 * p.WM[2 * 3 + c2]);
  }
  p.a = fma(p.A0[0], p.A0[0], fma(p.A0[1], p.A0[1], p.A0[2] * p.A0[2]));
  p.b = fma(p.A0[0], p.A1[0], fma(p.A0[1], p.A1[1], p.A0[2] * p.A1[2]));
  p.c = fma(p.A1[0], p.A1[0], fma(p.A1[1], p.A1[1], p.A1[2] * p.A1[2]));
  // det(A A^T) = sum of squared 2x2 minors of A (Cauchy-Binet): no a c - b^2 cancellation
  const double m01 = fma(p.A0[0], p.A1[1], -(p.A0[1] * p.A1[0]));
  const double m02 = fma(p.A0[0], p.A1[2], -(p.A0[2] * p.A1[0]));
  const double m12 = fma(p.A0[1], p.A1[2], -(p.A0[2] * p.A1[1]));
  p.det = fma(m01, m01, fma(m02, m02, m12 * m12));
  return (p.det > 0.0) && isfinite(p.det) && isfinite(p.a) && isfinite(p.c);
}

// Projected mean and 3-sigma pixel box (forward only).
__device__ __forceinline__ void project_geometry(const Cam& cam, const Rules& rules, double x,
                                                 double y, double z, const double* M,
                                                 ProjGeom& p) {
  p.ok = project_covariance(cam, rules, x, y, z, M, p);
  if (!p.ok) return;
  p.u = (double)cam.fx * p.tx * p.iz + (double)cam.cx;
  p.v = (double)cam.fy * p.ty * p.iz + (double)cam.cy;
  p.ok = isfinite(p.u) && isfinite(p.v);
  if (!p.ok) return;
  const double ext = (double)rules.ext;
  p.isa = rsqrt_d(p.a);
  p.sa = p.a * p.isa;
  const double rx = ext * p.sa, ry = ext * sqrt_d(p.c);
  // pixel i is covered iff its centre i + 0.5 lies in [u - rx, u + rx]
  const double Wm1 = cam.W - 1, Hm1 = cam.H - 1;
  const double ilo = ceil_clamped(p.u - rx - 0.5, 0.0, Wm1 + 1.0);
  const double ihi = floor_clamped(p.u + rx - 0.5, -1.0, Wm1);
  const double jlo = ceil_clamped(p.v - ry - 0.5, 0.0, Hm1 + 1.0);
  const double jhi = floor_clamped(p.v + ry - 0.5, -1.0, Hm1);
  p.i_lo = (int32_t)ilo;
  p.i_hi = (int32_t)ihi;
  p.j_lo = (int32_t)jlo;
  p.j_hi = (int32_t)jhi;
  p.ok = (p.i_lo <= p.i_hi) && (p.j_lo <= p.j_hi);
}

}  // namespace gs
