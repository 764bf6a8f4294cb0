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

template <int DEG>
__device__ __forceinline__ void sh_basis(double x, double y, double z, double* Y) {
  Y[0] = kY0;
  if constexpr (DEG >= 1) {
    Y[1] = kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = kY1 * x;
  }
  if constexpr (DEG >= 2) {
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kY2a * x * y;
    Y[5] = kY2a * y * z;
    Y[6] = kY2b * (3.0 * zz - 1.0);
    Y[7] = kY2a * x * z;
    Y[8] = kY2c * (xx - yy);
    if constexpr (DEG >= 3) {
      Y[9] = kY3a * y * (3.0 * xx - yy);
      Y[10] = kY3b * x * y * z;
      Y[11] = kY3c * y * (5.0 * zz - 1.0);
      Y[12] = kY3d * z * (5.0 * zz - 3.0);
      Y[13] = kY3c * x * (5.0 * zz - 1.0);
      Y[14] = kY3e * z * (xx - yy);
      Y[15] = kY3a * x * (xx - 3.0 * yy);
    }
  }
}

// Gradient of each basis polynomial with respect to (x, y, z): G[k][0..2].
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(double x, double y, double z, double (*G)[3]) {
  G[0][0] = G[0][1] = G[0][2] = 0.0;
  if constexpr (DEG >= 1) {
    G[1][0] = 0.0;  G[1][1] = kY1;  G[1][2] = 0.0;
    G[2][0] = 0.0;  G[2][1] = 0.0;  G[2][2] = kY1;
    G[3][0] = kY1;  G[3][1] = 0.0;  G[3][2] = 0.0;
  }
  if constexpr (DEG >= 2) {
    const double xx = x * x, yy = y * y, zz = z * z;
    G[4][0] = kY2a * y;        G[4][1] = kY2a * x;         G[4][2] = 0.0;
    G[5][0] = 0.0;             G[5][1] = kY2a * z;         G[5][2] = kY2a * y;
    G[6][0] = 0.0;             G[6][1] = 0.0;              G[6][2] = kY2b * 6.0 * z;
    G[7][0] = kY2a * z;        G[7][1] = 0.0;              G[7][2] = kY2a * x;
    G[8][0] = kY2c * 2.0 * x;  G[8][1] = -kY2c * 2.0 * y;  G[8][2] = 0.0;
    if constexpr (DEG >= 3) {
      G[9][0] = kY3a * 6.0 * x * y;
      G[9][1] = kY3a * (3.0 * xx - 3.0 * yy);
      G[9][2] = 0.0;
      G[10][0] = kY3b * y * z;
      G[10][1] = kY3b * x * z;
      G[10][2] = kY3b * x * y;
      G[11][0] = 0.0;
      G[11][1] = kY3c * (5.0 * zz - 1.0);
      G[11][2] = kY3c * 10.0 * y * z;
      G[12][0] = 0.0;
      G[12][1] = 0.0;
      G[12][2] = kY3d * (15.0 * zz - 3.0);
      G[13][0] = kY3c * (5.0 * zz - 1.0);
      G[13][1] = 0.0;
      G[13][2] = kY3c * 10.0 * x * z;
      G[14][0] = kY3e * 2.0 * x * z;
      G[14][1] = -kY3e * 2.0 * y * z;
      G[14][2] = kY3e * (xx - yy);
      G[15][0] = kY3a * (3.0 * xx - 3.0 * yy);
      G[15][1] = -kY3a * 6.0 * x * y;
      G[15][2] = 0.0;
    }
  }
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
  double tx, ty, tz;        // camera-space mean
  double WM[9];             // W * M, row-major
  double A0[3], A1[3];      // rows of A = J W M (Sigma' = A A^T)
  double a, b, c, det;      // Sigma' = [[a, b], [b, c]], det by Cauchy-Binet
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

__device__ __forceinline__ void project_geometry(const Cam& cam, const Rules& rules, double x,
                                                 double y, double z, const double* M,
                                                 ProjGeom& p) {
  p.tx = cam_row(cam.R + 0, cam.t[0], x, y, z);
  p.ty = cam_row(cam.R + 3, cam.t[1], x, y, z);
  p.tz = cam_row(cam.R + 6, cam.t[2], x, y, z);
  p.ok = ((float)p.tz >= rules.near_z);  // near cull on the FP32 depth
  if (!p.ok) return;
  for (int r = 0; r < 3; ++r)
    for (int c2 = 0; c2 < 3; ++c2)
      p.WM[r * 3 + c2] = (double)cam.R[r * 3 + 0] * M[0 * 3 + c2] +
                         (double)cam.R[r * 3 + 1] * M[1 * 3 + c2] +
                         (double)cam.R[r * 3 + 2] * M[2 * 3 + c2];
  const double fx = cam.fx, fy = cam.fy;
  const double iz = 1.0 / p.tz;
  const double J00 = fx * iz, J02 = -fx * p.tx * iz * iz;
  const double J11 = fy * iz, J12 = -fy * p.ty * iz * iz;
  for (int c2 = 0; c2 < 3; ++c2) {
    p.A0[c2] = J00 * p.WM[0 * 3 + c2] + J02 * p.WM[2 * 3 + c2];
    p.A1[c2] = J11 * p.WM[1 * 3 + c2] + J12 * p.WM[2 * 3 + c2];
  }
  p.a = p.A0[0] * p.A0[0] + p.A0[1] * p.A0[1] + p.A0[2] * p.A0[2];
  p.b = p.A0[0] * p.A1[0] + p.A0[1] * p.A1[1] + p.A0[2] * p.A1[2];
  p.c = p.A1[0] * p.A1[0] + p.A1[1] * p.A1[1] + p.A1[2] * p.A1[2];
  // det(A A^T) = sum of squared 2x2 minors of A (Cauchy-Binet): no a c - b^2 cancellation
  const double m01 = p.A0[0] * p.A1[1] - p.A0[1] * p.A1[0];
  const double m02 = p.A0[0] * p.A1[2] - p.A0[2] * p.A1[0];
  const double m12 = p.A0[1] * p.A1[2] - p.A0[2] * p.A1[1];
  p.det = m01 * m01 + m02 * m02 + m12 * m12;
  p.u = fx * p.tx / p.tz + (double)cam.cx;
  p.v = fy * p.ty / p.tz + (double)cam.cy;
  p.ok = (p.det > 0.0) && isfinite(p.det) && isfinite(p.a) && isfinite(p.c) &&
         isfinite(p.u) && isfinite(p.v);
  if (!p.ok) return;
  const double ext = (double)rules.ext;
  const double rx = ext * sqrt(p.a), ry = ext * sqrt(p.c);
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
