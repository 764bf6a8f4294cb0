// gs_project / gs_project_bwd: per-Gaussian projection into every view and its
// reverse-mode derivative. One thread per Gaussian; the parameters are read once
// (coalesced SoA planes) and reused from registers for every view. FP64 inside:
// the stage is HBM bound, and FP64 keeps the 2D mean and covariance far below
// the FP32 error of the blend.
#include "gs_device_math.h"

namespace gs {

constexpr int kProjBlock = 256;

template <int K>
__device__ __forceinline__ void load_sh(const float* __restrict__ sh, int64_t n, int64_t g,
                                        float (*shc)[3]) {
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) shc[k][ch] = sh[((int64_t)k * 3 + ch) * n + g];
}

template <int DEG>
__global__ void __launch_bounds__(kProjBlock)
project_kernel(const float* __restrict__ means, const float* __restrict__ log_scales,
               const float* __restrict__ quats, const float* __restrict__ logits,
               const float* __restrict__ sh, int64_t n, ProjViews views, Rules rules,
               uint32_t* __restrict__ depth_key, int32_t* __restrict__ tiles_touched,
               float* __restrict__ record) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int64_t g = (int64_t)blockIdx.x * kProjBlock + threadIdx.x;
  if (g >= n) return;
  const double x = means[g], y = means[n + g], z = means[2 * n + g];
  const float ls0 = log_scales[g], ls1 = log_scales[n + g], ls2 = log_scales[2 * n + g];
  const float q0 = quats[g], q1 = quats[n + g], q2 = quats[2 * n + g], q3 = quats[3 * n + g];
  const float lg = logits[g];
  const bool iso = rules.isotropic != 0;
  bool finite = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(ls0) && isfinite(ls1) &&
                isfinite(ls2) && isfinite(lg);
  if (!iso) finite = finite && isfinite(q0) && isfinite(q1) && isfinite(q2) && isfinite(q3);
  float shc[K][3];
  load_sh<K>(sh, n, g, shc);
#pragma unroll
  for (int k = 0; k < K; ++k) finite = finite && isfinite(shc[k][0] + shc[k][1] + shc[k][2]);
  // |q|^2 and 1/|q| (Newton-refined reciprocal square root, no IEEE divide or sqrt)
  const double qq = iso ? 1.0 : fma((double)q0, q0, fma((double)q1, q1, fma((double)q2, q2, (double)q3 * q3)));
  const bool alive = finite && qq > 0.0;
  double M[9];
  double opac = 0.0;
  if (alive) {
    double R[9];
    double s0, s1, s2;
    if (iso) {
      // one radius on all axes (Sec. 7.3 ablation): Sigma = s^2 I, no rotation
      R[0] = R[4] = R[8] = 1.0;
      R[1] = R[2] = R[3] = R[5] = R[6] = R[7] = 0.0;
      s0 = s1 = s2 = exp((((double)ls0 + (double)ls1) + (double)ls2) / 3.0);
    } else {
      const double iq = rsqrt_d(qq);
      quat_to_rot(q0 * iq, q1 * iq, q2 * iq, q3 * iq, R);
      s0 = exp((double)ls0);
      s1 = exp((double)ls1);
      s2 = exp((double)ls2);
    }
    for (int r = 0; r < 3; ++r) {
      M[r * 3 + 0] = R[r * 3 + 0] * s0;
      M[r * 3 + 1] = R[r * 3 + 1] * s1;
      M[r * 3 + 2] = R[r * 3 + 2] * s2;
    }
    opac = 1.0 / (1.0 + exp(-(double)lg));
  }
  for (int v = 0; v < views.n_views; ++v) {
    const int64_t idx = (int64_t)v * n + g;
    const Cam& cam = views.cam[v];
    ProjGeom p;
    bool ok = alive;
    if (ok) {
      project_geometry(cam, rules, x, y, z, M, p);
      ok = p.ok;
    }
    float d[3];
    if (ok) ok = view_dir(cam, x, y, z, d) > 0.0f;
    if (!ok) {
      // every (view, Gaussian) slot is written, a culled one with zeros: the stores of a
      // wave then fill whole cache lines, which costs less than the partial lines the
      // visible pairs alone would leave (0.354 against 0.386 ms at 3M Gaussians x 4
      // views, and the binning's reads of the depth keys are faster too)
      tiles_touched[idx] = 0;
      depth_key[idx] = 0u;
      float4* rec = reinterpret_cast<float4*>(record + idx * GS_RECORD_FLOATS);
      rec[0] = rec[1] = rec[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      continue;
    }
    float Y[K];
    sh_basis<DEG>(d[0], d[1], d[2], Y);
    const float r = fmaxf(sh_colour_raw<K>(shc, Y, 0), 0.0f);
    const float gc = fmaxf(sh_colour_raw<K>(shc, Y, 1), 0.0f);
    const float b = fmaxf(sh_colour_raw<K>(shc, Y, 2), 0.0f);
    const int ts = __builtin_ctz(views.tile);   // tiles are 8, 16 or 32 pixels wide
    tiles_touched[idx] = ((p.i_hi >> ts) - (p.i_lo >> ts) + 1) * ((p.j_hi >> ts) - (p.j_lo >> ts) + 1);
    const float z32 = (float)p.tz;
    depth_key[idx] = __float_as_uint(z32);
    // whitening L^-1 of Sigma' = L L^T: w00 = a^-1/2, w10 = -b / sqrt(a det), w11 = sqrt(a / det)
    const double sa = p.sa, isa = p.isa, isd = rsqrt_d(p.det);
    const double w00 = isa, w10 = -p.b * isa * isd, w11 = sa * isd;
    // whitened offset of the box's corner pixel centre from the mean, c = L^-1 (p0 - mean):
    // a pixel at p0 + D then has whitened offset L^-1 D + c, whose FP32 evaluation errs
    // in proportion to the whitened terms, not to the pixel distance from the mean
    const double ax = ((double)p.i_lo + 0.5) - p.u, ay = ((double)p.j_lo + 0.5) - p.v;
    float4* rec = reinterpret_cast<float4*>(record + idx * GS_RECORD_FLOATS);
    rec[0] = make_float4(__int_as_float(p.i_lo | (p.j_lo << 16)), __int_as_float(p.i_hi | (p.j_hi << 16)),
                         (float)(w00 * ax), (float)(w10 * ax + w11 * ay));
    rec[1] = make_float4((float)w00, (float)w10, (float)w11, (float)opac);
    rec[2] = make_float4(r, gc, b, z32);
  }
}

// ---------------------------------------------------------------------------
// backward: one loop over the views for the geometry (FP64) and one for the SH
// colour (FP32), so their registers are not live at the same time
// ---------------------------------------------------------------------------

// One view's inputs of the geometry backward: the tile count and the first six
// gradient components (2D mean, whitening, opacity).
struct GeomRow {
  int32_t touched;
  float gr[6];
};

__device__ __forceinline__ GeomRow load_geom_row(const int32_t* __restrict__ tiles_touched,
                                                 const float* __restrict__ grad2d, int64_t idx) {
  GeomRow r;
  r.touched = tiles_touched[idx];
  const float* gr = grad2d + idx * GS_GRAD2D_FLOATS;
#pragma unroll
  for (int k = 0; k < 6; ++k) r.gr[k] = gr[k];
  return r;
}

// The colour backward's: the tile count and the three colour components.
struct ColourRow {
  int32_t touched;
  float gr[3];
};

__device__ __forceinline__ ColourRow load_colour_row(const int32_t* __restrict__ tiles_touched,
                                                     const float* __restrict__ grad2d, int64_t idx) {
  ColourRow r;
  r.touched = tiles_touched[idx];
  const float* gr = grad2d + idx * GS_GRAD2D_FLOATS + 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) r.gr[k] = gr[k];
  return r;
}

// Three waves per SIMD: the kernel waits on memory most of its time, so the third wave
// pays (0.56 ms at two waves, 188 VGPRs; 0.51 ms at three with 84 bytes per lane
// spilled; 0.48 ms once the geometry loop fit 156 VGPRs without spills; 0.41 ms with
// each view's inputs loaded one view ahead, 167 VGPRs, at 3M Gaussians x 4 views).
// Four waves spill 112 bytes per lane and take 0.93 ms.
template <int DEG>
__global__ void __launch_bounds__(kProjBlock) __attribute__((amdgpu_waves_per_eu(3)))
project_bwd_kernel(const float* __restrict__ means, const float* __restrict__ log_scales,
                   const float* __restrict__ quats, const float* __restrict__ logits,
                   const float* __restrict__ sh, int64_t n, ProjViews views, Rules rules,
                   const int32_t* __restrict__ tiles_touched, const float* __restrict__ grad2d,
                   float* __restrict__ d_means, float* __restrict__ d_log_scales,
                   float* __restrict__ d_quats, float* __restrict__ d_logits,
                   float* __restrict__ d_sh) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int64_t g = (int64_t)blockIdx.x * kProjBlock + threadIdx.x;
  if (g >= n) return;
  // the first view's row is loaded before everything else (see the geometry loop);
  // bitwise ORs, so that every view's count is loaded at once, without branches
  const GeomRow first = load_geom_row(tiles_touched, grad2d, g);
  bool any = first.touched > 0;
  for (int v = 1; v < views.n_views; ++v) any = any | (tiles_touched[(int64_t)v * n + g] > 0);
  const double x = means[g], y = means[n + g], z = means[2 * n + g];
  float dmu_f[3] = {0.0f, 0.0f, 0.0f};
  {
  double ds[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, s[3] = {0, 0, 0};
  float dop = 0.0f;
  double opac = 0.0;
  const bool iso = rules.isotropic != 0;
  // the unit quaternion and 1 / |q|: formed before the view loop for R, and again after
  // it from the same inputs (not held through the loop, whose FP64 chain sets the
  // kernel's register peak)
  auto unit_quat = [&](double* qh) {
    const double q0 = quats[g], q1 = quats[n + g], q2 = quats[2 * n + g], q3 = quats[3 * n + g];
    const double iq = rsqrt_d(fma(q0, q0, fma(q1, q1, fma(q2, q2, q3 * q3))));
    qh[0] = q0 * iq;
    qh[1] = q1 * iq;
    qh[2] = q2 * iq;
    qh[3] = q3 * iq;
    return iq;
  };
  if (any) {
    double M[9];
    {
    double R[9];
    if (iso) {
      R[0] = R[4] = R[8] = 1.0;
      R[1] = R[2] = R[3] = R[5] = R[6] = R[7] = 0.0;
      s[0] = s[1] = s[2] = exp((((double)log_scales[g] + (double)log_scales[n + g]) +
                               (double)log_scales[2 * n + g]) / 3.0);
    } else {
      double qh[4];
      unit_quat(qh);
      quat_to_rot(qh[0], qh[1], qh[2], qh[3], R);
      s[0] = exp((double)log_scales[g]);
      s[1] = exp((double)log_scales[n + g]);
      s[2] = exp((double)log_scales[2 * n + g]);
    }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) M[r * 3 + c] = R[r * 3 + c] * s[c];
    }
    // the view loop accumulates in FP32 (the gradients' own precision); every
    // per-view term is formed in FP64
    float dM[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    // the next view's tile count and gradient row are loaded one view ahead, so that
    // their memory latency overlaps the current view's FP64 chain (every row exists:
    // grad2d holds V * n rows, zero where a pair is not visible)
    GeomRow nxt = first;
    for (int v = 0; v < views.n_views; ++v) {
      const GeomRow cur = nxt;
      if (v + 1 < views.n_views) nxt = load_geom_row(tiles_touched, grad2d, (int64_t)(v + 1) * n + g);
      if (cur.touched <= 0) continue;
      const Cam& cam = views.cam[v];
      ProjGeom p;
      project_covariance(cam, rules, x, y, z, M, p);
      const double du = cur.gr[0], dv = cur.gr[1], dw00 = cur.gr[2], dw10 = cur.gr[3],
                   dw11 = cur.gr[4];
      dop += cur.gr[5];
      // whitening W = L^-1: w00 = a^-1/2, w10 = -b / sqrt(a det), w11 = sqrt(a / det)
      const double a = p.a, b = p.b, c = p.c;
      const double sa = sqrt_d(a), isa = rcp_d(sa), isd = rsqrt_d(p.det);
      const double isasd = isa * isd, idet = isd * isd, ia = isa * isa;
      const double gA = dw00 * (-0.5 * ia * isa) +
                        dw10 * (0.5 * b * ia * isasd + 0.5 * b * c * isasd * idet) +
                        dw11 * (0.5 * isasd - 0.5 * sa * c * idet * isd);
      const double gB = dw10 * (-isasd - b * b * isasd * idet) + dw11 * (sa * b * idet * isd);
      const double gC = dw10 * (0.5 * b * sa * idet * isd) + dw11 * (-0.5 * a * sa * idet * isd);
      // Sigma' = A A^T: dA0 = 2 gA A0 + gB A1, dA1 = gB A0 + 2 gC A1
      double dA0[3], dA1[3];
      for (int k = 0; k < 3; ++k) {
        dA0[k] = 2.0 * gA * p.A0[k] + gB * p.A1[k];
        dA1[k] = gB * p.A0[k] + 2.0 * gC * p.A1[k];
      }
      const double fx = cam.fx, fy = cam.fy, tx = p.tx, ty = p.ty;
      const double iz = p.iz, iz2 = iz * iz, iz3 = iz2 * iz;
      const double J00 = fx * iz, J02 = -fx * tx * iz2, J11 = fy * iz, J12 = -fy * ty * iz2;
      // dJ_rc = dA_r . (W M)_c = W_c . (M dA_r): through M, so that W M need not stay
      // live from the covariance to here
      double m0[3], m1[3];
      for (int i = 0; i < 3; ++i) {
        m0[i] = M[i * 3 + 0] * dA0[0] + M[i * 3 + 1] * dA0[1] + M[i * 3 + 2] * dA0[2];
        m1[i] = M[i * 3 + 0] * dA1[0] + M[i * 3 + 1] * dA1[1] + M[i * 3 + 2] * dA1[2];
      }
      double dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
      for (int i = 0; i < 3; ++i) {
        dJ00 += (double)cam.R[0 * 3 + i] * m0[i];
        dJ02 += (double)cam.R[2 * 3 + i] * m0[i];
        dJ11 += (double)cam.R[1 * 3 + i] * m1[i];
        dJ12 += (double)cam.R[2 * 3 + i] * m1[i];
      }
      // A = U M with U = J W (rows U0 = J00 W0 + J02 W2, U1 = J11 W1 + J12 W2):
      // dM += U^T dA
      for (int i = 0; i < 3; ++i) {
        const double u0 = J00 * (double)cam.R[0 * 3 + i] + J02 * (double)cam.R[2 * 3 + i];
        const double u1 = J11 * (double)cam.R[1 * 3 + i] + J12 * (double)cam.R[2 * 3 + i];
        for (int j = 0; j < 3; ++j) dM[i * 3 + j] += (float)(u0 * dA0[j] + u1 * dA1[j]);
      }
      // camera-space mean through (u, v) and J
      const double dtx = du * fx * iz + dJ02 * (-fx * iz2);
      const double dty = dv * fy * iz + dJ12 * (-fy * iz2);
      const double dtz = du * (-fx * tx * iz2) + dv * (-fy * ty * iz2) + dJ00 * (-fx * iz2) +
                         dJ02 * (2.0 * fx * tx * iz3) + dJ11 * (-fy * iz2) +
                         dJ12 * (2.0 * fy * ty * iz3);
      for (int k = 0; k < 3; ++k)
        dmu_f[k] += (float)((double)cam.R[0 * 3 + k] * dtx + (double)cam.R[1 * 3 + k] * dty +
                            (double)cam.R[2 * 3 + k] * dtz);
    }
    opac = rcp_d(1.0 + exp(fmin(-(double)logits[g], 700.0)));   // exp capped: rcp_d(inf) is NaN
    // M = R diag(s): dR_ij = dM_ij s_j, ds_j = sum_i dM_ij R_ij (R recomputed here
    // rather than held through the view loop)
    double R[9];
    double qh[4] = {1.0, 0.0, 0.0, 0.0}, iq = 1.0;
    if (iso) {
      R[0] = R[4] = R[8] = 1.0;
      R[1] = R[2] = R[3] = R[5] = R[6] = R[7] = 0.0;
    } else {
      iq = unit_quat(qh);
      quat_to_rot(qh[0], qh[1], qh[2], qh[3], R);
    }
    double dR[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        dR[i * 3 + j] = dM[i * 3 + j] * s[j];
        ds[j] += dM[i * 3 + j] * R[i * 3 + j];
      }
    // derivative of Eq. (quat) with respect to (r, i, j, k), then the normalisation
    const double r = qh[0], i = qh[1], j = qh[2], k = qh[3];
    double dqh[4];
    dqh[0] = 2.0 * (-k * dR[1] + j * dR[2] + k * dR[3] - i * dR[5] - j * dR[6] + i * dR[7]);
    dqh[1] = 2.0 * (j * dR[1] + k * dR[2] + j * dR[3] - 2.0 * i * dR[4] - r * dR[5] + k * dR[6] +
                    r * dR[7] - 2.0 * i * dR[8]);
    dqh[2] = 2.0 * (-2.0 * j * dR[0] + i * dR[1] + r * dR[2] + i * dR[3] + k * dR[5] - r * dR[6] +
                    k * dR[7] - 2.0 * j * dR[8]);
    dqh[3] = 2.0 * (-2.0 * k * dR[0] - r * dR[1] + i * dR[2] + r * dR[3] - 2.0 * k * dR[4] +
                    j * dR[5] + i * dR[6] + j * dR[7]);
    const double dotq = qh[0] * dqh[0] + qh[1] * dqh[1] + qh[2] * dqh[2] + qh[3] * dqh[3];
    for (int c = 0; c < 4; ++c) dq[c] = iso ? 0.0 : (dqh[c] - qh[c] * dotq) * iq;
    if (iso) {
      // s = exp((l0 + l1 + l2) / 3): every row receives a third of dL/dlog s
      const double third = (ds[0] * s[0] + ds[1] * s[1] + ds[2] * s[2]) / 3.0;
      ds[0] = ds[1] = ds[2] = third / s[0];
    }
  }
  // the geometry gradients are final here; only the mean still gains the SH term
  d_log_scales[g] = (float)(ds[0] * s[0]);
  d_log_scales[n + g] = (float)(ds[1] * s[1]);
  d_log_scales[2 * n + g] = (float)(ds[2] * s[2]);
  for (int c = 0; c < 4; ++c) d_quats[(int64_t)c * n + g] = (float)dq[c];
  d_logits[g] = (float)((double)dop * opac * (1.0 - opac));
  }
  // SH colour: coefficient gradients and the view-direction term of the mean. The
  // barrier keeps the coefficient loads from being hoisted into the geometry loop.
  asm volatile("" ::: "memory");
  float dshc[K][3];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) dshc[kk][0] = dshc[kk][1] = dshc[kk][2] = 0.0f;
  if (any) {
    float shc[K][3];
    load_sh<K>(sh, n, g, shc);
    ColourRow nxt = load_colour_row(tiles_touched, grad2d, g);   // one view ahead, as above
    for (int v = 0; v < views.n_views; ++v) {
      const ColourRow cur = nxt;
      if (v + 1 < views.n_views) nxt = load_colour_row(tiles_touched, grad2d, (int64_t)(v + 1) * n + g);
      if (cur.touched <= 0) continue;
      const Cam& cam = views.cam[v];
      float d[3];
      const float dist = view_dir(cam, x, y, z, d);
      float Y[K];
      sh_basis<DEG>(d[0], d[1], d[2], Y);
      float dcol[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        // the forward clamped the colour at 0: no gradient through a clamped channel
        dcol[ch] = (sh_colour_raw<K>(shc, Y, ch) >= 0.0f) ? cur.gr[ch] : 0.0f;
#pragma unroll
        for (int kk = 0; kk < K; ++kk) dshc[kk][ch] = fmaf(Y[kk], dcol[ch], dshc[kk][ch]);
      }
      if constexpr (DEG > 0) {
        float w[K], ddir[3];
#pragma unroll
        for (int kk = 0; kk < K; ++kk)
          w[kk] = shc[kk][0] * dcol[0] + shc[kk][1] * dcol[1] + shc[kk][2] * dcol[2];
        sh_weighted_grad<DEG>(d[0], d[1], d[2], w, ddir);
        // d = e / |e|: dL/de = (I - d d^T) dL/dd / |e|
        const float radial = d[0] * ddir[0] + d[1] * ddir[1] + d[2] * ddir[2];
        const float idist = __builtin_amdgcn_rcpf(dist);
        dmu_f[0] += (ddir[0] - d[0] * radial) * idist;
        dmu_f[1] += (ddir[1] - d[1] * radial) * idist;
        dmu_f[2] += (ddir[2] - d[2] * radial) * idist;
      }
    }
  }
  d_means[g] = dmu_f[0];
  d_means[n + g] = dmu_f[1];
  d_means[2 * n + g] = dmu_f[2];
#pragma unroll
  for (int kk = 0; kk < K; ++kk)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) d_sh[((int64_t)kk * 3 + ch) * n + g] = dshc[kk][ch];
}

}  // namespace gs

using namespace gs;

extern "C" int gs_project(const gs_params* params, const gs_camera* cams, int32_t n_views,
                          const gs_config* cfg, const gs_projected* out, gs_stream_t stream) {
  if (!params || !cams || !cfg || !out) return GS_ERR_ARG;
  int rc = check_config(cfg);
  if (rc != GS_OK) return rc;
  if (params->n < 0) return GS_ERR_ARG;
  if (params->n == 0) return GS_OK;
  if (!params->means || !params->log_scales || !params->quats || !params->opacity_logits ||
      !params->sh || !out->depth_key || !out->tiles_touched || !out->record)
    return GS_ERR_ARG;
  if (params->n * (int64_t)n_views >= ((int64_t)1 << 32)) return GS_ERR_UNSUPPORTED;
  ProjViews pv;
  rc = fill_proj_views(cams, n_views, cfg->tile_size, &pv);
  if (rc != GS_OK) return rc;
  const Rules rules = make_rules(cfg);
  const int64_t n = params->n;
  const dim3 grid((unsigned)((n + kProjBlock - 1) / kProjBlock));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
#define GS_LAUNCH_PROJ(D)                                                                     \
  project_kernel<D><<<grid, kProjBlock, 0, s>>>(params->means, params->log_scales,            \
                                                params->quats, params->opacity_logits,        \
                                                params->sh, n, pv, rules, out->depth_key,     \
                                                out->tiles_touched, out->record)
  switch (cfg->sh_degree) {
    case 0: GS_LAUNCH_PROJ(0); break;
    case 1: GS_LAUNCH_PROJ(1); break;
    case 2: GS_LAUNCH_PROJ(2); break;
    default: GS_LAUNCH_PROJ(3); break;
  }
#undef GS_LAUNCH_PROJ
  return launch_status();
}

extern "C" int gs_project_bwd(const gs_params* params, const gs_camera* cams, int32_t n_views,
                              const gs_config* cfg, const gs_projected* proj,
                              const float* grad2d, const gs_params_grad* grads,
                              gs_stream_t stream) {
  if (!params || !cams || !cfg || !proj || !grads) return GS_ERR_ARG;
  int rc = check_config(cfg);
  if (rc != GS_OK) return rc;
  if (params->n < 0) return GS_ERR_ARG;
  if (params->n == 0) return GS_OK;
  if (!params->means || !params->log_scales || !params->quats || !params->opacity_logits ||
      !params->sh || !proj->tiles_touched || !grad2d || !grads->means || !grads->log_scales ||
      !grads->quats || !grads->opacity_logits || !grads->sh)
    return GS_ERR_ARG;
  if (params->n * (int64_t)n_views >= ((int64_t)1 << 32)) return GS_ERR_UNSUPPORTED;
  ProjViews pv;
  rc = fill_proj_views(cams, n_views, cfg->tile_size, &pv);
  if (rc != GS_OK) return rc;
  const Rules rules = make_rules(cfg);
  const int64_t n = params->n;
  const dim3 grid((unsigned)((n + kProjBlock - 1) / kProjBlock));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
#define GS_LAUNCH_PBWD(D)                                                                     \
  project_bwd_kernel<D><<<grid, kProjBlock, 0, s>>>(                                          \
      params->means, params->log_scales, params->quats, params->opacity_logits, params->sh,   \
      n, pv, rules, proj->tiles_touched, grad2d, grads->means, grads->log_scales,             \
      grads->quats, grads->opacity_logits, grads->sh)
  switch (cfg->sh_degree) {
    case 0: GS_LAUNCH_PBWD(0); break;
    case 1: GS_LAUNCH_PBWD(1); break;
    case 2: GS_LAUNCH_PBWD(2); break;
    default: GS_LAUNCH_PBWD(3); break;
  }
#undef GS_LAUNCH_PBWD
  return launch_status();
}
