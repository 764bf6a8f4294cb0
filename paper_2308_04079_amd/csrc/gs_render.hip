// gs_render_fwd / gs_render_bwd: per-tile front-to-back blending (Alg. 2
// BlendInOrder; Eq. front-to-back; App. C) and its back-to-front adjoint (Sec. 6).
//
// One workgroup per (view, tile); each 64-lane wave owns an 8x8 pixel block of
// the tile and walks the tile's instance list on its own: it gathers 64 entries
// (one per lane), keeps those whose 3-sigma pixel box meets its 8x8 block,
// compacts them into its LDS slice with a ballot, and blends them from LDS
// (broadcast reads). A wave stops as soon as all 64 of its pixels are saturated;
// waves never wait for each other, so no workgroup barrier is needed.
//
// The backward pass walks the same list back to front from the wave's last
// contributor, recovers T by dividing the stored final T by (1 - alpha), and
// reduces the nine per-pixel partial gradients of each Gaussian over the wave
// with lane exchanges before nine lanes issue the global atomics.
#include <algorithm>

#include "gs_internal.h"

namespace gs {

// Per-Gaussian LDS entry: geo = (box corner i_lo, j_lo as floats, mean - corner),
// shape = (w00, w10, w11, opacity), col = (r, g, b, instance position bits).
struct Eval {
  float dx, dy, e0, e1, m, G, alpha;
};

// The one alpha evaluation used by both passes: identical instruction sequences
// (the library is built with -ffp-contract=off), hence identical decisions.
__device__ __forceinline__ void eval_alpha(const float4& geo, const float4& shape, float fpx,
                                           float fpy, const Rules& r, Eval& e) {
  e.dx = (fpx - geo.x) - geo.z;  // fpx - geo.x is exact: both are integers or half-integers
  e.dy = (fpy - geo.y) - geo.w;
  e.e0 = shape.x * e.dx;
  e.e1 = fmaf(shape.y, e.dx, shape.z * e.dy);
  e.m = fmaf(e.e0, e.e0, e.e1 * e.e1);
  e.G = __expf(-0.5f * e.m);
  e.alpha = fminf(r.alpha_max, shape.w * e.G);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (kWave - lane));
}

struct WaveTile {
  int v, tile, W, H, x0, y0, x1, y1, px, py;
  uint32_t n_records;
  bool inside;
};

// Workgroup b renders tile tile_order[b] when an order is given (gs_sort writes the
// tiles longest list first, so the heaviest tiles start first and do not form the
// tail of the launch), else tile b.
template <int TS>
__device__ __forceinline__ bool wave_tile(const TileViews& tv, const uint32_t* tile_order,
                                          WaveTile& w) {
  w.tile = tile_order ? (int)tile_order[blockIdx.x] : (int)blockIdx.x;
  if ((uint32_t)w.tile >= (uint32_t)tv.tile_offset[tv.n_views]) return false;  // not a tile id
  w.n_records = tv.n_records;
  w.v = view_of_tile(tv, w.tile);
  const int lt = w.tile - tv.tile_offset[w.v];
  const int tx = lt % tv.tiles_x[w.v], ty = lt / tv.tiles_x[w.v];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  constexpr int WX = TS / 8;
  w.W = tv.W[w.v];
  w.H = tv.H[w.v];
  w.x0 = tx * TS + (wave % WX) * 8;
  w.y0 = ty * TS + (wave / WX) * 8;
  if (w.x0 >= w.W || w.y0 >= w.H) return false;
  w.x1 = min(w.x0 + 7, w.W - 1);
  w.y1 = min(w.y0 + 7, w.H - 1);
  w.px = w.x0 + (lane & 7);
  w.py = w.y0 + (lane >> 3);
  w.inside = (w.px < w.W) && (w.py < w.H);
  return true;
}

// The tile's instance list [start, end), clipped to the instance buffers, so that
// ranges not written by gs_sort cannot send the gathers out of range.
__device__ __forceinline__ void tile_range(const uint32_t* __restrict__ ranges, int tile,
                                           uint32_t n_inst, uint32_t& start, uint32_t& end) {
  end = min(ranges[2 * tile + 1], n_inst);
  start = min(ranges[2 * tile], end);
}

// One list entry as gathered by a lane: kept if some pixel of the wave's block can
// pass both per-pixel tests of the blend, m <= ext^2 and alpha >= alpha_min. With
// alpha = min(alpha_max, o exp(-m/2)) the second holds only for m <= 2 ln(o / alpha_min),
// so an entry is kept when the least m over the block is at most
// min(ext^2, 2 ln(o / alpha_min)) (a superset of the contributing entries, so the
// image and gradients do not change; faint Gaussians reach fewer blocks than their
// 3-sigma box). The least m of the convex m(d) = |W d|^2 over the rectangle of the
// block's pixel centres is 0 if the mean lies inside, else the least of its four edge
// minima, each a parabola minimised at its vertex clamped to the edge. A slack far
// above the FP32 rounding of both evaluations keeps the test conservative.
struct Entry {
  float4 r0, r1, r2;
  uint32_t g, i;
  int ilo, jlo;
  bool keep;
};

__device__ __forceinline__ float edge_min_m(float w00, float w10, float w11, float X, float ylo,
                                            float yhi, float i11) {
  // d = (X, dy): e1 = w10 X + w11 dy vanishes at dy = -w10 X / w11
  const float dy = fminf(fmaxf(-w10 * X * i11, ylo), yhi);
  const float e0 = w00 * X, e1 = fmaf(w10, X, w11 * dy);
  return fmaf(e0, e0, e1 * e1);
}

__device__ __forceinline__ float edge_min_m_y(float w00, float w10, float w11, float Y, float xlo,
                                              float xhi, float iq) {
  // d = (dx, Y): m = (w00^2 + w10^2) dx^2 + 2 w10 w11 Y dx + (w11 Y)^2, vertex at
  // dx = -w10 w11 Y / (w00^2 + w10^2)
  const float dx = fminf(fmaxf(-w10 * w11 * Y * iq, xlo), xhi);
  const float e0 = w00 * dx, e1 = fmaf(w10, dx, w11 * Y);
  return fmaf(e0, e0, e1 * e1);
}

__device__ __forceinline__ bool block_reachable(const float4& shape, float dxa, float dxb, float dya,
                                                float dyb, const Rules& r) {
  const float w00 = shape.x, w10 = shape.y, w11 = shape.z, o = shape.w;
  const float thr = fminf(r.ext2, 2.0f * (__logf(o) - r.log_alpha_min));
  const bool inside = dxa <= 0.0f && dxb >= 0.0f && dya <= 0.0f && dyb >= 0.0f;
  const float i11 = __builtin_amdgcn_rcpf(w11), iq = __builtin_amdgcn_rcpf(fmaf(w00, w00, w10 * w10));
  float mmin = fminf(fminf(edge_min_m(w00, w10, w11, dxa, dya, dyb, i11),
                           edge_min_m(w00, w10, w11, dxb, dya, dyb, i11)),
                     fminf(edge_min_m_y(w00, w10, w11, dya, dxa, dxb, iq),
                           edge_min_m_y(w00, w10, w11, dyb, dxa, dxb, iq)));
  mmin = inside ? 0.0f : mmin;
  // size of the terms whose rounding enters m: |e0|, |e1| <= S over the rectangle
  const float S = (fabsf(w00) + fabsf(w10)) * fmaxf(fabsf(dxa), fabsf(dxb)) +
                  fabsf(w11) * fmaxf(fabsf(dya), fabsf(dyb));
  const float slack = 1e-4f + S * (1e-4f + 1e-5f * S);
  return mmin <= thr + slack;
}

__device__ __forceinline__ void gather_entry(const float* __restrict__ record, uint32_t g,
                                             uint32_t i, const WaveTile& w, const Rules& rules,
                                             Entry& e) {
  e.keep = false;
  e.i = i;
  e.g = g;
  e.ilo = e.jlo = 0;
  e.r0 = make_float4(0, 0, 0, 0);
  e.r1 = e.r0;
  e.r2 = e.r0;
  if (g < w.n_records) {
    const float4* rec = reinterpret_cast<const float4*>(record + (size_t)e.g * GS_RECORD_FLOATS);
    e.r0 = rec[0];
    const int lo = __float_as_int(e.r0.x), hi = __float_as_int(e.r0.y);
    e.ilo = lo & 0xFFFF;
    e.jlo = (lo >> 16) & 0xFFFF;
    const int ihi = hi & 0xFFFF, jhi = (hi >> 16) & 0xFFFF;
    e.keep = (e.ilo <= w.x1) && (ihi >= w.x0) && (e.jlo <= w.y1) && (jhi >= w.y0);
    if (e.keep) {
      e.r1 = rec[1];
      // pixel centre minus mean at the block's edges, as the blend forms dx and dy
      const float mx = e.r0.z, my = e.r0.w;
      const float dxa = ((float)(w.x0 - e.ilo) + 0.5f) - mx, dxb = ((float)(w.x1 - e.ilo) + 0.5f) - mx;
      const float dya = ((float)(w.y0 - e.jlo) + 0.5f) - my, dyb = ((float)(w.y1 - e.jlo) + 0.5f) - my;
      e.keep = block_reachable(e.r1, dxa, dxb, dya, dyb, rules);
      if (e.keep) e.r2 = rec[2];
    }
  }
}

// Compact the kept entries of the wave into its LDS slice from slot `slot0` on, in
// lane order; returns the new fill level. The forward keeps the list position in
// col.w; the backward (s_pos given) keeps the record index there, so that it arrives
// with the colour for the atomics, and the position in s_pos.
__device__ __forceinline__ int commit_entries(const Entry& e, int slot0, float4* s_geo,
                                              float4* s_shape, float4* s_col, uint32_t* s_pos) {
  const uint64_t km = __ballot(e.keep);
  if (e.keep) {
    const int slot = slot0 + __popcll(km & lanemask_lt());
    s_geo[slot] = make_float4((float)e.ilo, (float)e.jlo, e.r0.z, e.r0.w);
    s_shape[slot] = e.r1;
    s_col[slot] = make_float4(e.r2.x, e.r2.y, e.r2.z, __uint_as_float(s_pos ? e.g : e.i));
    if (s_pos) s_pos[slot] = e.i;
  }
  return slot0 + __popcll(km);
}

// Instance values (Gaussian record indices) of one batch, loaded one batch ahead so
// that the first link of the gather chain (value, then record) is in flight while
// the wave blends the previous batch. Entries past the batch's end hold ~0u, which
// no record index reaches.
template <int R>
struct Ahead {
  uint32_t g[R];
};

template <int R>
__device__ __forceinline__ void load_ahead(const uint32_t* __restrict__ vals, int64_t first,
                                           int64_t last_ok, Ahead<R>& a) {
  const int lane = threadIdx.x % kWave;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = first + r * kWave + lane;
    a.g[r] = (i <= last_ok) ? vals[i] : ~0u;
  }
}

// Stage the R * 64 consecutive list entries [first, first + 64 R) whose values `a`
// holds into the wave's LDS slice (all gathers are issued before any ballot).
// Returns the kept count.
template <int R>
__device__ __forceinline__ int stage_batch(const float* __restrict__ record, const Ahead<R>& a,
                                           int64_t first, const WaveTile& w, const Rules& rules,
                                           float4* s_geo, float4* s_shape, float4* s_col,
                                           uint32_t* s_pos) {
  Entry e[R];
  const int lane = threadIdx.x % kWave;
#pragma unroll
  for (int r = 0; r < R; ++r)
    gather_entry(record, a.g[r], (uint32_t)(first + r * kWave + lane), w, rules, e[r]);
  int cnt = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) cnt = commit_entries(e[r], cnt, s_geo, s_shape, s_col, s_pos);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  return cnt;
}

template <int TS, int R>
__global__ void __launch_bounds__((TS / 8) * (TS / 8) * kWave)
render_fwd_kernel(const float* __restrict__ record, const uint32_t* __restrict__ vals,
                  const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ tile_order,
                  TileViews tv, Rules rules, float* __restrict__ image,
                  float* __restrict__ T_final, int32_t* __restrict__ last_idx) {
  constexpr int WPT = (TS / 8) * (TS / 8);
  constexpr int BATCH = R * kWave;
  __shared__ float4 s_geo[WPT][BATCH];
  __shared__ float4 s_shape[WPT][BATCH];
  __shared__ float4 s_col[WPT][BATCH];
  WaveTile w;
  if (!wave_tile<TS>(tv, tile_order, w)) return;
  const int wave = threadIdx.x / kWave;
  uint32_t start, end;
  tile_range(ranges, w.tile, tv.n_inst, start, end);
  const float fpx = (float)w.px + 0.5f, fpy = (float)w.py + 0.5f;
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  int32_t last = -1;
  // 1 while the pixel still blends, 0 once it stopped (or lies outside the image): a
  // float, so that every decision below is a compare feeding one select, with no
  // combining of lane masks
  float live = w.inside ? 1.0f : 0.0f;
  Ahead<R> ahead;
  load_ahead<R>(vals, start, (int64_t)end - 1, ahead);
  for (uint32_t base = start; base < end; base += BATCH) {
    if (__ballot(live > 0.0f) == 0ull) break;
    const Ahead<R> cur = ahead;
    const int cnt = stage_batch<R>(record, cur, base, w, rules, s_geo[wave], s_shape[wave],
                                   s_col[wave], nullptr);
    load_ahead<R>(vals, (int64_t)base + BATCH, (int64_t)end - 1, ahead);
    // groups of 8 entries; the saturation ballot runs once per group
    bool all_done = false;
    for (int k0 = 0; k0 < cnt && !all_done; k0 += 8) {
    const int kend = min(k0 + 8, cnt);
    for (int k = k0; k < kend; ++k) {
      const float4 geo = s_geo[wave][k];
      const float4 shape = s_shape[wave][k];
      const float4 col = s_col[wave][k];
      Eval e;
      eval_alpha(geo, shape, fpx, fpy, rules, e);
      // branch-free: every lane evaluates. a is alpha where the Gaussian is taken (inside
      // the extent, alpha >= alpha_min > 0, pixel live), else 0; an untaken entry then
      // leaves T * (1 - 0) = T >= T_min, so only a taken one can stop the pixel
      float a = (e.m <= rules.ext2) ? e.alpha : 0.0f;
      a = (a >= rules.alpha_min) ? a : 0.0f;
      a *= live;
      const float Tn = T * (1.0f - a);
      const bool stop = Tn < rules.T_min;
      const float ab = stop ? 0.0f : a;   // alpha of a blended entry, else 0
      const float wgt = T * ab;
      C0 = fmaf(wgt, col.x, C0);
      C1 = fmaf(wgt, col.y, C1);
      C2 = fmaf(wgt, col.z, C2);
      T = stop ? T : Tn;
      last = (ab > 0.0f) ? (int32_t)__float_as_uint(col.w) : last;
      live = stop ? 0.0f : live;
    }
    all_done = __ballot(live > 0.0f) == 0ull;
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (w.inside) {
    const int64_t P = tv.pix_offset[w.v];
    const int64_t HW = (int64_t)w.W * w.H;
    const int64_t p = (int64_t)w.py * w.W + w.px;
    float* img = image + 3 * P;
    img[p] = fmaf(T, rules.bg[0], C0);
    img[HW + p] = fmaf(T, rules.bg[1], C1);
    img[2 * HW + p] = fmaf(T, rules.bg[2], C2);
    if (T_final) T_final[P + p] = T;      // both NULL on the forward-only path
    if (last_idx) last_idx[P + p] = last;
  }
}

__device__ __forceinline__ int wave_max_int(int x) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) x = max(x, __shfl_xor(x, d, kWave));
  return x;
}

// Value of lane l ^ XM (XM < 16: a partner in the same 16-lane row) through ds_swizzle
// (bit mode, and-mask 0x1F): the exchange runs in the LDS crossbar, beside the VALU
// work of the other waves, where a DPP operand would occupy the VALU (measured ~3%
// faster on the backward blend than row_mirror / row_half_mirror / quad_perm DPP).
template <int XM>
__device__ __forceinline__ float lane_xor(float x) {
  static_assert(XM > 0 && XM < 16, "partner must be in the same row");
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, x), (XM << 10) | 0x1F));
}

// Wave sum of nine per-lane values as a reduce-scatter butterfly inside each 16-lane
// row: at every step a lane keeps half of its remaining values and adds its partner's
// copy of them (9 -> 5 -> 3 -> 2 -> 1 registers). The partners l ^ 15 and l ^ 7 differ
// in all low bits, so they come first (split on bit 3, then bit 2), then l ^ 2 and
// l ^ 1. Two cross-row exchanges finish the sum. In-row lane l then holds the total of
// value reduce_index(l) when bit l of kReduceLanes is set.
constexpr uint32_t kReduceLanes = 0x1737u;  // row lanes 0, 1, 2, 4, 5, 8, 9, 10, 12
__device__ __forceinline__ int reduce_index(uint32_t l) {
  return 5 * ((l >> 3) & 1) + 3 * ((l >> 2) & 1) + 2 * ((l >> 1) & 1) + (l & 1);
}

__device__ __forceinline__ float wave_reduce9_scatter(float a0, float a1, float a2, float a3,
                                                      float a4, float a5, float a6, float a7,
                                                      float a8) {
  const uint32_t l = __lane_id() & 15;
  const bool h3 = l & 8, h2 = l & 4, h1 = l & 2, h0 = l & 1;
  const float x0 = (h3 ? a5 : a0) + lane_xor<15>(h3 ? a0 : a5);
  const float x1 = (h3 ? a6 : a1) + lane_xor<15>(h3 ? a1 : a6);
  const float x2 = (h3 ? a7 : a2) + lane_xor<15>(h3 ? a2 : a7);
  const float x3 = (h3 ? a8 : a3) + lane_xor<15>(h3 ? a3 : a8);
  const float x4 = (h3 ? 0.0f : a4) + lane_xor<15>(h3 ? a4 : 0.0f);
  const float y0 = (h2 ? x3 : x0) + lane_xor<7>(h2 ? x0 : x3);
  const float y1 = (h2 ? x4 : x1) + lane_xor<7>(h2 ? x1 : x4);
  const float y2 = (h2 ? 0.0f : x2) + lane_xor<7>(h2 ? x2 : 0.0f);
  const float z0 = (h1 ? y2 : y0) + lane_xor<2>(h1 ? y0 : y2);
  const float z1 = (h1 ? 0.0f : y1) + lane_xor<2>(h1 ? y1 : 0.0f);
  float v = (h0 ? z1 : z0) + lane_xor<1>(h0 ? z0 : z1);
  v += __shfl_xor(v, 16, kWave);
  v += __shfl_xor(v, 32, kWave);
  return v;
}

template <int TS, int R, bool LIMIT>
__global__ void __launch_bounds__((TS / 8) * (TS / 8) * kWave)
render_bwd_kernel(const float* __restrict__ record, const uint32_t* __restrict__ vals,
                  const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ tile_order,
                  TileViews tv, Rules rules, const float* __restrict__ T_final,
                  const int32_t* __restrict__ last_idx, const float* __restrict__ dL_dimage,
                  float* __restrict__ grad2d) {
  constexpr int WPT = (TS / 8) * (TS / 8);
  constexpr int BATCH = R * kWave;
  __shared__ float4 s_geo[WPT][BATCH];
  __shared__ float4 s_shape[WPT][BATCH];
  __shared__ float4 s_col[WPT][BATCH];
  __shared__ uint32_t s_pos[WPT][BATCH];
  WaveTile w;
  if (!wave_tile<TS>(tv, tile_order, w)) return;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  uint32_t start, end;
  tile_range(ranges, w.tile, tv.n_inst, start, end);
  const float fpx = (float)w.px + 0.5f, fpy = (float)w.py + 0.5f;
  float T = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
  int32_t last = -1;
  if (w.inside) {
    const int64_t P = tv.pix_offset[w.v];
    const int64_t HW = (int64_t)w.W * w.H;
    const int64_t p = (int64_t)w.py * w.W + w.px;
    T = T_final[P + p];
    last = last_idx[P + p];
    const float* dimg = dL_dimage + 3 * P;
    g0 = dimg[p];
    g1 = dimg[HW + p];
    g2 = dimg[2 * HW + p];
  }
  // only g . B is ever needed, where B is the colour accumulated behind the current
  // Gaussian (initially T_final bg): dC/dalpha_i . g = T_i (g . c_i) - (g . B_i) / (1 - alpha_i)
  float S = T * (g0 * rules.bg[0] + g1 * rules.bg[1] + g2 * rules.bg[2]);
  // the walk starts at the wave's last contributor, bounded by the tile's list so that
  // a last_idx not written by the forward pass cannot send the gathers out of range
  const int64_t wave_last = std::min<int64_t>(wave_max_int(last), (int64_t)end - 1);
  if (wave_last < (int64_t)start) return;  // no pixel of this wave blended anything
  const bool atomic_lane = lane < 16 && ((kReduceLanes >> lane) & 1u);
  const int atomic_slot = reduce_index((uint32_t)lane);
  // limited-gradient ablation: count the pixel's blended Gaussians first, so the
  // back-to-front walk knows each one's front-to-back rank
  int n_blended = 0, from_back = 0;
  if constexpr (LIMIT) {
    for (int64_t top = wave_last; top >= (int64_t)start; top -= BATCH) {
      const int64_t bot = max((int64_t)start, top - (BATCH - 1));
      Ahead<R> cur;
      load_ahead<R>(vals, bot, top, cur);
      const int cnt = stage_batch<R>(record, cur, bot, w, rules, s_geo[wave], s_shape[wave],
                                     s_col[wave], s_pos[wave]);
      for (int k = cnt - 1; k >= 0; --k) {
        const int32_t pos = (int32_t)s_pos[wave][k];
        Eval e;
        eval_alpha(s_geo[wave][k], s_shape[wave][k], fpx, fpy, rules, e);
        n_blended += ((pos <= last) && (e.m <= rules.ext2) && (e.alpha >= rules.alpha_min)) ? 1 : 0;
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  Ahead<R> ahead;
  load_ahead<R>(vals, max((int64_t)start, wave_last - (BATCH - 1)), wave_last, ahead);
  for (int64_t top = wave_last; top >= (int64_t)start; top -= BATCH) {
    const int64_t bot = max((int64_t)start, top - (BATCH - 1));
    const Ahead<R> cur = ahead;
    const int cnt = stage_batch<R>(record, cur, bot, w, rules, s_geo[wave], s_shape[wave],
                                   s_col[wave], s_pos[wave]);
    const int64_t ntop = top - BATCH;   // the next batch, [max(start, ntop - BATCH + 1), ntop]
    load_ahead<R>(vals, max((int64_t)start, ntop - (BATCH - 1)), ntop, ahead);
    for (int k = cnt - 1; k >= 0; --k) {
      const float4 geo = s_geo[wave][k];
      const float4 shape = s_shape[wave][k];
      const float4 col = s_col[wave][k];
      const int32_t pos = (int32_t)s_pos[wave][k];
      Eval e;
      eval_alpha(geo, shape, fpx, fpy, rules, e);
      // branch-free: non-contributing lanes add zeros and keep their state
      const bool contrib = (pos <= last) && (e.m <= rules.ext2) && (e.alpha >= rules.alpha_min);
      bool grad_on = contrib;
      if constexpr (LIMIT) {
        grad_on = contrib && (n_blended - 1 - from_back) < rules.grad_limit;
        from_back += contrib ? 1 : 0;
      }
      const float inv = contrib ? __builtin_amdgcn_rcpf(1.0f - e.alpha) : 1.0f;
      T = T * inv;  // transmittance in front of this Gaussian
      const float wgt = contrib ? T * e.alpha : 0.0f;
      const float gwgt = grad_on ? wgt : 0.0f;
      const float d_r = gwgt * g0, d_g = gwgt * g1, d_b = gwgt * g2;
      const float gc = fmaf(g2, col.z, fmaf(g1, col.y, g0 * col.x));
      float dalpha = fmaf(T, gc, -S * inv);
      S = fmaf(wgt, gc, S);
      // alpha = min(alpha_max, o G): no gradient through a clamped alpha
      dalpha = (grad_on && shape.w * e.G <= rules.alpha_max) ? dalpha : 0.0f;
      const float d_o = dalpha * e.G;
      // dalpha/dm = -alpha / 2; m = e0^2 + e1^2, e0 = w00 dx, e1 = w10 dx + w11 dy, dx = pixel - mean
      const float q = -dalpha * e.alpha;
      const float t0 = q * e.e0, t1 = q * e.e1;
      const float d_mx = -fmaf(t0, shape.x, t1 * shape.y);
      const float d_my = -(t1 * shape.z);
      const float d_w00 = t0 * e.dx, d_w10 = t1 * e.dx, d_w11 = t1 * e.dy;
      if (__ballot(grad_on) != 0ull) {
        const float tot = wave_reduce9_scatter(d_mx, d_my, d_w00, d_w10, d_w11, d_o, d_r, d_g,
                                               d_b);
        if (atomic_lane)
          atomicAdd(grad2d + (size_t)__float_as_uint(col.w) * GS_GRAD2D_FLOATS + atomic_slot, tot);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// L1 loss gradient: a bounded grid per view (blockIdx.y) strides over its pixels;
// each block adds one partial loss.
__global__ void __launch_bounds__(256)
loss_l1_kernel(const float* __restrict__ image, const float* __restrict__ target, TileViews tv,
               float* __restrict__ dL, float* __restrict__ loss) {
  __shared__ float s_part[256 / kWave];
  const int v = blockIdx.y;
  const int64_t HW = tv.pix_offset[v + 1] - tv.pix_offset[v];
  const int64_t base = 3 * tv.pix_offset[v];
  const float inv = 1.0f / (3.0f * (float)HW);
  float part = 0.0f;
  for (int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x; pix < HW;
       pix += (int64_t)gridDim.x * 256) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t k = base + c * HW + pix;
      const float d = image[k] - target[k];
      dL[k] = (d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f));
      part += fabsf(d) * inv;
    }
  }
  if (loss) {
    part = wave_sum_to_lane63(part);
    if (__lane_id() == kWave - 1) s_part[threadIdx.x / kWave] = part;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss + v, s_part[0] + s_part[1] + s_part[2] + s_part[3]);
  }
}

}  // namespace gs

using namespace gs;

static int render_common(const gs_projected* proj, const gs_instances* inst,
                         const uint32_t* tile_ranges, const gs_camera* cams, int32_t n_views,
                         const gs_config* cfg, int64_t n, TileViews* tv) {
  if (!proj || !inst || !tile_ranges || !cams || !cfg || n < 0) return GS_ERR_ARG;
  int rc = check_config(cfg);
  if (rc != GS_OK) return rc;
  rc = fill_tile_views(cams, n_views, cfg->tile_size, tv);
  if (rc != GS_OK) return rc;
  if (n * (int64_t)n_views >= ((int64_t)1 << 32)) return GS_ERR_UNSUPPORTED;
  tv->n_records = (uint32_t)(n * n_views);
  if (!proj->record || !inst->vals) return GS_ERR_ARG;
  if (inst->capacity < 0 || inst->capacity > GS_MAX_INSTANCES) return GS_ERR_ARG;
  tv->n_inst = (uint32_t)inst->capacity;
  return GS_OK;
}

extern "C" int gs_render_fwd(const gs_projected* proj, const gs_instances* inst,
                             const uint32_t* tile_ranges, const uint32_t* tile_order,
                             const gs_camera* cams, int32_t n_views,
                             const gs_config* cfg, float* image, float* T_final, int32_t* last_idx,
                             int64_t n, gs_stream_t stream) {
  TileViews tv;
  int rc = render_common(proj, inst, tile_ranges, cams, n_views, cfg, n, &tv);
  if (rc != GS_OK) return rc;
  if (!image || (!T_final) != (!last_idx)) return GS_ERR_ARG;
  const Rules rules = make_rules(cfg);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const dim3 grid((unsigned)tv.tile_offset[n_views]);
#define GS_FWD(TS, R)                                                                          \
  render_fwd_kernel<TS, R><<<grid, (TS / 8) * (TS / 8) * kWave, 0, s>>>(                      \
      proj->record, inst->vals, tile_ranges, tile_order, tv, rules, image, T_final, last_idx)
  const bool two = cfg->lds_batch == 128;
  switch (cfg->tile_size) {
    case 8: if (two) GS_FWD(8, 2); else GS_FWD(8, 1); break;
    case 32: if (two) GS_FWD(32, 2); else GS_FWD(32, 1); break;
    default: if (two) GS_FWD(16, 2); else GS_FWD(16, 1); break;
  }
#undef GS_FWD
  return launch_status();
}

extern "C" int gs_loss_l1(const float* image, const float* target, const gs_camera* cams,
                          int32_t n_views, float* dL_dimage, float* loss, gs_stream_t stream) {
  if (!image || !target || !dL_dimage) return GS_ERR_ARG;
  TileViews tv;
  int rc = fill_tile_views(cams, n_views, 16, &tv);
  if (rc != GS_OK) return rc;
  int64_t max_hw = 0;
  for (int v = 0; v < n_views; ++v)
    max_hw = std::max<int64_t>(max_hw, tv.pix_offset[v + 1] - tv.pix_offset[v]);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const unsigned bx = (unsigned)std::min<int64_t>((max_hw + 255) / 256, 256);
  loss_l1_kernel<<<dim3(bx, (unsigned)n_views), 256, 0, s>>>(
      image, target, tv, dL_dimage, loss);
  return launch_status();
}

extern "C" int gs_render_bwd(const gs_projected* proj, const gs_instances* inst,
                             const uint32_t* tile_ranges, const uint32_t* tile_order,
                             const gs_camera* cams, int32_t n_views,
                             const gs_config* cfg, const float* T_final, const int32_t* last_idx,
                             const float* dL_dimage, float* grad2d, int64_t n,
                             gs_stream_t stream) {
  TileViews tv;
  int rc = render_common(proj, inst, tile_ranges, cams, n_views, cfg, n, &tv);
  if (rc != GS_OK) return rc;
  if (!T_final || !last_idx || !dL_dimage || !grad2d) return GS_ERR_ARG;
  const Rules rules = make_rules(cfg);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const dim3 grid((unsigned)tv.tile_offset[n_views]);
#define GS_BWD(TS, R)                                                                          \
  render_bwd_kernel<TS, R, false><<<grid, (TS / 8) * (TS / 8) * kWave, 0, s>>>(               \
      proj->record, inst->vals, tile_ranges, tile_order, tv, rules, T_final, last_idx,         \
      dL_dimage, grad2d)
#define GS_BWD_LIMITED(TS)                                                                     \
  render_bwd_kernel<TS, 1, true><<<grid, (TS / 8) * (TS / 8) * kWave, 0, s>>>(                \
      proj->record, inst->vals, tile_ranges, tile_order, tv, rules, T_final, last_idx,         \
      dL_dimage, grad2d)
  if (cfg->grad_limit > 0) {
    // the ablation path stages 64 entries per round whatever lds_batch says
    switch (cfg->tile_size) {
      case 8: GS_BWD_LIMITED(8); break;
      case 32: GS_BWD_LIMITED(32); break;
      default: GS_BWD_LIMITED(16); break;
    }
    return launch_status();
  }
#undef GS_BWD_LIMITED
  const bool two = cfg->lds_batch == 128;
  switch (cfg->tile_size) {
    case 8: if (two) GS_BWD(8, 2); else GS_BWD(8, 1); break;
    case 32: if (two) GS_BWD(32, 2); else GS_BWD(32, 1); break;
    default: if (two) GS_BWD(16, 2); else GS_BWD(16, 1); break;
  }
#undef GS_BWD
  return launch_status();
}
