// gs_render_fwd / gs_render_bwd: per-tile front-to-back blending (Alg. 2
// BlendInOrder; Eq. front-to-back; App. C) and its back-to-front adjoint (Sec. 6).
//
// One workgroup per (view, tile); each 64-lane wave owns an 8x8 pixel block of the
// tile and walks the tile's instance list in rounds of BATCH entries (one gathered per
// lane), keeping in its LDS slice only the entries that can reach a pixel of its block.
// Waves never wait for each other, so no workgroup barrier is needed.
//
// Forward: each 16-lane row of a wave owns a 4x4 block of the wave's block; every
// entry is tested against the four 4x4 blocks and each row gets the list of its own
// entries. The rows then blend their lists side by side, one entry per row per step
// (four Gaussians per wave instruction), and a wave stops as soon as all 64 of its
// pixels are saturated.
//
// Backward: the wave walks its kept entries back to front from the block's last
// contributor, one Gaussian per step over all 64 pixels, recovers T by dividing the
// stored final T by (1 - alpha), sums the nine per-pixel gradient terms over the wave
// with lane exchanges, and nine lanes issue the Gaussian's global atomics.
#include <algorithm>

#include "gs_internal.h"

namespace gs {

// Per-Gaussian LDS entry: geo = (centre of the box's corner pixel, whitened offset c of
// that centre from the mean), shape = (w00, w10, w11, opacity), col = (r, g, b, list
// position (forward) or record index (backward)), and for the backward the list
// position in pos.
struct Eval {
  float di, dj, e0, e1, m, G, alpha;
};

// exp(-m/2) = 2^(m * (-log2(e) / 2)): -0.5 times the FP32 log2(e) is exact, and so is
// the halving of m, so this one product equals the rounded (-m/2) * log2(e) of the
// two-multiply form bit for bit.
constexpr float kNegHalfLog2e = -0.5f * 1.44269502f;


// The one alpha evaluation used by both passes: identical instruction sequences
// (the library is built with -ffp-contract=off), hence identical decisions. The
// pixel's offset D from the corner centre is exact (integers), and its whitened offset
// from the mean is e = L^-1 D + c.
__device__ __forceinline__ void eval_alpha(const float4& geo, const float4& shape, float fpx,
                                           float fpy, float amax, Eval& e) {
  e.di = fpx - geo.x;
  e.dj = fpy - geo.y;
  e.e0 = fmaf(shape.x, e.di, geo.z);
  e.e1 = fmaf(shape.y, e.di, fmaf(shape.z, e.dj, geo.w));
  e.m = fmaf(e.e0, e.e0, e.e1 * e.e1);
  e.G = __builtin_amdgcn_exp2f(e.m * kNegHalfLog2e);
  // min(amax, o G) as one median-of-three (o G >= 0: opacity and G are in [0, 1]);
  // fminf would also re-canonicalise amax at every evaluation
  e.alpha = __builtin_amdgcn_fmed3f(shape.w * e.G, 0.0f, amax);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (kWave - lane));
}

constexpr int kRows = 4;       // 16-lane rows per wave, one 4x4 pixel block each
constexpr int kRowLanes = 16;

struct WaveTile {
  int v, tile, W, H, x0, y0, px, py, row;
  uint32_t n_records;
  bool inside;
};

// Workgroup b renders tile tile_order[b] when an order is given (gs_sort writes the
// tiles longest list first, so the heaviest tiles start first and do not form the
// tail of the launch), else tile b. Row r of a wave owns the 4x4 block at
// (x0 + 4 (r & 1), y0 + 4 (r >> 1)); lane l of the row its pixel (l & 3, l >> 2).
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
  w.row = lane / kRowLanes;
  const int l = lane % kRowLanes;
  w.px = w.x0 + 4 * (w.row & 1) + (l & 3);
  w.py = w.y0 + 4 * (w.row >> 1) + (l >> 2);
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

// One list entry as gathered by a lane (forward): kept for row r if its pixel box meets
// the row's 4x4 block and some pixel of the wave's block can pass both per-pixel tests
// of the blend, m <= ext^2 and alpha >= alpha_min. With alpha = min(alpha_max,
// o exp(-m/2)) the second holds only for m <= 2 ln(o / alpha_min), so the entry is kept
// when the least m over the pixel box clipped to the wave's block is at most
// min(ext^2, 2 ln(o / alpha_min)) (a superset of the contributing entries, so the image
// and gradients do not change; faint Gaussians reach fewer blocks than their 3-sigma
// box). Over a rectangle of pixel-centre offsets D from the corner centre,
// m = |L^-1 D + c|^2 is convex: its least value is 0 if the mean lies inside, else the
// least of the four edge minima, each a parabola minimised at its vertex clamped to the
// edge. A slack far above the FP32 rounding of both evaluations keeps the test
// conservative. (One test per entry on the clipped box costs less than one per row and
// keeps nearly all of the per-row cull: measured 0.59 against 0.62 ms.)
struct Entry {
  float4 r0, r1, r2;
  uint32_t g, i;
  int ilo, jlo;
  float ax, ay;    // offset of the mean from the corner centre, a = -L c
  uint32_t rows;   // bit r: kept for row r
};

struct Shape {
  float w00, w10, w11, c0, c1, i11, iq;   // i11 = 1 / w11, iq = 1 / (w00^2 + w10^2)
};

__device__ __forceinline__ float edge_min_m(const Shape& s, float X, float ylo, float yhi) {
  // D = (X, Dj): e1 = w11 Dj + (w10 X + c1) vanishes at Dj = -(w10 X + c1) / w11
  const float b = fmaf(s.w10, X, s.c1);
  const float dj = fminf(fmaxf(-b * s.i11, ylo), yhi);
  const float e0 = fmaf(s.w00, X, s.c0), e1 = fmaf(s.w11, dj, b);
  return fmaf(e0, e0, e1 * e1);
}

__device__ __forceinline__ float edge_min_m_y(const Shape& s, float Y, float xlo, float xhi) {
  // D = (Di, Y): m = (w00 Di + c0)^2 + (w10 Di + b)^2 with b = w11 Y + c1, vertex at
  // Di = -(w00 c0 + w10 b) / (w00^2 + w10^2)
  const float b = fmaf(s.w11, Y, s.c1);
  const float di = fminf(fmaxf(-fmaf(s.w00, s.c0, s.w10 * b) * s.iq, xlo), xhi);
  const float e0 = fmaf(s.w00, di, s.c0), e1 = fmaf(s.w10, di, b);
  return fmaf(e0, e0, e1 * e1);
}

// Reachability test of one block (offset rectangle [xa, xb] x [ya, yb] from the corner
// centre); thr = min(ext^2, 2 ln(o / alpha_min)).
__device__ __forceinline__ bool block_reachable(const Shape& s, float thr, float ax, float ay,
                                                float xa, float xb, float ya, float yb) {
  const bool inside = ax >= xa && ax <= xb && ay >= ya && ay <= yb;
  float mmin = fminf(fminf(edge_min_m(s, xa, ya, yb), edge_min_m(s, xb, ya, yb)),
                     fminf(edge_min_m_y(s, ya, xa, xb), edge_min_m_y(s, yb, xa, xb)));
  mmin = inside ? 0.0f : mmin;
  // size of the terms whose rounding enters m: |e0|, |e1| <= S over the rectangle
  const float S = fabsf(s.c0) + fabsf(s.c1) + (fabsf(s.w00) + fabsf(s.w10)) * fmaxf(fabsf(xa), fabsf(xb)) +
                  fabsf(s.w11) * fmaxf(fabsf(ya), fabsf(yb));
  const float slack = 1e-4f + S * (1e-4f + 1e-5f * S);
  return mmin <= thr + slack;
}

// Gather list entry i (record index g) and test it against the 4x4 blocks of the
// wave's four rows. row_lim[r]: the last list position row r still needs (the
// backward's row-wise last contributor; the forward's INT32_MAX while the row has a
// live pixel, else -1).
__device__ __forceinline__ void gather_entry(const float* __restrict__ record, uint32_t g,
                                             uint32_t i, const WaveTile& w, const Rules& rules,
                                             const int32_t* row_lim, Entry& e) {
  e.rows = 0;
  e.i = i;
  e.g = g;
  e.ilo = e.jlo = 0;
  e.ax = e.ay = 0.0f;
  e.r0 = make_float4(0, 0, 0, 0);
  e.r1 = e.r0;
  e.r2 = e.r0;
  if (g >= w.n_records) return;
  const float4* rec = reinterpret_cast<const float4*>(record + (size_t)e.g * GS_RECORD_FLOATS);
  e.r0 = rec[0];
  const int lo = __float_as_int(e.r0.x), hi = __float_as_int(e.r0.y);
  e.ilo = lo & 0xFFFF;
  e.jlo = (lo >> 16) & 0xFFFF;
  const int ihi = hi & 0xFFFF, jhi = (hi >> 16) & 0xFFFF;
  const int qx1 = min(w.x0 + 7, w.W - 1), qy1 = min(w.y0 + 7, w.H - 1);
  if (e.ilo > qx1 || ihi < w.x0 || e.jlo > qy1 || jhi < w.y0) return;
  e.r1 = rec[1];
  Shape sh;
  sh.w00 = e.r1.x;
  sh.w10 = e.r1.y;
  sh.w11 = e.r1.z;
  sh.c0 = e.r0.z;
  sh.c1 = e.r0.w;
  sh.i11 = __builtin_amdgcn_rcpf(sh.w11);
  sh.iq = __builtin_amdgcn_rcpf(fmaf(sh.w00, sh.w00, sh.w10 * sh.w10));
  // the mean's offset from the corner centre: L a = -c
  e.ax = -sh.c0 * __builtin_amdgcn_rcpf(sh.w00);
  e.ay = -fmaf(sh.w10, e.ax, sh.c1) * sh.i11;
  const float thr = fminf(rules.ext2, 2.0f * (__logf(e.r1.w) - rules.log_alpha_min));
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int sx0 = w.x0 + 4 * (r & 1), sy0 = w.y0 + 4 * (r >> 1);
    const int sx1 = min(sx0 + 3, w.W - 1), sy1 = min(sy0 + 3, w.H - 1);
    // an empty block (past the image edge) has sx0 > sx1 or sy0 > sy1 and fails here
    if ((int32_t)i > row_lim[r] || e.ilo > sx1 || ihi < sx0 || e.jlo > sy1 || jhi < sy0 ||
        sx0 > sx1 || sy0 > sy1)
      continue;
    e.rows |= 1u << r;
  }
  // one exact test on the pixel box clipped to the wave's 8x8 block (every pixel that can
  // take the entry lies in that rectangle): one test per entry, not one per row
  if (e.rows) {
    const int rx0 = max(w.x0, e.ilo), rx1 = min(qx1, ihi), ry0 = max(w.y0, e.jlo), ry1 = min(qy1, jhi);
    if (!block_reachable(sh, thr, e.ax, e.ay, (float)(rx0 - e.ilo), (float)(rx1 - e.ilo),
                         (float)(ry0 - e.jlo), (float)(ry1 - e.jlo)))
      e.rows = 0;
  }
  if (e.rows) e.r2 = rec[2];
}

// LDS slice of one wave: the staged entries of a round (slot BATCH holds a null entry
// that no pixel takes), and per row the slots of its entries in walk order, as bytes.
template <int BATCH>
struct WaveLds {
  float4 geo[BATCH + 1];
  float4 shape[BATCH + 1];
  float4 col[BATCH + 1];
  uint32_t idx[kRows * BATCH / 4];   // row r's k-th slot: byte k of idx[r * BATCH / 4 ...]
};

// The null entry: zero shape and opacity give alpha = 0 < alpha_min at every pixel.
template <int BATCH>
__device__ __forceinline__ void init_null_entry(WaveLds<BATCH>& s) {
  if (__lane_id() == 0) {
    s.geo[BATCH] = make_float4(0, 0, 0, 0);
    s.shape[BATCH] = make_float4(0, 0, 0, 0);
    s.col[BATCH] = make_float4(0, 0, 0, __uint_as_float(0xFFFFFFFFu));
  }
}

// Compact the kept entries of the wave into its LDS slice (slots in lane order) and
// write every row's slot list front to back. Slots of a row past its count point at
// the null entry. Returns the largest row count.
template <int BATCH, int R>
__device__ __forceinline__ int commit_round(const Entry* e, WaveLds<BATCH>& s, int& n_kept) {
  constexpr uint32_t kNull = (uint32_t)BATCH * 0x01010101u;
  const int lane = threadIdx.x % kWave;
  for (int w = lane; w < kRows * BATCH / 4; w += kWave) s.idx[w] = kNull;
  const uint64_t lt = lanemask_lt();
  // all ballots first, then the writes
  uint64_t km[R], br[R][kRows];
  int cnt[kRows] = {0, 0, 0, 0};
#pragma unroll
  for (int sub = 0; sub < R; ++sub) {
    km[sub] = __ballot(e[sub].rows != 0);
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      br[sub][r] = __ballot((e[sub].rows >> r) & 1u);
      cnt[r] += __popcll(br[sub][r]);
    }
  }
  uint8_t* idx8 = reinterpret_cast<uint8_t*>(s.idx);
  int slot0 = 0;
  int before[kRows] = {0, 0, 0, 0};
#pragma unroll
  for (int sub = 0; sub < R; ++sub) {
    const Entry& x = e[sub];
    const int slot = slot0 + __popcll(km[sub] & lt);
    if (x.rows) {
      s.geo[slot] = make_float4((float)x.ilo + 0.5f, (float)x.jlo + 0.5f, x.r0.z, x.r0.w);
      s.shape[slot] = x.r1;
      s.col[slot] = make_float4(x.r2.x, x.r2.y, x.r2.z, __uint_as_float(x.i));
    }
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      if ((x.rows >> r) & 1u) {
        const int q = before[r] + __popcll(br[sub][r] & lt);   // rank in list order
        idx8[r * BATCH + q] = (uint8_t)slot;
      }
      before[r] += __popcll(br[sub][r]);
    }
    slot0 += __popcll(km[sub]);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  n_kept = slot0;
  return max(max(cnt[0], cnt[1]), max(cnt[2], cnt[3]));
}

// Instance values (Gaussian record indices) of one round, loaded one round ahead so
// that the first link of the gather chain (value, then record) is in flight while the
// wave blends the previous round. Entries past the round's end hold ~0u, which no
// record index reaches.
template <int R>
struct Ahead {
  uint32_t g[R];
};

template <int BATCH>
constexpr int lanes_rounds() { return (BATCH + kWave - 1) / kWave; }

// Values of the BATCH entries [first, first + BATCH), entry r * 64 + lane in a.g[r]
// (a round of 32 entries leaves lanes 32..63 empty).
template <int BATCH>
__device__ __forceinline__ void load_ahead(const uint32_t* __restrict__ vals, int64_t first,
                                           int64_t last_ok, Ahead<lanes_rounds<BATCH>()>& a) {
  const int lane = threadIdx.x % kWave;
#pragma unroll
  for (int r = 0; r < lanes_rounds<BATCH>(); ++r) {
    const int64_t i = first + r * kWave + lane;
    a.g[r] = (r * kWave + lane < BATCH && i <= last_ok) ? vals[i] : ~0u;
  }
}

// Stage the BATCH consecutive list entries [first, first + BATCH) whose values `a`
// holds (all gathers are issued before any ballot). Returns the largest row count;
// n_kept receives the number of staged entries.
template <int BATCH>
__device__ __forceinline__ int stage_round(const float* __restrict__ record,
                                           const Ahead<lanes_rounds<BATCH>()>& a, int64_t first,
                                           const WaveTile& w, const Rules& rules,
                                           const int32_t* row_lim, WaveLds<BATCH>& s,
                                           int& n_kept) {
  constexpr int R = lanes_rounds<BATCH>();
  Entry e[R];
  const int lane = threadIdx.x % kWave;
#pragma unroll
  for (int r = 0; r < R; ++r)
    gather_entry(record, a.g[r], (uint32_t)(first + r * kWave + lane), w, rules, row_lim, e[r]);
  return commit_round<BATCH, R>(e, s, n_kept);
}

template <int TS, int BATCH>
__global__ void __launch_bounds__((TS / 8) * (TS / 8) * kWave)
render_fwd_kernel(const float* __restrict__ record, const uint32_t* __restrict__ vals,
                  const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ tile_order,
                  TileViews tv, Rules rules, float* __restrict__ image,
                  float* __restrict__ T_final, int32_t* __restrict__ last_idx) {
  constexpr int WPT = (TS / 8) * (TS / 8);
  constexpr int R = lanes_rounds<BATCH>();
  __shared__ WaveLds<BATCH> s_lds[WPT];
  WaveTile w;
  if (!wave_tile<TS>(tv, tile_order, w)) return;
  WaveLds<BATCH>& s = s_lds[threadIdx.x / kWave];
  init_null_entry(s);
  uint32_t start, end;
  tile_range(ranges, w.tile, tv.n_inst, start, end);
  const float fpx = (float)w.px + 0.5f, fpy = (float)w.py + 0.5f;
  const float amax = rules.alpha_max;
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  int32_t last = -1;
  // the smallest alpha the pixel still takes: alpha_min while it blends, +inf once it
  // stopped (or when it lies outside the image), so that one compare decides both
  float amin = w.inside ? rules.alpha_min : INFINITY;
  Ahead<R> ahead;
  load_ahead<BATCH>(vals, start, (int64_t)end - 1, ahead);
  for (uint32_t base = start; base < end; base += BATCH) {
    const uint64_t lv = __ballot(amin < INFINITY);
    if (lv == 0ull) break;
    int32_t row_lim[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) row_lim[r] = ((lv >> (kRowLanes * r)) & 0xFFFFull) ? INT32_MAX : -1;
    const Ahead<R> cur = ahead;
    int n_kept;
    const int n_steps = stage_round<BATCH>(record, cur, base, w, rules, row_lim, s, n_kept);
    load_ahead<BATCH>(vals, (int64_t)base + BATCH, (int64_t)end - 1, ahead);
    // groups of 8 steps; the saturation ballot runs once per group
    bool all_done = false;
    for (int k0 = 0; k0 < n_steps && !all_done; k0 += 8) {
      const int kend = min(k0 + 8, n_steps);
      uint32_t word = 0;
      for (int k = k0; k < kend; ++k) {
        if ((k & 3) == 0) word = s.idx[w.row * (BATCH / 4) + (k >> 2)];   // four steps' slots
        const int slot = (word >> (8 * (k & 3))) & 0xFF;
        const float4 geo = s.geo[slot];
        const float4 shape = s.shape[slot];
        const float4 col = s.col[slot];
        Eval e;
        eval_alpha(geo, shape, fpx, fpy, amax, e);
        // branch-free: every lane evaluates. a is alpha where the Gaussian is taken
        // (inside the extent, alpha >= alpha_min > 0, pixel live), else 0; an untaken
        // entry then leaves T * (1 - 0) = T >= T_min, so only a taken one can stop.
        // The two tests form one lane mask and one select; the blended mask (taken and
        // not stopping) selects the weight and the last contributor.
        const bool take = (e.m <= rules.ext2) & (e.alpha >= amin);
        const float a = take ? e.alpha : 0.0f;
        const float Tn = T * (1.0f - a);
        const bool stop = Tn < rules.T_min;
        const bool blend = take & !stop;
        const float wgt = T * (blend ? a : 0.0f);
        C0 = fmaf(wgt, col.x, C0);
        C1 = fmaf(wgt, col.y, C1);
        C2 = fmaf(wgt, col.z, C2);
        T = stop ? T : Tn;
        last = blend ? (int32_t)__float_as_uint(col.w) : last;
        amin = stop ? INFINITY : amin;
      }
      all_done = __ballot(amin < INFINITY) == 0ull;
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

// Value of lane l ^ XM (XM < 16: a partner in the same 16-lane row) through ds_swizzle
// (bit mode, and-mask 0x1F): the exchange runs in the LDS crossbar, beside the VALU
// work of the other waves, where a DPP operand would take a VALU issue slot (the
// backward blend is bound by its VALU issue; measured a few percent faster).
template <int XM>
__device__ __forceinline__ float lane_xor(float x) {
  static_assert(XM > 0 && XM < 16, "partner must be in the same row");
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, x), (XM << 10) | 0x1F));
}

template <int XM>
__device__ __forceinline__ int lane_xor_int(int x) {
  static_assert(XM > 0 && XM < 16, "partner must be in the same row");
  return __builtin_amdgcn_ds_swizzle(x, (XM << 10) | 0x1F);
}

// Largest value over the 16 lanes of each row.
__device__ __forceinline__ int row_max_int(int x) {
  x = max(x, lane_xor_int<1>(x));
  x = max(x, lane_xor_int<2>(x));
  x = max(x, lane_xor_int<4>(x));
  x = max(x, lane_xor_int<8>(x));
  return x;
}

// Row sum of nine per-lane values as a reduce-scatter butterfly inside each 16-lane
// row: at every step a lane keeps half of its remaining values and adds its partner's
// copy of them (9 -> 5 -> 3 -> 2 -> 1 registers). The partners l ^ 15 and l ^ 7 differ
// in all low bits, so they come first (split on bit 3, then bit 2), then l ^ 2 and
// l ^ 1. Row lane l then holds its row's total of value reduce_index(l) when bit l of
// kReduceLanes is set. A value without a partner at a step (a4, then x2, then y1) is
// added to its partner lane's copy on both lanes, with no selects: on the lanes that
// should hold nothing in that slot the copy lands in a slot past the ninth value, and
// every later partner shares the bits already split on, so it never reaches a kept lane
// (the kept lanes add the same operands as with an explicit zero).
constexpr uint32_t kReduceLanes = 0x1737u;  // row lanes 0, 1, 2, 4, 5, 8, 9, 10, 12
__device__ __forceinline__ int reduce_index(uint32_t l) {
  return 5 * ((l >> 3) & 1) + 3 * ((l >> 2) & 1) + 2 * ((l >> 1) & 1) + (l & 1);
}

// Value v of the butterfly is grad2d component (kSlotOfValue >> 4 v) & 15: the values
// are, in order, d_r, d_mx, d_my, d_w00, d_w11, d_g, d_o, d_b, d_w10, so that the first
// pair (values 0 and 5) is the red and green gradient, both the step's blend weight
// times a per-pixel constant: the lane's kept and sent constants of that pair are
// chosen once per pixel (k0 = w g_keep, s0 = w g_send), not selected at every step.
constexpr uint64_t kSlotOfValue = 0x385742106ull;

__device__ __forceinline__ float row_reduce9_scatter(float k0, float s0, float a1, float a2,
                                                     float a3, float a4, float a6, float a7,
                                                     float a8) {
  const uint32_t l = __lane_id() & 15;
  const bool h3 = l & 8, h2 = l & 4, h1 = l & 2, h0 = l & 1;
  const float x0 = k0 + lane_xor<15>(s0);
  const float x1 = (h3 ? a6 : a1) + lane_xor<15>(h3 ? a1 : a6);
  const float x2 = (h3 ? a7 : a2) + lane_xor<15>(h3 ? a2 : a7);
  const float x3 = (h3 ? a8 : a3) + lane_xor<15>(h3 ? a3 : a8);
  const float x4 = a4 + lane_xor<15>(a4);
  const float y0 = (h2 ? x3 : x0) + lane_xor<7>(h2 ? x0 : x3);
  const float y1 = (h2 ? x4 : x1) + lane_xor<7>(h2 ? x1 : x4);
  const float y2 = x2 + lane_xor<7>(x2);
  const float z0 = (h1 ? y2 : y0) + lane_xor<2>(h1 ? y0 : y2);
  const float z1 = y1 + lane_xor<2>(y1);
  return (h0 ? z1 : z0) + lane_xor<1>(h0 ? z0 : z1);
}

// ---------------------------------------------------------------------------
// backward: one Gaussian per step over the wave's whole 8x8 block
// ---------------------------------------------------------------------------

// LDS slice of one wave for the backward: the kept entries of a round in list order
// (geo, shape, colour with the record index, and aux = (offset a of the mean from the
// corner pixel centre, list position)).
template <int BATCH>
struct BwdLds {
  float4 geo[BATCH];
  float4 shape[BATCH];
  float4 col[BATCH];
  float4 aux[BATCH];
};

// List entry i (record g) for the backward: kept if some pixel of the wave's 8x8 block
// can take it (the block test of gather_entry over the whole block).
__device__ __forceinline__ bool gather_block_entry(const float* __restrict__ record, uint32_t g,
                                                   const WaveTile& w, const Rules& rules,
                                                   float4& r0, float4& r1, float4& r2,
                                                   float& ax, float& ay) {
  r0 = r1 = r2 = make_float4(0, 0, 0, 0);
  ax = ay = 0.0f;
  if (g >= w.n_records) return false;
  const float4* rec = reinterpret_cast<const float4*>(record + (size_t)g * GS_RECORD_FLOATS);
  r0 = rec[0];
  const int lo = __float_as_int(r0.x), hi = __float_as_int(r0.y);
  const int ilo = lo & 0xFFFF, jlo = (lo >> 16) & 0xFFFF;
  const int ihi = hi & 0xFFFF, jhi = (hi >> 16) & 0xFFFF;
  const int bx1 = min(w.x0 + 7, w.W - 1), by1 = min(w.y0 + 7, w.H - 1);
  if (ilo > bx1 || ihi < w.x0 || jlo > by1 || jhi < w.y0) return false;
  r1 = rec[1];
  Shape sh;
  sh.w00 = r1.x;
  sh.w10 = r1.y;
  sh.w11 = r1.z;
  sh.c0 = r0.z;
  sh.c1 = r0.w;
  sh.i11 = __builtin_amdgcn_rcpf(sh.w11);
  sh.iq = __builtin_amdgcn_rcpf(fmaf(sh.w00, sh.w00, sh.w10 * sh.w10));
  // the mean's offset from the corner centre: L^-1 a = -c
  ax = -sh.c0 * __builtin_amdgcn_rcpf(sh.w00);
  ay = -fmaf(sh.w10, ax, sh.c1) * sh.i11;
  const float thr = fminf(rules.ext2, 2.0f * (__logf(r1.w) - rules.log_alpha_min));
  if (!block_reachable(sh, thr, ax, ay, (float)(w.x0 - ilo), (float)(bx1 - ilo),
                       (float)(w.y0 - jlo), (float)(by1 - jlo)))
    return false;
  r2 = rec[2];
  return true;
}

// Stage the entries [first, first + BATCH) whose values `a` holds: the kept ones in
// list order from slot 0. Returns the kept count.
template <int BATCH>
__device__ __forceinline__ int stage_block_round(const float* __restrict__ record,
                                                 const Ahead<lanes_rounds<BATCH>()>& a,
                                                 int64_t first, const WaveTile& w,
                                                 const Rules& rules, BwdLds<BATCH>& s) {
  constexpr int R = lanes_rounds<BATCH>();
  const int lane = threadIdx.x % kWave;
  float4 r0[R], r1[R], r2[R];
  float ax[R], ay[R];
  bool keep[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
    keep[r] = gather_block_entry(record, a.g[r], w, rules, r0[r], r1[r], r2[r], ax[r], ay[r]);
  const uint64_t lt = lanemask_lt();
  int cnt = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t km = __ballot(keep[r]);
    if (keep[r]) {
      const int slot = cnt + __popcll(km & lt);
      const int lo = __float_as_int(r0[r].x);
      s.geo[slot] = make_float4((float)(lo & 0xFFFF) + 0.5f, (float)((lo >> 16) & 0xFFFF) + 0.5f,
                                r0[r].z, r0[r].w);
      s.shape[slot] = r1[r];
      s.col[slot] = make_float4(r2[r].x, r2[r].y, r2[r].z, __uint_as_float(a.g[r]));
      s.aux[slot] = make_float4(ax[r], ay[r], __uint_as_float((uint32_t)(first + r * kWave + lane)), 0.0f);
    }
    cnt += __popcll(km);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  return cnt;
}

// Largest value over the wave.
__device__ __forceinline__ int wave_max_int(int x) {
  x = row_max_int(x);
  x = max(x, __shfl_xor(x, 16, kWave));
  return max(x, __shfl_xor(x, 32, kWave));
}

// The L1 term of the loss taken inside the backward (L1 = true): each pixel's upstream
// gradient dL/dimage = sign(image - target) / (3 H W) (sign(0) = 0) is formed from the
// forward's image and the target, instead of being read from a stored dL/dimage, and
// the wave's share of the loss, mean |image - target| over 3 H W, goes to one slot per
// wave (tile * waves per tile + wave), summed per view by loss_parts_kernel.
struct L1In {
  const float* image;    // flat image layout
  const float* target;   // flat image layout
  float* part;           // [tiles * waves per tile] per-wave loss shares; NULL: no loss
};

template <int TS, int BATCH, bool LIMIT, bool L1>
__global__ void __launch_bounds__((TS / 8) * (TS / 8) * kWave)
render_bwd_kernel(const float* __restrict__ record, const uint32_t* __restrict__ vals,
                  const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ tile_order,
                  TileViews tv, Rules rules, const float* __restrict__ T_final,
                  const int32_t* __restrict__ last_idx, const float* __restrict__ dL_dimage,
                  float* __restrict__ grad2d, L1In l1) {
  constexpr int WPT = (TS / 8) * (TS / 8);
  __shared__ BwdLds<BATCH> s_lds[WPT];
  WaveTile w;
  if (!wave_tile<TS>(tv, tile_order, w)) {
    if constexpr (L1) {
      // a block outside the image still owns its loss slot: a zero share
      if (l1.part && (uint32_t)w.tile < (uint32_t)tv.tile_offset[tv.n_views] && __lane_id() == 0)
        l1.part[(int64_t)w.tile * WPT + threadIdx.x / kWave] = 0.0f;
    }
    return;
  }
  BwdLds<BATCH>& s = s_lds[threadIdx.x / kWave];
  const int lane = threadIdx.x % kWave;
  // the wave's 8x8 block: lane l owns pixel (l & 7, l >> 3) of it
  const int px = w.x0 + (lane & 7), py = w.y0 + (lane >> 3);
  const bool inside = px < w.W && py < w.H;
  uint32_t start, end;
  tile_range(ranges, w.tile, tv.n_inst, start, end);
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
  const float amax = rules.alpha_max;
  float T = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
  float loss_share = 0.0f;   // this pixel's share of the view's L1 loss (L1 only)
  int32_t last = -1;
  if (inside) {
    const int64_t P = tv.pix_offset[w.v];
    const int64_t HW = (int64_t)w.W * w.H;
    const int64_t p = (int64_t)py * w.W + px;
    T = T_final[P + p];
    last = last_idx[P + p];
    if constexpr (L1) {
      const float inv = 1.0f / (3.0f * (float)HW);
      const float* img = l1.image + 3 * P;
      const float* tgt = l1.target + 3 * P;
      const float d0 = img[p] - tgt[p], d1 = img[HW + p] - tgt[HW + p],
                  d2 = img[2 * HW + p] - tgt[2 * HW + p];
      g0 = d0 > 0.0f ? inv : (d0 < 0.0f ? -inv : 0.0f);
      g1 = d1 > 0.0f ? inv : (d1 < 0.0f ? -inv : 0.0f);
      g2 = d2 > 0.0f ? inv : (d2 < 0.0f ? -inv : 0.0f);
      loss_share = fabsf(d0) * inv + fabsf(d1) * inv + fabsf(d2) * inv;
    } else {
      const float* dimg = dL_dimage + 3 * P;
      g0 = dimg[p];
      g1 = dimg[HW + p];
      g2 = dimg[2 * HW + p];
    }
  }
  if constexpr (L1) {
    // before the early exit below: pixels that blended nothing still count in the loss
    if (l1.part) {
      loss_share = wave_sum_to_lane63(loss_share);
      if (lane == kWave - 1) l1.part[(int64_t)w.tile * WPT + threadIdx.x / kWave] = loss_share;
    }
  }
  // only g . B is ever needed, where B is the colour accumulated behind the current
  // Gaussian (initially T_final bg): dC/dalpha_i . g = T_i (g . c_i) - (g . B_i) / (1 - alpha_i)
  float S = T * (g0 * rules.bg[0] + g1 * rules.bg[1] + g2 * rules.bg[2]);
  // the walk starts at the wave's last contributor, bounded by the tile's list so that
  // a last_idx not written by the forward pass cannot send the gathers out of range
  const int32_t wave_last = min(wave_max_int(last), (int32_t)end - 1);
  if (wave_last < (int32_t)start) return;  // no pixel of this wave blended anything
  const bool atomic_lane = lane < kRowLanes && ((kReduceLanes >> lane) & 1u);
  const int atomic_slot = (int)((kSlotOfValue >> (4 * reduce_index((uint32_t)lane))) & 15u);
  // the red / green pair of the butterfly's first step: the colour constant this lane
  // keeps and the one it sends to its partner l ^ 15
  const bool upper = lane & 8;
  const float g_keep = upper ? g1 : g0, g_send = upper ? g0 : g1;
  // limited-gradient ablation: count the pixel's blended Gaussians first, so the
  // back-to-front walk knows each one's front-to-back rank
  int n_blended = 0, from_back = 0;
  if constexpr (LIMIT) {
    for (int64_t top = wave_last; top >= (int64_t)start; top -= BATCH) {
      const int64_t bot = max((int64_t)start, top - (BATCH - 1));
      Ahead<lanes_rounds<BATCH>()> cur;
      load_ahead<BATCH>(vals, bot, top, cur);
      const int cnt = stage_block_round<BATCH>(record, cur, bot, w, rules, s);
      for (int k = 0; k < cnt; ++k) {
        const int32_t pos = (int32_t)__float_as_uint(s.aux[k].z);
        Eval e;
        eval_alpha(s.geo[k], s.shape[k], fpx, fpy, amax, e);
        n_blended += ((pos <= last) && (e.m <= rules.ext2) && (e.alpha >= rules.alpha_min)) ? 1 : 0;
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  Ahead<lanes_rounds<BATCH>()> ahead;
  load_ahead<BATCH>(vals, max((int64_t)start, (int64_t)wave_last - (BATCH - 1)), wave_last, ahead);
  for (int64_t top = wave_last; top >= (int64_t)start; top -= BATCH) {
    const int64_t bot = max((int64_t)start, top - (BATCH - 1));
    const Ahead<lanes_rounds<BATCH>()> cur = ahead;
    const int cnt = stage_block_round<BATCH>(record, cur, bot, w, rules, s);
    const int64_t ntop = top - BATCH;   // the next round, [max(start, ntop - BATCH + 1), ntop]
    load_ahead<BATCH>(vals, max((int64_t)start, ntop - (BATCH - 1)), ntop, ahead);
    for (int k = cnt - 1; k >= 0; --k) {
      const float4 geo = s.geo[k];
      const float4 shape = s.shape[k];
      const float4 col = s.col[k];
      const float4 aux = s.aux[k];
      const int32_t pos = (int32_t)__float_as_uint(aux.z);
      Eval e;
      eval_alpha(geo, shape, fpx, fpy, amax, e);
      // branch-free: non-contributing lanes add zeros and keep their state
      const bool contrib = (pos <= last) && (e.m <= rules.ext2) && (e.alpha >= rules.alpha_min);
      bool grad_on = contrib;
      if constexpr (LIMIT) {
        grad_on = contrib && (n_blended - 1 - from_back) < rules.grad_limit;
        from_back += contrib ? 1 : 0;
      }
      // alpha of a contributing entry, else 0: then 1 / (1 - a) is exactly 1 (the hardware
      // reciprocal is exact at powers of two) and the weight 0, with one select
      const float a = contrib ? e.alpha : 0.0f;
      const float inv = __builtin_amdgcn_rcpf(1.0f - a);
      T = T * inv;  // transmittance in front of this Gaussian
      const float wgt = T * a;
      // wgt is already 0 where the entry does not contribute; only the limited-gradient
      // ablation drops contributing entries from the gradient
      float gwgt = wgt;
      if constexpr (LIMIT) gwgt = grad_on ? wgt : 0.0f;
      const float d_b = gwgt * g2;
      const float gc = fmaf(g2, col.z, fmaf(g1, col.y, g0 * col.x));
      float dalpha = fmaf(T, gc, -S * inv);
      S = fmaf(wgt, gc, S);
      // alpha = min(alpha_max, o G): no gradient through a clamped alpha
      dalpha = (grad_on && shape.w * e.G <= rules.alpha_max) ? dalpha : 0.0f;
      const float d_o = dalpha * e.G;
      // dalpha/dm = -alpha / 2; m = e0^2 + e1^2 with e = L^-1 d, d = pixel - mean
      // (d = D - a: the pixel's offset D from the corner centre, exact, minus the mean's)
      const float q = -dalpha * e.alpha;
      const float t0 = q * e.e0, t1 = q * e.e1;
      const float d_mx = -fmaf(t0, shape.x, t1 * shape.y);
      const float d_my = -(t1 * shape.z);
      const float dx = e.di - aux.x, dy = e.dj - aux.y;
      const float d_w00 = t0 * dx, d_w10 = t1 * dx, d_w11 = t1 * dy;
      if (__ballot(grad_on) != 0ull) {
        float tot = row_reduce9_scatter(gwgt * g_keep, gwgt * g_send, d_mx, d_my, d_w00, d_w11,
                                        d_o, d_b, d_w10);
        tot += __shfl_xor(tot, 16, kWave);
        tot += __shfl_xor(tot, 32, kWave);
        // staged entries hold record indices below n_records (gather_block_entry)
        const uint32_t rec = __float_as_uint(col.w);
        if (atomic_lane && tot != 0.0f)
          atomicAdd(grad2d + (size_t)rec * GS_GRAD2D_FLOATS + atomic_slot, tot);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Sum of one view's per-wave L1 shares (blockIdx.x = view), in a fixed order, so that
// the loss is the same on every run, added to loss[v]. Every wave of the view's tiles
// wrote its slot (zero for blocks outside the image).
constexpr int kPartThreads = 1024;

__global__ void __launch_bounds__(kPartThreads)
loss_parts_kernel(const float* __restrict__ part, TileViews tv, float* __restrict__ loss) {
  __shared__ float s_sum[kPartThreads / kWave];
  const int v = blockIdx.x;
  const int64_t wpt = (int64_t)(tv.tile / 8) * (tv.tile / 8);
  const int64_t b = (int64_t)tv.tile_offset[v] * wpt, e = (int64_t)tv.tile_offset[v + 1] * wpt;
  // eight independent loads in flight per pass, added in a fixed order
  float a[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  for (int64_t i = b + threadIdx.x; i < e; i += 8 * kPartThreads) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t k = i + (int64_t)j * kPartThreads;
      a[j] += (k < e) ? part[k] : 0.0f;
    }
  }
  float acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  acc = wave_sum_to_lane63(acc);
  if (__lane_id() == kWave - 1) s_sum[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int k = 0; k < kPartThreads / kWave; ++k) t += s_sum[k];
    atomicAdd(loss + v, t);
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
  const int batch = cfg->lds_batch == 0 ? 64 : cfg->lds_batch;
#define GS_FWD(TS, B)                                                                          \
  render_fwd_kernel<TS, B><<<grid, (TS / 8) * (TS / 8) * kWave, 0, s>>>(                      \
      proj->record, inst->vals, tile_ranges, tile_order, tv, rules, image, T_final, last_idx)
#define GS_FWD_BATCH(TS)                                                                       \
  switch (batch) {                                                                             \
    case 32: GS_FWD(TS, 32); break;                                                            \
    case 128: GS_FWD(TS, 128); break;                                                          \
    default: GS_FWD(TS, 64); break;                                                            \
  }
  switch (cfg->tile_size) {
    case 8: GS_FWD_BATCH(8); break;
    case 32: GS_FWD_BATCH(32); break;
    default: GS_FWD_BATCH(16); break;
  }
#undef GS_FWD_BATCH
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

template <bool L1>
static int render_bwd_launch(const gs_projected* proj, const gs_instances* inst,
                             const uint32_t* tile_ranges, const uint32_t* tile_order,
                             const TileViews& tv, const gs_config* cfg, const float* T_final,
                             const int32_t* last_idx, const float* dL_dimage, float* grad2d,
                             L1In l1, hipStream_t s) {
  const Rules rules = make_rules(cfg);
  const dim3 grid((unsigned)tv.tile_offset[tv.n_views]);
#define GS_BWD(TS, B)                                                                          \
  render_bwd_kernel<TS, B, false, L1><<<grid, (TS / 8) * (TS / 8) * kWave, 0, s>>>(           \
      proj->record, inst->vals, tile_ranges, tile_order, tv, rules, T_final, last_idx,         \
      dL_dimage, grad2d, l1)
#define GS_BWD_LIMITED(TS)                                                                     \
  render_bwd_kernel<TS, 64, true, L1><<<grid, (TS / 8) * (TS / 8) * kWave, 0, s>>>(           \
      proj->record, inst->vals, tile_ranges, tile_order, tv, rules, T_final, last_idx,         \
      dL_dimage, grad2d, l1)
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
  // 32x32 tiles stage at most 64 entries per wave and round: sixteen waves with
  // 128-entry rounds would not fit the workgroup's LDS
  const int batch = cfg->lds_batch == 0 ? 64 : cfg->lds_batch;
  switch (cfg->tile_size) {
    case 8:
      if (batch == 32) GS_BWD(8, 32); else if (batch == 128) GS_BWD(8, 128); else GS_BWD(8, 64);
      break;
    case 32:
      if (batch == 32) GS_BWD(32, 32); else GS_BWD(32, 64);
      break;
    default:
      if (batch == 32) GS_BWD(16, 32); else if (batch == 128) GS_BWD(16, 128); else GS_BWD(16, 64);
      break;
  }
#undef GS_BWD
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
  return render_bwd_launch<false>(proj, inst, tile_ranges, tile_order, tv, cfg, T_final, last_idx,
                                  dL_dimage, grad2d, L1In{nullptr, nullptr, nullptr},
                                  reinterpret_cast<hipStream_t>(stream));
}

extern "C" size_t gs_render_l1_workspace_bytes(const gs_camera* cams, int32_t n_views,
                                               const gs_config* cfg) {
  if (!cfg || check_config(cfg) != GS_OK) return 0;
  TileViews tv;
  if (fill_tile_views(cams, n_views, cfg->tile_size, &tv) != GS_OK) return 0;
  const size_t wpt = (size_t)(cfg->tile_size / 8) * (size_t)(cfg->tile_size / 8);
  return (size_t)tv.tile_offset[n_views] * wpt * sizeof(float);
}

extern "C" int gs_render_bwd_l1(const gs_projected* proj, const gs_instances* inst,
                                const uint32_t* tile_ranges, const uint32_t* tile_order,
                                const gs_camera* cams, int32_t n_views, const gs_config* cfg,
                                const float* T_final, const int32_t* last_idx, const float* image,
                                const float* target, float* grad2d, float* loss, void* workspace,
                                size_t workspace_bytes, int64_t n, gs_stream_t stream) {
  TileViews tv;
  int rc = render_common(proj, inst, tile_ranges, cams, n_views, cfg, n, &tv);
  if (rc != GS_OK) return rc;
  if (!T_final || !last_idx || !image || !target || !grad2d) return GS_ERR_ARG;
  float* part = nullptr;
  if (loss) {
    const size_t need = gs_render_l1_workspace_bytes(cams, n_views, cfg);
    if (need == 0 || !workspace || workspace_bytes < need) return GS_ERR_ARG;
    part = static_cast<float*>(workspace);
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  rc = render_bwd_launch<true>(proj, inst, tile_ranges, tile_order, tv, cfg, T_final, last_idx,
                               nullptr, grad2d, L1In{image, target, part}, s);
  if (rc != GS_OK || !loss) return rc;
  loss_parts_kernel<<<(unsigned)n_views, kPartThreads, 0, s>>>(part, tv, loss);
  return launch_status();
}
