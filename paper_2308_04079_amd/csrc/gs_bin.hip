// gs_bin: one (tile, value) instance per tile a visible (view, Gaussian) pair
// overlaps (Alg. 2 CreateTiles + DuplicateWithKeys; App. C "Sorting"), emitted in
// front-to-back order, so that gs_sort only has to sort the instances by tile:
//   1. compact the visible pairs (index order) with their depth keys;
//   2. stable radix sort of (depth, index) (31 key bits: depth > 0);
//   3. per depth-sorted pair, one gather of its tile rectangle from the record (its
//      tile count, first tile id and width, written densely in depth order), then
//      the exclusive scan of the counts (the instance count and the capacity check
//      come from an exact sum in step 1);
//   4. expansion of every pair into its tiles, row-major, writing the global tile id
//      and the pair's index, partitioned by output instance so every block does
//      the same work (the nearest pairs cover the most tiles and sort first); the
//      offsets pass of step 3 records the pair each output block starts in, and the
//      expansion reads only dense per-pair arrays.
// The result is the paper's per-instance (tile | depth) key order once sorted by tile.
#include <algorithm>

#include "gs_internal.h"

namespace gs {

constexpr int kBinBlock = 256;
constexpr int kBinItems = 8;                       // per thread
constexpr int kBinTile = kBinBlock * kBinItems;     // 2048 per block
constexpr int kExpandOut = 1024;                    // instances per expansion block
// misc words: [0] visible pairs, [1] the same clamped to the capacity, [4] the
// instances of the (clamped) depth-sorted pairs. The exact instance count over all
// pairs (64-bit, exact even when the capacity is short) is the sum of the per-block
// parts in the workspace's tile_parts.
constexpr int kMiscWords = 16;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = __lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, kWave);
    if (lane >= (uint32_t)d) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread over a 256-thread block; returns the
// block total through *total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* smem4, uint32_t* total) {
  const int wave = threadIdx.x / kWave;
  const uint32_t incl = wave_incl_scan(x);
  if (__lane_id() == kWave - 1) smem4[wave] = incl;
  __syncthreads();
  uint32_t base = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kBinBlock / kWave; ++w) {
    const uint32_t s = smem4[w];
    base += (w < wave) ? s : 0u;
    all += s;
  }
  __syncthreads();
  *total = all;
  return base + incl - x;
}

// Per block of the (view, Gaussian) pairs in index order: the number of visible pairs,
// and the block's instance count (64-bit) in instances_part[block].
__global__ void __launch_bounds__(kBinBlock)
bin_visible_sums(const int32_t* __restrict__ touched, int64_t n_items,
                 uint32_t* __restrict__ sums, unsigned long long* __restrict__ instances_part) {
  __shared__ uint32_t s4[kBinBlock / kWave];
  __shared__ unsigned long long s_tiles[kBinBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kBinTile;
  uint32_t acc = 0;
  unsigned long long tiles = 0;
#pragma unroll
  for (int j = 0; j < kBinItems; ++j) {
    const int64_t i = base + (int64_t)j * kBinBlock + threadIdx.x;
    const int32_t c = i < n_items ? touched[i] : 0;
    acc += c > 0 ? 1u : 0u;
    tiles += (unsigned long long)max(c, 0);
  }
  uint32_t tot;
  block_excl_scan(acc, s4, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
  // a per-block total, summed by the scan kernel, rather than one atomic per block on
  // a single counter
  unsigned long long t = tiles;
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) t += __shfl_xor(t, d, kWave);
  if (__lane_id() == 0) s_tiles[threadIdx.x / kWave] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long all = 0;
#pragma unroll
    for (int w = 0; w < kBinBlock / kWave; ++w) all += s_tiles[w];
    instances_part[blockIdx.x] = all;
  }
}

// Tile rectangle of a pair, from the pixel rectangle packed in its record: first
// column and row, width and height, in tiles.
struct TileRect {
  uint32_t tx0, ty0, w, h;
};

__device__ __forceinline__ TileRect tile_rect(int2 lohi, int T) {
  const int ts = __builtin_ctz(T);   // tiles are 8, 16 or 32 pixels wide
  TileRect r;
  r.tx0 = (uint32_t)((lohi.x & 0xFFFF) >> ts);
  r.ty0 = (uint32_t)(((lohi.x >> 16) & 0xFFFF) >> ts);
  r.w = (uint32_t)((lohi.y & 0xFFFF) >> ts) - r.tx0 + 1;
  r.h = (uint32_t)(((lohi.y >> 16) & 0xFFFF) >> ts) - r.ty0 + 1;
  return r;
}

__device__ __forceinline__ int view_of_pair(const TileViews& tv, uint32_t i, int64_t n) {
  int v = 0;
  while (v + 1 < tv.n_views && (int64_t)i >= (int64_t)(v + 1) * n) ++v;
  return v;
}

// Per depth-sorted pair, from its record's pixel rectangle (the same rectangle whose
// tile count the projection wrote to tiles_touched): width | height << 16 in tiles
// (both at most 4096: 32767 pixels over tiles of 8 or more) and the global id of its
// first tile, written densely in depth order; per block the instance count.
__global__ void __launch_bounds__(kBinBlock)
bin_pair_tiles(const uint32_t* __restrict__ sorted, const uint32_t* __restrict__ n_sorted_dev,
               int64_t max_items, const float* __restrict__ record, int64_t n, TileViews tv,
               uint32_t* __restrict__ sums, uint32_t* __restrict__ pair_wh,
               uint32_t* __restrict__ pair_base) {
  __shared__ uint32_t s4[kBinBlock / kWave];
  const int64_t n_items = min((int64_t)n_sorted_dev[0], max_items);
  const int64_t base = (int64_t)blockIdx.x * kBinTile;
  uint32_t g[kBinItems];
#pragma unroll
  for (int j = 0; j < kBinItems; ++j) {
    const int64_t s = base + (int64_t)j * kBinBlock + threadIdx.x;
    g[j] = s < n_items ? sorted[s] : ~0u;
  }
  int2 lohi[kBinItems];
#pragma unroll
  for (int j = 0; j < kBinItems; ++j)
    lohi[j] = g[j] != ~0u ? *reinterpret_cast<const int2*>(record + (int64_t)g[j] * GS_RECORD_FLOATS)
                          : make_int2(0, 0);
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kBinItems; ++j) {
    if (g[j] == ~0u) continue;
    const int64_t s = base + (int64_t)j * kBinBlock + threadIdx.x;
    const int v = view_of_pair(tv, g[j], n);
    const TileRect r = tile_rect(lohi[j], tv.tile);
    pair_wh[s] = r.w | (r.h << 16);
    pair_base[s] = (uint32_t)tv.tile_offset[v] + r.ty0 * (uint32_t)tv.tiles_x[v] + r.tx0;
    acc += r.w * r.h;
  }
  uint32_t tot;
  block_excl_scan(acc, s4, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One block: exclusive scan of the block sums in place. Writes the total (and,
// if clamped is given, the total clamped to `capacity`). With `exact` given (n_exact
// 64-bit per-block parts), the count written and checked against the capacity is
// their sum instead (the status flag is raised when it exceeds the capacity).
__global__ void __launch_bounds__(1024)
bin_scan_sums(uint32_t* __restrict__ sums, int64_t n_blocks, int64_t capacity,
              uint32_t* __restrict__ total_out, uint32_t* __restrict__ clamped,
              const unsigned long long* __restrict__ exact, int64_t n_exact,
              uint32_t* __restrict__ status, uint32_t* __restrict__ own_total) {
  __shared__ uint64_t part[1024];
  __shared__ uint64_t s_exact;
  const int t = threadIdx.x;
  if (exact) {
    uint64_t e = 0;
    for (int64_t i = t; i < n_exact; i += 1024) e += exact[i];
    part[t] = e;
    __syncthreads();
    for (int d = 512; d >= 1; d >>= 1) {
      if (t < d) part[t] += part[t + d];
      __syncthreads();
    }
    if (t == 0) s_exact = part[0];
    __syncthreads();
  }
  const int64_t per = (n_blocks + 1023) / 1024;
  const int64_t lo = (int64_t)t * per, hi = min(lo + per, n_blocks);
  uint64_t acc = 0;
  for (int64_t i = lo; i < hi; ++i) acc += sums[i];
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
    const uint64_t s = sums[i];
    sums[i] = (uint32_t)min(run, (uint64_t)0xFFFFFFFFu);
    run += s;
  }
  if (t == 1023) {
    const uint64_t total = exact ? s_exact : part[1023];
    total_out[0] = (uint32_t)min(total, (uint64_t)0xFFFFFFFFu);
    if (clamped) clamped[0] = (uint32_t)min(total, (uint64_t)capacity);
    if (status && total > (uint64_t)capacity) atomicOr(status, GS_STATUS_CAPACITY);
    if (own_total) own_total[0] = (uint32_t)min(part[1023], (uint64_t)0xFFFFFFFFu);
  }
}

// The visible pairs of each 2048-block in index order, as (depth key, index) for
// the sort. Eight rounds of 256 consecutive items; within a round a wave ballot
// and the per-wave totals give every visible item its position, so reads and
// writes stay contiguous.
__global__ void __launch_bounds__(kBinBlock)
bin_compact(const int32_t* __restrict__ touched, const uint32_t* __restrict__ depth_key,
            int64_t total_items, const uint32_t* __restrict__ block_offsets, int64_t capacity,
            uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ uint32_t s_wave[kBinItems][kBinBlock / kWave];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int64_t base = (int64_t)blockIdx.x * kBinTile;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  bool vis[kBinItems];
  uint32_t key[kBinItems];
  // every load of the block is issued before the first ballot (the depth keys of all
  // items, visible or not: at a third visible, their lines are read anyway)
  int32_t tc[kBinItems];
#pragma unroll
  for (int r = 0; r < kBinItems; ++r) {
    const int64_t i = base + (int64_t)r * kBinBlock + threadIdx.x;
    tc[r] = i < total_items ? touched[i] : 0;
    key[r] = i < total_items ? depth_key[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kBinItems; ++r) {
    vis[r] = tc[r] > 0;
    const uint64_t m = __ballot(vis[r]);
    if (lane == 0) s_wave[r][wave] = (uint32_t)__popcll(m);
  }
  __syncthreads();
  uint32_t run = block_offsets[blockIdx.x];
#pragma unroll
  for (int r = 0; r < kBinItems; ++r) {
    uint32_t before = 0, round = 0;
#pragma unroll
    for (int w = 0; w < kBinBlock / kWave; ++w) {
      const uint32_t c = s_wave[r][w];
      before += (w < wave) ? c : 0u;
      round += c;
    }
    const uint64_t m = __ballot(vis[r]);
    const uint32_t pos = run + before + (uint32_t)__popcll(m & below);
    if (vis[r] && (int64_t)pos < capacity) {
      keys[pos] = key[r];
      vals[pos] = (uint32_t)(base + (int64_t)r * kBinBlock + threadIdx.x);
    }
    run += round;
  }
}

// LDS word of item i of a 2048-item block, padded by one word per 32 items so that
// lanes reading kBinItems consecutive items each fall in different banks
__device__ __forceinline__ int padded(int i) { return i + (i >> 5); }

// Start offset of every depth-sorted pair's instances: the block-local scan of the
// tile counts plus the block's offset. Every pair also records itself as the head of
// each expansion block whose first output (a multiple of kExpandOut below n_out)
// falls in its range, so that block needs no search for its first pair.
__global__ void __launch_bounds__(kBinBlock)
bin_pair_offsets(const uint32_t* __restrict__ pair_wh,
                 const uint32_t* __restrict__ n_sorted_dev, int64_t max_items,
                 const uint32_t* __restrict__ block_offsets, const uint32_t* __restrict__ n_out_dev,
                 int64_t capacity, uint32_t* __restrict__ offs, uint32_t* __restrict__ heads) {
  // the block's counts pass through LDS (one padded word per item) so that the global
  // reads and writes are coalesced while each thread scans kBinItems consecutive items
  __shared__ uint32_t s_t[kBinTile + kBinTile / 32];
  __shared__ uint32_t s4[kBinBlock / kWave];
  const int64_t n_sorted = min((int64_t)n_sorted_dev[0], max_items);
  const uint64_t n_out = (uint64_t)min((int64_t)n_out_dev[0], capacity);
  const int64_t blk = (int64_t)blockIdx.x * kBinTile;
  if (blk >= n_sorted) return;   // uniform over the block
#pragma unroll
  for (int r = 0; r < kBinItems; ++r) {
    const int q = r * kBinBlock + threadIdx.x;
    const uint32_t wh = blk + q < n_sorted ? pair_wh[blk + q] : 0u;
    s_t[padded(q)] = (wh & 0xFFFFu) * (wh >> 16);
  }
  __syncthreads();
  const int q0 = threadIdx.x * kBinItems;
  uint32_t cnt[kBinItems], local = 0;
#pragma unroll
  for (int j = 0; j < kBinItems; ++j) {
    cnt[j] = s_t[padded(q0 + j)];
    local += cnt[j];
  }
  uint32_t tot;
  uint64_t run = (uint64_t)block_offsets[blockIdx.x] + block_excl_scan(local, s4, &tot);
  // each thread now overwrites only the 16 words it read: no barrier needed before
#pragma unroll
  for (int j = 0; j < kBinItems; ++j) {
    s_t[padded(q0 + j)] = (uint32_t)run;
    if (blk + q0 + j < n_sorted) {
      const uint64_t end = min(run + cnt[j], n_out);
      for (uint64_t h = (run + kExpandOut - 1) / kExpandOut; h * kExpandOut < end; ++h)
        heads[h] = (uint32_t)(blk + q0 + j);
    }
    run += cnt[j];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kBinItems; ++r) {
    const int q = r * kBinBlock + threadIdx.x;
    if (blk + q < n_sorted) offs[blk + q] = s_t[padded(q)];
  }
}

// Expansion partitioned by output: block b writes instances [o0, o0 + kExpandOut),
// o0 = kExpandOut b. Its pairs run from heads[b] to heads[b + 1] (the pair holding
// the next block's first output), at most kExpandOut + 1 of them; they are staged in
// LDS (offset, value, first tile id, width and tiles per row, all read densely), and
// each output finds its pair by binary search over the staged offsets. Every block does the same amount of
// work whatever the tile counts (the nearest Gaussians cover the most tiles and sort
// first).
__global__ void __launch_bounds__(kBinBlock)
bin_expand(const uint32_t* __restrict__ sorted, const uint32_t* __restrict__ n_sorted_dev,
           int64_t max_items, int64_t n, TileViews tv, const uint32_t* __restrict__ offs,
           const uint32_t* __restrict__ pair_wh, const uint32_t* __restrict__ pair_base,
           const uint32_t* __restrict__ heads,
           const uint32_t* __restrict__ n_out_dev, int64_t capacity,
           uint32_t* __restrict__ tiles, uint32_t* __restrict__ vals) {
  constexpr int kStage = kExpandOut + 1;
  __shared__ uint32_t s_off[kStage];
  __shared__ uint32_t s_val[kStage];
  __shared__ uint32_t s_base[kStage];   // global id of the pair's first tile
  __shared__ uint32_t s_wx[kStage];     // rectangle width | tiles per row << 16
  const int64_t n_sorted = min((int64_t)n_sorted_dev[0], max_items);
  const int64_t n_out = min((int64_t)n_out_dev[0], capacity);
  const int64_t o0 = (int64_t)blockIdx.x * kExpandOut;
  if (o0 >= n_out || n_sorted <= 0) return;   // uniform over the block
  const int64_t o1 = min(o0 + kExpandOut, n_out);
  const int64_t p0 = min((int64_t)heads[blockIdx.x], n_sorted - 1);
  const int64_t p1 = o1 < n_out ? min((int64_t)heads[blockIdx.x + 1], n_sorted - 1) : n_sorted - 1;
  // outputs [o0, o1) touch at most kExpandOut consecutive pairs from p0 on
  const int n_pairs = (int)std::max<int64_t>(1, std::min<int64_t>(p1 - p0 + 1, kStage));
  for (int j = threadIdx.x; j < n_pairs; j += kBinBlock) {
    const uint32_t i = sorted[p0 + j];
    const uint32_t tx = (uint32_t)tv.tiles_x[view_of_pair(tv, i, n)];
    s_off[j] = offs[p0 + j];
    s_val[j] = i;
    s_base[j] = pair_base[p0 + j];
    s_wx[j] = (pair_wh[p0 + j] & 0xFFFFu) | (tx << 16);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kExpandOut / kBinBlock; ++r) {
    const int64_t o = o0 + r * kBinBlock + threadIdx.x;
    if (o < o1) {
      int lo = 0, hi = n_pairs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)s_off[mid] <= o) lo = mid; else hi = mid - 1;
      }
      const uint32_t k = (uint32_t)(o - (int64_t)s_off[lo]);
      const uint32_t wx = s_wx[lo], wdt = wx & 0xFFFFu;
      tiles[o] = s_base[lo] + (k / wdt) * (wx >> 16) + k % wdt;
      vals[o] = s_val[lo];
    }
  }
}

struct BinWs {
  uint32_t* misc;
  uint32_t* vis_sums;
  uint32_t* exp_sums;
  uint32_t* offs;            // instance offset of every pair in depth order
  uint32_t* pair_wh;         // tile rectangle width | height << 16 of every pair in depth order
  unsigned long long* tile_parts;   // instance count of each 2048-pair block (index order)
  void* radix;
  size_t radix_bytes;
  int64_t nb;
};

static size_t align_words(size_t w) { return (w + 63) & ~(size_t)63; }

static size_t bin_ws_layout(int64_t n_total, int db, BinWs* out, void* base) {
  const int64_t nb = (n_total + kBinTile - 1) / kBinTile;
  const size_t w_misc = kMiscWords;
  const size_t w_sums = align_words((size_t)nb + 1);
  const size_t offs_off = align_words(w_misc + 2 * w_sums);
  const size_t scounts_off = align_words(offs_off + (size_t)n_total);
  const size_t parts_off = align_words(scounts_off + (size_t)n_total);
  const size_t radix_off = align_words(parts_off + 2 * ((size_t)nb + 1));
  const size_t radix_bytes = radix_workspace_bytes(n_total, radix_passes(kDepthKeyBits, db));
  if (out) {
    uint32_t* p = static_cast<uint32_t*>(base);
    out->misc = p;
    out->vis_sums = p + w_misc;
    out->exp_sums = p + w_misc + w_sums;
    out->offs = p + offs_off;
    out->pair_wh = p + scounts_off;
    out->tile_parts = reinterpret_cast<unsigned long long*>(p + parts_off);
    out->radix = p + radix_off;
    out->radix_bytes = radix_bytes;
    out->nb = nb;
  }
  return radix_off * sizeof(uint32_t) + radix_bytes;
}

}  // namespace gs

using namespace gs;

extern "C" size_t gs_bin_workspace_bytes(int64_t n_total, const gs_config* cfg) {
  if (n_total < 0 || !cfg || check_config(cfg) != GS_OK) return 0;
  return bin_ws_layout(n_total, cfg->sort_digit_bits, nullptr, nullptr);
}

extern "C" int gs_bin(const gs_projected* proj, int64_t n, const gs_camera* cams, int32_t n_views,
                      const gs_config* cfg, const gs_instances* inst, void* workspace,
                      size_t workspace_bytes, gs_stream_t stream) {
  if (!proj || !cams || !cfg || !inst || n < 0) return GS_ERR_ARG;
  int rc = check_config(cfg);
  if (rc != GS_OK) return rc;
  TileViews tv;
  rc = fill_tile_views(cams, n_views, cfg->tile_size, &tv);
  if (rc != GS_OK) return rc;
  if (!inst->keys || !inst->vals || !inst->keys_alt || !inst->vals_alt || !inst->count ||
      !inst->status || inst->capacity < 0)
    return GS_ERR_ARG;
  if (inst->capacity > GS_MAX_INSTANCES) return GS_ERR_UNSUPPORTED;
  const int64_t total = n * (int64_t)n_views;
  if (total >= ((int64_t)1 << 32)) return GS_ERR_UNSUPPORTED;
  if (total > 0 && (!proj->tiles_touched || !proj->depth_key || !proj->record)) return GS_ERR_ARG;
  if (!workspace || workspace_bytes < gs_bin_workspace_bytes(total, cfg)) return GS_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  BinWs w;
  bin_ws_layout(total, cfg->sort_digit_bits, &w, workspace);
  const int64_t cap = inst->capacity;
  const int db = cfg->sort_digit_bits;
  const InstanceBufs b =
      instance_bufs(inst, radix_passes(tile_key_bits(tv.tile_offset[n_views]), db));
  // 1. visible pairs in index order (and the exact instance count); the scans write
  // every misc word that is read later, so it needs no clearing
  if (w.nb > 0)
    bin_visible_sums<<<dim3((unsigned)w.nb), kBinBlock, 0, s>>>(proj->tiles_touched, total,
                                                                w.vis_sums, w.tile_parts);
  bin_scan_sums<<<1, 1024, 0, s>>>(w.vis_sums, w.nb, cap, w.misc, w.misc + 1, nullptr, 0,
                                   nullptr, nullptr);
  if (w.nb > 0)
    bin_compact<<<dim3((unsigned)w.nb), kBinBlock, 0, s>>>(
        proj->tiles_touched, proj->depth_key, total, w.vis_sums, cap, b.depth.keys[0],
        b.depth.vals[0]);
  // 2. by depth (stable: ties keep index order)
  const int64_t max_vis = std::min(total, cap);
  rc = radix_sort(b.depth, 0, w.misc + 1, max_vis, kDepthKeyBits, db, w.radix, w.radix_bytes, s);
  if (rc != GS_OK) return rc;
  const uint32_t* sorted = b.depth.vals[radix_passes(kDepthKeyBits, db) & 1];
  // 3. tile rectangles in depth order -> instance offsets, count and capacity check.
  // The first tile ids and the block heads go to regions of the instance buffers that
  // are dead once the depth sort is done: its first key array (max_vis <= capacity
  // words) and its other value array (one word per kExpandOut outputs, at most
  // capacity words). The expansion writes the tile sort's set 0 (keys_alt, vals or
  // vals_alt), which overlaps neither.
  const int depth_passes = radix_passes(kDepthKeyBits, db);
  uint32_t* pair_base = b.depth.keys[0];
  uint32_t* heads = b.depth.vals[(depth_passes + 1) & 1];
  const int64_t nbe = (max_vis + kBinTile - 1) / kBinTile;
  if (nbe > 0)
    bin_pair_tiles<<<dim3((unsigned)nbe), kBinBlock, 0, s>>>(
        sorted, w.misc + 1, max_vis, proj->record, n, tv, w.exp_sums, w.pair_wh, pair_base);
  bin_scan_sums<<<1, 1024, 0, s>>>(w.exp_sums, nbe, cap, inst->count, nullptr, w.tile_parts,
                                   w.nb, inst->status, w.misc + 4);
  // 4. the instances, front to back: pair offsets and block heads, then an
  // output-partitioned expansion
  if (nbe > 0)
    bin_pair_offsets<<<dim3((unsigned)nbe), kBinBlock, 0, s>>>(
        w.pair_wh, w.misc + 1, max_vis, w.exp_sums, w.misc + 4, cap, w.offs, heads);
  const int64_t nbo = (cap + kExpandOut - 1) / kExpandOut;
  if (nbe > 0 && nbo > 0)
    bin_expand<<<dim3((unsigned)nbo), kBinBlock, 0, s>>>(
        sorted, w.misc + 1, max_vis, n, tv, w.offs, w.pair_wh, pair_base, heads, w.misc + 4,
        cap, b.tiles.keys[0], b.tiles.vals[0]);
  return launch_status();
}
