// Sorting (Alg. 2 SortByKeys + IdentifyTileRanges; App. C "Sorting"). The paper
// sorts all instances once by a 64-bit (tile | depth) key. Here the same order is
// produced by two stable radix sorts of 32-bit keys: gs_bin sorts the visible
// (view, Gaussian) pairs by depth and expands them into instances in that order;
// gs_sort then sorts the instances by tile id alone. A stable sort by tile of a
// sequence already in (depth, index) order is the (tile, depth, index) order, and
// the instance pass moves 8 bytes per instance over the tile bits only instead of
// 12 bytes over tile + depth bits.
//
// Each radix digit pass is reduce-then-scan, in three launches: a counting pass in
// which every 256-thread block counts the digits of its 3072 keys (wave ballots find
// the lanes sharing a digit), a scan with one workgroup per digit over the blocks'
// counts, and a scatter pass in which every block ranks its keys again, reorders them
// through LDS and writes each digit's run contiguously at its scanned offset. The keys
// are read twice per pass, but no block waits on another: a single-launch pass with a
// decoupled look-back (onesweep) chains every block to its predecessors through
// device-scope loads, which on this chip cross the eight XCDs' L2s.
#include <algorithm>
#include <mutex>

#include "gs_internal.h"

namespace gs {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 12;
constexpr int kSortTile = kSortBlock * kSortItems;   // 3072 keys per block
constexpr int kSortWaves = kSortBlock / kWave;
constexpr int kMaxPasses = 8;
constexpr int kMaxRadix = 256;
constexpr int kScanChunk = 16;                      // counts per scan load batch

// Workspace: counts[RADIX][n_blocks], digit-major: the count pass writes how many keys
// of block b have digit d, the scan replaces each with the block's exclusive offset
// inside its digit; totals[RADIX] holds each digit's total. One set serves every pass.
struct RadixWs {
  uint32_t* counts;
  uint32_t* totals;
  int64_t n_blocks;   // row length of counts: blocks of the largest item count
};

static int64_t radix_blocks(int64_t max_items) {
  return std::max<int64_t>(1, (max_items + kSortTile - 1) / kSortTile);
}

size_t radix_workspace_bytes(int64_t max_items, int passes) {
  (void)passes;   // the passes run one after the other on the same counts
  return (size_t)(kMaxRadix * radix_blocks(max_items) + kMaxRadix) * sizeof(uint32_t);
}

static RadixWs carve(void* ws, int64_t max_items) {
  RadixWs w;
  uint32_t* p = static_cast<uint32_t*>(ws);
  w.n_blocks = radix_blocks(max_items);
  w.counts = p;
  w.totals = p + (size_t)kMaxRadix * w.n_blocks;
  return w;
}

__device__ __forceinline__ int64_t item_count(const uint32_t* count, int64_t max_items) {
  return min((int64_t)count[0], max_items);
}

// Logical block (the run of keys [b * kSortTile, +kSortTile)) of workgroup blockIdx.x.
// Workgroups go to the eight XCDs in turn, so workgroup p runs on XCD p % 8; block b
// is given to workgroup (b % chunk) * 8 + b / chunk, with chunk = ceil(nb / 8) for the nb
// blocks that hold keys: each XCD takes a contiguous range of blocks, and the
// neighbouring blocks whose digit runs share cache lines in the scatter write them
// through the same L2, which merges the partial lines before they go to memory (bin
// 0.415 -> 0.38 ms, sort 0.185 -> 0.16 ms at 3M Gaussians x 4 views, against
// workgroup b taking block b). The grid is a multiple of 8 of at least nb workgroups;
// a workgroup without a block returns -1.
__device__ __forceinline__ int64_t logical_block(int64_t M) {
  const int64_t nb = (M + kSortTile - 1) / kSortTile;
  const int64_t chunk = (nb + 7) / 8;
  const int64_t x = blockIdx.x % 8, i = blockIdx.x / 8;
  const int64_t b = x * chunk + i;
  return (i < chunk && b < nb) ? b : -1;
}

// The block's keys: wave w owns the contiguous run [b*3072 + w*768, +768), round r
// lane l its item r*64 + l. Digits of missing items are RADIX (no digit).
template <int DB>
__device__ __forceinline__ void load_block_keys(const uint32_t* __restrict__ keys, int64_t b,
                                                int64_t M, int shift, uint32_t* k, uint32_t* dig) {
  constexpr int RADIX = 1 << DB;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int64_t wbase = b * kSortTile + (int64_t)wave * (kSortTile / kSortWaves);
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = wbase + (int64_t)r * kWave + lane;
    const bool valid = i < M;
    k[r] = valid ? keys[i] : 0u;
    dig[r] = valid ? ((k[r] >> shift) & (RADIX - 1)) : (uint32_t)RADIX;
  }
}

// Rank of every item among the wave's items of the same digit, in input order (round,
// then lane): lanes sharing a digit are found with one ballot per digit bit. whist
// (the wave's RADIX counters, zero on entry) ends holding the wave's digit counts.
template <int DB>
__device__ __forceinline__ void wave_rank(const uint32_t* dig, uint32_t* rank, uint32_t* whist) {
  constexpr int RADIX = 1 << DB;
  const int lane = threadIdx.x % kWave;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const bool valid = dig[r] < (uint32_t)RADIX;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < DB; ++b) {
      const bool bit = (dig[r] >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    uint32_t base = 0;
    if (valid) {
      base = whist[dig[r]];
      rank[r] = base + (uint32_t)__popcll(peers & lt_mask);
    }
    __builtin_amdgcn_wave_barrier();
    // the highest lane of each peer group writes the new count
    if (valid && (peers >> lane) == 1ull) whist[dig[r]] = base + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
}

// Exclusive scan of one value per thread over the block (256 threads); *total receives
// the sum. s holds kSortWaves words.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t x, uint32_t* s, uint32_t* total) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  uint32_t incl = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += y;
  }
  if (lane == kWave - 1) s[wave] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kSortWaves; ++w) {
    before += (w < wave) ? s[w] : 0u;
    all += s[w];
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

// Counting pass: block b's digit counts to counts[d][b]. Workgroups without a block
// write nothing (the scan and the scatter stop at the last block holding keys).
template <int DB>
__global__ void __launch_bounds__(kSortBlock)
radix_count(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ count,
            int64_t max_items, int shift, int64_t n_blocks, uint32_t* __restrict__ counts) {
  constexpr int RADIX = 1 << DB;
  __shared__ uint32_t s_whist[kSortWaves][RADIX];
  const int64_t M = item_count(count, max_items);
  const int64_t b = logical_block(M);
  if (b < 0) return;   // uniform over the block
  const int tid = threadIdx.x, wave = tid / kWave;
  for (int i = tid; i < kSortWaves * RADIX; i += kSortBlock) (&s_whist[0][0])[i] = 0;
  uint32_t k[kSortItems], dig[kSortItems];
  load_block_keys<DB>(keys, b, M, shift, k, dig);
  __syncthreads();
  // counts need no ranks: LDS adds into the wave's own counters. Lanes of one add that
  // share a digit serialise on its word, so the lanes holding lane 0's digit (the
  // common digit of a skewed pass, such as the top bits of the depth keys) are counted
  // with one ballot and one add, and only the others add one each.
  const int lane = tid % kWave;
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t d = dig[r];
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
    const uint64_t same = __ballot(d == d0);
    if (lane == 0 && d0 < (uint32_t)RADIX) atomicAdd(&s_whist[wave][d0], (uint32_t)__popcll(same));
    if (d != d0 && d < (uint32_t)RADIX) atomicAdd(&s_whist[wave][d], 1u);
  }
  __syncthreads();
  if (tid < RADIX) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) c += s_whist[w][tid];
    counts[(int64_t)tid * n_blocks + b] = c;
  }
}

// One workgroup per digit d: exclusive scan of counts[d][0..nb) in place (nb = blocks
// holding keys), the digit's total to totals[d]. Thread t takes a contiguous run of
// blocks and loads it kScanChunk counts at a time; the first chunk stays in registers.
__global__ void __launch_bounds__(kSortBlock)
radix_scan_counts(uint32_t* __restrict__ counts, const uint32_t* __restrict__ count,
                  int64_t max_items, int64_t n_blocks, uint32_t* __restrict__ totals) {
  __shared__ uint32_t s_scan[kSortWaves];
  const int64_t M = item_count(count, max_items);
  const int64_t nb = (M + kSortTile - 1) / kSortTile;
  uint32_t* col = counts + (int64_t)blockIdx.x * n_blocks;
  const int64_t per = (nb + kSortBlock - 1) / kSortBlock;
  const int64_t lo = min(nb, (int64_t)threadIdx.x * per), hi = min(nb, lo + per);
  uint32_t first[kScanChunk];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) {
    first[j] = (lo + j < hi) ? col[lo + j] : 0u;
    sum += first[j];
  }
  for (int64_t i0 = lo + kScanChunk; i0 < hi; i0 += kScanChunk) {
    uint32_t x[kScanChunk];
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) x[j] = (i0 + j < hi) ? col[i0 + j] : 0u;
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) sum += x[j];
  }
  uint32_t total;
  uint32_t run = block_excl_scan256(sum, s_scan, &total);
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) {
    if (lo + j < hi) col[lo + j] = run;
    run += first[j];
  }
  for (int64_t i0 = lo + kScanChunk; i0 < hi; i0 += kScanChunk) {
    uint32_t x[kScanChunk];
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) x[j] = (i0 + j < hi) ? col[i0 + j] : 0u;
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) {
      if (i0 + j < hi) col[i0 + j] = run;
      run += x[j];
    }
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

// Scatter pass: block b ranks its keys again as the counting pass did, places them in
// block-sorted order through LDS, and writes each digit's run contiguously at
// start[d] + offsets[d][b], start being the exclusive scan of the digit totals.
template <int DB>
__global__ void __launch_bounds__(kSortBlock)
radix_scatter(const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
              uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
              const uint32_t* __restrict__ count, int64_t max_items, int shift, int64_t n_blocks,
              const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ totals) {
  constexpr int RADIX = 1 << DB;
  __shared__ uint32_t s_keys[kSortTile];
  __shared__ uint32_t s_vals[kSortTile];
  __shared__ uint32_t s_whist[kSortWaves][RADIX];
  __shared__ uint32_t s_local_base[RADIX];
  __shared__ uint32_t s_global_base[RADIX];
  __shared__ uint32_t s_scan[kSortWaves];

  const int64_t M = item_count(count, max_items);
  const int64_t b = logical_block(M);
  if (b < 0) return;   // uniform over the block
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  // this block's offsets and the digit totals, in flight while the keys load
  const uint32_t my_off = (tid < RADIX) ? offsets[(int64_t)tid * n_blocks + b] : 0u;
  const uint32_t dtot = (tid < RADIX) ? totals[tid] : 0u;
  for (int i = tid; i < kSortWaves * RADIX; i += kSortBlock) (&s_whist[0][0])[i] = 0;
  uint32_t k[kSortItems], val[kSortItems], dig[kSortItems], rank[kSortItems];
  load_block_keys<DB>(keys_in, b, M, shift, k, dig);
  {
    const int64_t wbase = b * kSortTile + (int64_t)wave * (kSortTile / kSortWaves);
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const int64_t i = wbase + (int64_t)r * kWave + lane;
      val[r] = (i < M) ? vals_in[i] : 0u;
    }
  }
  __syncthreads();
  wave_rank<DB>(dig, rank, s_whist[wave]);
  __syncthreads();
  // per digit: exclusive offsets of the waves, block total
  uint32_t total = 0;
  if (tid < RADIX) {
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
      const uint32_t c = s_whist[w][tid];
      s_whist[w][tid] = total;
      total += c;
    }
  }
  uint32_t unused;
  const uint32_t start = block_excl_scan256(dtot, s_scan, &unused);
  const uint32_t local = block_excl_scan256(total, s_scan, &unused);
  if (tid < RADIX) {
    s_local_base[tid] = local;
    s_global_base[tid] = start + my_off;
  }
  __syncthreads();
  // reorder through LDS into block-sorted order
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    if (dig[r] < (uint32_t)RADIX) {
      const uint32_t pos = s_local_base[dig[r]] + s_whist[wave][dig[r]] + rank[r];
      s_keys[pos] = k[r];
      s_vals[pos] = val[r];
    }
  }
  __syncthreads();
  const int n_valid = (int)min((int64_t)kSortTile, M - b * kSortTile);
  for (int i = tid; i < n_valid; i += kSortBlock) {
    const uint32_t kk = s_keys[i];
    const uint32_t d = (kk >> shift) & (RADIX - 1);
    const uint32_t g = s_global_base[d] + ((uint32_t)i - s_local_base[d]);
    keys_out[g] = kk;
    vals_out[g] = s_vals[i];
  }
}

int radix_passes(int key_bits, int digit_bits) {
  return (key_bits + digit_bits - 1) / digit_bits;
}

int radix_sort(const RadixBufs& b, int start, const uint32_t* count, int64_t max_items,
               int key_bits, int db, void* ws, size_t ws_bytes, hipStream_t s) {
  const int passes = radix_passes(key_bits, db);
  if (passes > kMaxPasses) return GS_ERR_UNSUPPORTED;
  if (passes == 0 || max_items <= 0) return GS_OK;
  if (ws_bytes < radix_workspace_bytes(max_items, passes)) return GS_ERR_ARG;
  RadixWs w = carve(ws, max_items);
  const dim3 grid((unsigned)((w.n_blocks + 7) / 8 * 8));   // a multiple of 8: logical_block
  for (int p = 0; p < passes; ++p) {
    const int src = (start + p) & 1, dst = src ^ 1;
#define GS_LAUNCH_PASS(D)                                                                        \
  radix_count<D><<<grid, kSortBlock, 0, s>>>(b.keys[src], count, max_items, p * db, w.n_blocks,  \
                                             w.counts);                                          \
  radix_scan_counts<<<dim3(1u << D), kSortBlock, 0, s>>>(w.counts, count, max_items, w.n_blocks, \
                                                         w.totals);                              \
  radix_scatter<D><<<grid, kSortBlock, 0, s>>>(b.keys[src], b.vals[src], b.keys[dst],            \
                                               b.vals[dst], count, max_items, p * db,            \
                                               w.n_blocks, w.counts, w.totals)
    switch (db) {
      case 4: GS_LAUNCH_PASS(4); break;
      case 5: GS_LAUNCH_PASS(5); break;
      case 6: GS_LAUNCH_PASS(6); break;
      case 7: GS_LAUNCH_PASS(7); break;
      default: GS_LAUNCH_PASS(8); break;
    }
#undef GS_LAUNCH_PASS
  }
  return GS_OK;
}

// IdentifyTileRanges: [start, end) of every global tile by binary search of the
// sorted tile ids (equivalent to comparing neighbouring ids; no zero-fill needed).
__global__ void __launch_bounds__(256)
sort_ranges(const uint32_t* __restrict__ tiles, const uint32_t* __restrict__ count,
            int64_t capacity, int64_t n_tiles, uint32_t* __restrict__ ranges) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_tiles) return;
  const int64_t M = min((int64_t)count[0], capacity);
  auto lower = [&](uint32_t key) {
    int64_t lo = 0, hi = M;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (tiles[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  ranges[2 * t] = (uint32_t)lower((uint32_t)t);
  ranges[2 * t + 1] = (uint32_t)lower((uint32_t)(t + 1));
}

// Issue order for the render launches: tiles bucketed by floor(log2(list length)),
// longest bucket first (order inside a bucket is arbitrary; it changes no result).
__device__ __forceinline__ int length_bucket(uint32_t len) { return len ? 32 - __clz(len) : 0; }

// The order is built by blocks of 1024 tiles over the whole chip (a single block
// serialises the LDS atomics of the few, crowded length buckets on one CU): each block
// first writes its tiles' bucket counts as one row of a table in the workspace; then
// bucket b starts after every tile of the longer buckets, the blocks follow one
// another inside it, and LDS atomics hand out the positions inside a block.
constexpr int kOrderBlock = 256;
constexpr int kOrderItems = 4;
constexpr int kOrderTiles = kOrderBlock * kOrderItems;
constexpr int kBuckets = 33;

static int64_t order_blocks(int64_t n_tiles) { return (n_tiles + kOrderTiles - 1) / kOrderTiles; }

__device__ __forceinline__ int tile_bucket(const uint32_t* __restrict__ ranges, int64_t i) {
  const uint2 r = reinterpret_cast<const uint2*>(ranges)[i];
  return length_bucket(r.y - r.x);
}

__global__ void __launch_bounds__(kOrderBlock)
sort_order_counts(const uint32_t* __restrict__ ranges, int64_t n_tiles, uint32_t* __restrict__ counts) {
  __shared__ uint32_t c[kBuckets];
  const int t = threadIdx.x;
  if (t < kBuckets) c[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kOrderTiles;
#pragma unroll
  for (int j = 0; j < kOrderItems; ++j) {
    const int64_t i = base + j * kOrderBlock + t;
    if (i < n_tiles) atomicAdd(&c[tile_bucket(ranges, i)], 1u);
  }
  __syncthreads();
  if (t < kBuckets) counts[(int64_t)blockIdx.x * kBuckets + t] = c[t];
}

__global__ void __launch_bounds__(kOrderBlock)
sort_order_place(const uint32_t* __restrict__ ranges, int64_t n_tiles,
                 const uint32_t* __restrict__ counts, int n_blocks, uint32_t* __restrict__ order) {
  __shared__ uint32_t total[kBuckets], before[kBuckets], cursor[kBuckets];
  const int t = threadIdx.x;
  if (t < kBuckets) total[t] = before[t] = 0;
  __syncthreads();
  // column sums of the table: over all blocks, and over the blocks before this one
  const int n_entries = n_blocks * kBuckets;   // < 2^27: n_tiles < 2^31
  const int mine = (int)blockIdx.x * kBuckets;
  for (int e = t; e < n_entries; e += kOrderBlock) {
    const uint32_t v = counts[e];
    if (v) {
      const int b = e % kBuckets;
      atomicAdd(&total[b], v);
      if (e < mine) atomicAdd(&before[b], v);
    }
  }
  __syncthreads();
  if (t == 0) {
    uint32_t run = 0;
    for (int b = kBuckets - 1; b >= 0; --b) {
      cursor[b] = run + before[b];
      run += total[b];
    }
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kOrderTiles;
#pragma unroll
  for (int j = 0; j < kOrderItems; ++j) {
    const int64_t i = base + j * kOrderBlock + t;
    if (i < n_tiles) order[atomicAdd(&cursor[tile_bucket(ranges, i)], 1u)] = (uint32_t)i;
  }
}

int tile_key_bits(int64_t n_tiles_total) {
  int tb = 0;
  while (tb < 40 && ((int64_t)1 << tb) < n_tiles_total) ++tb;
  return tb;
}

InstanceBufs instance_bufs(const gs_instances* inst, int tile_passes) {
  // keys / keys_alt hold capacity 64-bit words each; each is used as two u32 arrays
  InstanceBufs b;
  uint32_t* k0 = reinterpret_cast<uint32_t*>(inst->keys);
  uint32_t* k1 = reinterpret_cast<uint32_t*>(inst->keys_alt);
  const int64_t cap = inst->capacity;
  b.depth = {{k0, k1}, {k0 + cap, k1 + cap}};
  // the expansion writes (k1, vals or vals_alt) so that the tile passes end in vals
  const bool odd = tile_passes & 1;
  b.tiles = {{k1, k0}, {odd ? inst->vals_alt : inst->vals, odd ? inst->vals : inst->vals_alt}};
  b.sorted_tiles = odd ? k0 : k1;
  return b;
}

// The tile-order count table follows the radix sort's workspace.
static size_t order_table_offset(int64_t capacity, int passes) {
  return (radix_workspace_bytes(capacity, passes) + 255) & ~(size_t)255;
}

}  // namespace gs

using namespace gs;

extern "C" int32_t gs_sort_key_bits(int64_t n_tiles_total) { return tile_key_bits(n_tiles_total); }

extern "C" size_t gs_sort_workspace_bytes(int64_t capacity, int64_t n_tiles_total,
                                          const gs_config* cfg) {
  if (capacity < 0 || !cfg || check_config(cfg) != GS_OK) return 0;
  const int passes = radix_passes(tile_key_bits(n_tiles_total), cfg->sort_digit_bits);
  return order_table_offset(capacity, passes) +
         (size_t)std::max<int64_t>(0, order_blocks(n_tiles_total)) * kBuckets * sizeof(uint32_t);
}

extern "C" const uint32_t* gs_sorted_tile_ids(const gs_instances* inst, int64_t n_tiles_total,
                                              const gs_config* cfg) {
  if (!inst || !cfg || check_config(cfg) != GS_OK || !inst->keys || !inst->keys_alt) return nullptr;
  return instance_bufs(inst, radix_passes(tile_key_bits(n_tiles_total), cfg->sort_digit_bits))
      .sorted_tiles;
}

// Enqueue the sort into the given workspace (the caller's, or the static scratch).
static int sort_impl(const gs_instances* inst, int64_t n_tiles_total, const gs_config* cfg,
                     uint32_t* tile_ranges, uint32_t* tile_order, void* workspace,
                     size_t workspace_bytes, hipStream_t s) {
  const int bits = tile_key_bits(n_tiles_total);
  const int passes = radix_passes(bits, cfg->sort_digit_bits);
  if (passes > kMaxPasses) return GS_ERR_UNSUPPORTED;
  const InstanceBufs b = instance_bufs(inst, passes);
  const int64_t cap = inst->capacity;
  int rc = radix_sort(b.tiles, 0, inst->count, cap, bits, cfg->sort_digit_bits, workspace,
                      workspace_bytes, s);
  if (rc != GS_OK) return rc;
  sort_ranges<<<dim3((unsigned)((n_tiles_total + 255) / 256)), 256, 0, s>>>(
      b.sorted_tiles, inst->count, cap, n_tiles_total, tile_ranges);
  if (tile_order) {
    const int64_t nb = order_blocks(n_tiles_total);
    uint32_t* table = reinterpret_cast<uint32_t*>(static_cast<char*>(workspace) +
                                                  order_table_offset(cap, passes));
    sort_order_counts<<<dim3((unsigned)nb), kOrderBlock, 0, s>>>(tile_ranges, n_tiles_total, table);
    sort_order_place<<<dim3((unsigned)nb), kOrderBlock, 0, s>>>(tile_ranges, n_tiles_total, table,
                                                               (int)nb, tile_order);
  }
  return launch_status();
}

static int check_sort_args(const gs_instances* inst, int64_t n_tiles_total, const gs_config* cfg,
                           const uint32_t* tile_ranges) {
  if (!inst || !cfg || !tile_ranges || n_tiles_total < 1) return GS_ERR_ARG;
  const int rc = check_config(cfg);
  if (rc != GS_OK) return rc;
  if (!inst->keys || !inst->vals || !inst->keys_alt || !inst->vals_alt || !inst->count ||
      !inst->status || inst->capacity < 0)
    return GS_ERR_ARG;
  if (inst->capacity > GS_MAX_INSTANCES) return GS_ERR_UNSUPPORTED;
  if (n_tiles_total >= ((int64_t)1 << 31)) return GS_ERR_UNSUPPORTED;
  return GS_OK;
}

extern "C" int gs_sort(const gs_instances* inst, int64_t n_tiles_total, const gs_config* cfg,
                       uint32_t* tile_ranges, uint32_t* tile_order, void* workspace,
                       size_t workspace_bytes, gs_stream_t stream) {
  int rc = check_sort_args(inst, n_tiles_total, cfg, tile_ranges);
  if (rc != GS_OK) return rc;
  if (!workspace) return GS_ERR_ARG;
  if (workspace_bytes < gs_sort_workspace_bytes(inst->capacity, n_tiles_total, cfg)) return GS_ERR_ARG;
  return sort_impl(inst, n_tiles_total, cfg, tile_ranges, tile_order, workspace, workspace_bytes,
                   reinterpret_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------
// gs_sort_noalloc: the same sort with the library's static scratch as workspace
// ---------------------------------------------------------------------------

// The static scratch: each GPU the library runs on holds its own copy. In host code
// this name is only a handle for hipGetSymbolAddress, never a device address.
static __device__ __align__(256) unsigned char scratch[GS_SORT_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

// Device address of the current device's copy of the scratch, looked up on the first
// call on that device.
static int scratch_for_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GS_ERR_HIP;
  if (dev < 0 || dev >= kMaxScratchDevices) return GS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GS_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GS_OK;
}

extern "C" int gs_sort_noalloc(const gs_instances* inst, int64_t n_tiles_total,
                               const gs_config* cfg, uint32_t* tile_ranges, uint32_t* tile_order,
                               gs_stream_t stream) {
  int rc = check_sort_args(inst, n_tiles_total, cfg, tile_ranges);
  if (rc != GS_OK) return rc;
  if (gs_sort_workspace_bytes(inst->capacity, n_tiles_total, cfg) > GS_SORT_SCRATCH_BYTES)
    return GS_ERR_SCRATCH;
  void* ws = nullptr;
  rc = scratch_for_current_device(&ws);
  if (rc != GS_OK) return rc;
  return sort_impl(inst, n_tiles_total, cfg, tile_ranges, tile_order, ws, GS_SORT_SCRATCH_BYTES,
                   reinterpret_cast<hipStream_t>(stream));
}
