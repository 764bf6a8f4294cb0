// Sorting (Alg. 2 SortByKeys + IdentifyTileRanges; App. C "Sorting"). The paper
// sorts all instances once by a 64-bit (tile | depth) key. Here the same order is
// produced by two stable radix sorts of 32-bit keys: gs_bin sorts the visible
// (view, Gaussian) pairs by depth and expands them into instances in that order;
// gs_sort then sorts the instances by tile id alone. A stable sort by tile of a
// sequence already in (depth, index) order is the (tile, depth, index) order, and
// the instance pass moves 8 bytes per instance over the tile bits only instead of
// 12 bytes over tile + depth bits.
//
// Each radix sort has the onesweep structure (Adinets and Merrill, 2022): one
// histogram pass over the keys computes the digit counts of every pass at once; then
// each digit pass is a single launch in which a 256-thread block takes 4096 keys in
// ticket order, ranks them in LDS (wave ballots find the lanes sharing a digit),
// publishes its digit counts, resolves its global digit offsets by decoupled
// look-back over the blocks before it, and scatters the pairs, staged through LDS so
// the writes of a digit run are contiguous.
#include <algorithm>
#include <mutex>

#include "gs_internal.h"

namespace gs {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;   // 4096 keys per block
constexpr int kLookback = 8;                        // predecessors examined per step
constexpr int kMaxPasses = 8;
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagInc = 2u << 30;
constexpr uint32_t kValueMask = (1u << 30) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;
// The histogram pass adds its block counts into one of kHistCopies copies, chosen by
// block index: consecutive blocks are dispatched to different XCDs (eight on MI355X),
// so each copy collects the atomics of one XCD instead of all blocks contending for
// the same words; the scan kernel sums the copies.
constexpr int kHistCopies = 8;
constexpr int kHistWords = kMaxPasses * 256;

struct RadixWs {
  uint32_t* hist;      // [kHistCopies][kMaxPasses][256] digit counts; copy 0 then holds
                       // the exclusive scan of their sum
  uint32_t* ticket;    // [kMaxPasses]
  uint32_t* lookback;  // [passes][n_blocks][256]
  int64_t n_blocks;
};

static int64_t radix_blocks(int64_t max_items) {
  return std::max<int64_t>(1, (max_items + kSortTile - 1) / kSortTile);
}

size_t radix_workspace_bytes(int64_t max_items, int passes) {
  return (size_t)(kHistCopies * kHistWords + 64 + (int64_t)passes * radix_blocks(max_items) * 256) *
         sizeof(uint32_t);
}

static RadixWs carve(void* ws, int64_t max_items) {
  RadixWs w;
  uint32_t* p = static_cast<uint32_t*>(ws);
  w.n_blocks = radix_blocks(max_items);
  w.hist = p;
  w.ticket = p + kHistCopies * kHistWords;
  w.lookback = w.ticket + 64;
  return w;
}

__device__ __forceinline__ int64_t item_count(const uint32_t* count, int64_t max_items) {
  return min((int64_t)count[0], max_items);
}

__global__ void __launch_bounds__(256)
radix_init(RadixWs w, int passes, const uint32_t* __restrict__ count, int64_t max_items) {
  const int64_t M = item_count(count, max_items);
  const int64_t nb = (M + kSortTile - 1) / kSortTile;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < (int64_t)kHistCopies * kHistWords; i += stride) w.hist[i] = 0;
  for (int64_t i = t0; i < 64; i += stride) w.ticket[i] = 0;
  for (int p = 0; p < passes; ++p) {
    uint32_t* lb = w.lookback + (size_t)p * w.n_blocks * 256;
    for (int64_t i = t0; i < nb * 256; i += stride) lb[i] = 0;
  }
}

// Digit counts of every pass in one read of the keys: blocks take 4096-key tiles in
// turn (sixteen loads in flight per thread), count in LDS, then add their counts to
// their XCD's copy of the histogram.
__global__ void __launch_bounds__(256)
radix_histogram(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ count,
                int64_t max_items, int passes, int db, uint32_t* __restrict__ hist) {
  __shared__ uint32_t sh[kMaxPasses][256];
  for (int i = threadIdx.x; i < kMaxPasses * 256; i += 256) (&sh[0][0])[i] = 0;
  __syncthreads();
  const int64_t M = item_count(count, max_items);
  const uint32_t mask = (1u << db) - 1;
  for (int64_t base = (int64_t)blockIdx.x * kSortTile; base < M;
       base += (int64_t)gridDim.x * kSortTile) {
    uint32_t k[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const int64_t i = base + (int64_t)r * 256 + threadIdx.x;
      k[r] = i < M ? keys[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      if (base + (int64_t)r * 256 + threadIdx.x >= M) break;
      for (int p = 0; p < passes; ++p) atomicAdd(&sh[p][(k[r] >> (p * db)) & mask], 1u);
    }
  }
  __syncthreads();
  uint32_t* mine = hist + (size_t)(blockIdx.x % kHistCopies) * kHistWords;
  for (int i = threadIdx.x; i < passes * 256; i += 256) {
    const uint32_t c = (&sh[0][0])[i];
    if (c) atomicAdd(&mine[i], c);
  }
}

__global__ void __launch_bounds__(256)
radix_scan_hist(uint32_t* __restrict__ hist, int passes) {
  __shared__ uint32_t s[256];
  const int t = threadIdx.x;
  for (int p = 0; p < passes; ++p) {
    uint32_t x = 0;
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c) x += hist[c * kHistWords + p * 256 + t];
    s[t] = x;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
      const uint32_t y = (t >= d) ? s[t - d] : 0u;
      __syncthreads();
      s[t] += y;
      __syncthreads();
    }
    hist[p * 256 + t] = s[t] - x;
    __syncthreads();
  }
}

template <int DB>
__global__ void __launch_bounds__(kSortBlock)
radix_pass(const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
           uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
           const uint32_t* __restrict__ count, int64_t max_items, int shift,
           const uint32_t* __restrict__ digit_start, uint32_t* __restrict__ lookback,
           uint32_t* __restrict__ ticket, uint32_t* __restrict__ status) {
  constexpr int RADIX = 1 << DB;
  constexpr int WAVES = kSortBlock / kWave;
  constexpr int WAVE_ITEMS = kSortTile / WAVES;
  __shared__ uint32_t s_keys[kSortTile];
  __shared__ uint32_t s_vals[kSortTile];
  __shared__ uint32_t s_whist[WAVES][RADIX];
  __shared__ uint32_t s_local_base[RADIX];
  __shared__ uint32_t s_global_base[RADIX];
  __shared__ uint32_t s_scan[WAVES];
  __shared__ uint32_t s_tile;

  const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  if (tid == 0) s_tile = atomicAdd(ticket, 1u);
  for (int i = tid; i < WAVES * RADIX; i += kSortBlock) (&s_whist[0][0])[i] = 0;
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t M = item_count(count, max_items);
  if (tile * kSortTile >= M) return;  // uniform over the block

  // load: wave w owns the contiguous run [tile*4096 + w*1024, +1024), round r lane l
  const int64_t wbase = tile * kSortTile + (int64_t)wave * WAVE_ITEMS;
  uint32_t k[kSortItems], val[kSortItems], dig[kSortItems], rank[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = wbase + (int64_t)r * kWave + lane;
    const bool valid = i < M;
    k[r] = valid ? keys_in[i] : 0u;
    val[r] = valid ? vals_in[i] : 0u;
    dig[r] = valid ? ((k[r] >> shift) & (RADIX - 1)) : (uint32_t)RADIX;
  }
  // rank in input order (round-major, then lane): stable
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
      base = s_whist[wave][dig[r]];
      rank[r] = base + (uint32_t)__popcll(peers & lt_mask);
    }
    __builtin_amdgcn_wave_barrier();
    // the highest lane of each peer group writes the new count
    if (valid && (peers >> lane) == 1ull) s_whist[wave][dig[r]] = base + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();

  // per digit: exclusive offsets of the waves, block total
  uint32_t total = 0;
  if (tid < RADIX) {
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      const uint32_t c = s_whist[w][tid];
      s_whist[w][tid] = total;
      total += c;
    }
  }
  // decoupled look-back: thread d resolves digit d
  if (tid < RADIX) {
    uint32_t* mine = lookback + tile * RADIX + tid;
    uint32_t excl = 0;
    if (tile == 0) {
      __hip_atomic_store(mine, kFlagInc | total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(mine, kFlagAgg | total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // windowed look-back: load kLookback predecessors at once (independent loads, one
      // latency), add them nearest first up to the first inclusive prefix; on a
      // not-yet-published entry, keep what was added and re-poll from that entry
      int64_t t = tile - 1;
      uint32_t spins = 0;
      bool found = false;
      while (!found) {
        uint32_t wv[kLookback];
#pragma unroll
        for (int j = 0; j < kLookback; ++j)
          wv[j] = (t - j >= 0) ? __hip_atomic_load(lookback + (t - j) * RADIX + tid, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT)
                               : kFlagInc;  // before block 0: an empty inclusive prefix
        int j = 0;
        for (; j < kLookback; ++j) {
          const uint32_t flag = wv[j] & ~kValueMask;
          if (flag == 0) break;
          excl += wv[j] & kValueMask;
          if (flag == kFlagInc) {
            found = true;
            break;
          }
        }
        if (found) break;
        t -= j;
        if (j < kLookback) {  // entry t not published yet
          if (++spins > kSpinLimit) {  // never expected; bounded so the grid always drains
            atomicOr(status, GS_STATUS_SORT);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __hip_atomic_store(mine, kFlagInc | ((excl + total) & kValueMask), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    s_global_base[tid] = digit_start[tid] + excl;
  }
  // block-local exclusive scan of the digit totals: wave prefix sums, then the waves
  uint32_t incl = (tid < RADIX) ? total : 0u;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += y;
  }
  if (lane == kWave - 1) s_scan[wave] = incl;
  __syncthreads();
  uint32_t wbase_sum = 0;
#pragma unroll
  for (int w2 = 0; w2 < WAVES; ++w2) wbase_sum += (w2 < wave) ? s_scan[w2] : 0u;
  if (tid < RADIX) s_local_base[tid] = wbase_sum + incl - total;
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
  const int n_valid = (int)min((int64_t)kSortTile, M - tile * kSortTile);
  for (int s = tid; s < n_valid; s += kSortBlock) {
    const uint32_t kk = s_keys[s];
    const uint32_t d = (kk >> shift) & (RADIX - 1);
    const uint32_t g = s_global_base[d] + ((uint32_t)s - s_local_base[d]);
    keys_out[g] = kk;
    vals_out[g] = s_vals[s];
  }
}

int radix_passes(int key_bits, int digit_bits) {
  return (key_bits + digit_bits - 1) / digit_bits;
}

int radix_sort(const RadixBufs& b, int start, const uint32_t* count, int64_t max_items,
               int key_bits, int db, void* ws, size_t ws_bytes, uint32_t* status,
               hipStream_t s) {
  const int passes = radix_passes(key_bits, db);
  if (passes > kMaxPasses) return GS_ERR_UNSUPPORTED;
  if (passes == 0 || max_items <= 0) return GS_OK;
  if (ws_bytes < radix_workspace_bytes(max_items, passes)) return GS_ERR_ARG;
  RadixWs w = carve(ws, max_items);
  radix_init<<<dim3((unsigned)std::min<int64_t>(w.n_blocks, 1024)), 256, 0, s>>>(
      w, passes, count, max_items);
  const int src0 = start & 1;
  const unsigned hb = (unsigned)std::min<int64_t>(w.n_blocks, 2048);
  radix_histogram<<<dim3(hb), 256, 0, s>>>(b.keys[src0], count, max_items, passes, db, w.hist);
  radix_scan_hist<<<1, 256, 0, s>>>(w.hist, passes);
  const dim3 grid((unsigned)w.n_blocks);
  for (int p = 0; p < passes; ++p) {
    const int src = (start + p) & 1, dst = src ^ 1;
    uint32_t* lb = w.lookback + (size_t)p * w.n_blocks * 256;
#define GS_LAUNCH_PASS(D)                                                                        \
  radix_pass<D><<<grid, kSortBlock, 0, s>>>(b.keys[src], b.vals[src], b.keys[dst], b.vals[dst],  \
                                            count, max_items, p * db, w.hist + p * 256, lb,      \
                                            w.ticket + p, status)
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
                      workspace_bytes, inst->status, s);
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
