// gs_bin: exclusive scan of tiles_touched over all (view, Gaussian) pairs and one
// (key, value) instance per covered tile (Alg. 2 CreateTiles + DuplicateWithKeys;
// App. C "Sorting"). Three launches: per-block sums, a one-block scan of those
// sums (which also writes the instance count and the capacity check), and a
// block-local scan fused with the scatter of the instances, so the per-Gaussian
// offsets never go to memory.
#include "gs_internal.h"

namespace gs {

constexpr int kBinBlock = 256;
constexpr int kBinItems = 16;                       // per thread
constexpr int kBinTile = kBinBlock * kBinItems;     // 4096 per block

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

__global__ void __launch_bounds__(kBinBlock)
bin_block_sums(const int32_t* __restrict__ touched, int64_t total_items, uint32_t* __restrict__ sums) {
  __shared__ uint32_t s4[kBinBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kBinTile;
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kBinItems; ++j) {
    const int64_t i = base + (int64_t)j * kBinBlock + threadIdx.x;
    if (i < total_items) acc += (uint32_t)max(touched[i], 0);
  }
  uint32_t tot;
  block_excl_scan(acc, s4, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One block: exclusive scan of the block sums in place; writes the instance
// count and flags overflow of the capacity.
__global__ void __launch_bounds__(1024)
bin_scan_sums(uint32_t* __restrict__ sums, int64_t n_blocks, int64_t capacity,
              uint32_t* __restrict__ count, uint32_t* __restrict__ status) {
  __shared__ uint64_t part[1024];
  const int t = threadIdx.x;
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
    const uint64_t total = part[1023];
    count[0] = (uint32_t)min(total, (uint64_t)0xFFFFFFFFu);
    if (total > (uint64_t)capacity) atomicOr(status, GS_STATUS_CAPACITY);
  }
}

// Load-balanced expansion: the block's 4096 counts are scanned in LDS, then each
// thread produces output instances o = tid, tid + 256, ... of the block's range,
// finding its Gaussian by binary search over the LDS prefix sums. Writes are
// contiguous across the block.
__global__ void __launch_bounds__(kBinBlock)
bin_duplicate(const int32_t* __restrict__ touched, const uint32_t* __restrict__ depth_key,
              const float* __restrict__ record, int64_t n, int64_t total_items, TileViews tv,
              const uint32_t* __restrict__ block_offsets, int64_t capacity,
              uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ uint32_t s_off[kBinTile + 1];
  __shared__ uint32_t s4[kBinBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kBinTile;
#pragma unroll
  for (int j = 0; j < kBinItems; ++j) {
    const int64_t i = base + (int64_t)j * kBinBlock + threadIdx.x;
    s_off[j * kBinBlock + threadIdx.x] = (i < total_items) ? (uint32_t)max(touched[i], 0) : 0u;
  }
  __syncthreads();
  // thread t scans the 16 consecutive counts [16 t, 16 t + 16)
  uint32_t c[kBinItems], local = 0;
#pragma unroll
  for (int j = 0; j < kBinItems; ++j) {
    c[j] = s_off[threadIdx.x * kBinItems + j];
    local += c[j];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan(local, s4, &tot);
#pragma unroll
  for (int j = 0; j < kBinItems; ++j) {
    s_off[threadIdx.x * kBinItems + j] = run;
    run += c[j];
  }
  if (threadIdx.x == 0) s_off[kBinTile] = tot;
  __syncthreads();
  const uint32_t out0 = block_offsets[blockIdx.x];
  const int T = tv.tile;
  for (uint32_t o = threadIdx.x; o < tot; o += kBinBlock) {
    const uint64_t dst = (uint64_t)out0 + o;
    if (dst >= (uint64_t)capacity) break;   // o only grows
    // largest j with s_off[j] <= o (counts of zero give equal neighbours: take the last)
    int lo = 0, hi = kBinTile - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= o) lo = mid; else hi = mid - 1;
    }
    const int64_t i = base + lo;
    const uint32_t k = o - s_off[lo];
    const int v = (int)(i / n);
    const int2 lohi = *reinterpret_cast<const int2*>(record + i * GS_RECORD_FLOATS);
    const int ilo = lohi.x & 0xFFFF, jlo = (lohi.x >> 16) & 0xFFFF;
    const int ihi = lohi.y & 0xFFFF;
    const int tx0 = ilo / T, ty0 = jlo / T;
    const uint32_t wdt = (uint32_t)(ihi / T - tx0 + 1);
    const uint32_t ty = (uint32_t)ty0 + k / wdt, tx = (uint32_t)tx0 + k % wdt;
    keys[dst] = ((uint64_t)(uint32_t)(tv.tile_offset[v] + ty * tv.tiles_x[v] + tx) << 32) |
                (uint64_t)depth_key[i];
    vals[dst] = (uint32_t)i;
  }
}

}  // namespace gs

using namespace gs;

extern "C" size_t gs_bin_workspace_bytes(int64_t n_total) {
  if (n_total < 0) return 0;
  const int64_t nb = (n_total + kBinTile - 1) / kBinTile;
  return (size_t)(nb + 1) * sizeof(uint32_t);
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
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t nb = (total + kBinTile - 1) / kBinTile;
  if (total > 0 && (!proj->tiles_touched || !proj->depth_key || !proj->record)) return GS_ERR_ARG;
  if (workspace_bytes < gs_bin_workspace_bytes(total) || (nb > 0 && !workspace)) return GS_ERR_ARG;
  uint32_t* sums = static_cast<uint32_t*>(workspace);
  if (nb > 0)
    bin_block_sums<<<dim3((unsigned)nb), kBinBlock, 0, s>>>(proj->tiles_touched, total, sums);
  bin_scan_sums<<<1, 1024, 0, s>>>(sums, nb, inst->capacity, inst->count, inst->status);
  // the sort ping-pongs between the two buffers and must finish in keys/vals
  const bool odd = sort_passes(tv.tile_offset[n_views], cfg->sort_digit_bits) & 1;
  if (nb > 0)
    bin_duplicate<<<dim3((unsigned)nb), kBinBlock, 0, s>>>(
        proj->tiles_touched, proj->depth_key, proj->record, n, total, tv, sums, inst->capacity,
        odd ? inst->keys_alt : inst->keys, odd ? inst->vals_alt : inst->vals);
  return launch_status();
}
