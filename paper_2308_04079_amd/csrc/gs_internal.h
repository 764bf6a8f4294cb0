// Internal declarations shared by the HIP sources of libgs_mi355x (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"
#include "gs_host.h"

namespace gs {

constexpr int kWave = 64;

// Radix sort of (key, value) u32 pairs (gs_sort.hip): buffers of the two ping-pong sets.
struct RadixBufs {
  uint32_t* keys[2];
  uint32_t* vals[2];
};
// Where the two sorts of the instance pipeline keep their data inside gs_instances:
// the depth sort of visible pairs uses keys and keys_alt as u32 arrays, the tile sort
// the first half of each for the tile ids and vals / vals_alt for the values.
struct InstanceBufs {
  RadixBufs depth;
  RadixBufs tiles;             // set 0 is what the expansion writes
  uint32_t* sorted_tiles;      // tile ids after the tile sort
};
int radix_passes(int key_bits, int digit_bits);
size_t radix_workspace_bytes(int64_t max_items, int passes);
// Sorts min(*count, max_items) pairs on their low key_bits bits, starting in set
// `start`; the result is in set (start + passes) & 1. Enqueue only.
int radix_sort(const RadixBufs& b, int start, const uint32_t* count, int64_t max_items,
               int key_bits, int digit_bits, void* ws, size_t ws_bytes, hipStream_t s);
int tile_key_bits(int64_t n_tiles_total);
InstanceBufs instance_bufs(const gs_instances* inst, int tile_passes);
constexpr int kDepthKeyBits = 31;   // depth > 0: the sign bit of its float word is 0

inline int launch_status() {
  return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

// view index of a global tile id (tile_offset is ascending)
__device__ __forceinline__ int view_of_tile(const TileViews& tv, int tile) {
  int v = 0;
  for (int k = 1; k < tv.n_views; ++k) v += (tile >= tv.tile_offset[k]) ? 1 : 0;
  return v;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Sum over the 64 lanes of a wave with DPP row operations; the total lands in lane 63.
// Every lane must be active.
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
  // quad butterflies (xor 1, xor 2), then half-row and row mirrors: row sum in every lane
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false));
  // row_bcast:15 into rows 1 and 3, then row_bcast:31 into rows 2 and 3
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xA, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xC, 0xF, false));
  return v;
}

}  // namespace gs
