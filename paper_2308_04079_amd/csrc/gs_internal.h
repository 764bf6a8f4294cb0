// Internal declarations shared by the HIP sources of libgs_mi355x (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

namespace gs {

constexpr int kWave = 64;

// Per-view camera as the kernels see it (passed by value in the kernel arguments).
struct Cam {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t W, H;
};

// Camera table for the projection kernels.
struct ProjViews {
  int32_t n_views;
  int32_t tile;
  Cam cam[GS_MAX_VIEWS];
};

// Image and tile geometry of every view for the binning and render kernels.
struct TileViews {
  int32_t n_views;
  int32_t tile;
  int32_t W[GS_MAX_VIEWS];
  int32_t H[GS_MAX_VIEWS];
  int32_t tiles_x[GS_MAX_VIEWS];
  int32_t tile_offset[GS_MAX_VIEWS + 1];
  int64_t pix_offset[GS_MAX_VIEWS + 1];
  uint32_t n_records;  // V * N: instance values at or above it are ignored
};

struct Rules {
  float near_z, ext, ext2, alpha_min, alpha_max, T_min;
  float bg[3];
  int32_t isotropic;   // Sigma = s^2 I, s = exp(mean log-scale)
  int32_t grad_limit;  // > 0: only the N front-most blended Gaussians get gradients
};

static_assert(sizeof(ProjViews) < 3000, "kernel argument block too large");
static_assert(sizeof(TileViews) < 1000, "kernel argument block too large");

// host-side helpers (gs_api.cpp)
int fill_proj_views(const gs_camera* cams, int32_t n_views, int32_t tile, ProjViews* out);
int fill_tile_views(const gs_camera* cams, int32_t n_views, int32_t tile, TileViews* out);
int check_config(const gs_config* cfg);
Rules make_rules(const gs_config* cfg);
int sort_passes(int64_t n_tiles_total, int32_t digit_bits);

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
