// Host-side structures and argument checks of libgs_mi355x: plain C++ with no HIP
// dependency, so that the validation code also builds (and is checked under the
// address and undefined-behaviour sanitizers) as an ordinary CPU program.
#pragma once

#include <stdint.h>

#include "gs.h"

namespace gs {

// Per-view camera as the kernels see it (passed by value in the kernel arguments).
struct Cam {
  double C[3];   // camera centre -R^T t in world space (FP64, computed once per view)
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
  uint32_t n_inst;     // instance capacity: tile ranges are clipped to it
};

struct Rules {
  float near_z, ext, ext2, alpha_min, alpha_max, T_min;
  float bg[3];
  int32_t isotropic;   // Sigma = s^2 I, s = exp(mean log-scale)
  int32_t grad_limit;  // > 0: only the N front-most blended Gaussians get gradients
  float log_alpha_min; // ln(alpha_min): below opacity o, alpha < alpha_min once m > 2 ln(o / alpha_min)
};

static_assert(sizeof(ProjViews) < 3600, "kernel argument block too large");
static_assert(sizeof(TileViews) < 1000, "kernel argument block too large");

// host-side helpers (gs_host.cpp)
int fill_proj_views(const gs_camera* cams, int32_t n_views, int32_t tile, ProjViews* out);
int fill_tile_views(const gs_camera* cams, int32_t n_views, int32_t tile, TileViews* out);
int check_config(const gs_config* cfg);
Rules make_rules(const gs_config* cfg);

}  // namespace gs
