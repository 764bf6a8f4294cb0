// Host-side argument checking and the small helpers of the C ABI (no HIP calls:
// built with the host compiler, and also as a CPU program under the sanitizers).
#include <math.h>
#include <string.h>

#include "gs_host.h"

namespace gs {

int check_config(const gs_config* cfg) {
  if (!cfg) return GS_ERR_ARG;
  if (cfg->sh_degree < 0 || cfg->sh_degree > 3) return GS_ERR_ARG;
  if (cfg->tile_size != 8 && cfg->tile_size != 16 && cfg->tile_size != 32) return GS_ERR_ARG;
  if (!(cfg->near_z > 0.0f) || !(cfg->sigma_extent > 0.0f)) return GS_ERR_ARG;
  if (!(cfg->alpha_min > 0.0f) || !(cfg->alpha_max < 1.0f) || !(cfg->alpha_min <= cfg->alpha_max))
    return GS_ERR_ARG;
  if (!(cfg->T_min > 0.0f) || !(cfg->T_min < 1.0f)) return GS_ERR_ARG;
  if (cfg->sort_digit_bits < 4 || cfg->sort_digit_bits > 8) return GS_ERR_ARG;
  if (cfg->lds_batch != 0 && cfg->lds_batch != 32 && cfg->lds_batch != 64 && cfg->lds_batch != 128)
    return GS_ERR_ARG;
  if (cfg->isotropic != 0 && cfg->isotropic != 1) return GS_ERR_ARG;
  if (cfg->grad_limit < 0) return GS_ERR_ARG;
  for (int c = 0; c < 3; ++c)
    if (!isfinite(cfg->bg[c])) return GS_ERR_ARG;
  return GS_OK;
}

Rules make_rules(const gs_config* cfg) {
  Rules r;
  r.near_z = cfg->near_z;
  r.ext = cfg->sigma_extent;
  r.ext2 = cfg->sigma_extent * cfg->sigma_extent;
  r.alpha_min = cfg->alpha_min;
  r.alpha_max = cfg->alpha_max;
  r.T_min = cfg->T_min;
  r.bg[0] = cfg->bg[0];
  r.bg[1] = cfg->bg[1];
  r.bg[2] = cfg->bg[2];
  r.isotropic = cfg->isotropic;
  r.grad_limit = cfg->grad_limit;
  r.log_alpha_min = logf(cfg->alpha_min);
  return r;
}

static int check_cams(const gs_camera* cams, int32_t n_views) {
  if (!cams || n_views < 1) return GS_ERR_ARG;
  if (n_views > GS_MAX_VIEWS) return GS_ERR_UNSUPPORTED;
  for (int v = 0; v < n_views; ++v) {
    const gs_camera& c = cams[v];
    if (c.width < 1 || c.height < 1) return GS_ERR_ARG;
    if (c.width > GS_MAX_DIM || c.height > GS_MAX_DIM) return GS_ERR_UNSUPPORTED;
    if (!isfinite(c.fx) || !isfinite(c.fy) || !isfinite(c.cx) || !isfinite(c.cy)) return GS_ERR_ARG;
    for (int k = 0; k < 9; ++k)
      if (!isfinite(c.R[k])) return GS_ERR_ARG;
    for (int k = 0; k < 3; ++k)
      if (!isfinite(c.t[k])) return GS_ERR_ARG;
  }
  return GS_OK;
}

int fill_proj_views(const gs_camera* cams, int32_t n_views, int32_t tile, ProjViews* out) {
  int rc = check_cams(cams, n_views);
  if (rc != GS_OK) return rc;
  memset(out, 0, sizeof(*out));
  out->n_views = n_views;
  out->tile = tile;
  for (int v = 0; v < n_views; ++v) {
    memcpy(out->cam[v].R, cams[v].R, sizeof(float) * 9);
    memcpy(out->cam[v].t, cams[v].t, sizeof(float) * 3);
    out->cam[v].fx = cams[v].fx;
    out->cam[v].fy = cams[v].fy;
    out->cam[v].cx = cams[v].cx;
    out->cam[v].cy = cams[v].cy;
    out->cam[v].W = cams[v].width;
    out->cam[v].H = cams[v].height;
    for (int k = 0; k < 3; ++k)
      out->cam[v].C[k] = -((double)cams[v].R[0 * 3 + k] * cams[v].t[0] +
                           (double)cams[v].R[1 * 3 + k] * cams[v].t[1] +
                           (double)cams[v].R[2 * 3 + k] * cams[v].t[2]);
  }
  return GS_OK;
}

int fill_tile_views(const gs_camera* cams, int32_t n_views, int32_t tile, TileViews* out) {
  int rc = check_cams(cams, n_views);
  if (rc != GS_OK) return rc;
  memset(out, 0, sizeof(*out));
  out->n_views = n_views;
  out->tile = tile;
  int64_t toff = 0, poff = 0;
  for (int v = 0; v < n_views; ++v) {
    out->W[v] = cams[v].width;
    out->H[v] = cams[v].height;
    out->tiles_x[v] = (cams[v].width + tile - 1) / tile;
    out->tile_offset[v] = (int32_t)toff;
    out->pix_offset[v] = poff;
    toff += (int64_t)out->tiles_x[v] * ((cams[v].height + tile - 1) / tile);
    poff += (int64_t)cams[v].width * cams[v].height;
  }
  if (toff >= ((int64_t)1 << 31)) return GS_ERR_UNSUPPORTED;
  out->tile_offset[n_views] = (int32_t)toff;
  out->pix_offset[n_views] = poff;
  return GS_OK;
}


}  // namespace gs

using namespace gs;

extern "C" void gs_default_config(gs_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->sh_degree = 3;
  cfg->tile_size = 16;
  cfg->near_z = 0.2f;
  cfg->sigma_extent = 3.0f;
  cfg->alpha_min = 1.0f / 255.0f;
  cfg->alpha_max = 0.99f;
  cfg->T_min = 1e-4f;
  cfg->sort_digit_bits = 8;
  cfg->lds_batch = 64;
}

extern "C" int64_t gs_tile_layout(const gs_camera* cams, int32_t n_views, int32_t tile_size,
                                  int64_t* tile_offset) {
  if (tile_size != 8 && tile_size != 16 && tile_size != 32) return GS_ERR_ARG;
  TileViews tv;
  int rc = fill_tile_views(cams, n_views, tile_size, &tv);
  if (rc != GS_OK) return rc;
  if (tile_offset)
    for (int v = 0; v <= n_views; ++v) tile_offset[v] = tv.tile_offset[v];
  return tv.tile_offset[n_views];
}


extern "C" const char* gs_status_string(int code) {
  switch (code) {
    case GS_OK: return "ok";
    case GS_ERR_ARG: return "invalid argument";
    case GS_ERR_CAPACITY: return "instance count exceeds capacity";
    case GS_ERR_HIP: return "HIP launch failed";
    case GS_ERR_UNSUPPORTED: return "size beyond a documented limit";
    case GS_ERR_SORT: return "sort look-back did not complete";
    case GS_ERR_SCRATCH: return "needs more than the library's static scratch";
    default: return "unknown status";
  }
}
