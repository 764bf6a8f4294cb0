// CPU driver for the host-side argument checks of the C ABI (gs_host.cpp), built with
// the address and undefined-behaviour sanitizers by tests/test_host_sanitizers.py.
// Every call must return one of the documented codes without touching memory it was
// not given; accepted inputs must produce consistent tile and pixel layouts.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gs.h"
#include "gs_host.h"

static int failures = 0;
#define EXPECT(cond)                                                       \
  do {                                                                     \
    if (!(cond)) {                                                         \
      fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                          \
    }                                                                      \
  } while (0)

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64() {  // splitmix64
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static float pick_float() {
  static const float special[] = {0.0f, -0.0f, 1.0f, -1.0f, 0.5f, 1e-30f, 1e30f, 3.0f, 0.99f,
                                  1.0f / 255.0f, 1e-4f, 0.2f, INFINITY, -INFINITY, NAN};
  const uint64_t r = next_u64();
  if (r & 1) return special[(r >> 1) % (sizeof(special) / sizeof(special[0]))];
  return (float)((double)(r >> 11) / (double)(1ull << 53) * 20.0 - 10.0);
}
static int32_t pick_int(int32_t lo, int32_t hi) {
  return lo + (int32_t)(next_u64() % (uint64_t)(hi - lo + 1));
}

static gs_camera camera(int w, int h) {
  gs_camera c;
  memset(&c, 0, sizeof(c));
  c.R[0] = c.R[4] = c.R[8] = 1.0f;
  c.fx = c.fy = 100.0f;
  c.cx = 0.5f * w;
  c.cy = 0.5f * h;
  c.width = w;
  c.height = h;
  return c;
}

static void check_layout(const gs_camera* cams, int n, int tile, const gs::TileViews& tv) {
  int64_t t = 0, p = 0;
  for (int v = 0; v < n; ++v) {
    EXPECT(tv.tile_offset[v] == t);
    EXPECT(tv.pix_offset[v] == p);
    EXPECT(tv.tiles_x[v] == (cams[v].width + tile - 1) / tile);
    t += (int64_t)tv.tiles_x[v] * ((cams[v].height + tile - 1) / tile);
    p += (int64_t)cams[v].width * cams[v].height;
  }
  EXPECT(tv.tile_offset[n] == t && tv.pix_offset[n] == p);
}

int main() {
  // the default configuration is valid and is the method's
  gs_config cfg;
  gs_default_config(&cfg);
  gs_default_config(nullptr);
  EXPECT(gs::check_config(&cfg) == GS_OK);
  EXPECT(gs::check_config(nullptr) == GS_ERR_ARG);
  gs::Rules r = gs::make_rules(&cfg);
  EXPECT(r.ext2 == 9.0f && r.alpha_max == cfg.alpha_max && r.log_alpha_min < 0.0f);

  // every field perturbed at random: a valid code, and GS_OK only for sane values
  for (int it = 0; it < 20000; ++it) {
    gs_config c = cfg;
    switch (next_u64() % 13) {
      case 0: c.sh_degree = pick_int(-3, 6); break;
      case 1: c.tile_size = pick_int(-4, 40); break;
      case 2: c.near_z = pick_float(); break;
      case 3: c.sigma_extent = pick_float(); break;
      case 4: c.alpha_min = pick_float(); break;
      case 5: c.alpha_max = pick_float(); break;
      case 6: c.T_min = pick_float(); break;
      case 7: c.bg[next_u64() % 3] = pick_float(); break;
      case 8: c.sort_digit_bits = pick_int(-2, 14); break;
      case 9: c.lds_batch = pick_int(-64, 300); break;
      case 10: c.isotropic = pick_int(-2, 3); break;
      case 11: c.grad_limit = pick_int(-5, 5); break;
      default: memcpy(&c, &cfg, sizeof(c)); break;
    }
    const int rc = gs::check_config(&c);
    EXPECT(rc == GS_OK || rc == GS_ERR_ARG);
    if (rc == GS_OK) {
      EXPECT(c.sh_degree >= 0 && c.sh_degree <= 3);
      EXPECT(c.tile_size == 8 || c.tile_size == 16 || c.tile_size == 32);
      EXPECT(c.alpha_min > 0.0f && c.alpha_min <= c.alpha_max && c.alpha_max < 1.0f);
      EXPECT(c.T_min > 0.0f && c.T_min < 1.0f && c.near_z > 0.0f && c.sigma_extent > 0.0f);
      for (int k = 0; k < 3; ++k) EXPECT(isfinite(c.bg[k]));
      gs::Rules rr = gs::make_rules(&c);
      EXPECT(isfinite(rr.log_alpha_min));
    }
  }

  // camera tables: sizes, counts, non-finite fields, NULL
  gs::TileViews tv;
  gs::ProjViews pv;
  EXPECT(gs::fill_tile_views(nullptr, 1, 16, &tv) == GS_ERR_ARG);
  EXPECT(gs::fill_proj_views(nullptr, 1, 16, &pv) == GS_ERR_ARG);
  gs_camera cams[GS_MAX_VIEWS + 2];
  for (int v = 0; v < GS_MAX_VIEWS + 2; ++v) cams[v] = camera(64 + v, 48 + 3 * v);
  EXPECT(gs::fill_tile_views(cams, 0, 16, &tv) == GS_ERR_ARG);
  EXPECT(gs::fill_tile_views(cams, GS_MAX_VIEWS + 1, 16, &tv) == GS_ERR_UNSUPPORTED);
  EXPECT(gs::fill_tile_views(cams, GS_MAX_VIEWS, 16, &tv) == GS_OK);
  check_layout(cams, GS_MAX_VIEWS, 16, tv);
  EXPECT(gs::fill_proj_views(cams, GS_MAX_VIEWS, 16, &pv) == GS_OK);
  for (int it = 0; it < 20000; ++it) {
    const int n = pick_int(-1, GS_MAX_VIEWS + 1);
    const int tile = (int[]){8, 16, 32}[next_u64() % 3];
    for (int v = 0; v < GS_MAX_VIEWS + 2; ++v) {
      cams[v] = camera(pick_int(1, 2000), pick_int(1, 2000));
      const uint64_t r2 = next_u64() % 8;
      if (r2 == 0) cams[v].width = pick_int(-5, 40000);
      if (r2 == 1) cams[v].height = pick_int(-5, 40000);
      if (r2 == 2) cams[v].fx = pick_float();
      if (r2 == 3) cams[v].R[next_u64() % 9] = pick_float();
      if (r2 == 4) cams[v].t[next_u64() % 3] = pick_float();
    }
    const int rc = gs::fill_tile_views(cams, n, tile, &tv);
    EXPECT(rc == GS_OK || rc == GS_ERR_ARG || rc == GS_ERR_UNSUPPORTED);
    if (rc == GS_OK) check_layout(cams, n, tile, tv);
    const int rc2 = gs::fill_proj_views(cams, n, tile, &pv);
    EXPECT(rc2 == rc || (rc == GS_ERR_UNSUPPORTED && rc2 == GS_OK));
    if (rc2 == GS_OK)
      for (int v = 0; v < n; ++v) EXPECT(isfinite(pv.cam[v].C[0]) && pv.cam[v].W == cams[v].width);
    int64_t off[GS_MAX_VIEWS + 2];
    const int64_t t = gs_tile_layout(cams, n, tile, (next_u64() & 1) ? off : nullptr);
    EXPECT(t == (rc == GS_OK ? (int64_t)tv.tile_offset[n] : (int64_t)rc));
  }
  EXPECT(gs_tile_layout(cams, 1, 12, nullptr) == GS_ERR_ARG);
  // the largest images: a 32767 x 32767 view has 4096^2 tiles of 8 pixels
  cams[0] = camera(GS_MAX_DIM, GS_MAX_DIM);
  EXPECT(gs::fill_tile_views(cams, 1, 8, &tv) == GS_OK);
  cams[0].width = GS_MAX_DIM + 1;
  EXPECT(gs::fill_tile_views(cams, 1, 8, &tv) == GS_ERR_UNSUPPORTED);

  for (int code = -10; code <= 10; ++code) EXPECT(gs_status_string(code) != nullptr);
  if (failures) {
    fprintf(stderr, "%d expectation(s) failed\n", failures);
    return 1;
  }
  printf("host checks ok\n");
  return 0;
}
