/*
 * gs.h - C ABI of the MI355X (gfx950) tile rasterizer for 3D Gaussian splats.
 *
 * The method is the differentiable tile rasterizer of Kerbl et al., "3D Gaussian
 * Splatting for Real-Time Radiance Field Rendering" (SIGGRAPH 2023), Sec. 6 and
 * App. C and the rasterization procedure of Alg. 2: an image of given size from the
 * Gaussians' means, covariances (stored as scales and rotation quaternions, Sec. 4),
 * SH colours (Sec. 5) and opacities, seen from one camera; and its backward pass
 * (Sec. 6 and App. A).
 *
 * One forward pass is
 *     gs_project -> gs_bin -> gs_sort -> gs_render_fwd
 * and the matching backward pass is
 *     gs_render_bwd -> gs_project_bwd.
 * Every stage accepts V >= 1 views at once: Gaussians are projected into all
 * views, instances of all views are sorted together under a global tile id,
 * and the render kernels process the tiles of all views in one launch.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Memory: every pointer inside the structs below is a DEVICE pointer owned by
 *   the caller (e.g. a torch tensor). The structs themselves, the camera array
 *   and the config are HOST memory, read during the call and not retained. The
 *   library never allocates, frees or synchronises; scratch memory is passed in
 *   as a caller-owned workspace whose size the *_workspace_bytes queries give.
 * - Streams: every call only enqueues kernels on `stream` (0 = the null stream)
 *   and returns; the sequence is capturable into a HIP graph.
 * - Errors: the return value reports argument errors found on the host
 *   (GS_ERR_ARG, GS_ERR_UNSUPPORTED) and launch failures (GS_ERR_HIP). Errors that
 *   can only be known on the device (too many instances for the capacity) are OR-ed
 *   into the device status word
 *   gs_instances.status; read it after the stream completes (gs_read_status).
 *   On a device-side error the outputs are unspecified but every kernel stays
 *   inside the caller's buffers.
 * - Culled or degenerate Gaussians (non-finite input, zero quaternion, depth
 *   below near_z, non-positive-definite 2D covariance, empty pixel box) are not
 *   errors: they get tiles_touched = 0 and zero gradients.
 * - Parameter layout is structure-of-arrays (coalesced per plane):
 *     means [3][N], log_scales [3][N], quats [4][N] as (r, i, j, k),
 *     opacity_logits [N], sh [K][3][N] with K = (sh_degree + 1)^2.
 * - Camera: world-to-camera rotation R (row-major) and translation t, pinhole
 *   intrinsics in pixels, OpenCV axes (x right, y down, z forward); pixel (i, j)
 *   has its centre at (i + 0.5, j + 0.5).
 */
#ifndef GS_MI355X_H
#define GS_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* gs_stream_t; /* identical to hipStream_t */

#define GS_MAX_VIEWS 32        /* views per call */
#define GS_MAX_DIM 32767       /* largest image width or height */
#define GS_RECORD_FLOATS 12    /* floats per projected Gaussian record */
#define GS_GRAD2D_FLOATS 9     /* floats per screen-space gradient record */
#define GS_MAX_INSTANCES (((int64_t)1 << 30) - 1) /* largest instance capacity (instance
                                                     positions are int32 in last_idx) */

enum {
  GS_OK = 0,
  GS_ERR_ARG = -1,         /* null pointer, negative size, bad config value */
  GS_ERR_CAPACITY = -2,    /* device status: more instances than capacity */
  GS_ERR_HIP = -3,         /* a HIP launch failed */
  GS_ERR_UNSUPPORTED = -4, /* size beyond a documented limit */
  GS_ERR_SORT = -5,        /* device status GS_STATUS_SORT (reserved: the current sort
                              has no device-side failure and never raises it) */
  GS_ERR_SCRATCH = -6      /* the call needs more than the library's static scratch */
};

/* bits of the device status word */
#define GS_STATUS_CAPACITY 1u
#define GS_STATUS_SORT 2u

typedef struct gs_camera {
  float R[9];            /* world -> camera rotation, row-major (W in Sec. 4) */
  float t[3];            /* world -> camera translation */
  float fx, fy, cx, cy;  /* focal lengths and principal point, pixels */
  int32_t width, height; /* image size, 1..GS_MAX_DIM */
} gs_camera;

/* The fixed numerical rules (App. C "Numerical stability"; Sec. 6) and the
 * tuning knobs. gs_default_config fills the values the method uses. */
typedef struct gs_config {
  int32_t sh_degree;       /* 0..3 (Sec. 7.1: up to 4 bands) */
  int32_t tile_size;       /* 8, 16 (the paper's value) or 32 pixels */
  float near_z;            /* near cull on camera depth, 0.2 */
  float sigma_extent;      /* a Gaussian touches a pixel iff m <= sigma_extent^2; 3 */
  float alpha_min;         /* skip alpha below this, 1/255 */
  float alpha_max;         /* clamp alpha to at most this, 0.99 */
  float T_min;             /* stop before transmittance falls below this, 1e-4 */
  float bg[3];             /* background colour added as T_final * bg */
  int32_t sort_digit_bits; /* radix digit width of gs_sort: 4..8, default 8 */
  int32_t lds_batch;       /* list entries each wave stages in LDS per round: 32, 64 or
                              128 (0 = 64); changes speed only */
  /* Ablation switches of Sec. 7.3 (0 in the method itself): */
  int32_t isotropic;       /* 1: one radius on all axes, Sigma = s^2 I with s = exp of the
                              mean of the three log-scales; quaternions unused, zero
                              gradient, each log-scale row gets a third of the gradient */
  int32_t grad_limit;      /* N > 0: a pixel passes gradient only to its N front-most
                              blended Gaussians (image unchanged); 0: to all of them */
} gs_config;

typedef struct gs_params {
  const float* means;          /* [3][N] */
  const float* log_scales;     /* [3][N]; scale = exp(log_scale) (Sec. 5.1) */
  const float* quats;          /* [4][N] (r, i, j, k), normalised inside */
  const float* opacity_logits; /* [N]; opacity = sigmoid(logit) (Sec. 5.1) */
  const float* sh;             /* [K][3][N] */
  int64_t n;                   /* N >= 0 */
} gs_params;

typedef struct gs_params_grad { /* same layouts as gs_params; overwritten */
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  float* sh;
} gs_params_grad;

/* Per view and Gaussian (index v * N + g), written by gs_project:
 *   depth_key     FP32 bit pattern of the camera-space depth (sort key low word)
 *   tiles_touched tiles covered by the Gaussian's 3-sigma pixel box; 0 = culled
 *   record        GS_RECORD_FLOATS floats:
 *     [0] pixel box low corner  (i_lo | j_lo << 16) as int32 bits
 *     [1] pixel box high corner (i_hi | j_hi << 16) as int32 bits
 *     [2] c0, [3] c1               c = L^-1 ((i_lo + 0.5, j_lo + 0.5) - (u, v)), the
 *                                  whitened offset of the box's corner pixel centre
 *                                  from the 2D mean (u, v)
 *     [4] w00, [5] w10, [6] w11    L^-1 = [[w00, 0], [w10, w11]] with Sigma' = L L^T
 *                                  (Cholesky); the pixel (i_lo + Di, j_lo + Dj) has
 *                                  m = (w00 Di + c0)^2 + (w10 Di + w11 Dj + c1)^2
 *     [7] opacity, [8..10] RGB colour, [11] camera depth (FP32)
 * Valid only where tiles_touched > 0. */
typedef struct gs_projected {
  uint32_t* depth_key;     /* [V*N] */
  int32_t* tiles_touched;  /* [V*N] */
  float* record;           /* [V*N][GS_RECORD_FLOATS] */
} gs_projected;

/* Instance arrays (App. C "Sorting"): one instance per visible (view, Gaussian)
 * pair and tile it overlaps, value v * N + g. After gs_sort, vals[0..M) lists the
 * instances in (global tile id, depth, index) order: the order of the paper's
 * single sort by the key (tile << 32) | depth. The pipeline reaches it with two
 * stable 32-bit sorts (gs_bin: pairs by depth; gs_sort: instances by tile id) and
 * uses keys and keys_alt as scratch (each as two uint32 arrays of capacity
 * entries); gs_sorted_tile_ids locates the sorted tile id of every instance. */
typedef struct gs_instances {
  uint64_t* keys;       /* [capacity] */
  uint32_t* vals;       /* [capacity] */
  uint64_t* keys_alt;   /* [capacity] */
  uint32_t* vals_alt;   /* [capacity] */
  int64_t capacity;     /* 0..GS_MAX_INSTANCES */
  uint32_t* count;      /* device [1]: instance count M (the required count on overflow) */
  uint32_t* status;     /* device [1]: GS_STATUS_* bits, OR-ed; the caller zeroes it */
} gs_instances;

/* Fill *cfg with the method's rules: SH degree 3, 16x16 tiles, near 0.2, 3 sigma,
 * alpha in [1/255, 0.99], T_min 1e-4, black background, 8-bit sort digits, LDS
 * batches of 64 entries per wave. */
void gs_default_config(gs_config* cfg);

/* Global tile ids: view v owns ids [tile_offset[v], tile_offset[v+1]) laid out
 * row-major over ceil(W/T) x ceil(H/T) tiles. Returns the total tile count
 * (tile_offset[n_views]), or a negative GS_ERR_* on bad arguments.
 * tile_offset may be NULL; otherwise it has n_views + 1 entries (host). */
int64_t gs_tile_layout(const gs_camera* cams, int32_t n_views, int32_t tile_size,
                       int64_t* tile_offset);

/* Bits of the tile-id key that gs_sort sorts on (those of the largest global tile
 * id); gs_bin's depth sort uses 31 bits (depth > 0 keeps the float's sign bit 0). */
int32_t gs_sort_key_bits(int64_t n_tiles_total);

/* Project (Alg. 2 CullGaussian + ScreenspaceGaussians; Sec. 4 Eq. volume-render;
 * Sec. 5 activations and SH colour). Reads params once and projects every
 * Gaussian into every view: depth, near cull, Sigma' = J W Sigma W^T J^T, the
 * 3-sigma pixel box, its Cholesky whitening, opacity and view-dependent colour.
 * Arithmetic is FP64 inside; the outputs are FP32. */
int gs_project(const gs_params* params, const gs_camera* cams, int32_t n_views,
               const gs_config* cfg, const gs_projected* out, gs_stream_t stream);

/* Workspace bytes of gs_bin for V*N projected Gaussians (0 on a bad config). */
size_t gs_bin_workspace_bytes(int64_t n_total, const gs_config* cfg);

/* Bin (Alg. 2 CreateTiles + DuplicateWithKeys; App. C "Sorting"): the visible
 * (view, Gaussian) pairs, stably sorted by depth (radix, cfg->sort_digit_bits per
 * pass), then one instance per pair and covered tile in that order (tiles of a pair
 * row-major). Writes the instance count to *inst->count; if it exceeds
 * inst->capacity, ORs GS_STATUS_CAPACITY into *inst->status and writes nothing
 * past capacity. n is N (per view). */
int gs_bin(const gs_projected* proj, int64_t n, const gs_camera* cams, int32_t n_views,
           const gs_config* cfg, const gs_instances* inst, void* workspace,
           size_t workspace_bytes, gs_stream_t stream);

/* Workspace bytes of gs_sort. */
size_t gs_sort_workspace_bytes(int64_t capacity, int64_t n_tiles_total, const gs_config* cfg);

/* Sort (Alg. 2 SortByKeys + IdentifyTileRanges; App. C): stable LSD radix sort of
 * the M = min(*count, capacity) instances of gs_bin by global tile id (per digit a
 * counting pass, a scan of the per-block counts, and a scatter pass), which
 * completes the (tile, depth, index) order, then per global tile the range
 * [start, end) of its instances, written to tile_ranges[t][2] (uint32). If tile_order (device, [n_tiles_total])
 * is not NULL it receives a permutation of the tile ids, longest list first
 * (bucketed by floor(log2(length))), the issue order for the render calls. */
int gs_sort(const gs_instances* inst, int64_t n_tiles_total, const gs_config* cfg,
            uint32_t* tile_ranges, uint32_t* tile_order, void* workspace,
            size_t workspace_bytes, gs_stream_t stream);

/* gs_sort without a workspace argument, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): identical
 * arguments, results and errors, but the scratch memory is the library's own static
 * device array of GS_SORT_SCRATCH_BYTES, one per GPU, held until the process ends. The
 * call allocates and frees nothing. Limit: gs_sort_workspace_bytes(inst->capacity,
 * n_tiles_total, cfg) must not exceed GS_SORT_SCRATCH_BYTES (else GS_ERR_SCRATCH and
 * nothing is enqueued); 16 MiB covers about 50M instances (1 KiB per 3072).
 * The array belongs to the device current at the call (the stream must be on it); the
 * first call on a device looks up its address there (hipGetSymbolAddress: make that
 * first call outside graph capture). No part of the array needs to start at zero
 * (every call writes what it reads), but all calls on one GPU share it: calls that overlap in time on one GPU (on
 * different streams) race and give wrong results. */
#define GS_SORT_SCRATCH_BYTES ((size_t)16 << 20)
int gs_sort_noalloc(const gs_instances* inst, int64_t n_tiles_total, const gs_config* cfg,
                    uint32_t* tile_ranges, uint32_t* tile_order, gs_stream_t stream);

/* Device address of the sorted global tile id of every instance after gs_sort
 * (uint32 [M], inside inst->keys or inst->keys_alt), or NULL on bad arguments. */
const uint32_t* gs_sorted_tile_ids(const gs_instances* inst, int64_t n_tiles_total,
                                   const gs_config* cfg);

/* Forward blend (Alg. 2 BlendInOrder; Eq. front-to-back; App. C rules): for every
 * pixel of every view, front to back over its tile's instances: skip pixels
 * outside the 3-sigma ellipse, alpha = min(alpha_max, o exp(-m/2)), skip
 * alpha < alpha_min, stop before T (1 - alpha) < T_min, then add T_final * bg.
 * Per view v the outputs start at pixel offset P_v = sum_{u<v} W_u H_u:
 *   image    [3][H][W] planar FP32 at image + 3 P_v
 *   T_final  [H][W] at T_final + P_v        final transmittance
 *   last_idx [H][W] at last_idx + P_v       instance position of the last
 *                                           blended Gaussian, -1 if none
 * n is N (per view); instance values >= V*N are ignored, and tile ranges are
 * clipped to [0, inst->capacity] (GS_ERR_ARG for a capacity outside
 * 0..GS_MAX_INSTANCES), so ranges not written by gs_sort give wrong images but
 * no out-of-range access. tile_order (device, nullable) is the order in which
 * tiles are issued (from gs_sort, a permutation of the tile ids); it changes no
 * output. */
int gs_render_fwd(const gs_projected* proj, const gs_instances* inst,
                  const uint32_t* tile_ranges, const uint32_t* tile_order,
                  const gs_camera* cams, int32_t n_views,
                  const gs_config* cfg, float* image, float* T_final, int32_t* last_idx,
                  int64_t n, gs_stream_t stream);

/* Backward blend (Sec. 6: back to front from each pixel's last contributor,
 * transmittance recovered by dividing the stored T_final by (1 - alpha); App. C):
 * given dL/dimage in the image layout, accumulates per view and Gaussian the
 * screen-space gradient record grad2d[v*N + g][9] =
 *   d(u, v), d(w00, w10, w11), d(opacity), d(r, g, b).
 * The gradients are ADDED to grad2d: the caller zeroes it first. T_final and
 * last_idx are the forward pass's outputs for the same inputs; a last_idx beyond
 * its tile's instance list is treated as the list's end (the walk never leaves
 * the list), other values give meaningless gradients but no out-of-range access. */
int gs_render_bwd(const gs_projected* proj, const gs_instances* inst,
                  const uint32_t* tile_ranges, const uint32_t* tile_order,
                  const gs_camera* cams, int32_t n_views,
                  const gs_config* cfg, const float* T_final, const int32_t* last_idx,
                  const float* dL_dimage, float* grad2d, int64_t n, gs_stream_t stream);

/* gs_render_bwd with the L1 photometric term of Sec. 5.1 taken inside it, for steps
 * whose loss is L1 alone: instead of a stored dL/dimage, each pixel's upstream gradient
 * is sign(image - target) / (3 H W) (sign(0) = 0), from the forward pass's image and the
 * target (device, the image layout), exactly what gs_loss_l1 writes; grad2d receives
 * what gs_render_bwd would add for that dL/dimage. If loss (device, V floats) is not
 * NULL, each view's mean |image - target| over 3 H W is ADDED to loss[v], summed in a
 * fixed order (the same bits on every run; equal to gs_loss_l1's up to that order);
 * workspace: device scratch of gs_render_l1_workspace_bytes(cams, n_views, cfg) bytes
 * (one float per 8x8 pixel block), owned by the caller and overwritten, unused (may be
 * NULL) when loss is NULL; the query returns 0 for invalid cameras or config.
 * image, target, T_final, last_idx or grad2d NULL, or a loss with a missing or short
 * workspace: GS_ERR_ARG. */
size_t gs_render_l1_workspace_bytes(const gs_camera* cams, int32_t n_views,
                                    const gs_config* cfg);
int gs_render_bwd_l1(const gs_projected* proj, const gs_instances* inst,
                     const uint32_t* tile_ranges, const uint32_t* tile_order,
                     const gs_camera* cams, int32_t n_views, const gs_config* cfg,
                     const float* T_final, const int32_t* last_idx, const float* image,
                     const float* target, float* grad2d, float* loss, void* workspace,
                     size_t workspace_bytes, int64_t n, gs_stream_t stream);

/* Projection backward (App. A chain rule, the quaternion normalisation, the
 * activations, SH and its view direction): gradients of the raw parameters,
 * summed over views, written (not accumulated) to *grads. grad2d (device) holds
 * n_views * n rows of GS_GRAD2D_FLOATS as gs_render_bwd leaves them; every row may
 * be read, and the values of rows whose pair has tiles_touched <= 0 are ignored. */
int gs_project_bwd(const gs_params* params, const gs_camera* cams, int32_t n_views,
                   const gs_config* cfg, const gs_projected* proj, const float* grad2d,
                   const gs_params_grad* grads, gs_stream_t stream);

/* L1 photometric loss of Sec. 5.1 (the L1 term of L = (1 - lambda) L1 +
 * lambda D-SSIM), per view the mean over 3 H W values of |image - target|:
 * writes dL/dimage = sign(image - target) / (3 H W) (sign(0) = 0) in the image
 * layout and, if loss is not NULL, ADDS each view's loss to loss[v] (device,
 * caller zeroes it). image and target are device arrays in the gs_render_fwd
 * image layout. */
int gs_loss_l1(const float* image, const float* target, const gs_camera* cams, int32_t n_views,
               float* dL_dimage, float* loss, gs_stream_t stream);

/* The full photometric loss of Sec. 5.1, L = (1 - lambda) L1 + lambda L_D-SSIM per
 * view (the paper uses lambda = 0.2), with L1 as in gs_loss_l1 and L_D-SSIM =
 * 1 - mean SSIM over the 3 H W values. SSIM (structural similarity, per channel) uses
 * an 11 x 11 Gaussian window of standard deviation 1.5 normalised to sum 1, zero
 * values outside the image (no renormalisation at the borders), C1 = 0.01^2,
 * C2 = 0.03^2 (dynamic range 1); the paper names D-SSIM without these constants.
 * Writes dL/dimage (image layout) and, if loss is not NULL, ADDS each view's loss to
 * loss[v]. workspace: device scratch of gs_loss_workspace_bytes(cams, n_views)
 * bytes (9 floats per pixel), owned by the caller and overwritten.
 * lambda outside [0, 1] or a short workspace: GS_ERR_ARG. */
size_t gs_loss_workspace_bytes(const gs_camera* cams, int32_t n_views);
int gs_loss_photometric(const float* image, const float* target, const gs_camera* cams,
                        int32_t n_views, float lambda, float* dL_dimage, float* loss,
                        void* workspace, size_t workspace_bytes, gs_stream_t stream);

/* ---------------------------------------------------------------------------
 * Adaptive density control (Sec. 5.2, Alg. 1). Readings where the paper gives no
 * number: the view-space positional gradient is taken in normalised device
 * coordinates, |(W/2 dL/du, H/2 dL/dv)| per view, averaged over the views where the
 * Gaussian was visible; a clone is an exact copy (the next optimiser step moves it);
 * a split replaces a Gaussian by two children mu + R diag(s) z, z ~ N(0, I) given by
 * the caller, with log-scales lowered by log(split_factor).
 * ------------------------------------------------------------------------- */
typedef struct gs_densify_config {
  float grad_threshold;    /* tau_pos: densify above this average gradient, 0.0002 */
  float min_opacity;       /* epsilon_alpha: remove below this opacity, 0.005 */
  float split_scale;       /* split (not clone) when the largest scale exceeds this */
  float max_world_scale;   /* remove above this largest scale; <= 0 disables */
  float max_screen_radius; /* remove above this pixel-box half-extent; <= 0 disables */
  float split_factor;      /* phi: scale divisor of split children, 1.6 */
} gs_densify_config;

/* grad_threshold 0.0002, min_opacity 0.005, split_scale 0.01, no size removal, phi 1.6. */
void gs_default_densify_config(gs_densify_config* cfg);

/* Statistics after a backward pass: for every Gaussian visible in some view (tiles
 * touched > 0 in proj), ADD to grad_sum[g] the NDC gradient norms of its projected
 * mean from grad2d (the gs_render_bwd output), to view_count[g] the number of such
 * views, and raise max_radius[g] to its largest pixel-box half-extent. The caller
 * zeroes the three device arrays [N] when it resets the statistics. */
int gs_densify_accumulate(const gs_projected* proj, const float* grad2d, const gs_camera* cams,
                          int32_t n_views, int64_t n, float* grad_sum, int32_t* view_count,
                          float* max_radius, gs_stream_t stream);

size_t gs_densify_workspace_bytes(int64_t n);

/* The plan (Alg. 1): per Gaussian action[g] = 0 remove (opacity below min_opacity,
 * or too large), 1 keep, 2 clone (average gradient above grad_threshold, largest
 * scale at most split_scale), 3 split (above both); offsets[g] = exclusive prefix of
 * the output counts (0, 1, 2, 2); *n_out (device) = the new Gaussian count. */
int gs_densify_plan(const gs_params* params, const float* grad_sum, const int32_t* view_count,
                    const float* max_radius, const gs_densify_config* cfg, uint8_t* action,
                    uint32_t* offsets, uint32_t* n_out, void* workspace, size_t workspace_bytes,
                    gs_stream_t stream);

/* Write the new parameter arrays (layouts of gs_params with N' = n_out rows, in the
 * gs_params_grad struct of output pointers) in Gaussian order: kept Gaussians once,
 * clones twice, split children from normals[g][2][3]. src_index (nullable, [n_out])
 * receives each output's source Gaussian (for gathering optimiser state). */
int gs_densify_apply(const gs_params* params, int32_t sh_degree, const uint8_t* action,
                     const uint32_t* offsets, const float* normals, const gs_densify_config* cfg,
                     const gs_params_grad* out, int64_t n_out, uint32_t* src_index,
                     gs_stream_t stream);

/* Opacity reset (Sec. 5.2: every 3000 iterations): opacity <- min(opacity, max_opacity),
 * applied to the logits in place. */
int gs_reset_opacity(float* opacity_logits, int64_t n, float max_opacity, gs_stream_t stream);

/* Carry per-Gaussian state laid out like gs_params (e.g. the optimiser's moments)
 * through the densification planned by gs_densify_plan: output j of a Gaussian g
 * takes state[g], or zeros when zero_created != 0 and g was cloned or split.
 * out is sized like gs_densify_apply's output (n_out Gaussians). */
int gs_densify_gather(const gs_params* state, int32_t sh_degree, const uint8_t* action,
                      const uint32_t* offsets, int32_t zero_created, const gs_params_grad* out,
                      int64_t n_out, gs_stream_t stream);

/* One Adam step (the optimiser of Alg. 1; Kingma and Ba) over n values, in place:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * param -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t >= 1 the step count.
 * All four are device arrays of n floats (float4 accesses when all are 16-byte aligned). */
int gs_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, float lr,
                 float beta1, float beta2, float eps, int32_t t, gs_stream_t stream);

/* Copy the device status word to the host after synchronising `stream`
 * (the only synchronising call; not for use under graph capture). */
int gs_read_status(const gs_instances* inst, uint32_t* status, uint32_t* count,
                   gs_stream_t stream);

const char* gs_status_string(int code);

#ifdef __cplusplus
}
#endif
#endif /* GS_MI355X_H */
