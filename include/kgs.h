/*
 * kgs.h -- C ABI of the MI355X (gfx950) differentiable Gaussian rasterizer and
 * the multi-view densify / prune statistics of lifecycle-managed Gaussian
 * mapping (KiloGS-SLAM, arXiv 2606.30436).
 *
 * Conventions shared by every entry point
 *   * Plain C types only.  Arrays are caller-owned DEVICE memory unless a
 *     comment says "host".  Nothing here allocates device memory: every
 *     scratch buffer lives in the caller-allocated workspace handed to
 *     kgs_create, except the 1 MiB static device array of
 *     kgs_accumulate_stats_static (library-owned, one per GPU).
 *   * Work is enqueued on the caller's stream (hipStream_t passed as void*;
 *     NULL means the default stream).  Calls return after enqueueing; results
 *     are valid after the stream is synchronised.
 *   * Argument errors are found on the host before anything is enqueued and
 *     return KGS_ERR_INVALID_ARG.  HIP launch errors return KGS_ERR_HIP.
 *     Conditions found on the device (capacity overflow, non-finite input)
 *     set bits of a device status word read by kgs_status_read.
 *   * One context per stream; a context is not thread safe.
 *   * Gaussian parameters are structure-of-arrays, Gaussian index fastest:
 *       means [3][N], log_scales [3][N], quats [4][N] (w, x, y, z; any
 *       non-zero length), opacity_logits [N], sh [K][3][N] with
 *       K = (sh_degree + 1)^2 real spherical-harmonic coefficients per colour
 *       channel (index l^2 + l + m, Condon-Shortley phase).
 *   * Images are planar: colour [V][3][H][W], depth / t_final / last [V][H][W].
 *     Pixel (x, y) samples the image plane at (x + 0.5, y + 0.5).
 *
 * The method computed (paper sections cited per entry point below):
 *   pose        T' = Exp(xi) T  for a world->camera pose T and a tangent
 *               xi = (rho, phi) in se(3).
 *   project     EWA splatting of each Gaussian: camera point, 2D covariance
 *               J W Sigma W^T J^T + eps I, its inverse (conic), pixel centre,
 *               opacity o = sigmoid(logit), view-dependent colour
 *               max(0, SH(dir) + 0.5), depth = camera z.
 *   bin + sort  one (tile, Gaussian) pair per tile of the Gaussian's
 *               opacity-aware pixel rectangle, sorted by
 *               (view, tile, fp32 depth, Gaussian index): records sorted by
 *               (view, depth), pairs emitted in that order, then sorted
 *               stably by tile.
 *   render_fwd  front-to-back alpha compositing of colour and depth with
 *               transmittance T_j = prod_{m<j}(1 - alpha_m) (appendix,
 *               "Depth Volume Rendering"): D = sum_j T_j alpha_j z_j.
 *   render_bwd  exact gradient of render_fwd + project for all Gaussian
 *               parameters and the 6-DoF pose, recomputing the per-pixel
 *               sequences; plus per Gaussian the footprint |Omega_v(i)| (pixels
 *               where it is blended) and kappa_v(i), the number of those pixels
 *               with ||I_v - I^_v||_1 > tau_err (appendix, "Densification
 *               Score").
 *   stats       chunk scores S_d and S_p and their global OR / max merge
 *               (Sec. 3.3 "Global Densification / Pruning Rules"; appendix
 *               "Densification Score", "Pruning Score").
 *   decide      PRUNE if S_p(i) > tau_p, else DENSIFY if S_d(i), else KEEP.
 */
#ifndef KGS_H
#define KGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KGS_OK = 0,
  KGS_ERR_INVALID_ARG = 1,
  KGS_ERR_HIP = 2,
  KGS_ERR_CAPACITY = 3,   /* a device capacity was exceeded: outputs undefined, regrow and rerun */
  KGS_ERR_NONFINITE = 4,  /* a non-finite parameter was met */
  KGS_ERR_STATE = 5       /* call order violated (e.g. render before project) */
} kgs_status;

/* device status word bits (kgs_status_read) */
#define KGS_FLAG_SLOT_OVERFLOW 0x1u
#define KGS_FLAG_PAIR_OVERFLOW 0x2u
#define KGS_FLAG_NONFINITE 0x4u

/* decision codes written by kgs_densify_prune_decide */
#define KGS_KEEP 0
#define KGS_DENSIFY 1
#define KGS_PRUNE 2

/* Pinhole camera, world->camera: x_cam = R x_world + t, R row major.
 * Camera axes: x right, y down, z forward.  72 bytes. */
typedef struct kgs_camera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
} kgs_camera;

/* Rasterizer configuration.  The paper inherits its rasterizer from 3DGS and
 * states none of these constants; kgs_config_default fills the readings
 * alpha_min = 1/255, alpha_max = 0.99, t_min = 1e-4, near_z = 0.2,
 * eps2d = 0.3 px^2, guard = 1.3, rect_margin = 1/256, bg = 0, and
 * far_z = 1e30.  far_z is the single-level form of the paper's distance mask
 * (appendix, "Level-of-Detail (LoD) Mask Computation": a Gaussian is rendered
 * only inside its level's distance range): camera depths >= far_z are culled. */
typedef struct kgs_config {
  int32_t tile_w, tile_h;   /* 16x16, 8x32, 32x8 (four waves per compositing workgroup)
                               or 32x16, 16x32 (eight waves); the backward with two
                               pixels per lane runs half as many */
  int32_t batch;            /* Gaussians staged per LDS batch of the backward: 32, 64
                               or 128 (at most 64 with 512-pixel tiles); the forward
                               stages 64 at a time in every wave */
  int32_t sh_degree;        /* 0..3 */
  float alpha_min, alpha_max, t_min, near_z, eps2d, guard, rect_margin, far_z;
  float bg[3];
  int32_t width, height;    /* image size of every view */
  int32_t max_views;        /* 1..64 views per call */
  int32_t px_per_lane;      /* compositing backward: pixels per lane, 1 (a wave per 8x8 block) or 2 (a
                               wave per 16x8 block, tiles at least 16 wide); 0 picks 2 where the
                               launch has at least 4096 such waves (16 per CU), else 1 */
  int64_t max_gaussians;
  int64_t slot_capacity;    /* visible (view, Gaussian) records per call */
  int64_t pair_capacity;    /* (tile, Gaussian) pairs per call, < 2^32 */
} kgs_config;

typedef struct kgs_gaussians {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity_logits;
  const float* sh;
  int64_t n;
  int32_t sh_degree;
  int32_t pad_;
} kgs_gaussians;

typedef struct kgs_image {
  float* color;     /* [V][3][H][W] = composited colour + t_final * bg */
  float* depth;     /* [V][H][W]   = sum_j T_j alpha_j z_j (not normalised) */
  float* t_final;   /* [V][H][W]   transmittance after the last blended Gaussian */
  int32_t* last;    /* [V][H][W]   1 + position, in the pixel's tile list, of its last blended Gaussian (0: none) */
} kgs_image;

/* Gradients, ADDED to (caller zeroes them).  Same layouts as the parameters;
 * pose_xi [V][6] with (rho, phi) order.  Any pointer may be NULL to skip it. */
typedef struct kgs_grads {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  float* sh;
  float* pose_xi;
} kgs_grads;

/* Per-Gaussian statistics accumulated over the views of a chunk ([N] each,
 * ADDED to; the caller zeroes them at the start of a chunk).  Any may be NULL.
 *   kappa_sum      sum_v kappa_v(i)
 *   omega_sum      sum_v |Omega_v(i)|
 *   gamma_sum      sum_v L_v |Omega_v(i)|   (L_v: the view's photometric loss)
 *   grad_norm_sum  sum_v ||dL/d mu2D_v(i)||_2 in pixels (3DGS positional statistic)
 *   view_count     number of views in which i is visible
 *   max_radius     max_v of the larger pixel half-extent of i (MAX-merged) */
typedef struct kgs_view_stats {
  uint32_t* kappa_sum;
  uint32_t* omega_sum;
  double* gamma_sum;
  float* grad_norm_sum;
  uint32_t* view_count;
  int32_t* max_radius;
} kgs_view_stats;

/* Global lifecycle state, [N] each: S_d(i) as 0/1 and S_p(i). */
typedef struct kgs_lifecycle_state {
  uint8_t* densify;
  double* prune_score;
} kgs_lifecycle_state;

/* Device buffers of the last project / bin_sort call (for tests and tools).
 * All pointers are into the workspace; counts are device pointers. */
typedef struct kgs_buffers {
  const uint32_t* n_slots;      /* device scalar */
  const uint32_t* n_pairs;      /* device scalar */
  const float* slot_rec;        /* [S][16]: mu_x-0.5-floor(W/2), mu_y-0.5-floor(H/2), P', k, E', log2 o,
                                   depth, -, r, g, b, -, first pair (u32 bits), -, -, -  with the conic as
                                   q = P (dx + k dy)^2 + E dy^2, P' = -P log2(e) / 2, E' = -E log2(e) / 2;
                                   64 bytes per record, one aligned line segment per read */
  const uint32_t* slot_gid;     /* [S] Gaussian index */
  const uint32_t* slot_view;    /* [S] view */
  const int32_t* slot_pix;      /* [S][4]: floor(mu_x), floor(mu_y), rx, ry */
  const uint32_t* slot_pairoff; /* [S] first pair (emission order) */
  const uint32_t* keys;         /* [P] sorted pair keys: (view << tile_bits) | tile.  Pairs are grouped by
                                   tile, then view; depth order within a (view, tile) group */
  const uint32_t* sorted_slot;  /* [P] slot of each sorted pair */
  const uint32_t* ranges;       /* [V*tiles][2] start, end in the sorted pairs, index view * tiles + tile */
  int32_t tiles_x, tiles_y;
  int32_t tile_bits;            /* tiles < 2^tile_bits */
  int32_t n_views;              /* views of the last kgs_project */
} kgs_buffers;

/* A whole pass over one chunk of views: zero the accumulators (optional),
 * project, bin + sort, render_fwd, L1 loss, render_bwd with statistics, then
 * (optional) close the chunk into the lifecycle state and decide. */
typedef struct kgs_chunk_desc {
  kgs_gaussians gaussians;
  const kgs_camera* cams;   /* device [V] */
  const float* pose_xi;     /* device [V][6] or NULL */
  int32_t n_views;
  float tau_err;
  const float* target;      /* device [V][3][H][W] */
  kgs_image image;          /* outputs */
  float* dl_dcolor;         /* device [V][3][H][W] scratch: dL/dC of the L1 loss */
  float* view_loss;         /* device [V]: mean |C - I| per view */
  kgs_grads grads;
  kgs_view_stats stats;
  int32_t zero_accumulators; /* != 0: grads and stats start from zero (the backward writes them instead of adding) */
  float tau_d;
  kgs_lifecycle_state state; /* densify != NULL: kgs_accumulate_stats(reset = 1) after the backward */
  uint8_t* decision;         /* != NULL: kgs_densify_prune_decide after that */
  double tau_p;
} kgs_chunk_desc;

typedef struct kgs_ctx kgs_ctx;
typedef struct kgs_graph kgs_graph;

/* Fill cfg with the default readings for an image of width x height. */
void kgs_config_default(kgs_config* cfg, int32_t width, int32_t height);

/* Bytes of device workspace a context with this configuration needs (host only). */
kgs_status kgs_workspace_size(const kgs_config* cfg, size_t* bytes);

/* Create a context over caller-owned device memory of at least
 * kgs_workspace_size bytes (256-byte aligned).  The context is host memory
 * owned by the library; free it with kgs_destroy (the workspace stays the
 * caller's). */
kgs_status kgs_create(const kgs_config* cfg, void* workspace, size_t bytes, kgs_ctx** out);
kgs_status kgs_destroy(kgs_ctx* ctx);

/* Change the tile shape and LDS batch of an existing context (the workspace
 * is sized for every supported shape).  Takes effect at the next project.
 * KGS_ERR_INVALID_ARG for a shape or batch the configuration does not allow. */
kgs_status kgs_set_tiling(kgs_ctx* ctx, int32_t tile_w, int32_t tile_h, int32_t batch);

/* EWA projection of every Gaussian into every view (Sec. 3.2 map
 * representation, rasterized as in 3DGS; depth is the camera z used by the
 * appendix's depth rendering).  cams: device [V]; pose_xi: device [V][6] or
 * NULL.  Culls z <= near_z, o < alpha_min and empty tile rectangles, and
 * writes compact per-(view, Gaussian) records into the workspace.  Slot
 * overflow sets KGS_FLAG_SLOT_OVERFLOW. */
kgs_status kgs_project(kgs_ctx* ctx, const kgs_gaussians* g, const kgs_camera* cams, int32_t n_views,
                       const float* pose_xi, void* stream);

/* Tile binning and depth sort of the projected records ("sorted Gaussians",
 * appendix, Depth Volume Rendering): the records are radix-sorted by
 * (view, fp32 depth bits), one pair per tile of each record's rectangle is
 * emitted in that order, and the pairs are radix-sorted stably by their tile
 * within the view, which leaves each (view, tile) group contiguous and in
 * depth order; equal depths keep Gaussian-index order.  Then per-(view, tile)
 * ranges.  Pair overflow sets KGS_FLAG_PAIR_OVERFLOW (at kgs_project).
 * KGS_ERR_INVALID_ARG if the tile count per view needs more than 25 bits. */
kgs_status kgs_bin_sort(kgs_ctx* ctx, void* stream);

/* Front-to-back compositing of every tile of every view (appendix, Depth
 * Volume Rendering; colour composited with the same weights). */
kgs_status kgs_render_fwd(kgs_ctx* ctx, const kgs_image* out, void* stream);

/* L1 photometric loss per view (harness for the paper's photometric loss,
 * Sec. 3.2 mapping loss): view_loss[v] = mean |C - I| over pixels and
 * channels; dl_dcolor = sign(C - I) / (3 H W).  target: device [V][3][H][W]. */
kgs_status kgs_loss_l1(kgs_ctx* ctx, const float* target, const kgs_image* img, float* dl_dcolor,
                       float* view_loss, void* stream);

/* Mapping loss of the sliding-window optimisation (Sec. 3.2, Eq. mapping loss;
 * appendix "Rendering Objectives") over n_views rendered views:
 *   view_loss[v] = L_photo,v = w_l1 mean|I - C| + w_ssim (1 - mean SSIM(I, C))
 *   geo_loss[v]  = L_geo,v   = mean|D_target - D|        (if target_depth)
 * means over the view's 3 H W (colour) or H W (depth) values; SSIM with an
 * 11x11 Gaussian window (sigma 1.5), C1 = 0.01^2, C2 = 0.03^2, per channel,
 * zero padding.  Gradients of sum_v (L_photo,v + lambda_g L_geo,v) are
 * WRITTEN: dl_dcolor [V][3][H][W]; dl_ddepth [V][H][W] when target_depth is
 * given (required then).  The paper's weights are w_l1 = 0.8, w_ssim = 0.2,
 * lambda_g = 0.01.  img: colour [V][3][H][W] (and depth [V][H][W]) of the
 * configured image size; target [V][3][H][W]; target_depth [V][H][W] or NULL;
 * geo_loss [V] or NULL.  Uses the workspace; deterministic. */
kgs_status kgs_loss_mapping(kgs_ctx* ctx, int32_t n_views, const kgs_image* img, const float* target,
                            const float* target_depth, float w_l1, float w_ssim, float lambda_g, float* dl_dcolor,
                            float* dl_ddepth, float* view_loss, float* geo_loss, void* stream);

/* Isotropy regulariser (appendix "Rendering Objectives"):
 *   L_iso = sum_i sum_k |s_ik - mean_k s_ik|,  s = exp(log_scales)
 * written to loss (device scalar, unweighted); lambda_iso dL_iso/dlog_scales
 * is ADDED to grad_log_scales [3][N] (or NULL).  The paper's lambda_iso = 10. */
kgs_status kgs_loss_iso(kgs_ctx* ctx, const kgs_gaussians* g, float lambda_iso, float* grad_log_scales, float* loss,
                        void* stream);

/* ------------------------------------------------------------------------
 * Probabilistic Gaussian initialisation (Sec. 3.3, "Probabilistic Gaussian
 * Initialization") with the level-of-detail voxel rule of Sec. 3.2
 * ("Hierarchical Anchor Management"), for a batch of keyframes:
 *   DoG  = min(|(G_s1 - G_s2) * I|, 1),   I the mean of the three channels
 *   P    = min(0.9 DoG + 0.1 norm(||grad D||), 1)   (lambda = 0.9, hyper-parameter table)
 *   P_kf = max(P - P^, 0)    with P^ the same map of the rendered colour and depth
 * A pixel spawns if P_kf > 0 is not below any in-image 3x3 neighbour (the
 * suppression), u < P_kf for the caller's uniform u, and its depth is
 * positive.  It is unprojected at its pixel centre, x = R^T (d K^-1 (x+.5,
 * y+.5, 1) - t), and quantised at the level l of its camera distance,
 * voxel = floor(x / eps_l).  Readings: s1 = 1, s2 = 1.6, blur radius
 * round(3 s) with the border pixel repeated; central depth differences inside
 * the image, one-sided on its border; min-max normalisation per image;
 * eps = (0.1, 0.25, 1, 5, 25) m (the printed third size, 0.1, read as 1) and
 * level l for camera distances below 100 eps_l (the last level unbounded).
 * Every decision is taken in FP64.
 * ------------------------------------------------------------------------ */
typedef struct kgs_spawn_list {
  int32_t* pixel;    /* [capacity][2]: keyframe, pixel index y * width + x */
  int32_t* level;    /* [capacity]: level 0..4 */
  int32_t* voxel;    /* [capacity][3]: floor(x / eps_level) */
  float* point;      /* [capacity][3]: the unprojected world point */
  float* color;      /* [capacity][3]: the keyframe's colour at the pixel (or NULL) */
  uint32_t* count;   /* device scalar: spawning pixels, which may exceed capacity (then only the first
                        capacity, in (keyframe, row, column) order, are written) */
  int64_t capacity;
} kgs_spawn_list;

/* Bytes of device workspace kgs_init_spawn needs (host only). */
kgs_status kgs_init_workspace_size(int32_t width, int32_t height, int32_t n_views, size_t* bytes);

/* color [V][3][H][W] in [0, 1]; depth [V][H][W] (the depth prior D, metres);
 * rendered [V][3][H][W] and rendered_depth [V][H][W] (the map's render of each
 * keyframe) or both NULL (a first keyframe: P_kf = P); uniforms [V][H][W] in
 * [0, 1); cams: device [V] world->camera pinhole cameras; workspace of
 * kgs_init_workspace_size bytes, 256-byte aligned; p_kf [V][H][W] (FP32 copy
 * of P_kf) or NULL.  Writes the spawning pixels to out in (keyframe, row,
 * column) order.  Deterministic. */
kgs_status kgs_init_spawn(const float* color, const float* depth, const float* rendered, const float* rendered_depth,
                          const float* uniforms, const kgs_camera* cams, int32_t n_views, int32_t width,
                          int32_t height, void* workspace, size_t workspace_bytes, float* p_kf,
                          const kgs_spawn_list* out, void* stream);

/* ------------------------------------------------------------------------
 * Map maintenance (appendix "Dynamic Map Expansion" and "Global Map
 * Alignment"; Sec. 3.3 densify / prune decisions acting on the map).  With
 * explicit Gaussians an anchor is one Gaussian.
 *   * A voxel is (level l, idx = floor(x / eps_l)); its 64-bit key packs l in
 *     bits 60..62 and idx + 2^19 in three 20-bit fields (indices outside
 *     [-2^19, 2^19) give the key ~0, which is skipped).
 *   * The spatial hash is a caller-allocated table of 2^log2_capacity slots
 *     (kgs_map_table_bytes), cleared once with kgs_map_table_clear; it maps each
 *     occupied voxel to its anchor.
 *   * A batch insertion creates one anchor per new voxel, numbered n_anchors_in,
 *     n_anchors_in + 1, ... in the order of each new voxel's first candidate;
 *     a voxel already present keeps its anchor.  Deterministic.
 *   * New Gaussians (readings): mean idx eps_l, log-scales ln(eps_l), identity
 *     rotation, opacity 0.1, SH degree-0 colour of the spawning pixel, higher
 *     bands zero.
 *   * Densify points (reading): mu +- s_max a_max of every Gaussian whose
 *     decision is DENSIFY (its largest scale along its axis), + before -, in
 *     Gaussian order; their level from the distance to a camera centre.
 *   * Poses are world->camera (R, t); alignment moves the Gaussians of keyframe m
 *     by p' = R_new^T (R_old p + t_old - t_new) and turns them by R_new^T R_old.
 *   * Re-voxelisation keeps, of the anchors sharing a voxel at their level, the
 *     one with the lowest index.
 * Status bits (device word, OR-ed): 1 the hash table is full, 2 the parameter
 * arrays are full.  Every integer decision is taken in FP64.
 * ------------------------------------------------------------------------ */

/* Writable structure-of-arrays Gaussians of capacity n (the stride of every plane). */
typedef struct kgs_gaussians_out {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  float* sh;
  int64_t n;
  int32_t sh_degree;
  int32_t pad_;
} kgs_gaussians_out;

/* Bytes of a table of 2^log2_capacity slots, log2_capacity in 4..31 (host only). */
kgs_status kgs_map_table_bytes(int32_t log2_capacity, size_t* bytes);
/* Mark every slot empty. */
kgs_status kgs_map_table_clear(void* table, int32_t log2_capacity, void* stream);
/* Bytes of device workspace the insertion, densify-point and re-voxelisation
 * calls need for up to max_items keys or Gaussians (host only). */
kgs_status kgs_map_workspace_size(int64_t max_items, size_t* bytes);
/* keys[i] of (level[i], voxel[i][3]). */
kgs_status kgs_map_voxel_keys(const int32_t* level, const int32_t* voxel, int64_t n, uint64_t* keys, void* stream);
/* Insert keys[n].  anchor[i] (or NULL): the anchor of key i (~0 for a skipped
 * key or a full table); created[k] (or NULL): the key index that created
 * anchor n_anchors_in + k; n_anchors_in / n_anchors_out: device scalars (must
 * not alias); status: device word. */
kgs_status kgs_map_insert(void* table, int32_t log2_capacity, const uint64_t* keys, int64_t n,
                          const uint32_t* n_anchors_in, uint32_t* anchor, uint32_t* created, uint32_t* n_anchors_out,
                          uint32_t* status, void* workspace, size_t workspace_bytes, void* stream);
/* Parameters of the anchors n_anchors_in .. n_anchors_out - 1 created by an
 * insertion, from the level, voxel and colour [3] of their creating key; written
 * at their anchor index in out (status bit 2 past out->n). */
kgs_status kgs_map_spawn(const uint32_t* created, const uint32_t* n_anchors_in, const uint32_t* n_anchors_out,
                         const int32_t* level, const int32_t* voxel, const float* color, int64_t n_candidates,
                         const kgs_gaussians_out* out, uint32_t* status, void* stream);
/* Densify points of the DENSIFY decisions: level [cap], voxel [cap][3],
 * point [cap][3], source [cap] (the Gaussian); count: device scalar, the full
 * number (2 per Gaussian), of which the first capacity are written.
 * centre: host [3] camera centre for the levels. */
kgs_status kgs_map_densify_points(const kgs_gaussians* g, const uint8_t* decision, const double centre[3],
                                  int64_t capacity, int32_t* level, int32_t* voxel, float* point, uint32_t* source,
                                  uint32_t* count, void* workspace, size_t workspace_bytes, void* stream);
/* Survivors of the decision (not PRUNE) gathered to out at keep_map[i] (the
 * exclusive prefix count kgs_densify_prune_decide writes). */
kgs_status kgs_map_compact(const kgs_gaussians* g, const uint8_t* decision, const uint32_t* keep_map,
                           const kgs_gaussians_out* out, void* stream);
/* In place: Gaussian i of keyframe m = keyframe_of[i] (-1: none) moves with
 * T_new^(m) (T_old^(m))^-1; old_poses / new_poses: device [n_keyframes]
 * cameras (only R and t are used). */
kgs_status kgs_map_align(float* means, float* quats, int64_t n, const int32_t* keyframe_of, const kgs_camera* old_poses,
                         const kgs_camera* new_poses, int32_t n_keyframes, void* stream);
/* Re-voxelise n anchors (means [3][n], level [n]) into a freshly cleared table:
 * keep[i] = 1 for the lowest index of each voxel, anchor[i] = the survivor's
 * new index (rank among the survivors), n_keep (device) their number. */
kgs_status kgs_map_revoxelize(const float* means, const int32_t* level, int64_t n, void* table, int32_t log2_capacity,
                              uint8_t* keep, uint32_t* anchor, uint32_t* n_keep, uint32_t* status, void* workspace,
                              size_t workspace_bytes, void* stream);

/* One Adam step (bias-corrected, step >= 1) over n map parameters: the
 * gradient steps of the sliding-window optimisation (Sec. 3.2; the paper
 * names no optimiser).  m and v are the caller's moment buffers (zeroed before
 * step 1). */
kgs_status kgs_adam(float* theta, float* m, float* v, const float* grad, int64_t n, int32_t step, float lr, float beta1,
                    float beta2, float eps, void* stream);

/* ------------------------------------------------------------------------
 * Anchors (appendix "Voxelized Representation and MLP Decoding" and
 * "Level-of-Detail (LoD) Mask Computation"; per-anchor scores of appendix
 * "Densification Score" / "Pruning Score").
 * An anchor i holds a position p_i, a feature f_i in R^32, a local scale
 * l_i = exp(log_l_i) and K offsets O_ik; its level l_i selects the distance
 * band [D_min, D_max) in which it is rendered (D_max = 100 eps_level,
 * eps = (0.1, 0.25, 1, 5, 25), D_min the previous level's D_max).
 * Decoding for a camera centre c: d = |p - c|, d^ = (p - c) / d; one network
 *   36 inputs (f, d^, d) -> 32 ReLU -> 14 K outputs, child k taking outputs
 *   14k..14k+13 as (alpha, colour[3], rotation[4], ds[3], dO[3]);
 *   theta = W1 [32][36], b1 [32], W2 [14K][32], b2 [14K] (FP32, row major);
 *   BF16 operands on the matrix cores, FP32 accumulation.
 * Child k of anchor a is Gaussian a K + k, with
 *   mean p + (O_k + dO_k) * l,  log-scale log l + log sigmoid(ds),
 *   rotation as decoded, opacity tanh(alpha) * (1 inside the band, else 0)
 *   (logit -100 when not positive), colour sigmoid(.) as a degree-0 SH
 *   coefficient (c - 0.5) / Y_00.
 * ------------------------------------------------------------------------ */
typedef struct kgs_anchors {
  const float* p;         /* [3][A] */
  const float* feat;      /* [A][32], 16-byte aligned rows */
  const float* log_l;     /* [3][A] */
  const float* offsets;   /* [K][3][A] */
  const int32_t* level;   /* [A], 0..4 */
  int64_t n;              /* A */
  int32_t k;              /* children per anchor, 1..16 */
  int32_t pad_;
} kgs_anchors;
#define KGS_DECODER_PARAMS(K) (32 * 36 + 32 + 14 * (K) * 32 + 14 * (K))

/* The Gaussians one view sees: out (sh_degree 0, capacity out->n >= A K)
 * receives child a K + k of every anchor; camera: device pointer to the view's
 * camera (its centre -R^T t).  Deterministic. */
kgs_status kgs_anchor_decode(const kgs_anchors* a, const float* theta, const kgs_camera* camera,
                             const kgs_gaussians_out* out, void* stream);

/* Per-anchor footprint statistics of the last projected, binned and rendered
 * views (fwd: their kgs_render_fwd outputs): for every anchor a, |Omega_v(a)|
 * is the number of pixels where at least one Gaussian g with anchor_of[g] == a
 * is blended, and kappa_v(a) those of them where the error mask is set
 * (sum over channels of |target - colour| > tau_err).  Added to the chunk sums
 * of stats (arrays of n_anchors): omega_sum += |Omega_v|, kappa_sum += kappa_v,
 * gamma_sum += view_loss[v] |Omega_v| (if view_loss and gamma_sum).
 * anchor_of [N] of the projected Gaussians; counts: device scratch of
 * 2 V n_anchors u32 (per-view counts, zeroed by the call); status [2] u32:
 * bit 4 of status[0] if a sub-block's anchors could not be split to fit (its
 * counts are then incomplete), status[1] counts the re-walks. */
kgs_status kgs_anchor_stats(kgs_ctx* ctx, const kgs_image* fwd, const uint32_t* anchor_of, int64_t n_anchors,
                            const float* target, float tau_err, const float* view_loss, uint32_t* counts,
                            const kgs_view_stats* stats, uint32_t* status, void* stream);

/* Backward of render_fwd and project for the last projected views, plus the
 * per-view footprint statistics (appendix, densification and pruning
 * scores: Omega_v(i), M_v, kappa_v(i), gamma_v(i) = L_v |Omega_v(i)|).
 * dl_dcolor [V][3][H][W] (required), dl_ddepth [V][H][W] (or NULL),
 * dl_dtfinal [V][H][W] (or NULL): the gradient with respect to the final
 * transmittance t_final (the opacity image is 1 - t_final);
 * target [V][3][H][W] or NULL (then kappa is not counted); view_loss [V] or
 * NULL (then gamma is not accumulated).  g, cams and pose_xi must be those of
 * the matching kgs_project.  grads and stats are ADDED to. */
kgs_status kgs_render_bwd(kgs_ctx* ctx, const kgs_gaussians* g, const kgs_camera* cams, int32_t n_views,
                          const float* pose_xi, const kgs_image* fwd, const float* dl_dcolor,
                          const float* dl_ddepth, const float* dl_dtfinal, const float* target, float tau_err,
                          const float* view_loss, const kgs_grads* grads, const kgs_view_stats* stats,
                          void* stream);

/* The two halves of kgs_render_bwd, for callers that time or schedule them
 * separately.  kgs_render_bwd_pixels: the compositing backward (recomputes
 * each pixel's sequence, writes per-pair gradients and footprint counts into
 * the workspace).  kgs_project_bwd: per Gaussian, the sum over its pairs and
 * views, the chain rule to the parameters and the pose, and the statistics.
 * Called in this order they equal kgs_render_bwd; kgs_project_bwd returns
 * KGS_ERR_STATE unless kgs_render_bwd_pixels has run since the last
 * kgs_project / kgs_bin_sort / kgs_set_tiling. */
kgs_status kgs_render_bwd_pixels(kgs_ctx* ctx, const kgs_image* fwd, const float* dl_dcolor, const float* dl_ddepth,
                                 const float* dl_dtfinal, const float* target, float tau_err, void* stream);
kgs_status kgs_project_bwd(kgs_ctx* ctx, const kgs_gaussians* g, const kgs_camera* cams, int32_t n_views,
                           const float* pose_xi, const float* view_loss, const kgs_grads* grads,
                           const kgs_view_stats* stats, void* stream);

/* Close a chunk (appendix, Densification Score and Pruning Score; Sec. 3.3
 * global rules):  S_d = kappa_sum / n_views,  L = ln(1 + gamma_sum),
 * S_p = (L - min_A L) / (max_A L - min_A L) over A = {omega_sum > 0} (0 off A
 * and when max == min);  densify |= S_d > tau_d;  prune_score = max(prune_score, S_p).
 * L, S_p and the min / max are computed in FP64.  If reset != 0 the chunk sums
 * (kappa, omega, gamma) are zeroed afterwards. */
kgs_status kgs_accumulate_stats(kgs_ctx* ctx, const kgs_view_stats* stats, int64_t n, int32_t n_views,
                                const kgs_lifecycle_state* state, float tau_d, int32_t reset, void* stream);

/* kgs_accumulate_stats for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments and results as kgs_accumulate_stats, no context:
 * the min / max partials of the chunk's L live in a static device array that
 * the library holds on each GPU it runs on until the process ends (1 MiB), so
 * nothing is allocated.  n may be at most KGS_ACCUMULATE_STATIC_MAX_N
 * (65535 blocks of 256 Gaussians), else KGS_ERR_INVALID_ARG.  The array keeps
 * the last call's contents and needs no clearing; calls that overlap on one
 * GPU (concurrent streams, threads) share it and race.  KGS_ERR_HIP if the
 * array's device address cannot be obtained on the current device. */
#define KGS_ACCUMULATE_STATIC_MAX_N 16776960LL
kgs_status kgs_accumulate_stats_static(const kgs_view_stats* stats, int64_t n, int32_t n_views,
                                       const kgs_lifecycle_state* state, float tau_d, int32_t reset, void* stream);

/* decision[i] = PRUNE if prune_score > tau_p, else DENSIFY if densify, else
 * KEEP (Sec. 3.3).  keep_map (or NULL): exclusive prefix count of survivors;
 * n_keep (device scalar, or NULL).  tau_p is a double so that 0.99 is not
 * moved by float rounding (prune scores are FP64). */
kgs_status kgs_densify_prune_decide(kgs_ctx* ctx, const kgs_lifecycle_state* state, int64_t n, double tau_p,
                                    uint8_t* decision, uint32_t* keep_map, uint32_t* n_keep, void* stream);

/* ------------------------------------------------------------------------
 * Learned prune / keep / densify head.  A small network predicts the plain
 * criterion's decision (kgs_densify_prune_decide, Sec. 3.3 and App. D) from a
 * Gaussian's statistics; it is trained on that criterion's decisions, which
 * stay the fallback and the reference for its agreement.  MLP 16 -> 64 -> 64 -> 3,
 * ReLU after both hidden layers, logits out; every GEMM takes BF16 operands
 * (round to nearest even) on the matrix cores with FP32 accumulation.
 * Parameters: one FP32 device vector theta[KGS_HEAD_PARAMS] laid out as
 * W1 [64][16], b1 [64], W2 [64][64], b2 [64], W3 [3][64], b3 [3].
 * Features: [N][KGS_HEAD_FEATURES] BF16 bit patterns (16-byte aligned rows).
 * ------------------------------------------------------------------------ */
#define KGS_HEAD_FEATURES 16
#define KGS_HEAD_PARAMS 5443

/* Bytes of device workspace kgs_head_loss_grad needs (host only). */
kgs_status kgs_head_workspace_size(size_t* bytes);

/* Features of every Gaussian from a chunk's statistics, before the chunk is
 * merged (call it before kgs_accumulate_stats, which may reset the sums):
 *   0 S_d^(i,c) = kappa / n_views      1 L = ln(1 + gamma)     2 S_p^(i,c)
 *   3 ln(1 + |Omega|)                  4 kappa / |Omega|       5 views seen / n_views
 *   6 mean |dL/dmu2D| per view seen    7 ln(1 + max radius)    8 opacity
 *   9-11 log-scales, largest first     12 S_p(i) and 13 S_d(i) of `before` (0 if NULL)
 *   14 gamma / |Omega|                 15 1 if |Omega| > 0
 * (App. D: footprint, error mask, densification and pruning scores.)  stats
 * must hold all six accumulators; features: device [N][16] BF16. */
kgs_status kgs_head_features(kgs_ctx* ctx, const kgs_gaussians* g, const kgs_view_stats* stats, int32_t n_views,
                             const kgs_lifecycle_state* before, uint16_t* features, void* stream);

/* logits [N][3] (or NULL) and decision [N] = argmax, lower class on ties (or NULL). */
kgs_status kgs_head_forward(const float* theta, const uint16_t* features, int64_t n, float* logits,
                            uint8_t* decision, void* stream);

/* Class-weighted mean cross-entropy L = sum_n w_{y_n} CE_n / sum_n w_{y_n}
 * against labels [N] (0 KEEP, 1 DENSIFY, 2 PRUNE) with class_w device [3]:
 * writes grad [KGS_HEAD_PARAMS] = dL/dtheta and loss [1] (device).  The
 * backward rounds its GEMM operands (dL/dlogits and the masked hidden
 * gradients) to BF16 as the forward does.  Deterministic. */
kgs_status kgs_head_loss_grad(const float* theta, const uint16_t* features, const uint8_t* labels, int64_t n,
                              const float* class_w, void* workspace, size_t workspace_bytes, float* grad, float* loss,
                              void* stream);

/* One Adam step (bias-corrected, step >= 1) on theta with moments m, v. */
kgs_status kgs_head_adam(float* theta, float* m, float* v, const float* grad, int32_t step, float lr, float beta1,
                         float beta2, float eps, void* stream);

/* The whole chunk as described by kgs_chunk_desc. */
kgs_status kgs_chunk_run(kgs_ctx* ctx, const kgs_chunk_desc* desc, void* stream);

/* Record kgs_chunk_run into a HIP graph (stream capture) and launch it.  The
 * graph refers to ctx's workspace and state: destroy it before ctx, and run
 * no other work of ctx concurrently with a launch. */
kgs_status kgs_chunk_capture(kgs_ctx* ctx, const kgs_chunk_desc* desc, kgs_graph** out);
kgs_status kgs_chunk_launch(kgs_graph* graph, void* stream);
kgs_status kgs_graph_destroy(kgs_graph* graph);

/* Synchronous reads (the caller synchronises the stream first). */
kgs_status kgs_status_read(kgs_ctx* ctx, uint32_t* flags);
kgs_status kgs_status_clear(kgs_ctx* ctx, void* stream);
kgs_status kgs_counts_read(kgs_ctx* ctx, int64_t* n_slots, int64_t* n_pairs);
/* Device pointers into the workspace (valid until the next call on ctx).  It
 * first fills the slot_pairoff view from the records on the null stream and
 * waits for the device. */
kgs_status kgs_get_buffers(kgs_ctx* ctx, kgs_buffers* out);

const char* kgs_status_string(kgs_status s);

#ifdef __cplusplus
}
#endif
#endif /* KGS_H */
