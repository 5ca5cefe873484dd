// C ABI of the library: contexts over a caller-owned workspace, argument
// checks, the entry points declared in include/kgs.h, and HIP graph capture
// of a whole chunk.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "kgs_internal.h"

kgs_status kgs_launch_project(kgs_ctx*, const kgs_gaussians*, const kgs_camera*, int, const float*, hipStream_t);
kgs_status kgs_launch_bin_sort(kgs_ctx*, hipStream_t);
kgs_status kgs_launch_pairoff_copy(kgs_ctx*, hipStream_t);
kgs_status kgs_launch_pair_keys(kgs_ctx*, hipStream_t);
kgs_status kgs_launch_slot_view_copy(kgs_ctx*, hipStream_t);
kgs_status kgs_launch_render_fwd(kgs_ctx*, const kgs_image*, hipStream_t);
kgs_status kgs_launch_loss(kgs_ctx*, const float*, const kgs_image*, float*, float*, hipStream_t);
kgs_status kgs_launch_render_bwd(kgs_ctx*, const kgs_image*, const float*, const float*, const float*,
                                 const float*, float, hipStream_t, bool fuse_l1 = false, float* dl_out = nullptr);
void kgs_launch_loss_final(kgs_ctx*, float*, hipStream_t);
kgs_status kgs_launch_project_bwd(kgs_ctx*, const kgs_gaussians*, const kgs_camera*, int, const float*,
                                  const float*, const kgs_grads*, const kgs_view_stats*, hipStream_t, bool overwrite = false);
kgs_status kgs_launch_accumulate(kgs_ctx*, const kgs_view_stats*, int64_t, int, const kgs_lifecycle_state*, float,
                                 int, hipStream_t);
kgs_status kgs_launch_decide(kgs_ctx*, const kgs_lifecycle_state*, int64_t, double, uint8_t*, uint32_t*, uint32_t*,
                             hipStream_t);

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v);

kgs_status kgs_check_launch() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? KGS_OK : KGS_ERR_HIP;
}

namespace {

bool tile_ok(int w, int h) {
  return (w == 16 && h == 16) || (w == 8 && h == 32) || (w == 32 && h == 8) || (w == 32 && h == 16) ||
         (w == 16 && h == 32);
}
// 512-pixel tiles (eight waves per workgroup) stage at most 64 records at a time
bool tiling_ok(int w, int h, int batch) { return tile_ok(w, h) && !(w * h == 512 && batch > 64); }
bool batch_ok(int b) { return b == 32 || b == 64 || b == 128; }

int tiles_for(int W, int H, int tw, int th) { return ((W + tw - 1) / tw) * ((H + th - 1) / th); }

int max_tiles_of(int W, int H) {
  return std::max(tiles_for(W, H, 16, 16), std::max(tiles_for(W, H, 8, 32), tiles_for(W, H, 32, 8)));
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Walk the workspace layout; with base == nullptr only the size is computed.
size_t layout(const kgs_config& c, char* base, kgs_ctx* ctx) {
  const int64_t V = c.max_views, N = std::max<int64_t>(c.max_gaussians, 1);
  const int64_t nb = (N + KGS_BLOCK - 1) / KGS_BLOCK;
  const int64_t S = std::max<int64_t>(c.slot_capacity, 1), P = std::max<int64_t>(c.pair_capacity, 1);
  const int64_t T = (int64_t)max_tiles_of(c.width, c.height);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  char* p;
  p = take(sizeof(CamDev) * V);                 if (ctx) ctx->cams = (CamDev*)p;
  p = take(4 * V * N);                          if (ctx) ctx->vis = (uint32_t*)p;
  p = take(8 * V * nb);                         if (ctx) ctx->blk_cnt = (uint32_t*)p;
  p = take(8 * V * nb);                         if (ctx) ctx->blk_base = (uint32_t*)p;
  p = take(4 * 64);                             if (ctx) ctx->counters = (uint32_t*)p;
  p = take(64 * S);                             if (ctx) ctx->slot_rec = (float4*)p;
  p = take(4 * S);                              if (ctx) ctx->slot_gid = (uint32_t*)p;
  p = take(4 * S);                              if (ctx) ctx->slot_view = (uint32_t*)p;
  p = take(16 * S);                             if (ctx) ctx->slot_pix = (int4*)p;
  p = take(4 * S);                              if (ctx) ctx->slot_pairoff = (uint32_t*)p;
  p = take(4 * S);                              if (ctx) ctx->slot_ntiles = (uint32_t*)p;
  p = take(4 * P);                              if (ctx) ctx->keys[0] = (uint32_t*)p;
  p = take(4 * P);                              if (ctx) ctx->keys[1] = (uint32_t*)p;
  p = take(4 * P);                              if (ctx) ctx->vals[0] = (uint32_t*)p;
  p = take(4 * P);                              if (ctx) ctx->vals[1] = (uint32_t*)p;
  p = take(8 * S);                              if (ctx) ctx->slot_keys[0] = (uint64_t*)p;
  p = take(8 * S);                              if (ctx) ctx->slot_keys[1] = (uint64_t*)p;
  p = take(4 * S);                              if (ctx) ctx->slot_vals[0] = (uint32_t*)p;
  p = take(4 * S);                              if (ctx) ctx->slot_vals[1] = (uint32_t*)p;
  p = take(4 * (S / 64 + 2));                   if (ctx) ctx->group_part = (uint32_t*)p;
  p = take(8 * V * T);                          if (ctx) ctx->ranges = (uint2*)p;
  p = take(4 * V * T);                          if (ctx) ctx->tile_order = (uint32_t*)p;
  p = take(48 * P);                             if (ctx) ctx->pair_grad = (float4*)p;
  p = take(P + 16);                             if (ctx) ctx->pair_live = (uint8_t*)p;
  p = take(4 * KGS_RADIX_BUCKETS * KGS_SORT_BLOCKS); if (ctx) ctx->radix_hist = (uint32_t*)p;
  p = take(4 * KGS_RADIX_BUCKETS * KGS_MAX_PASSES); if (ctx) ctx->radix_total = (uint32_t*)p;
  p = take(4 * KGS_SLOT_WORDS * S);             if (ctx) ctx->slot_bwd = (float4*)p;
  p = take(4 * P);                              if (ctx) ctx->pair_slot = (uint32_t*)p;
  p = take(64 * (P / 64 + 2));                  if (ctx) ctx->seg_head = (float4*)p;
  p = take(64 * (P / 64 + 2));                  if (ctx) ctx->seg_tail = (float4*)p;
  p = take(24 * S);                             if (ctx) ctx->slot_pose = (float2*)p;
  p = take(4 * S);                              if (ctx) ctx->slot_live = (uint32_t*)p;
  p = take(4 * S);                              if (ctx) ctx->slot_om = (uint32_t*)p;
  p = take(4 * (P / 2048 + 2));                 if (ctx) ctx->chunk_first = (uint32_t*)p;
  p = take(16 * S);                             if (ctx) ctx->emit_rec = (uint4*)p;
  p = take(16 * S);                             if (ctx) ctx->emit_desc = (uint4*)p;
  {
    const int64_t st = std::max(kgs_scan_tiles(V * nb), kgs_scan_tiles(S / 64 + 2)) + 1;
    p = take(16 * st);                          if (ctx) ctx->scan_part = (unsigned long long*)p;
    p = take(16);                               if (ctx) ctx->scan_totals = (unsigned long long*)p;
  }
  p = take(48 * V * KGS_POSE_BLOCKS);           if (ctx) ctx->pose_partial = (double*)p;
  p = take(8 * V * T);                          if (ctx) ctx->loss_partial = (double*)p;
  p = take(4 * 9 * V * (int64_t)c.width * c.height); if (ctx) ctx->ssim_aux = (float*)p;
  p = take(8 * 9 * V * (int64_t)kgs_maploss_tiles(c.width, c.height)); if (ctx) ctx->ssim_partial = (double*)p;
  p = take(16 * (nb + 1));                      if (ctx) ctx->mm_partial = (double*)p;
  p = take(4 * (nb + 1));                       if (ctx) ctx->keep_partial = (uint32_t*)p;
  return off;
}

kgs_status config_check(const kgs_config* c) {
  if (!c) return KGS_ERR_INVALID_ARG;
  if (!tiling_ok(c->tile_w, c->tile_h, c->batch) || !batch_ok(c->batch)) return KGS_ERR_INVALID_ARG;
  if (c->sh_degree < 0 || c->sh_degree > 3) return KGS_ERR_INVALID_ARG;
  if (c->px_per_lane < 0 || c->px_per_lane > 2) return KGS_ERR_INVALID_ARG;
  if (c->width <= 0 || c->height <= 0 || c->width > 32000 || c->height > 32000) return KGS_ERR_INVALID_ARG;
  if (c->max_views < 1 || c->max_views > KGS_MAX_VIEWS) return KGS_ERR_INVALID_ARG;
  if (c->max_gaussians < 0 || c->max_gaussians >= (int64_t(1) << 32)) return KGS_ERR_INVALID_ARG;
  if (c->slot_capacity < 0 || c->slot_capacity >= (int64_t(1) << 32)) return KGS_ERR_INVALID_ARG;
  if (c->pair_capacity < 0 || c->pair_capacity >= (int64_t(1) << 32)) return KGS_ERR_INVALID_ARG;
  if (!(c->alpha_min > 0.f && c->alpha_min < 1.f) || !(c->alpha_max > 0.f && c->alpha_max <= 1.f))
    return KGS_ERR_INVALID_ARG;
  if (!(c->far_z > c->near_z)) return KGS_ERR_INVALID_ARG;
  if (!(c->t_min >= 0.f) || !(c->near_z > 0.f) || !(c->eps2d >= 0.f) || !(c->guard > 0.f)) return KGS_ERR_INVALID_ARG;
  // keys hold the global tile index in 32 bits
  if ((int64_t)c->max_views * max_tiles_of(c->width, c->height) >= (int64_t(1) << 31)) return KGS_ERR_INVALID_ARG;
  return KGS_OK;
}

void set_tiling(kgs_ctx* ctx) {
  ctx->tiles_x = (ctx->cfg.width + ctx->cfg.tile_w - 1) / ctx->cfg.tile_w;
  ctx->tiles_y = (ctx->cfg.height + ctx->cfg.tile_h - 1) / ctx->cfg.tile_h;
  ctx->n_tiles = ctx->tiles_x * ctx->tiles_y;
}

__global__ void k_clear_status(uint32_t* counters) {
  if (threadIdx.x < 3) counters[threadIdx.x] = 0u;
}

bool gaussians_ok(const kgs_ctx* ctx, const kgs_gaussians* g) {
  if (!g) return false;
  if (g->n < 0 || g->n > ctx->cfg.max_gaussians) return false;
  if (g->sh_degree < 0 || g->sh_degree > 3) return false;
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh)) return false;
  return true;
}

bool image_ok(const kgs_image* im) { return im && im->color && im->depth && im->t_final && im->last; }

}  // namespace

struct kgs_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
  kgs_ctx* ctx;
};

extern "C" {

void kgs_config_default(kgs_config* c, int32_t width, int32_t height) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->tile_w = 16;
  c->tile_h = 16;
  c->batch = 128;
  c->sh_degree = 3;
  c->alpha_min = 1.0f / 255.0f;
  c->alpha_max = 0.99f;
  c->t_min = 1e-4f;
  c->near_z = 0.2f;
  c->eps2d = 0.3f;
  c->guard = 1.3f;
  c->rect_margin = 1.0f / 256.0f;
  c->far_z = 1e30f;
  c->width = width;
  c->height = height;
  c->max_views = 1;
  c->max_gaussians = 0;
  c->slot_capacity = 0;
  c->pair_capacity = 0;
}

kgs_status kgs_workspace_size(const kgs_config* cfg, size_t* bytes) {
  const kgs_status s = config_check(cfg);
  if (s != KGS_OK || !bytes) return KGS_ERR_INVALID_ARG;
  *bytes = layout(*cfg, nullptr, nullptr);
  return KGS_OK;
}

kgs_status kgs_create(const kgs_config* cfg, void* workspace, size_t bytes, kgs_ctx** out) {
  if (config_check(cfg) != KGS_OK || !out || !workspace) return KGS_ERR_INVALID_ARG;
  if (((uintptr_t)workspace & 255u) != 0) return KGS_ERR_INVALID_ARG;
  if (bytes < layout(*cfg, nullptr, nullptr)) return KGS_ERR_INVALID_ARG;
  kgs_ctx* ctx = new (std::nothrow) kgs_ctx();
  if (!ctx) return KGS_ERR_INVALID_ARG;
  ctx->cfg = *cfg;
  ctx->ws = (char*)workspace;
  ctx->ws_bytes = bytes;
  ctx->max_tiles = max_tiles_of(cfg->width, cfg->height);
  ctx->nb_max = (std::max<int64_t>(cfg->max_gaussians, 1) + KGS_BLOCK - 1) / KGS_BLOCK;
  layout(*cfg, (char*)workspace, ctx);
  set_tiling(ctx);
  *out = ctx;
  return KGS_OK;
}

kgs_status kgs_destroy(kgs_ctx* ctx) {
  delete ctx;
  return KGS_OK;
}

kgs_status kgs_set_tiling(kgs_ctx* ctx, int32_t tile_w, int32_t tile_h, int32_t batch) {
  if (!ctx || !tiling_ok(tile_w, tile_h, batch) || !batch_ok(batch)) return KGS_ERR_INVALID_ARG;
  ctx->cfg.tile_w = tile_w;
  ctx->cfg.tile_h = tile_h;
  ctx->cfg.batch = batch;
  set_tiling(ctx);
  ctx->projected = 0;
  ctx->binned = 0;
  ctx->pixels_done = 0;
  return KGS_OK;
}

kgs_status kgs_project(kgs_ctx* ctx, const kgs_gaussians* g, const kgs_camera* cams, int32_t n_views,
                       const float* pose_xi, void* stream) {
  if (!ctx || !gaussians_ok(ctx, g) || !cams || n_views < 1 || n_views > ctx->cfg.max_views)
    return KGS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, st, ctx->counters);
  ctx->last_views = n_views;
  ctx->last_n = g->n;
  ctx->last_degree = g->sh_degree;
  ctx->proj_tile_w = ctx->cfg.tile_w;
  ctx->proj_tile_h = ctx->cfg.tile_h;
  const kgs_status s = kgs_launch_project(ctx, g, cams, n_views, pose_xi, st);
  ctx->projected = (s == KGS_OK);
  ctx->binned = 0;
  ctx->pixels_done = 0;
  return s;
}

kgs_status kgs_bin_sort(kgs_ctx* ctx, void* stream) {
  if (!ctx) return KGS_ERR_INVALID_ARG;
  if (!ctx->projected) return KGS_ERR_STATE;
  const kgs_status s = kgs_launch_bin_sort(ctx, (hipStream_t)stream);
  ctx->binned = (s == KGS_OK);
  ctx->pixels_done = 0;
  return s;
}

kgs_status kgs_render_fwd(kgs_ctx* ctx, const kgs_image* out, void* stream) {
  if (!ctx || !image_ok(out)) return KGS_ERR_INVALID_ARG;
  if (!ctx->binned) return KGS_ERR_STATE;
  return kgs_launch_render_fwd(ctx, out, (hipStream_t)stream);
}

kgs_status kgs_loss_l1(kgs_ctx* ctx, const float* target, const kgs_image* img, float* dl_dcolor, float* view_loss,
                       void* stream) {
  if (!ctx || !target || !img || !img->color || !dl_dcolor || !view_loss) return KGS_ERR_INVALID_ARG;
  if (!ctx->projected) return KGS_ERR_STATE;
  return kgs_launch_loss(ctx, target, img, dl_dcolor, view_loss, (hipStream_t)stream);
}

kgs_status kgs_loss_mapping(kgs_ctx* ctx, int32_t n_views, const kgs_image* img, const float* target,
                            const float* target_depth, float w_l1, float w_ssim, float lambda_g, float* dl_dcolor,
                            float* dl_ddepth, float* view_loss, float* geo_loss, void* stream) {
  if (!ctx || !img || !img->color || !target || !dl_dcolor || !view_loss) return KGS_ERR_INVALID_ARG;
  if (n_views < 1 || n_views > ctx->cfg.max_views) return KGS_ERR_INVALID_ARG;
  if (target_depth && (!img->depth || !dl_ddepth)) return KGS_ERR_INVALID_ARG;
  if (!(w_l1 >= 0.f) || !(w_ssim >= 0.f) || !(lambda_g >= 0.f)) return KGS_ERR_INVALID_ARG;
  return kgs_launch_loss_mapping(ctx, n_views, target, target_depth, img, w_l1, w_ssim, lambda_g, dl_dcolor,
                                 dl_ddepth, view_loss, geo_loss, (hipStream_t)stream);
}

kgs_status kgs_loss_iso(kgs_ctx* ctx, const kgs_gaussians* g, float lambda_iso, float* grad_log_scales, float* loss,
                        void* stream) {
  if (!ctx || !g || !g->log_scales || !loss || g->n < 0 || g->n > ctx->cfg.max_gaussians) return KGS_ERR_INVALID_ARG;
  if (!(lambda_iso >= 0.f)) return KGS_ERR_INVALID_ARG;
  return kgs_launch_loss_iso(ctx, g, lambda_iso, grad_log_scales, loss, (hipStream_t)stream);
}

kgs_status kgs_init_workspace_size(int32_t width, int32_t height, int32_t n_views, size_t* bytes) {
  if (!bytes || width <= 0 || height <= 0 || width > 32000 || height > 32000 || n_views < 1 || n_views > 65535)
    return KGS_ERR_INVALID_ARG;
  *bytes = kgs_init_ws_bytes(width, height, n_views);
  return KGS_OK;
}

kgs_status kgs_init_spawn(const float* color, const float* depth, const float* rendered, const float* rendered_depth,
                          const float* uniforms, const kgs_camera* cams, int32_t n_views, int32_t width,
                          int32_t height, void* workspace, size_t workspace_bytes, float* p_kf,
                          const kgs_spawn_list* out, void* stream) {
  if (!color || !depth || !uniforms || !cams || !workspace || !out) return KGS_ERR_INVALID_ARG;
  if (!out->pixel || !out->level || !out->voxel || !out->point || !out->count || out->capacity < 0)
    return KGS_ERR_INVALID_ARG;
  if ((rendered == nullptr) != (rendered_depth == nullptr)) return KGS_ERR_INVALID_ARG;
  size_t need = 0;
  if (kgs_init_workspace_size(width, height, n_views, &need) != KGS_OK || workspace_bytes < need)
    return KGS_ERR_INVALID_ARG;
  if (((uintptr_t)workspace & 255) != 0) return KGS_ERR_INVALID_ARG;
  return kgs_launch_init_spawn(color, depth, rendered, rendered_depth, uniforms, cams, n_views, width, height,
                               (char*)workspace, p_kf, out, (hipStream_t)stream);
}

// ---------------------------------------------------------------- map maintenance
namespace {
bool log2_cap_ok(int32_t l) { return l >= 4 && l <= 31; }
bool map_ws_ok(const void* ws, size_t bytes, int64_t n) {
  return ws && ((uintptr_t)ws & 255) == 0 && n >= 0 && bytes >= kgs_map_ws_bytes(n);
}
bool gout_ok(const kgs_gaussians_out* o) {
  return o && o->means && o->log_scales && o->quats && o->opacity_logits && o->sh && o->n >= 0 && o->sh_degree >= 0 &&
         o->sh_degree <= 3;
}
}  // namespace

kgs_status kgs_map_table_bytes(int32_t log2_capacity, size_t* bytes) {
  if (!bytes || !log2_cap_ok(log2_capacity)) return KGS_ERR_INVALID_ARG;
  *bytes = kgs_map_slot_bytes() << log2_capacity;
  return KGS_OK;
}

kgs_status kgs_map_table_clear(void* table, int32_t log2_capacity, void* stream) {
  if (!table || !log2_cap_ok(log2_capacity)) return KGS_ERR_INVALID_ARG;
  kgs_launch_map_clear(table, 1ull << log2_capacity, (hipStream_t)stream);
  return kgs_check_launch();
}

kgs_status kgs_map_workspace_size(int64_t max_items, size_t* bytes) {
  if (!bytes || max_items < 0 || max_items >= (int64_t(1) << 32)) return KGS_ERR_INVALID_ARG;
  *bytes = kgs_map_ws_bytes(max_items);
  return KGS_OK;
}

kgs_status kgs_map_voxel_keys(const int32_t* level, const int32_t* voxel, int64_t n, uint64_t* keys, void* stream) {
  if (n < 0 || (n > 0 && (!level || !voxel || !keys))) return KGS_ERR_INVALID_ARG;
  return kgs_launch_map_voxel_keys(level, voxel, n, (unsigned long long*)keys, (hipStream_t)stream);
}

kgs_status kgs_map_insert(void* table, int32_t log2_capacity, const uint64_t* keys, int64_t n,
                          const uint32_t* n_anchors_in, uint32_t* anchor, uint32_t* created, uint32_t* n_anchors_out,
                          uint32_t* status, void* workspace, size_t workspace_bytes, void* stream) {
  if (!table || !log2_cap_ok(log2_capacity) || !n_anchors_in || !n_anchors_out || !status) return KGS_ERR_INVALID_ARG;
  if (n < 0 || n >= (int64_t(1) << 32) || (n > 0 && !keys) || n_anchors_in == n_anchors_out) return KGS_ERR_INVALID_ARG;
  if (!map_ws_ok(workspace, workspace_bytes, n)) return KGS_ERR_INVALID_ARG;
  return kgs_launch_map_insert(table, 1ull << log2_capacity, (const unsigned long long*)keys, n, n_anchors_in, anchor,
                               created, n_anchors_out, status, (char*)workspace, (hipStream_t)stream);
}

kgs_status kgs_map_spawn(const uint32_t* created, const uint32_t* n_anchors_in, const uint32_t* n_anchors_out,
                         const int32_t* level, const int32_t* voxel, const float* color, int64_t n_candidates,
                         const kgs_gaussians_out* out, uint32_t* status, void* stream) {
  if (!created || !n_anchors_in || !n_anchors_out || !level || !voxel || !color || !gout_ok(out) || !status ||
      n_candidates < 0)
    return KGS_ERR_INVALID_ARG;
  return kgs_launch_map_spawn(created, n_anchors_in, n_anchors_out, level, voxel, color, n_candidates, out, status,
                              (hipStream_t)stream);
}

kgs_status kgs_map_densify_points(const kgs_gaussians* g, const uint8_t* decision, const double centre[3],
                                  int64_t capacity, int32_t* level, int32_t* voxel, float* point, uint32_t* source,
                                  uint32_t* count, void* workspace, size_t workspace_bytes, void* stream) {
  if (!g || !g->means || !g->log_scales || !g->quats || !decision || !centre || !level || !voxel || !point ||
      !source || !count || capacity < 0)
    return KGS_ERR_INVALID_ARG;
  if (!map_ws_ok(workspace, workspace_bytes, g->n)) return KGS_ERR_INVALID_ARG;
  return kgs_launch_map_densify(g, decision, centre, capacity, level, voxel, point, source, count, (char*)workspace,
                                (hipStream_t)stream);
}

kgs_status kgs_map_compact(const kgs_gaussians* g, const uint8_t* decision, const uint32_t* keep_map,
                           const kgs_gaussians_out* out, void* stream) {
  if (!g || !g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh || g->n < 0 || !decision ||
      !keep_map || !gout_ok(out) || out->sh_degree != g->sh_degree)
    return KGS_ERR_INVALID_ARG;
  return kgs_launch_map_compact(g, decision, keep_map, out, (hipStream_t)stream);
}

kgs_status kgs_map_align(float* means, float* quats, int64_t n, const int32_t* keyframe_of, const kgs_camera* old_poses,
                         const kgs_camera* new_poses, int32_t n_keyframes, void* stream) {
  if (n < 0 || n_keyframes < 1 || (n > 0 && (!means || !quats || !keyframe_of || !old_poses || !new_poses)))
    return KGS_ERR_INVALID_ARG;
  return kgs_launch_map_align(means, quats, n, keyframe_of, old_poses, new_poses, n_keyframes, (hipStream_t)stream);
}

kgs_status kgs_map_revoxelize(const float* means, const int32_t* level, int64_t n, void* table, int32_t log2_capacity,
                              uint8_t* keep, uint32_t* anchor, uint32_t* n_keep, uint32_t* status, void* workspace,
                              size_t workspace_bytes, void* stream) {
  if (!table || !log2_cap_ok(log2_capacity) || !n_keep || !status || n < 0 || n >= (int64_t(1) << 32))
    return KGS_ERR_INVALID_ARG;
  if (n > 0 && (!means || !level || !keep || !anchor)) return KGS_ERR_INVALID_ARG;
  if (!map_ws_ok(workspace, workspace_bytes, n)) return KGS_ERR_INVALID_ARG;
  return kgs_launch_map_revoxelize(means, level, n, table, 1ull << log2_capacity, keep, anchor, n_keep, status,
                                   (char*)workspace, (hipStream_t)stream);
}

kgs_status kgs_adam(float* theta, float* m, float* v, const float* grad, int64_t n, int32_t step, float lr, float beta1,
                    float beta2, float eps, void* stream) {
  if (n < 0 || step < 1 || (n > 0 && (!theta || !m || !v || !grad)) || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return KGS_ERR_INVALID_ARG;
  return kgs_launch_adam(theta, m, v, grad, n, step, lr, beta1, beta2, eps, (hipStream_t)stream);
}

kgs_status kgs_anchor_decode(const kgs_anchors* a, const float* theta, const kgs_camera* camera,
                             const kgs_gaussians_out* out, void* stream) {
  if (!a || !theta || !camera || !out || a->n < 0 || a->k < 1 || a->k > 16) return KGS_ERR_INVALID_ARG;
  if (a->n > 0 && (!a->p || !a->feat || !a->log_l || !a->offsets || !a->level)) return KGS_ERR_INVALID_ARG;
  if (((uintptr_t)a->feat & 15) != 0) return KGS_ERR_INVALID_ARG;
  if (!out->means || !out->log_scales || !out->quats || !out->opacity_logits || !out->sh || out->sh_degree != 0 ||
      out->n < a->n * a->k)
    return KGS_ERR_INVALID_ARG;
  return kgs_launch_anchor_decode(a, theta, *camera, out, (hipStream_t)stream);
}

kgs_status kgs_anchor_stats(kgs_ctx* ctx, const kgs_image* fwd, const uint32_t* anchor_of, int64_t n_anchors,
                            const float* target, float tau_err, const float* view_loss, uint32_t* counts,
                            const kgs_view_stats* stats, uint32_t* status, void* stream) {
  if (!ctx || !fwd || !fwd->color || !anchor_of || !target || !counts || !stats || !status || n_anchors < 0 ||
      n_anchors >= (int64_t(1) << 32) - 1)
    return KGS_ERR_INVALID_ARG;
  if (!ctx->binned) return KGS_ERR_STATE;
  return kgs_launch_anchor_stats(ctx, fwd, anchor_of, n_anchors, target, tau_err, view_loss, counts, stats, status,
                                 (hipStream_t)stream);
}

kgs_status kgs_render_bwd(kgs_ctx* ctx, const kgs_gaussians* g, const kgs_camera* cams, int32_t n_views,
                          const float* pose_xi, const kgs_image* fwd, const float* dl_dcolor, const float* dl_ddepth,
                          const float* dl_dtfinal, const float* target, float tau_err, const float* view_loss,
                          const kgs_grads* grads,
                          const kgs_view_stats* stats, void* stream) {
  if (!ctx || !gaussians_ok(ctx, g) || !cams || !image_ok(fwd) || !dl_dcolor || !grads) return KGS_ERR_INVALID_ARG;
  if (!ctx->binned) return KGS_ERR_STATE;
  if (n_views != ctx->last_views || g->n != ctx->last_n || g->sh_degree != ctx->last_degree) return KGS_ERR_STATE;
  hipStream_t st = (hipStream_t)stream;
  kgs_status s = kgs_launch_render_bwd(ctx, fwd, dl_dcolor, dl_ddepth, dl_dtfinal, target, tau_err, st);
  if (s != KGS_OK) return s;
  ctx->pixels_done = 1;
  return kgs_launch_project_bwd(ctx, g, cams, n_views, pose_xi, view_loss, grads, stats, st);
}

kgs_status kgs_render_bwd_pixels(kgs_ctx* ctx, const kgs_image* fwd, const float* dl_dcolor, const float* dl_ddepth,
                                 const float* dl_dtfinal, const float* target, float tau_err, void* stream) {
  if (!ctx || !image_ok(fwd) || !dl_dcolor) return KGS_ERR_INVALID_ARG;
  if (!ctx->binned) return KGS_ERR_STATE;
  const kgs_status s = kgs_launch_render_bwd(ctx, fwd, dl_dcolor, dl_ddepth, dl_dtfinal, target, tau_err,
                                             (hipStream_t)stream);
  ctx->pixels_done = (s == KGS_OK);
  return s;
}

kgs_status kgs_project_bwd(kgs_ctx* ctx, const kgs_gaussians* g, const kgs_camera* cams, int32_t n_views,
                           const float* pose_xi, const float* view_loss, const kgs_grads* grads,
                           const kgs_view_stats* stats, void* stream) {
  if (!ctx || !gaussians_ok(ctx, g) || !cams || !grads) return KGS_ERR_INVALID_ARG;
  // the per-pair records and live flags it sums come from kgs_render_bwd_pixels on this binning
  if (!ctx->binned || !ctx->pixels_done) return KGS_ERR_STATE;
  if (n_views != ctx->last_views || g->n != ctx->last_n || g->sh_degree != ctx->last_degree) return KGS_ERR_STATE;
  return kgs_launch_project_bwd(ctx, g, cams, n_views, pose_xi, view_loss, grads, stats, (hipStream_t)stream);
}

kgs_status kgs_accumulate_stats(kgs_ctx* ctx, const kgs_view_stats* stats, int64_t n, int32_t n_views,
                                const kgs_lifecycle_state* state, float tau_d, int32_t reset, void* stream) {
  if (!ctx || !stats || !state || n < 0 || n > ctx->cfg.max_gaussians || n_views < 1) return KGS_ERR_INVALID_ARG;
  if (!stats->kappa_sum || !stats->omega_sum || !stats->gamma_sum || !state->densify || !state->prune_score)
    return KGS_ERR_INVALID_ARG;
  return kgs_launch_accumulate(ctx, stats, n, n_views, state, tau_d, reset, (hipStream_t)stream);
}

kgs_status kgs_densify_prune_decide(kgs_ctx* ctx, const kgs_lifecycle_state* state, int64_t n, double tau_p,
                                    uint8_t* decision, uint32_t* keep_map, uint32_t* n_keep, void* stream) {
  if (!ctx || !state || !state->densify || !state->prune_score || !decision || n < 0 ||
      n > ctx->cfg.max_gaussians)
    return KGS_ERR_INVALID_ARG;
  return kgs_launch_decide(ctx, state, n, tau_p, decision, keep_map, n_keep, (hipStream_t)stream);
}

// ---------------------------------------------------------------- learned head
kgs_status kgs_head_workspace_size(size_t* bytes) {
  if (!bytes) return KGS_ERR_INVALID_ARG;
  *bytes = kgs_head_ws_bytes();
  return KGS_OK;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

kgs_status kgs_head_features(kgs_ctx* ctx, const kgs_gaussians* g, const kgs_view_stats* stats, int32_t n_views,
                             const kgs_lifecycle_state* before, uint16_t* features, void* stream) {
  if (!ctx || !gaussians_ok(ctx, g) || !stats || !features || !aligned16(features) || n_views < 1) return KGS_ERR_INVALID_ARG;
  if (!stats->kappa_sum || !stats->omega_sum || !stats->gamma_sum || !stats->grad_norm_sum || !stats->view_count ||
      !stats->max_radius)
    return KGS_ERR_INVALID_ARG;
  if (before && (!before->densify || !before->prune_score)) return KGS_ERR_INVALID_ARG;
  return kgs_launch_head_features(ctx, g, stats, n_views, before, features, (hipStream_t)stream);
}

kgs_status kgs_head_forward(const float* theta, const uint16_t* features, int64_t n, float* logits,
                            uint8_t* decision, void* stream) {
  if (!theta || n < 0 || (n > 0 && !features) || !aligned16(features)) return KGS_ERR_INVALID_ARG;
  return kgs_launch_head_forward(theta, features, n, logits, decision, (hipStream_t)stream);
}

kgs_status kgs_head_loss_grad(const float* theta, const uint16_t* features, const uint8_t* labels, int64_t n,
                              const float* class_w, void* workspace, size_t workspace_bytes, float* grad, float* loss,
                              void* stream) {
  if (!theta || n < 1 || !features || !aligned16(features) || !labels || !class_w || !workspace || !grad)
    return KGS_ERR_INVALID_ARG;
  if (workspace_bytes < kgs_head_ws_bytes() || ((uintptr_t)workspace & 255u)) return KGS_ERR_INVALID_ARG;
  return kgs_launch_head_train(theta, features, labels, n, class_w, (char*)workspace, grad, loss, (hipStream_t)stream);
}

kgs_status kgs_head_adam(float* theta, float* m, float* v, const float* grad, int32_t step, float lr, float beta1,
                         float beta2, float eps, void* stream) {
  if (!theta || !m || !v || !grad || step < 1 || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f))
    return KGS_ERR_INVALID_ARG;
  return kgs_launch_head_adam(theta, m, v, grad, step, lr, beta1, beta2, eps, (hipStream_t)stream);
}

static void fill_zero(void* p, uint64_t bytes, hipStream_t st) {
  if (!p || bytes == 0) return;
  const uint64_t words = bytes / 4;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<uint64_t>((words + 255) / 256, 2048)), dim3(256), 0, st,
                     (uint32_t*)p, words, 0u);
}

kgs_status kgs_chunk_run(kgs_ctx* ctx, const kgs_chunk_desc* d, void* stream) {
  if (!ctx || !d || !d->target || !d->dl_dcolor || !d->view_loss) return KGS_ERR_INVALID_ARG;
  if (!gaussians_ok(ctx, &d->gaussians) || d->n_views < 1 || d->n_views > ctx->cfg.max_views)
    return KGS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const uint64_t n = (uint64_t)d->gaussians.n;
  const uint64_t K = (uint64_t)(d->gaussians.sh_degree + 1) * (d->gaussians.sh_degree + 1);
  // with zero_accumulators the gather writes every Gaussian's gradients and
  // statistics and the pose reduction writes the pose gradient, so nothing
  // needs clearing first unless there are no Gaussians to gather over
  if (d->zero_accumulators && n == 0) {
    fill_zero(d->grads.means, 12 * n, st);
    fill_zero(d->grads.log_scales, 12 * n, st);
    fill_zero(d->grads.quats, 16 * n, st);
    fill_zero(d->grads.opacity_logits, 4 * n, st);
    fill_zero(d->grads.sh, 12 * K * n, st);
    fill_zero(d->grads.pose_xi, 24 * (uint64_t)d->n_views, st);
    fill_zero(d->stats.kappa_sum, 4 * n, st);
    fill_zero(d->stats.omega_sum, 4 * n, st);
    fill_zero(d->stats.gamma_sum, 8 * n, st);
    fill_zero(d->stats.grad_norm_sum, 4 * n, st);
    fill_zero(d->stats.view_count, 4 * n, st);
    fill_zero(d->stats.max_radius, 4 * n, st);
  }
  kgs_status s = kgs_project(ctx, &d->gaussians, d->cams, d->n_views, d->pose_xi, stream);
  if (s != KGS_OK) return s;
  if ((s = kgs_bin_sort(ctx, stream)) != KGS_OK) return s;
  if ((s = kgs_render_fwd(ctx, &d->image, stream)) != KGS_OK) return s;
  // the L1 loss and its gradient are formed inside the compositing backward
  // (the same values and partial sums as kgs_loss_l1), then the per-view losses
  if ((s = kgs_launch_render_bwd(ctx, &d->image, nullptr, nullptr, nullptr, d->target, d->tau_err, st, true,
                                 d->dl_dcolor)) != KGS_OK)
    return s;
  kgs_launch_loss_final(ctx, d->view_loss, st);
  s = kgs_launch_project_bwd(ctx, &d->gaussians, d->cams, d->n_views, d->pose_xi, d->view_loss, &d->grads, &d->stats,
                             st, d->zero_accumulators != 0 && n > 0);
  if (s != KGS_OK) return s;
  if (d->state.densify) {
    s = kgs_accumulate_stats(ctx, &d->stats, d->gaussians.n, d->n_views, &d->state, d->tau_d, 1, stream);
    if (s != KGS_OK) return s;
    if (d->decision)
      s = kgs_densify_prune_decide(ctx, &d->state, d->gaussians.n, d->tau_p, d->decision, nullptr, nullptr, stream);
  }
  return s;
}

kgs_status kgs_chunk_capture(kgs_ctx* ctx, const kgs_chunk_desc* d, kgs_graph** out) {
  if (!ctx || !d || !out) return KGS_ERR_INVALID_ARG;
  hipStream_t st;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return KGS_ERR_HIP;
  kgs_graph* g = new (std::nothrow) kgs_graph();
  if (!g) {
    hipStreamDestroy(st);
    return KGS_ERR_INVALID_ARG;
  }
  kgs_status s = KGS_OK;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) s = KGS_ERR_HIP;
  kgs_status run = KGS_OK;
  if (s == KGS_OK) run = kgs_chunk_run(ctx, d, st);
  hipGraph_t graph = nullptr;
  if (s == KGS_OK && hipStreamEndCapture(st, &graph) != hipSuccess) s = KGS_ERR_HIP;
  if (s == KGS_OK && run != KGS_OK) s = run;
  if (s == KGS_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) s = KGS_ERR_HIP;
  hipStreamDestroy(st);
  if (s != KGS_OK) {
    if (graph) hipGraphDestroy(graph);
    delete g;
    return s;
  }
  g->graph = graph;
  g->ctx = ctx;
  *out = g;
  return KGS_OK;
}

kgs_status kgs_chunk_launch(kgs_graph* g, void* stream) {
  if (!g) return KGS_ERR_INVALID_ARG;
  // the graph's own sort uses the depth keys its projection writes: a later
  // sort outside the graph builds them again
  g->ctx->slot_keys_ready = 0;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? KGS_OK : KGS_ERR_HIP;
}

kgs_status kgs_graph_destroy(kgs_graph* g) {
  if (!g) return KGS_OK;
  hipGraphExecDestroy(g->exec);
  hipGraphDestroy(g->graph);
  delete g;
  return KGS_OK;
}

kgs_status kgs_status_read(kgs_ctx* ctx, uint32_t* flags) {
  if (!ctx || !flags) return KGS_ERR_INVALID_ARG;
  return hipMemcpy(flags, ctx->counters + 2, sizeof(uint32_t), hipMemcpyDeviceToHost) == hipSuccess ? KGS_OK
                                                                                                       : KGS_ERR_HIP;
}

kgs_status kgs_status_clear(kgs_ctx* ctx, void* stream) {
  if (!ctx) return KGS_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, (hipStream_t)stream, ctx->counters);
  return kgs_check_launch();
}

kgs_status kgs_counts_read(kgs_ctx* ctx, int64_t* n_slots, int64_t* n_pairs) {
  if (!ctx) return KGS_ERR_INVALID_ARG;
  uint32_t c[2];
  if (hipMemcpy(c, ctx->counters, sizeof c, hipMemcpyDeviceToHost) != hipSuccess) return KGS_ERR_HIP;
  if (n_slots) *n_slots = c[0];
  if (n_pairs) *n_pairs = c[1];
  return KGS_OK;
}

kgs_status kgs_get_buffers(kgs_ctx* ctx, kgs_buffers* b) {
  if (!ctx || !b) return KGS_ERR_INVALID_ARG;
  // the per-record first pairs live in the records, the slots' views in their
  // emission descriptors, and a single-pass tile sort leaves the sorted keys
  // implicit in the ranges: the flat views are filled here
  if (kgs_launch_pairoff_copy(ctx, nullptr) != KGS_OK || kgs_launch_pair_keys(ctx, nullptr) != KGS_OK ||
      kgs_launch_slot_view_copy(ctx, nullptr) != KGS_OK || hipDeviceSynchronize() != hipSuccess)
    return KGS_ERR_HIP;
  b->n_slots = ctx->counters;
  b->n_pairs = ctx->counters + 1;
  b->slot_rec = (const float*)ctx->slot_rec;
  b->slot_gid = ctx->slot_gid;
  b->slot_view = ctx->slot_view;
  b->slot_pix = (const int32_t*)ctx->slot_pix;
  b->slot_pairoff = ctx->slot_pairoff;
  b->keys = ctx->keys[ctx->sorted_buf];
  b->sorted_slot = ctx->sorted_slot;
  b->ranges = (const uint32_t*)ctx->ranges;
  b->tiles_x = ctx->tiles_x;
  b->tiles_y = ctx->tiles_y;
  b->tile_bits = ctx->tile_bits;
  b->n_views = ctx->last_views;
  return KGS_OK;
}

const char* kgs_status_string(kgs_status s) {
  switch (s) {
    case KGS_OK: return "ok";
    case KGS_ERR_INVALID_ARG: return "invalid argument";
    case KGS_ERR_HIP: return "HIP error";
    case KGS_ERR_CAPACITY: return "device capacity exceeded";
    case KGS_ERR_NONFINITE: return "non-finite parameter";
    case KGS_ERR_STATE: return "call order violated";
  }
  return "unknown status";
}

}  // extern "C"
