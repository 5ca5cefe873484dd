// Internal definitions of the gfx950 rasterizer library: workspace layout,
// context, device camera, and the device helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/kgs.h"

#define KGS_BLOCK 256                 // threads per block for per-Gaussian / per-tile kernels
#define KGS_MAX_VIEWS 64
#define KGS_CNT_LIVE 4                  // counters[] word of the live-slot count
#define KGS_SORT_BLOCKS 1024          // fixed grid (one partition per block) of the radix sort passes
#define KGS_MAX_PASSES 8
#define KGS_RADIX_BUCKETS 1024      // widest digit of a radix pass: 10 bits
#define KGS_BWD_TWO_PX_MIN_WAVES 4096  // compositing backward, px_per_lane 0: two pixels per lane from 16 waves per CU
#define KGS_POSE_BLOCKS 256           // pieces per view of the pose reduction
#define KGS_SLOT_WORDS 24             // words of a slot's backward record

// ---------------------------------------------------------------- device camera
// Pose already applied.  The camera point of a Gaussian is R' mu + t' in
// FP64 (Rd, td).  The camera centre -R'^T t' (the origin of the view
// direction) is held as an unevaluated sum ctr + ctr_lo of two floats so that
// mu - centre keeps its accuracy for maps whose coordinates run to kilometres.
struct CamDev {
  float R[9];
  float ctr_lo[3];
  float ctr[3];
  float fx, fy, cx, cy;
  float lox, hix, loy, hiy;           // guard band on x/z and y/z
  int32_t W, H;
  int32_t pad0, pad1;
  double Jl[36];                      // SE(3) left Jacobian at xi, row major, (rho, phi) order
  double Rd[9], td[3];                // the posed world->camera transform in FP64
};

// Records hold the pixel-plane centre relative to the pixel (floor(W/2),
// floor(H/2)), so the FP32 value stays within half the image (plus the guard
// band) in magnitude.
__device__ __forceinline__ int pix_origin(int extent) { return extent >> 1; }

// Layout of the record depth-sort key: the view above the bits of the FP32
// depth minus those of a value just below near (depths are positive, so their
// bit patterns order like the values); 4-byte keys when both fit in 32 bits.
struct SlotKeyLayout {
  uint32_t depth_lo;
  int depth_bits, view_bits;
  bool key32() const { return depth_bits + view_bits <= 32; }
};
static inline SlotKeyLayout slot_key_layout(float near_z, float far_z, int V) {
  uint32_t near_b, far_b;
  __builtin_memcpy(&near_b, &near_z, 4);
  __builtin_memcpy(&far_b, &far_z, 4);
  SlotKeyLayout L;
  L.depth_lo = near_b > 4096u ? near_b - 4096u : 0u;
  const uint64_t span = (uint64_t)(far_b < 0x7f800000u ? far_b : 0x7f800000u) + 4096u - L.depth_lo;
  L.depth_bits = 1;
  while (L.depth_bits < 32 && (1ull << L.depth_bits) <= span) ++L.depth_bits;
  L.view_bits = 0;
  while ((1 << L.view_bits) < V) ++L.view_bits;
  return L;
}

// ---------------------------------------------------------------- context
struct kgs_ctx {
  kgs_config cfg;
  char* ws;
  size_t ws_bytes;
  int tiles_x, tiles_y, n_tiles;      // current tiling, per view
  int max_tiles;                      // max over supported tilings, per view
  int64_t nb_max;                     // blocks of 256 over max_gaussians
  // workspace carve-out
  CamDev* cams;                       // [max_views]
  uint32_t* vis;                      // [V][N] tile count after counting; slot index + 1 (0: none) after emission
  uint32_t* blk_cnt;                  // [max_views][nb][2] visible count, tile count
  uint32_t* blk_base;                 // [max_views][nb][2] exclusive bases
  uint32_t* counters;                 // [64]: 0 n_slots, 1 n_pairs, 2 status, 4 live slots, others free
  float4* slot_rec;                   // [S][4] compositing records, 64 bytes (the last: first pair)
  uint32_t* slot_gid;                 // [S]
  uint32_t* slot_view;                // [S] debug view only (filled from emit_desc on request)
  uint32_t* slot_ntiles;              // [S] tiles of each slot's rectangle (also in emit_desc.w)
  int4* slot_pix;                     // [S]
  uint32_t* slot_pairoff;             // [S]
  uint32_t* keys[2];                  // [P] ping-pong: global tile index of each pair
  uint32_t* vals[2];                  // [P] ping-pong (pair emission position)
  uint64_t* slot_keys[2];             // [S] ping-pong: (view << 32) | depth bits
  uint32_t* slot_vals[2];             // [S] ping-pong: slot index
  uint32_t* group_part;               // [S / 64 + 2] group partials of the pair-offset scan
  uint32_t* sorted_slot;              // [P] slot of each sorted pair (the sort's value buffer)
  uint2* ranges;                      // [max_views * max_tiles]
  uint32_t* tile_order;               // [max_views * max_tiles] compositing launch order, heaviest first
  float4* pair_grad;                  // [P][3] per-pair record-space gradients + counts
  uint8_t* pair_live;                 // [P] 1 where the compositing backward wrote the pair's record
  uint32_t* radix_hist;               // [KGS_RADIX_BUCKETS][KGS_SORT_BLOCKS] digit counts, then offsets, per partition
  uint32_t* radix_total;              // [KGS_MAX_PASSES][KGS_RADIX_BUCKETS]
  float4* slot_bwd;                   // [S][KGS_SLOT_WORDS / 4] per-slot backward records
  uint32_t* pair_slot;                // [P] slot of every pair, emission order
  float4* seg_head;                   // [P / 64 + 1][4] per 64-pair window: its first segment's partial sum
  float4* seg_tail;                   // [P / 64 + 1][4] and its last segment's
  float2* slot_pose;                  // [S][3] pose contributions (rho, phi) of every slot
  uint32_t* slot_live;                // [S] slots whose pixels blended somewhere, for the chain rule
  uint32_t* slot_om;                  // [S] pixels the slot blended (|Omega|): cleared by each compositing backward, set by its pair sums
  uint32_t* chunk_first;              // [P / 2048 + 2] record owning the first pair of each emission chunk
  uint4* emit_rec;                    // [S] emission descriptor of each record, in depth order
  uint4* emit_desc;                   // [S] the same without the record index, in record order (projection)
  int slot_keys_ready;                // the projection wrote the depth-sort keys; no sort has used them yet
  unsigned long long* scan_part;      // tile sums of the device-wide scans
  unsigned long long* scan_totals;    // [2] their totals
  double* pose_partial;               // [max_views][KGS_POSE_BLOCKS][6]
  double* loss_partial;               // [max_views * max_tiles] L1 loss per (view, tile)
  float* ssim_aux;                    // [max_views][3][3][H][W] SSIM derivative maps of the mapping loss
  double* ssim_partial;               // [max_views][3][mapping-loss tiles][3] per-tile loss sums
  double* mm_partial;                 // [nb][2]
  uint32_t* keep_partial;             // [nb + 1]
  // state
  int last_views;
  int64_t last_n;
  int last_degree;
  int tile_bits;                      // pair keys: (view << tile_bits) | tile, from the last bin_sort
  int sorted_buf;                     // which ping-pong buffer holds the sorted pairs
  int pair_keys_written;              // 0: the sorted keys were not written (single-pass tile sort)
  const uint32_t* perm;               // slots in (view, depth) order, from the last bin_sort
  int projected, binned, pixels_done;   // call order: project, bin_sort, (render_fwd,) render_bwd_pixels, project_bwd
  int proj_tile_w, proj_tile_h;
};

// ---------------------------------------------------------------- helpers
// floor(a / b) for b a power of two (every tile width and height is): an
// arithmetic shift, which rounds toward minus infinity like the floor
__device__ __forceinline__ int floordiv_pow2(int a, int b) { return a >> __builtin_ctz((unsigned)b); }

// lanes of the wave where pred holds (of those active); the compiler builtin
// takes the condition as a lane mask, so a compare feeds it without a round
// trip through a vector register
__device__ __forceinline__ uint64_t ballot64(bool pred) { return __builtin_amdgcn_ballot_w64(pred); }

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t mask_lt_count(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int l = (int)lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T u = __shfl_up(v, o, 64);
    if (l >= o) v += u;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// threads of the small per-view reductions (the loss finals)
#define KGS_FINAL_THREADS 256

// Sum over a KGS_FINAL_THREADS workgroup in a fixed order: a butterfly in each
// wave, then the four wave sums as (w0 + w1) + (w2 + w3).  Thread 0 gets the
// total; sh holds four values.  Every thread of the workgroup must call it.
__device__ __forceinline__ double block_sum_fixed(double v, double* sh) {
  static_assert(KGS_FINAL_THREADS == 256, "four waves");
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Block-wide (256 threads) exclusive scan of two u32 values in thread order.
// Returns the exclusive prefixes and the block totals.  Uses 16 words of LDS.
__device__ __forceinline__ void block_scan2(uint32_t a, uint32_t b, uint32_t* sh, uint32_t& ea, uint32_t& eb,
                                            uint32_t& ta, uint32_t& tb) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  uint32_t ia = wave_inclusive_scan(a), ib = wave_inclusive_scan(b);
  if (l == 63) { sh[w] = ia; sh[4 + w] = ib; }
  __syncthreads();
  uint32_t oa = 0, ob = 0;
  for (int k = 0; k < w; ++k) { oa += sh[k]; ob += sh[4 + k]; }
  ta = sh[0] + sh[1] + sh[2] + sh[3];
  tb = sh[4] + sh[5] + sh[6] + sh[7];
  ea = oa + ia - a;
  eb = ob + ib - b;
  __syncthreads();
}

// ---------------------------------------------------------------- projection
// Everything that decides visibility and the pixel rectangle of Gaussian i in
// one view.  Shared by the counting, emitting and backward kernels so that all
// three take identical decisions.
struct ProjCore {
  float tx, ty, tz;
  float ux, uy;          // x/z, y/z after the guard-band clamp
  int clx, cly;          // clamp active
  float J00, J02, J11, J12;
  float T0[3], T1[3];    // rows of J R'
  float a0[3], a1[3];    // Rq^T T0, Rq^T T1 (the rows of J R' Rq, before the scales)
  float v[3];            // Rq^T R'^T (ux, uy, 1)
  float K;               // fx fy / z^2
  float Sp00, Sp11;      // diagonal of J R' Sigma R'^T J^T (no low-pass term)
  float S00, S01, S11;   // 2D covariance with the low-pass term
  float det;
  float Pc, kc, Ec;      // conic as P (dx + k dy)^2 + E dy^2
  float rmx, rmy;        // pixel-plane centre minus 0.5 minus the record origin
  int fxi, fyi, rx, ry;  // integer centre and half extents
  int x0, x1, y0, y1;    // tile rectangle [x0, x1) x [y0, y1)
};

// x - camera centre, with the low part of the centre subtracted second.
__device__ __forceinline__ void cam_offset(const CamDev& c, const float x[3], float d[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) d[k] = (x[k] - c.ctr[k]) - c.ctr_lo[k];
}

// The 2D covariance S = M M^T + eps I with M = J R' Rq diag(s) (2x3), in a
// form FP32 keeps accurate for the long thin splats of nearby surfaces:
//   * the diagonal entries are sums of squares of the rows m0, m1 of M;
//   * det(M M^T) = |m0 x m1|^2 (Lagrange), and m0 x m1 = cof(diag s) Rq^T
//     (T0 x T1) with T0 x T1 = (fx fy / z^2) R'^T (ux, uy, 1) for a rotation
//     R', so det = K^2 |cof(s) v|^2 + eps (S'00 + S'11) + eps^2 is a sum of
//     non-negative terms (the textbook S00 S11 - S01^2 cancels to nothing in
//     FP32 when the splat is a thousand times longer than wide);
//   * the conic is kept in pivoted form q = P (dx + k dy)^2 + E dy^2 with
//     P = S11 / det, k = -S01 / S11, E = 1 / S11, which is the same quadratic
//     form with no cancellation between its terms.
// o: opacity.  Returns visibility.
__device__ __forceinline__ bool project_core(const CamDev& c, const float mu[3], const float Rq[9], const float s[3],
                                             float o, float near_z, float far_z, float eps2d, float rect_margin,
                                             float log_qscale,
                                             int tile_w, int tile_h, int tiles_x, int tiles_y, ProjCore& p) {
  // camera point and pixel-plane centre in FP64 (a few operations per
  // Gaussian and view; the centre's FP32 rounding error otherwise moves alpha
  // at the alpha_min contour by ~1e-3 for sharp splats at x ~ 1000)
  const double m0 = mu[0], m1 = mu[1], m2 = mu[2];
  const double X = c.Rd[0] * m0 + c.Rd[1] * m1 + c.Rd[2] * m2 + c.td[0];
  const double Y = c.Rd[3] * m0 + c.Rd[4] * m1 + c.Rd[5] * m2 + c.td[1];
  const double Z = c.Rd[6] * m0 + c.Rd[7] * m1 + c.Rd[8] * m2 + c.td[2];
  p.tx = (float)X;
  p.ty = (float)Y;
  p.tz = (float)Z;
  // near plane and the single-level distance mask, decided on the FP64 camera depth
  if (!(Z > (double)near_z) || !(Z < (double)far_z)) return false;
  const float iz = 1.0f / p.tz;
  float ux = p.tx * iz, uy = p.ty * iz;
  p.clx = 0;
  p.cly = 0;
  if (ux < c.lox) { ux = c.lox; p.clx = -1; } else if (ux > c.hix) { ux = c.hix; p.clx = 1; }
  if (uy < c.loy) { uy = c.loy; p.cly = -1; } else if (uy > c.hiy) { uy = c.hiy; p.cly = 1; }
  p.ux = ux;
  p.uy = uy;
  p.J00 = c.fx * iz;
  p.J02 = -c.fx * ux * iz;
  p.J11 = c.fy * iz;
  p.J12 = -c.fy * uy * iz;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    p.T0[k] = p.J00 * c.R[k] + p.J02 * c.R[6 + k];
    p.T1[k] = p.J11 * c.R[3 + k] + p.J12 * c.R[6 + k];
  }
  float w[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) w[k] = c.R[k] * ux + c.R[3 + k] * uy + c.R[6 + k];
  float q0[3], q1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    p.a0[k] = Rq[k] * p.T0[0] + Rq[3 + k] * p.T0[1] + Rq[6 + k] * p.T0[2];
    p.a1[k] = Rq[k] * p.T1[0] + Rq[3 + k] * p.T1[1] + Rq[6 + k] * p.T1[2];
    p.v[k] = Rq[k] * w[0] + Rq[3 + k] * w[1] + Rq[6 + k] * w[2];
    q0[k] = s[k] * p.a0[k];
    q1[k] = s[k] * p.a1[k];
  }
  p.Sp00 = q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2];
  p.Sp11 = q1[0] * q1[0] + q1[1] * q1[1] + q1[2] * q1[2];
  p.S01 = q0[0] * q1[0] + q0[1] * q1[1] + q0[2] * q1[2];
  p.S00 = p.Sp00 + eps2d;
  p.S11 = p.Sp11 + eps2d;
  p.K = c.fx * c.fy * iz * iz;
  const float h0 = s[1] * s[2] * p.v[0], h1 = s[0] * s[2] * p.v[1], h2 = s[0] * s[1] * p.v[2];
  const float Kh = p.K * p.K;
  p.det = Kh * (h0 * h0 + h1 * h1 + h2 * h2) + eps2d * (p.Sp00 + p.Sp11) + eps2d * eps2d;
  if (!(p.det > 0.0f) || !(p.S11 > 0.0f)) return false;
  p.Ec = 1.0f / p.S11;
  p.Pc = p.S11 / p.det;
  p.kc = -p.S01 * p.Ec;
  const double izd = 1.0 / Z;
  const double mxd = (double)c.fx * X * izd + (double)c.cx, myd = (double)c.fy * Y * izd + (double)c.cy;
  const float BIG = 16777216.0f;
  if (!(fabs(mxd) < (double)BIG && fabs(myd) < (double)BIG)) return false;
  p.rmx = (float)(mxd - 0.5 - (double)pix_origin(c.W));
  p.rmy = (float)(myd - 0.5 - (double)pix_origin(c.H));
  // alpha >= alpha_min needs q <= qmax = 2 ln(o / alpha_min); on that ellipse
  // |dx| <= sqrt(qmax Sxx) and |dy| <= sqrt(qmax Syy).
  const float qmax = 2.0f * (__logf(o) - log_qscale);
  float ex = ceilf(sqrtf(qmax * p.S00) * (1.0f + rect_margin));
  float ey = ceilf(sqrtf(qmax * p.S11) * (1.0f + rect_margin));
  ex = fminf(ex, BIG);
  ey = fminf(ey, BIG);
  p.rx = (int)ex;
  p.ry = (int)ey;
  p.fxi = (int)floor(mxd);
  p.fyi = (int)floor(myd);
  int x0 = floordiv_pow2(p.fxi - p.rx, tile_w), x1 = floordiv_pow2(p.fxi + p.rx, tile_w) + 1;
  int y0 = floordiv_pow2(p.fyi - p.ry, tile_h), y1 = floordiv_pow2(p.fyi + p.ry, tile_h) + 1;
  p.x0 = max(x0, 0);
  p.y0 = max(y0, 0);
  p.x1 = min(x1, tiles_x);
  p.y1 = min(y1, tiles_y);
  return p.x0 < p.x1 && p.y0 < p.y1;
}

// Unit quaternion (w, x, y, z) -> rotation.
__device__ __forceinline__ void quat_rotation(const float q[4], float R[9]) {
  const float w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
}


// Per-Gaussian, view-independent quantities.
struct GaussLocal {
  float mu[3];
  float qn[4], qnorm;
  float s[3];
  float Rq[9];
  float o;
  bool ok;
};

__device__ __forceinline__ void load_gaussian(const kgs_gaussians& g, int64_t i, float alpha_min, GaussLocal& G,
                                              bool& nonfinite) {
  const int64_t n = g.n;
  G.mu[0] = g.means[i];
  G.mu[1] = g.means[n + i];
  G.mu[2] = g.means[2 * n + i];
  float q[4] = {g.quats[i], g.quats[n + i], g.quats[2 * n + i], g.quats[3 * n + i]};
  float ls[3] = {g.log_scales[i], g.log_scales[n + i], g.log_scales[2 * n + i]};
  const float lg = g.opacity_logits[i];
  float chk = G.mu[0] + G.mu[1] + G.mu[2] + q[0] + q[1] + q[2] + q[3] + ls[0] + ls[1] + ls[2] + lg;
  nonfinite = !isfinite(chk);
  G.qnorm = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float iq = 1.0f / G.qnorm;
#pragma unroll
  for (int k = 0; k < 4; ++k) G.qn[k] = q[k] * iq;
#pragma unroll
  for (int k = 0; k < 3; ++k) G.s[k] = __expf(ls[k]);
  quat_rotation(G.qn, G.Rq);
  G.o = 1.0f / (1.0f + __expf(-lg));
  G.ok = !nonfinite && G.qnorm > 0.0f && G.o >= alpha_min;
}

// ---------------------------------------------------------------- spherical harmonics
// Real SH, Condon-Shortley phase, index l^2 + l + m, of a unit direction.
namespace sh {
constexpr float PI_F = 3.14159265358979323846f;
}
#define KGS_SQRT(x) __builtin_sqrtf(x)

__device__ __forceinline__ void sh_basis(int degree, float x, float y, float z, float* Y) {
  const float c0 = 0.5f * KGS_SQRT(1.0f / sh::PI_F);
  Y[0] = c0;
  if (degree < 1) return;
  const float c1 = KGS_SQRT(3.0f / (4.0f * sh::PI_F));
  Y[1] = -c1 * y;
  Y[2] = c1 * z;
  Y[3] = -c1 * x;
  if (degree < 2) return;
  const float a = 0.5f * KGS_SQRT(15.0f / sh::PI_F), b = 0.25f * KGS_SQRT(5.0f / sh::PI_F),
              cc = 0.25f * KGS_SQRT(15.0f / sh::PI_F);
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = a * x * y;
  Y[5] = -a * y * z;
  Y[6] = b * (2.f * zz - xx - yy);
  Y[7] = -a * x * z;
  Y[8] = cc * (xx - yy);
  if (degree < 3) return;
  const float d3a = 0.25f * KGS_SQRT(35.0f / (2.0f * sh::PI_F)), d3b = 0.5f * KGS_SQRT(105.0f / sh::PI_F),
              d3c = 0.25f * KGS_SQRT(21.0f / (2.0f * sh::PI_F)), d3d = 0.25f * KGS_SQRT(7.0f / sh::PI_F),
              d3e = 0.25f * KGS_SQRT(105.0f / sh::PI_F);
  Y[9] = -d3a * y * (3.f * xx - yy);
  Y[10] = d3b * x * y * z;
  Y[11] = -d3c * y * (4.f * zz - xx - yy);
  Y[12] = d3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
  Y[13] = -d3c * x * (4.f * zz - xx - yy);
  Y[14] = d3e * z * (xx - yy);
  Y[15] = -d3a * x * (xx - 3.f * yy);
}

// Gradient of the polynomial extensions above: dY[k] = (d/dx, d/dy, d/dz).
__device__ __forceinline__ void sh_basis_grad(int degree, float x, float y, float z, float (*dY)[3]) {
  dY[0][0] = dY[0][1] = dY[0][2] = 0.f;
  if (degree < 1) return;
  const float c1 = KGS_SQRT(3.0f / (4.0f * sh::PI_F));
  dY[1][0] = 0.f; dY[1][1] = -c1; dY[1][2] = 0.f;
  dY[2][0] = 0.f; dY[2][1] = 0.f; dY[2][2] = c1;
  dY[3][0] = -c1; dY[3][1] = 0.f; dY[3][2] = 0.f;
  if (degree < 2) return;
  const float a = 0.5f * KGS_SQRT(15.0f / sh::PI_F), b = 0.25f * KGS_SQRT(5.0f / sh::PI_F),
              cc = 0.25f * KGS_SQRT(15.0f / sh::PI_F);
  dY[4][0] = a * y;         dY[4][1] = a * x;         dY[4][2] = 0.f;
  dY[5][0] = 0.f;           dY[5][1] = -a * z;        dY[5][2] = -a * y;
  dY[6][0] = -2.f * b * x;  dY[6][1] = -2.f * b * y;  dY[6][2] = 4.f * b * z;
  dY[7][0] = -a * z;        dY[7][1] = 0.f;           dY[7][2] = -a * x;
  dY[8][0] = 2.f * cc * x;  dY[8][1] = -2.f * cc * y; dY[8][2] = 0.f;
  if (degree < 3) return;
  const float d3a = 0.25f * KGS_SQRT(35.0f / (2.0f * sh::PI_F)), d3b = 0.5f * KGS_SQRT(105.0f / sh::PI_F),
              d3c = 0.25f * KGS_SQRT(21.0f / (2.0f * sh::PI_F)), d3d = 0.25f * KGS_SQRT(7.0f / sh::PI_F),
              d3e = 0.25f * KGS_SQRT(105.0f / sh::PI_F);
  const float xx = x * x, yy = y * y, zz = z * z;
  dY[9][0] = -6.f * d3a * x * y;              dY[9][1] = -3.f * d3a * (xx - yy);          dY[9][2] = 0.f;
  dY[10][0] = d3b * y * z;                    dY[10][1] = d3b * x * z;                    dY[10][2] = d3b * x * y;
  dY[11][0] = 2.f * d3c * x * y;              dY[11][1] = -d3c * (4.f * zz - xx - 3.f * yy); dY[11][2] = -8.f * d3c * y * z;
  dY[12][0] = -6.f * d3d * x * z;             dY[12][1] = -6.f * d3d * y * z;             dY[12][2] = d3d * (6.f * zz - 3.f * xx - 3.f * yy);
  dY[13][0] = -d3c * (4.f * zz - 3.f * xx - yy); dY[13][1] = 2.f * d3c * x * y;           dY[13][2] = -8.f * d3c * x * z;
  dY[14][0] = 2.f * d3e * x * z;              dY[14][1] = -2.f * d3e * y * z;             dY[14][2] = d3e * (xx - yy);
  dY[15][0] = -3.f * d3a * (xx - yy);         dY[15][1] = 6.f * d3a * x * y;              dY[15][2] = 0.f;
}

// sum_k w[k] grad Y_k (gradient of the polynomial extensions of sh_basis).
__device__ __forceinline__ void sh_dir_grad(int degree, float x, float y, float z, const float* w, float g[3]) {
  g[0] = g[1] = g[2] = 0.f;
  if (degree < 1) return;
  const float c1 = KGS_SQRT(3.0f / (4.0f * sh::PI_F));
  g[1] -= c1 * w[1];
  g[2] += c1 * w[2];
  g[0] -= c1 * w[3];
  if (degree < 2) return;
  const float a = 0.5f * KGS_SQRT(15.0f / sh::PI_F), b = 0.25f * KGS_SQRT(5.0f / sh::PI_F),
              cc = 0.25f * KGS_SQRT(15.0f / sh::PI_F);
  g[0] += w[4] * a * y - w[6] * 2.f * b * x - w[7] * a * z + w[8] * 2.f * cc * x;
  g[1] += w[4] * a * x - w[5] * a * z - w[6] * 2.f * b * y - w[8] * 2.f * cc * y;
  g[2] += -w[5] * a * y + w[6] * 4.f * b * z - w[7] * a * x;
  if (degree < 3) return;
  const float d3a = 0.25f * KGS_SQRT(35.0f / (2.0f * sh::PI_F)), d3b = 0.5f * KGS_SQRT(105.0f / sh::PI_F),
              d3c = 0.25f * KGS_SQRT(21.0f / (2.0f * sh::PI_F)), d3d = 0.25f * KGS_SQRT(7.0f / sh::PI_F),
              d3e = 0.25f * KGS_SQRT(105.0f / sh::PI_F);
  const float xx = x * x, yy = y * y, zz = z * z;
  g[0] += -w[9] * 6.f * d3a * x * y + w[10] * d3b * y * z + w[11] * 2.f * d3c * x * y - w[12] * 6.f * d3d * x * z -
          w[13] * d3c * (4.f * zz - 3.f * xx - yy) + w[14] * 2.f * d3e * x * z - w[15] * 3.f * d3a * (xx - yy);
  g[1] += -w[9] * 3.f * d3a * (xx - yy) + w[10] * d3b * x * z - w[11] * d3c * (4.f * zz - xx - 3.f * yy) -
          w[12] * 6.f * d3d * y * z + w[13] * 2.f * d3c * x * y - w[14] * 2.f * d3e * y * z +
          w[15] * 6.f * d3a * x * y;
  g[2] += w[10] * d3b * x * y - w[11] * 8.f * d3c * y * z + w[12] * d3d * (6.f * zz - 3.f * xx - 3.f * yy) -
          w[13] * 8.f * d3c * x * z + w[14] * d3e * (xx - yy);
}

// ---------------------------------------------------------------- compositing
// Record of a projected Gaussian in the pixel loop (3 x float4):
//   r0 = (mu_x - 0.5 - ox, mu_y - 0.5 - oy, P', k)   r1 = (E', log2 o, depth, -)   r2 = (r, g, b, -)
// with (ox, oy) = (floor(W/2), floor(H/2)), P' = -P/2 log2(e), E' = -E/2 log2(e)
// for the pivoted conic q = P (dx + k dy)^2 + E dy^2.  For the pixel
// (px, py) = (x + ox, y + oy):  log2 alpha = log2 o + P' u^2 + E' dy^2 with
// u = dx + k dy, dx = x - r0.x, dy = y - r0.y (pixel centres at +0.5).  The
// same function is used by the forward and the backward pass so both take
// identical decisions.
__device__ __forceinline__ float log2_alpha(float px, float py, const float4& r0, float E, float lo, float& dy,
                                            float& u) {
  const float dx = px - r0.x;
  dy = py - r0.y;
  u = __fmaf_rn(r0.w, dy, dx);
  const float t = __fmaf_rn(E * dy, dy, lo);
  return __fmaf_rn(r0.z * u, u, t);
}

__device__ __forceinline__ float exp2_approx(float e) { return __builtin_amdgcn_exp2f(e); }

// Pixel of lane `l` of wave `w` in a tile: a tile of 64 NW pixels is NW 8x8
// sub-blocks, one per wave of its workgroup (NW = 4 for 16x16, 32x8, 8x32;
// NW = 8 for 32x16, 16x32).
__device__ __forceinline__ void tile_subblock(int tile_w, int w, int& sx, int& sy) {
  const int nsx = tile_w >> 3;  // sub-blocks per tile row, in row-major order
  sx = (w % nsx) * 8;
  sy = (w / nsx) * 8;
}

// Host-side kernel launch helpers (defined in kgs_api.hip).
kgs_status kgs_check_launch();

// Launch helpers of the lifecycle statistics and the learned head.
const double* kgs_launch_chunk_minmax(kgs_ctx* ctx, const kgs_view_stats* s, int64_t n, hipStream_t st);
int kgs_maploss_tiles(int W, int H);
size_t kgs_init_ws_bytes(int W, int H, int V);
kgs_status kgs_launch_adam(float* theta, float* m, float* v, const float* g, int64_t n, int32_t step, float lr,
                           float b1, float b2, float eps, hipStream_t st);
kgs_status kgs_launch_anchor_decode(const kgs_anchors* a, const float* theta, const kgs_camera& cam,
                                    const kgs_gaussians_out* out, hipStream_t st);
kgs_status kgs_launch_anchor_stats(kgs_ctx* ctx, const kgs_image* fwd, const uint32_t* anchor_of, int64_t n_anchor,
                                   const float* target, float tau_err, const float* view_loss, uint32_t* counts,
                                   const kgs_view_stats* stats, uint32_t* status, hipStream_t st);
size_t kgs_map_ws_bytes(int64_t n);
size_t kgs_map_slot_bytes();
void kgs_launch_map_clear(void* table, uint64_t cap, hipStream_t st);
kgs_status kgs_launch_map_insert(void* table, uint64_t cap, const unsigned long long* keys, int64_t n,
                                 const uint32_t* n_in, uint32_t* anchor, uint32_t* created, uint32_t* n_out,
                                 uint32_t* status, char* ws, hipStream_t st);
kgs_status kgs_launch_map_voxel_keys(const int32_t* level, const int32_t* vox, int64_t n, unsigned long long* keys,
                                     hipStream_t st);
kgs_status kgs_launch_map_spawn(const uint32_t* created, const uint32_t* n_in, const uint32_t* n_out,
                                const int32_t* level, const int32_t* vox, const float* color, int64_t n_cand,
                                const kgs_gaussians_out* g, uint32_t* status, hipStream_t st);
kgs_status kgs_launch_map_densify(const kgs_gaussians* g, const uint8_t* decision, const double centre[3],
                                  int64_t cap, int32_t* level, int32_t* vox, float* point, uint32_t* source,
                                  uint32_t* count, char* ws, hipStream_t st);
kgs_status kgs_launch_map_compact(const kgs_gaussians* g, const uint8_t* decision, const uint32_t* keep_map,
                                  const kgs_gaussians_out* out, hipStream_t st);
kgs_status kgs_launch_map_align(float* means, float* quats, int64_t n, const int32_t* keyframe_of,
                                const kgs_camera* old_pose, const kgs_camera* new_pose, int n_kf, hipStream_t st);
kgs_status kgs_launch_map_revoxelize(const float* means, const int32_t* level, int64_t n, void* table, uint64_t cap,
                                     uint8_t* keep, uint32_t* anchor, uint32_t* n_keep, uint32_t* status, char* ws,
                                     hipStream_t st);
kgs_status kgs_launch_init_spawn(const float* color, const float* depth, const float* rcolor, const float* rdepth,
                                 const float* u, const kgs_camera* cams, int V, int W, int H, char* ws,
                                 float* pkf_out, const kgs_spawn_list* out, hipStream_t st);
kgs_status kgs_launch_loss_mapping(kgs_ctx* ctx, int V, const float* target, const float* target_depth,
                                   const kgs_image* img, float w_l1, float w_ssim, float lambda_g,
                                   float* dl_dcolor, float* dl_ddepth, float* view_loss, float* geo_loss,
                                   hipStream_t st);
kgs_status kgs_launch_loss_iso(kgs_ctx* ctx, const kgs_gaussians* g, float lambda, float* grad, float* loss,
                               hipStream_t st);
size_t kgs_head_ws_bytes();
kgs_status kgs_launch_head_forward(const float* theta, const uint16_t* feat, int64_t n, float* logits,
                                   uint8_t* decision, hipStream_t st);
kgs_status kgs_launch_head_train(const float* theta, const uint16_t* feat, const uint8_t* labels, int64_t n,
                                 const float* cw, char* ws, float* grad, float* loss, hipStream_t st);
kgs_status kgs_launch_head_adam(float* theta, float* m, float* v, const float* grad, int32_t step, float lr,
                                float b1, float b2, float eps, hipStream_t st);
kgs_status kgs_launch_head_features(kgs_ctx* ctx, const kgs_gaussians* g, const kgs_view_stats* stats, int V,
                                    const kgs_lifecycle_state* before, uint16_t* feat, hipStream_t st);

// ---------------------------------------------------------------- compositing (kgs_render.hip, kgs_anchor.hip)
// a compile-time flag passed as a value (selects a variant of a generic lambda)
template <bool V>
struct BoolC {
  static constexpr bool value = V;
};

struct RenderParams {
  int W, H, tile_w, tile_h, tiles_x, tiles_y, n_tiles;
  float log2_amin, amax, tmin;
  float bg0, bg1, bg2;
  // a record with log2 o below this reaches alpha_max at no pixel (see render_params)
  float log2_amax_lo;
};

// Whether the footprint {log2 alpha >= log2 alpha_min} of a record can reach
// the pixel-centre box [x0, x1] x [y0, y1] (record coordinates): the minimum
// of q = A (x + k y)^2 + C y^2 over the box (A = -P', C = -E') against
// tau = log2 o - log2 alpha_min.  q is convex, so the minimum is 0 with the
// centre inside the box, else on an edge: y = y0 or y1 at x = clamp(-k y),
// x = x0 or x1 at y = clamp(-A k x / (A k^2 + C)).  The margin keeps the test
// conservative against the rounding of the per-pixel evaluation.
__device__ __forceinline__ bool footprint_meets_box(float x0, float x1, float y0, float y1, const float4& r0,
                                                    const float4& r1, float log2_amin) {
  const float A = -r0.z, k = r0.w, C = -r1.x;
  const float tau = r1.y - log2_amin;
  if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return true;
  const float s = A * k * __builtin_amdgcn_rcpf(fmaf(A * k, k, C));
  float f;
  {
    const float xa = fminf(fmaxf(-k * y0, x0), x1), ua = fmaf(k, y0, xa);
    const float xb = fminf(fmaxf(-k * y1, x0), x1), ub = fmaf(k, y1, xb);
    f = fminf(fmaf(A * ua, ua, C * y0 * y0), fmaf(A * ub, ub, C * y1 * y1));
  }
  {
    const float ya = fminf(fmaxf(-s * x0, y0), y1), ua = fmaf(k, ya, x0);
    const float yb = fminf(fmaxf(-s * x1, y0), y1), ub = fmaf(k, yb, x1);
    f = fminf(f, fminf(fmaf(A * ua, ua, C * ya * ya), fmaf(A * ub, ub, C * yb * yb)));
  }
  return f <= tau + 1e-3f * (1.0f + tau);
}

// Bits of the tile index in a pair key: tiles < 2^bits, so the padding key
// (all ones) sorts after every tile of its view.
static inline int kgs_tile_bits(int n_tiles) {
  int b = 1;
  while ((1u << b) <= (uint32_t)n_tiles) ++b;
  return b;
}

static inline int tile_waves(const kgs_ctx* ctx) { return ctx->cfg.tile_w * ctx->cfg.tile_h / 64; }

static inline RenderParams render_params(const kgs_ctx* ctx) {
  RenderParams P;
  P.W = ctx->cfg.width;
  P.H = ctx->cfg.height;
  P.tile_w = ctx->cfg.tile_w;
  P.tile_h = ctx->cfg.tile_h;
  P.tiles_x = ctx->tiles_x;
  P.tiles_y = ctx->tiles_y;
  P.n_tiles = ctx->n_tiles;
  P.log2_amin = log2f(ctx->cfg.alpha_min);
  P.amax = ctx->cfg.alpha_max;
  P.tmin = ctx->cfg.t_min;
  P.bg0 = ctx->cfg.bg[0];
  P.bg1 = ctx->cfg.bg[1];
  P.bg2 = ctx->cfg.bg[2];
  // log2 alpha <= log2 o at every pixel (the quadratic form is negative
  // semi-definite and its rounded terms keep their signs), and the hardware
  // exp2 errs by a few ulp, far below the 1e-3 margin: below this bound
  // exp2(log2 alpha) < alpha_max, so the clamp at alpha_max is the identity
  P.log2_amax_lo = log2f(ctx->cfg.alpha_max) - 1e-3f;
  return P;
}


// Device-wide exclusive scan (kgs_scan.hip): W (1 or 2) interleaved u32 values
// per entry, u64 accumulation, outputs clamped at cap0 / cap1; in may equal
// out.  part needs W * kgs_scan_tiles(entries) u64, totals W u64.
int64_t kgs_scan_tiles(int64_t entries);
void kgs_launch_scan(const uint32_t* in, uint32_t* out, int64_t entries, int W, unsigned long long cap0,
                     unsigned long long cap1, unsigned long long* part, unsigned long long* totals, hipStream_t st);
