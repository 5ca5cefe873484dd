// Probabilistic Gaussian initialisation (Sec. 3.3, "Probabilistic Gaussian
// Initialization") and the level-of-detail voxel rule (Sec. 3.2, "Hierarchical
// Anchor Management") for a batch of keyframes:
//   DoG   = min(|(G_s1 - G_s2) * I|, 1)                I: mean of the three channels
//   P     = min(lambda DoG + (1 - lambda) norm(||grad D||), 1)
//   P_kf  = max(P - P^, 0)                             P^: the same map of the render
//   3x3 non-maximum suppression over P_kf; a kept pixel spawns when u < P_kf
//   and its depth is positive; it is unprojected at its pixel centre and
//   quantised at the level of its camera distance, idx = floor(x / eps_l).
// Readings (the paper names none of these): s1 = 1, s2 = 1.6, blur radius
// round(3 s) with the border pixel repeated; central differences of D inside
// the image, one-sided on its border; min-max normalisation over the image;
// eps = (0.1, 0.25, 1, 5, 25) and level l for distances below 100 eps_l.
//
// Everything that decides an integer (the suppression, u < P_kf, the level and
// the floor) is evaluated in FP64, with the products and sums in the order of
// the definitions and no fused multiply-adds, so the GPU's decisions are the
// FP64 ones.  The image work is a few hundred FP64 operations per pixel on
// 1242x375 keyframes: the passes are bound by their HBM traffic and launches.
//
// Passes: (1) per 32x16 tile of each keyframe (and of its render), the two
// blurs from an LDS-staged halo, the DoG, the depth-gradient norm and its tile
// min / max; (2) min / max per keyframe; (3) P_kf per pixel; (4) per 256-pixel
// row segment the spawning flags and their count; (5) a device-wide scan of the
// counts; (6) the spawning pixels again, each written at its segment's offset
// plus its rank, so the list is in (keyframe, row, column) order.
#include <cmath>

#include "kgs_internal.h"

#define IN_TW 32
#define IN_TH 16
#define IN_R 5                       // radius of the wider blur
#define IN_RW (IN_TW + 2 * IN_R)
#define IN_RH (IN_TH + 2 * IN_R)
#define IN_R1 3                      // radius of the narrower blur
#define IN_SEG 256

struct InitParams {
  double w1[2 * IN_R1 + 1];
  double w2[2 * IN_R + 1];
  double lambda, one_minus_lambda;
  double eps[5], dmax[4];
  int W, H, V, tiles_x, n_tiles, n_seg;
  int has_render;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Pass 1.  grid (tiles, V, 1 + has_render); z = 0 the keyframe, z = 1 its render.
__global__ __launch_bounds__(256) void k_init_saliency(InitParams P, const float* __restrict__ color,
                                                       const float* __restrict__ depth,
                                                       const float* __restrict__ rcolor,
                                                       const float* __restrict__ rdepth, double* __restrict__ dog,
                                                       double* __restrict__ gnorm, double* __restrict__ part) {
#pragma clang fp contract(off)
  __shared__ double sg[IN_RH][IN_RW];
  __shared__ double h1[IN_RH][IN_TW], h2[IN_RH][IN_TW];
  __shared__ double rmin[4], rmax[4];
  const int tile = blockIdx.x, v = blockIdx.y, which = blockIdx.z;
  const int tx = tile % P.tiles_x, ty = tile / P.tiles_x;
  const size_t npix = (size_t)P.W * P.H;
  const float* C = (which ? rcolor : color) + (size_t)v * 3 * npix;
  const float* D = (which ? rdepth : depth) + (size_t)v * npix;
  for (int i = threadIdx.x; i < IN_RH * IN_RW; i += 256) {
    const int r = i / IN_RW, c = i - r * IN_RW;
    const int gx = clampi(tx * IN_TW - IN_R + c, 0, P.W - 1), gy = clampi(ty * IN_TH - IN_R + r, 0, P.H - 1);
    const size_t q = (size_t)gy * P.W + gx;
    sg[r][c] = (((double)C[q] + (double)C[npix + q]) + (double)C[2 * npix + q]) / 3.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < IN_RH * IN_TW; i += 256) {
    const int r = i / IN_TW, c = i - r * IN_TW;
    double a = 0.0, b = 0.0;
    for (int j = 0; j <= 2 * IN_R1; ++j) a = a + P.w1[j] * sg[r][c + IN_R - IN_R1 + j];
    for (int j = 0; j <= 2 * IN_R; ++j) b = b + P.w2[j] * sg[r][c + j];
    h1[r][c] = a;
    h2[r][c] = b;
  }
  __syncthreads();
  double lo = INFINITY, hi = -INFINITY;
  for (int k = 0; k < 2; ++k) {
    const int oy = (threadIdx.x >> 5) + 8 * k, ox = threadIdx.x & 31;
    const int px = tx * IN_TW + ox, py = ty * IN_TH + oy;
    if (px >= P.W || py >= P.H) continue;
    double a = 0.0, b = 0.0;
    for (int j = 0; j <= 2 * IN_R1; ++j) a = a + P.w1[j] * h1[oy + IN_R - IN_R1 + j][ox];
    for (int j = 0; j <= 2 * IN_R; ++j) b = b + P.w2[j] * h2[oy + j][ox];
    const size_t q = (size_t)py * P.W + px;
    const size_t o = ((size_t)which * P.V + v) * npix + q;
    dog[o] = fmin(fabs(a - b), 1.0);
    double gx = 0.0, gy = 0.0;
    if (P.W > 1) {
      if (px == 0) gx = (double)D[q + 1] - (double)D[q];
      else if (px == P.W - 1) gx = (double)D[q] - (double)D[q - 1];
      else gx = ((double)D[q + 1] - (double)D[q - 1]) / 2.0;
    }
    if (P.H > 1) {
      if (py == 0) gy = (double)D[q + P.W] - (double)D[q];
      else if (py == P.H - 1) gy = (double)D[q] - (double)D[q - P.W];
      else gy = ((double)D[q + P.W] - (double)D[q - P.W]) / 2.0;
    }
    const double g = sqrt(gx * gx + gy * gy);
    gnorm[o] = g;
    lo = fmin(lo, g);
    hi = fmax(hi, g);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    rmin[threadIdx.x >> 6] = lo;
    rmax[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* pp = part + (((size_t)which * P.V + v) * P.n_tiles + tile) * 2;
    pp[0] = fmin(fmin(rmin[0], rmin[1]), fmin(rmin[2], rmin[3]));
    pp[1] = fmax(fmax(rmax[0], rmax[1]), fmax(rmax[2], rmax[3]));
  }
}

// Pass 2.  grid (V, 1 + has_render): min / max of the depth-gradient norm over the image.
__global__ __launch_bounds__(256) void k_init_minmax(InitParams P, const double* __restrict__ part,
                                                     double* __restrict__ mm) {
  __shared__ double rmin[4], rmax[4];
  const int v = blockIdx.x, which = blockIdx.y;
  const double* pp = part + ((size_t)which * P.V + v) * P.n_tiles * 2;
  double lo = INFINITY, hi = -INFINITY;
  for (int t = threadIdx.x; t < P.n_tiles; t += 256) {
    lo = fmin(lo, pp[2 * t]);
    hi = fmax(hi, pp[2 * t + 1]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    rmin[threadIdx.x >> 6] = lo;
    rmax[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = mm + ((size_t)which * P.V + v) * 2;
    o[0] = fmin(fmin(rmin[0], rmin[1]), fmin(rmin[2], rmin[3]));
    o[1] = fmax(fmax(rmax[0], rmax[1]), fmax(rmax[2], rmax[3]));
  }
}

__device__ __forceinline__ double prob_at(const InitParams& P, const double* dog, const double* gnorm,
                                          const double* mm, int which, int v, size_t q) {
#pragma clang fp contract(off)
  const size_t npix = (size_t)P.W * P.H;
  const size_t o = ((size_t)which * P.V + v) * npix + q;
  const double lo = mm[((size_t)which * P.V + v) * 2], hi = mm[((size_t)which * P.V + v) * 2 + 1];
  const double n = hi > lo ? (gnorm[o] - lo) / (hi - lo) : 0.0;
  return fmin(P.lambda * dog[o] + P.one_minus_lambda * n, 1.0);
}

// Pass 3.  P_kf per pixel (FP64 map; an FP32 copy on request).
__global__ __launch_bounds__(256) void k_init_pkf(InitParams P, const double* __restrict__ dog,
                                                  const double* __restrict__ gnorm, const double* __restrict__ mm,
                                                  double* __restrict__ pkf, float* __restrict__ pkf_out) {
#pragma clang fp contract(off)
  const size_t npix = (size_t)P.W * P.H;
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int v = blockIdx.y;
  if (q >= npix) return;
  double p = prob_at(P, dog, gnorm, mm, 0, v, q);
  if (P.has_render) p = fmax(p - prob_at(P, dog, gnorm, mm, 1, v, q), 0.0);
  pkf[(size_t)v * npix + q] = p;
  if (pkf_out) pkf_out[(size_t)v * npix + q] = (float)p;
}

// A pixel spawns: P_kf > 0, not below any in-image 3x3 neighbour, u < P_kf and depth > 0.
__device__ __forceinline__ bool spawns(const InitParams& P, const double* pkf, const float* u, const float* depth,
                                       int v, int x, int y) {
  const size_t npix = (size_t)P.W * P.H;
  const double* M = pkf + (size_t)v * npix;
  const size_t q = (size_t)y * P.W + x;
  const double p = M[q];
  if (!(p > 0.0)) return false;
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      const int xx = x + dx, yy = y + dy;
      if ((dx || dy) && xx >= 0 && xx < P.W && yy >= 0 && yy < P.H && p < M[(size_t)yy * P.W + xx]) return false;
    }
  return (double)u[(size_t)v * npix + q] < p && (double)depth[(size_t)v * npix + q] > 0.0;
}

// Pass 4.  grid (n_seg, H, V): spawning pixels per 256-pixel row segment.
__global__ __launch_bounds__(IN_SEG) void k_init_count(InitParams P, const double* __restrict__ pkf,
                                                       const float* __restrict__ u, const float* __restrict__ depth,
                                                       uint32_t* __restrict__ counts) {
  __shared__ uint32_t sc[IN_SEG / 64];
  const int seg = blockIdx.x, y = blockIdx.y, v = blockIdx.z;
  const int x = seg * IN_SEG + threadIdx.x;
  const bool f = x < P.W && spawns(P, pkf, u, depth, v, x, y);
  const uint32_t c = (uint32_t)__popcll(ballot64(f));
  if ((threadIdx.x & 63) == 0) sc[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0)
    counts[((size_t)v * P.H + y) * P.n_seg + seg] = (sc[0] + sc[1]) + (sc[2] + sc[3]);
}

// Pass 6.  The spawning pixels at their segment's offset plus their rank in the segment.
__global__ __launch_bounds__(IN_SEG) void k_init_emit(InitParams P, const double* __restrict__ pkf,
                                                      const float* __restrict__ u, const float* __restrict__ color,
                                                      const float* __restrict__ depth,
                                                      const kgs_camera* __restrict__ cams,
                                                      const uint32_t* __restrict__ offsets, int64_t cap,
                                                      int32_t* __restrict__ o_pixel, int32_t* __restrict__ o_level,
                                                      int32_t* __restrict__ o_voxel, float* __restrict__ o_point,
                                                      float* __restrict__ o_color) {
#pragma clang fp contract(off)
  __shared__ uint32_t sc[IN_SEG / 64];
  const int seg = blockIdx.x, y = blockIdx.y, v = blockIdx.z;
  const int x = seg * IN_SEG + threadIdx.x;
  const bool f = x < P.W && spawns(P, pkf, u, depth, v, x, y);
  const uint64_t b = ballot64(f);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sc[w] = (uint32_t)__popcll(b);
  __syncthreads();
  if (!f) return;
  uint32_t rank = mask_lt_count(b);
  for (int k = 0; k < w; ++k) rank += sc[k];
  const uint64_t slot = (uint64_t)offsets[((size_t)v * P.H + y) * P.n_seg + seg] + rank;
  if (slot >= (uint64_t)cap) return;
  const kgs_camera c = cams[v];
  const size_t npix = (size_t)P.W * P.H;
  const size_t q = (size_t)y * P.W + x;
  const double z = (double)depth[(size_t)v * npix + q];
  const double xc0 = z * ((double)x + 0.5 - (double)c.cx) / (double)c.fx;
  const double xc1 = z * ((double)y + 0.5 - (double)c.cy) / (double)c.fy;
  const double xc2 = z;
  const double d0 = xc0 - (double)c.t[0], d1 = xc1 - (double)c.t[1], d2 = xc2 - (double)c.t[2];
  double X[3], ctr[3];
  for (int i = 0; i < 3; ++i) {
    // world point R^T (x_cam - t) and camera centre -R^T t
    X[i] = ((double)c.R[i] * d0 + (double)c.R[3 + i] * d1) + (double)c.R[6 + i] * d2;
    ctr[i] = -(((double)c.R[i] * (double)c.t[0] + (double)c.R[3 + i] * (double)c.t[1]) +
               (double)c.R[6 + i] * (double)c.t[2]);
  }
  const double e0 = X[0] - ctr[0], e1 = X[1] - ctr[1], e2 = X[2] - ctr[2];
  const double dist = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
  int lev = 4;
  for (int l = 3; l >= 0; --l)
    if (dist < P.dmax[l]) lev = l;
  const double eps = P.eps[lev];
  o_pixel[2 * slot] = v;
  o_pixel[2 * slot + 1] = (int32_t)q;
  o_level[slot] = lev;
  for (int i = 0; i < 3; ++i) {
    o_voxel[3 * slot + i] = (int32_t)floor(X[i] / eps);
    o_point[3 * slot + i] = (float)X[i];
    if (o_color) o_color[3 * slot + i] = color[((size_t)v * 3 + i) * npix + q];
  }
}

__global__ void k_init_total(const unsigned long long* __restrict__ tot, uint32_t* __restrict__ count) {
  if (threadIdx.x == 0) *count = (uint32_t)min(*tot, 0xffffffffull);
}

// ---------------------------------------------------------------- host side
namespace {
struct InitLayout {
  size_t dog, gnorm, pkf, part, mm, counts, offsets, scan_part, scan_tot, total;
};
InitLayout init_layout(int W, int H, int V) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t npix = (size_t)W * H;
  const int n_tiles = ((W + IN_TW - 1) / IN_TW) * ((H + IN_TH - 1) / IN_TH);
  const int64_t n_seg = (W + IN_SEG - 1) / IN_SEG;
  const int64_t entries = (int64_t)V * H * n_seg;
  InitLayout L;
  size_t off = 0;
  L.dog = off; off = al(off + 8 * 2 * (size_t)V * npix);
  L.gnorm = off; off = al(off + 8 * 2 * (size_t)V * npix);
  L.pkf = off; off = al(off + 8 * (size_t)V * npix);
  L.part = off; off = al(off + 16 * 2 * (size_t)V * n_tiles);
  L.mm = off; off = al(off + 16 * 2 * (size_t)V);
  L.counts = off; off = al(off + 4 * (size_t)entries);
  L.offsets = off; off = al(off + 4 * (size_t)entries);
  L.scan_part = off; off = al(off + 16 * (size_t)(kgs_scan_tiles(entries) + 1));
  L.scan_tot = off; off = al(off + 16);
  L.total = off;
  return L;
}
}  // namespace

size_t kgs_init_ws_bytes(int W, int H, int V) { return init_layout(W, H, V).total; }

kgs_status kgs_launch_init_spawn(const float* color, const float* depth, const float* rcolor, const float* rdepth,
                                 const float* u, const kgs_camera* cams, int V, int W, int H, char* ws,
                                 float* pkf_out, const kgs_spawn_list* out, hipStream_t st) {
  const InitLayout L = init_layout(W, H, V);
  InitParams P;
  const double s1 = 1.0, s2 = 1.6;
  {
    double a = 0.0, b = 0.0;
    for (int j = 0; j <= 2 * IN_R1; ++j) {
      const double x = j - IN_R1;
      P.w1[j] = exp(-x * x / (2.0 * s1 * s1));
      a += P.w1[j];
    }
    for (int j = 0; j <= 2 * IN_R1; ++j) P.w1[j] /= a;
    for (int j = 0; j <= 2 * IN_R; ++j) {
      const double x = j - IN_R;
      P.w2[j] = exp(-x * x / (2.0 * s2 * s2));
      b += P.w2[j];
    }
    for (int j = 0; j <= 2 * IN_R; ++j) P.w2[j] /= b;
  }
  P.lambda = 0.9;
  P.one_minus_lambda = 1.0 - P.lambda;
  const double eps[5] = {0.1, 0.25, 1.0, 5.0, 25.0};
  for (int l = 0; l < 5; ++l) P.eps[l] = eps[l];
  for (int l = 0; l < 4; ++l) P.dmax[l] = 100.0 * eps[l];
  P.W = W;
  P.H = H;
  P.V = V;
  P.tiles_x = (W + IN_TW - 1) / IN_TW;
  P.n_tiles = P.tiles_x * ((H + IN_TH - 1) / IN_TH);
  P.n_seg = (W + IN_SEG - 1) / IN_SEG;
  P.has_render = rcolor != nullptr;
  double* dog = reinterpret_cast<double*>(ws + L.dog);
  double* gnorm = reinterpret_cast<double*>(ws + L.gnorm);
  double* pkf = reinterpret_cast<double*>(ws + L.pkf);
  double* part = reinterpret_cast<double*>(ws + L.part);
  double* mm = reinterpret_cast<double*>(ws + L.mm);
  uint32_t* counts = reinterpret_cast<uint32_t*>(ws + L.counts);
  uint32_t* offsets = reinterpret_cast<uint32_t*>(ws + L.offsets);
  const int which = P.has_render ? 2 : 1;
  hipLaunchKernelGGL(k_init_saliency, dim3((unsigned)P.n_tiles, (unsigned)V, (unsigned)which), dim3(256), 0, st, P,
                     color, depth, rcolor, rdepth, dog, gnorm, part);
  hipLaunchKernelGGL(k_init_minmax, dim3((unsigned)V, (unsigned)which), dim3(256), 0, st, P, (const double*)part, mm);
  const size_t npix = (size_t)W * H;
  hipLaunchKernelGGL(k_init_pkf, dim3((unsigned)((npix + 255) / 256), (unsigned)V), dim3(256), 0, st, P,
                     (const double*)dog, (const double*)gnorm, (const double*)mm, pkf, pkf_out);
  const dim3 sg((unsigned)P.n_seg, (unsigned)H, (unsigned)V);
  hipLaunchKernelGGL(k_init_count, sg, dim3(IN_SEG), 0, st, P, (const double*)pkf, u, depth, counts);
  const int64_t entries = (int64_t)V * H * P.n_seg;
  unsigned long long* tot = reinterpret_cast<unsigned long long*>(ws + L.scan_tot);
  kgs_launch_scan(counts, offsets, entries, 1, 0xffffffffull, 0xffffffffull,
                  reinterpret_cast<unsigned long long*>(ws + L.scan_part), tot, st);
  hipLaunchKernelGGL(k_init_emit, sg, dim3(IN_SEG), 0, st, P, (const double*)pkf, u, color, depth, cams,
                     (const uint32_t*)offsets, out->capacity, out->pixel, out->level, out->voxel, out->point,
                     out->color);
  // the total, saturated at 2^32 - 1
  hipLaunchKernelGGL(k_init_total, dim3(1), dim3(64), 0, st, (const unsigned long long*)tot, out->count);
  return kgs_check_launch();
}
