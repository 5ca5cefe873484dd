// Mapping loss of the sliding-window optimisation (Sec. 3.2, Eq. "mapping loss";
// appendix "Rendering Objectives"):
//   L_photo,v = w_l1 mean|I - I^| + w_ssim (1 - mean SSIM(I, I^))      per view
//   L_geo,v   = mean|D - D^|                                           per view
//   L_iso     = sum_i sum_k |s_ik - mean_k s_ik|,  s = exp(log-scales)
// and their gradients dL/dI^, dL/dD^, dL/dlog s for the chunk loss
// sum_v (L_photo,v + lambda_g L_geo,v) + lambda_iso L_iso.
//
// SSIM: 11x11 Gaussian window (sigma 1.5, normalised), C1 = 0.01^2,
// C2 = 0.03^2, per channel, zero padding.  With mu = G*x, E = G*(products):
//   S = A1 A2 / (B1 B2),  A1 = 2 mu_x mu_y + C1,  A2 = 2 (E_xy - mu_x mu_y) + C2,
//   B1 = mu_x^2 + mu_y^2 + C1,  B2 = E_xx - mu_x^2 + E_yy - mu_y^2 + C2,
// and the derivative of sum_p S(p) with respect to x(q) is
//   (G * dS/dmu_x)(q) + 2 x(q) (G * dS/dE_xx)(q) + y(q) (G * dS/dE_xy)(q)
// (the window is symmetric, so the adjoint of the zero-padded filter is the
// same filter over maps that are zero outside the image).  Two passes: the
// first filters x, y and their products and writes the three derivative maps,
// the second filters those and forms the gradient.  Each is a 32x16 output tile
// per (view, channel) with a 5-pixel halo staged in LDS, the separable window
// run along rows (a thread takes four neighbouring outputs of a row from its 14
// inputs, read once into registers), then columns (two neighbouring rows per
// thread), so each LDS value read serves several taps.  Bound: plain FP32 ALU (about 400 flop per
// pixel and channel against 44 bytes of HBM traffic).
#include <cmath>

#include "kgs_internal.h"

#define ML_TW 32
#define ML_TH 16
#define ML_R 5
#define ML_RW (ML_TW + 2 * ML_R)   // 42
#define ML_RH (ML_TH + 2 * ML_R)   // 26

struct MapLossParams {
  float w[11];
  int W, H, tiles_x, n_tiles;
  float c1, c2;
  float g_l1;     // w_l1 / (3 H W)
  float g_ssim;   // -w_ssim / (3 H W)
  float g_depth;  // lambda_g / (H W)
};

__device__ __forceinline__ float sgnf(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

// block of 256 threads: sum of two floats (per wave) then of the waves in order, in FP64
__device__ __forceinline__ void block_sum3(float a, float b, float c, double* sh, double* out) {
  const int w = threadIdx.x >> 6;
  const float ra = wave_sum(a), rb = wave_sum(b), rc = wave_sum(c);
  if ((threadIdx.x & 63) == 0) {
    sh[3 * w + 0] = ra;
    sh[3 * w + 1] = rb;
    sh[3 * w + 2] = rc;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    out[k] = (sh[k] + sh[3 + k]) + (sh[6 + k] + sh[9 + k]);
  }
}

// Pass 1: per (tile, channel, view) block.  aux [V][3 ch][3][H][W] receives dS/dmu_x, dS/dE_xx, dS/dE_xy;
// partial [V][3][n_tiles][3] receives (sum 1 - S, sum |x - y|, sum |D^ - D| (channel 0 only)).
__global__ __launch_bounds__(256) void k_ssim_fwd(MapLossParams P, const float* __restrict__ img,
                                                  const float* __restrict__ target,
                                                  const float* __restrict__ depth,
                                                  const float* __restrict__ target_depth,
                                                  float* __restrict__ dl_ddepth, float* __restrict__ aux,
                                                  double* __restrict__ partial) {
  __shared__ float sx[ML_RH][ML_RW], sy[ML_RH][ML_RW];
  __shared__ float hq[5][ML_RH][ML_TW];
  __shared__ double red[12];
  const int tile = blockIdx.x, ch = blockIdx.y, v = blockIdx.z;
  const int tx = tile % P.tiles_x, ty = tile / P.tiles_x;
  const int x0 = tx * ML_TW - ML_R, y0 = ty * ML_TH - ML_R;
  const size_t npix = (size_t)P.W * P.H;
  const float* X = img + ((size_t)v * 3 + ch) * npix;
  const float* Y = target + ((size_t)v * 3 + ch) * npix;
  for (int i = threadIdx.x; i < ML_RH * ML_RW; i += 256) {
    const int r = i / ML_RW, c = i - r * ML_RW;
    const int gx = x0 + c, gy = y0 + r;
    float a = 0.f, b = 0.f;
    if (gx >= 0 && gx < P.W && gy >= 0 && gy < P.H) {
      a = X[(size_t)gy * P.W + gx];
      b = Y[(size_t)gy * P.W + gx];
    }
    sx[r][c] = a;
    sy[r][c] = b;
  }
  __syncthreads();
  // rows: the five products filtered along x for every halo row; a thread
  // takes four neighbouring outputs of a row, reading its 14 inputs once
  if (threadIdx.x < ML_RH * (ML_TW / 4)) {
    const int r = threadIdx.x / (ML_TW / 4), c0 = 4 * (threadIdx.x - r * (ML_TW / 4));
    float a[14], b[14], aa[14], bb[14], ab[14];
#pragma unroll
    for (int i = 0; i < 14; ++i) {
      a[i] = sx[r][c0 + i];
      b[i] = sy[r][c0 + i];
      aa[i] = a[i] * a[i];
      bb[i] = b[i] * b[i];
      ab[i] = a[i] * b[i];
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      float ax = 0.f, ay = 0.f, axx = 0.f, ayy = 0.f, axy = 0.f;
#pragma unroll
      for (int k = 0; k < 11; ++k) {
        const float wk = P.w[k];
        ax = fmaf(wk, a[o + k], ax);
        ay = fmaf(wk, b[o + k], ay);
        axx = fmaf(wk, aa[o + k], axx);
        ayy = fmaf(wk, bb[o + k], ayy);
        axy = fmaf(wk, ab[o + k], axy);
      }
      hq[0][r][c0 + o] = ax;
      hq[1][r][c0 + o] = ay;
      hq[2][r][c0 + o] = axx;
      hq[3][r][c0 + o] = ayy;
      hq[4][r][c0 + o] = axy;
    }
  }
  __syncthreads();
  // columns: a thread takes two neighbouring rows of a column, reading its 12 inputs of each map once
  float s_sum = 0.f, l1_sum = 0.f, geo_sum = 0.f;
  const int ox = threadIdx.x & 31, oy0 = 2 * (threadIdx.x >> 5);
  float col[5][2];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    float t[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) t[i] = hq[m][oy0 + i][ox];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < 11; ++k) acc = fmaf(P.w[k], t[h + k], acc);
      col[m][h] = acc;
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int oy = oy0 + h;
    const int px = tx * ML_TW + ox, py = ty * ML_TH + oy;
    if (px < P.W && py < P.H) {
      const float mx = col[0][h], my = col[1][h], exx = col[2][h], eyy = col[3][h], exy = col[4][h];
      const float a1 = 2.f * mx * my + P.c1, a2 = 2.f * (exy - mx * my) + P.c2;
      const float b1 = mx * mx + my * my + P.c1, b2 = (exx - mx * mx) + (eyy - my * my) + P.c2;
      const float inv_d = 1.0f / (b1 * b2);
      const float S = a1 * a2 * inv_d;
      s_sum += 1.0f - S;   // D-SSIM summed directly: no cancellation against the pixel count
      const size_t q = (size_t)py * P.W + px;
      float* A = aux + (((size_t)v * 3 + ch) * 3) * npix;
      A[q] = 2.f * inv_d * (my * (a2 - a1) - S * mx * (b2 - b1));   // dS/dmu_x
      A[npix + q] = -S / b2;                                        // dS/dE_xx
      A[2 * npix + q] = 2.f * a1 * inv_d;                           // dS/dE_xy
      l1_sum += fabsf(sx[oy + ML_R][ox + ML_R] - sy[oy + ML_R][ox + ML_R]);
      if (ch == 0 && depth && target_depth) {
        const size_t dq = (size_t)v * npix + q;
        const float d = depth[dq] - target_depth[dq];
        geo_sum += fabsf(d);
        if (dl_ddepth) dl_ddepth[dq] = P.g_depth * sgnf(d);
      }
    }
  }
  double* out = partial + (((size_t)v * 3 + ch) * P.n_tiles + tile) * 3;
  block_sum3(s_sum, l1_sum, geo_sum, red, out);
}

// Pass 2: dL/dx = g_ssim (G*A + 2 x G*B + y G*C) + g_l1 sign(x - y).
__global__ __launch_bounds__(256) void k_ssim_bwd(MapLossParams P, const float* __restrict__ img,
                                                  const float* __restrict__ target, const float* __restrict__ aux,
                                                  float* __restrict__ dl_dcolor) {
  __shared__ float sa[3][ML_RH][ML_RW];
  __shared__ float hq[3][ML_RH][ML_TW];
  const int tile = blockIdx.x, ch = blockIdx.y, v = blockIdx.z;
  const int tx = tile % P.tiles_x, ty = tile / P.tiles_x;
  const int x0 = tx * ML_TW - ML_R, y0 = ty * ML_TH - ML_R;
  const size_t npix = (size_t)P.W * P.H;
  const float* A = aux + (((size_t)v * 3 + ch) * 3) * npix;
  for (int i = threadIdx.x; i < ML_RH * ML_RW; i += 256) {
    const int r = i / ML_RW, c = i - r * ML_RW;
    const int gx = x0 + c, gy = y0 + r;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    if (gx >= 0 && gx < P.W && gy >= 0 && gy < P.H) {
      const size_t q = (size_t)gy * P.W + gx;
      a0 = A[q];
      a1 = A[npix + q];
      a2 = A[2 * npix + q];
    }
    sa[0][r][c] = a0;
    sa[1][r][c] = a1;
    sa[2][r][c] = a2;
  }
  __syncthreads();
  // rows, four neighbouring outputs per thread (as in the first pass)
  if (threadIdx.x < ML_RH * (ML_TW / 4)) {
    const int r = threadIdx.x / (ML_TW / 4), c0 = 4 * (threadIdx.x - r * (ML_TW / 4));
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      float t[14];
#pragma unroll
      for (int i = 0; i < 14; ++i) t[i] = sa[m][r][c0 + i];
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < 11; ++k) acc = fmaf(P.w[k], t[o + k], acc);
        hq[m][r][c0 + o] = acc;
      }
    }
  }
  __syncthreads();
  const float* X = img + ((size_t)v * 3 + ch) * npix;
  const float* Y = target + ((size_t)v * 3 + ch) * npix;
  float* G = dl_dcolor + ((size_t)v * 3 + ch) * npix;
  // columns, two neighbouring rows per thread
  const int ox = threadIdx.x & 31, oy0 = 2 * (threadIdx.x >> 5);
  float col[3][2];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    float t[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) t[i] = hq[m][oy0 + i][ox];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < 11; ++k) acc = fmaf(P.w[k], t[h + k], acc);
      col[m][h] = acc;
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int oy = oy0 + h;
    const int px = tx * ML_TW + ox, py = ty * ML_TH + oy;
    if (px < P.W && py < P.H) {
      const float ga = col[0][h], gb = col[1][h], gc = col[2][h];
      const size_t q = (size_t)py * P.W + px;
      const float x = X[q], y = Y[q];
      G[q] = P.g_ssim * (ga + 2.f * x * gb + y * gc) + P.g_l1 * sgnf(x - y);
    }
  }
}

// One workgroup per view: the (channel, tile) partials summed in a fixed order
// (per thread, then a fixed tree over the workgroup).
__global__ __launch_bounds__(KGS_FINAL_THREADS) void k_maploss_final(int n_tiles, double inv_n3, double inv_n,
                                                                     float w_l1, float w_ssim,
                                                                     const double* __restrict__ partial,
                                                                     float* __restrict__ view_loss,
                                                                     float* __restrict__ geo_loss) {
  __shared__ double sh[3][KGS_FINAL_THREADS / 64];
  const int v = blockIdx.x, l = threadIdx.x;
  double s = 0.0, a = 0.0, g = 0.0;
  for (int ch = 0; ch < 3; ++ch) {
    const double* p = partial + ((size_t)v * 3 + ch) * n_tiles * 3;
    for (int t = l; t < n_tiles; t += KGS_FINAL_THREADS) {
      s += p[3 * t];
      a += p[3 * t + 1];
      g += p[3 * t + 2];
    }
  }
  s = block_sum_fixed(s, sh[0]);
  a = block_sum_fixed(a, sh[1]);
  g = block_sum_fixed(g, sh[2]);
  if (l == 0) {
    view_loss[v] = (float)((double)w_l1 * a * inv_n3 + (double)w_ssim * s * inv_n3);
    if (geo_loss) geo_loss[v] = (float)(g * inv_n);
  }
}

// Isotropy: per Gaussian |s_k - m| summed over k, m = mean_k s_k, s = exp(log s);
// dL_iso / dlog s_j = s_j (sign(s_j - m) - (1/3) sum_k sign(s_k - m)), scaled by lambda and ADDED.
__global__ __launch_bounds__(KGS_BLOCK) void k_iso(int64_t n, const float* __restrict__ log_scales, float lambda,
                                                   float* __restrict__ grad, double* __restrict__ partial) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * KGS_BLOCK + threadIdx.x;
  float li = 0.f;
  if (i < n) {
    const float s0 = expf(log_scales[i]), s1 = expf(log_scales[n + i]), s2 = expf(log_scales[2 * n + i]);
    const float m = (s0 + s1 + s2) * (1.0f / 3.0f);
    const float g0 = sgnf(s0 - m), g1 = sgnf(s1 - m), g2 = sgnf(s2 - m);
    li = (fabsf(s0 - m) + fabsf(s1 - m)) + fabsf(s2 - m);
    if (grad) {
      const float c = (g0 + g1 + g2) * (1.0f / 3.0f);
      grad[i] += lambda * s0 * (g0 - c);
      grad[n + i] += lambda * s1 * (g1 - c);
      grad[2 * n + i] += lambda * s2 * (g2 - c);
    }
  }
  const float r = wave_sum(li);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(1024) void k_iso_final(int64_t nb, const double* __restrict__ partial,
                                                    float* __restrict__ loss) {
  __shared__ double sh[16];
  double a = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += 1024) a += partial[b];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < 16; ++k) t += sh[k];
    *loss = (float)t;
  }
}

// ---------------------------------------------------------------- host side
int kgs_maploss_tiles(int W, int H) { return ((W + ML_TW - 1) / ML_TW) * ((H + ML_TH - 1) / ML_TH); }

kgs_status kgs_launch_loss_mapping(kgs_ctx* ctx, int V, const float* target, const float* target_depth,
                                   const kgs_image* img, float w_l1, float w_ssim, float lambda_g,
                                   float* dl_dcolor, float* dl_ddepth, float* view_loss, float* geo_loss,
                                   hipStream_t st) {
  MapLossParams P;
  {
    double w[11], s = 0.0;
    for (int k = 0; k < 11; ++k) {
      const double x = k - 5;
      w[k] = exp(-x * x / (2.0 * 1.5 * 1.5));
      s += w[k];
    }
    for (int k = 0; k < 11; ++k) P.w[k] = (float)(w[k] / s);
  }
  P.W = ctx->cfg.width;
  P.H = ctx->cfg.height;
  P.tiles_x = (P.W + ML_TW - 1) / ML_TW;
  P.n_tiles = kgs_maploss_tiles(P.W, P.H);
  P.c1 = 1e-4f;
  P.c2 = 9e-4f;
  const double npix = (double)P.W * (double)P.H;
  P.g_l1 = (float)(w_l1 / (3.0 * npix));
  P.g_ssim = (float)(-w_ssim / (3.0 * npix));
  P.g_depth = (float)(lambda_g / npix);
  const dim3 grid((unsigned)P.n_tiles, 3, (unsigned)V);
  const bool with_depth = target_depth && img->depth;
  hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, st, P, (const float*)img->color, target,
                     with_depth ? (const float*)img->depth : (const float*)nullptr,
                     with_depth ? target_depth : (const float*)nullptr, with_depth ? dl_ddepth : (float*)nullptr,
                     ctx->ssim_aux, ctx->ssim_partial);
  hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, st, P, (const float*)img->color, target,
                     (const float*)ctx->ssim_aux, dl_dcolor);
  hipLaunchKernelGGL(k_maploss_final, dim3((unsigned)V), dim3(KGS_FINAL_THREADS), 0, st, P.n_tiles, 1.0 / (3.0 * npix), 1.0 / npix,
                     w_l1, w_ssim, (const double*)ctx->ssim_partial, view_loss,
                     with_depth ? geo_loss : (float*)nullptr);
  return kgs_check_launch();
}

kgs_status kgs_launch_loss_iso(kgs_ctx* ctx, const kgs_gaussians* g, float lambda, float* grad, float* loss,
                               hipStream_t st) {
  const int64_t n = g->n, nb = (n + KGS_BLOCK - 1) / KGS_BLOCK;
  if (nb == 0) return KGS_OK;
  hipLaunchKernelGGL(k_iso, dim3((unsigned)nb), dim3(KGS_BLOCK), 0, st, n, g->log_scales, lambda, grad,
                     ctx->mm_partial);
  hipLaunchKernelGGL(k_iso_final, dim3(1), dim3(1024), 0, st, nb, (const double*)ctx->mm_partial, loss);
  return kgs_check_launch();
}
