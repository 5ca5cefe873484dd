// The learned prune / keep / densify head: a 16 -> 64 -> 64 -> 3 MLP over
// per-Gaussian statistics, trained on the decisions of the plain multi-view
// criterion (Sec. 3.3, App. D) and usable in its place.
//
// Every GEMM runs on the matrix cores (v_mfma_f32_16x16x16_bf16: BF16
// operands, FP32 accumulation).  Gaussians are the N dimension of every
// product, so a layer's output tile (lane (a, b) holds rows 4b..4b+3 of
// column a) is already the B operand of the next layer: no transposes in the
// forward pass or in the backward's data gradients.  The weight gradients
// sum over Gaussians (K dimension); their operands are transposed through a
// per-wave LDS tile.  Weights live in LDS as BF16 (plus transposed copies for
// the backward); the FP32 master vector stays in HBM.
//
// Gradients are summed per wave in registers, written as per-wave partials and
// added in a fixed order, so a training step is deterministic.
#include "kgs_internal.h"

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define HD_OFF_W1 0
#define HD_OFF_B1 1024
#define HD_OFF_W2 1088
#define HD_OFF_B2 5184
#define HD_OFF_W3 5248
#define HD_OFF_B3 5440
#define HD_STRIDE (KGS_HEAD_PARAMS + 1)   // per-wave partial: gradient, then the weighted loss
#define HD_BLOCKS 256
#define HD_WAVES (HD_BLOCKS * 4)
#define HD_LD 68                          // padded row of the 64-wide BF16 tiles in LDS

// FP32 -> BF16, round to nearest even (finite values)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x4 pack4(float v0, float v1, float v2, float v3) {
  bf16x4 r;
  r[0] = (short)f2bf(v0);
  r[1] = (short)f2bf(v1);
  r[2] = (short)f2bf(v2);
  r[3] = (short)f2bf(v3);
  return r;
}

__device__ __forceinline__ bf16x4 ld4(const uint16_t* p) { return *reinterpret_cast<const bf16x4*>(p); }

struct HeadLds {
  uint16_t w1[64][16];       // layer 1 A: row = hidden unit, 16 inputs
  uint16_t w2[64][HD_LD];    // layer 2 A: row = hidden2 unit, 64 inputs
  uint16_t w3[16][HD_LD];    // layer 3 A: rows 0-2 the outputs, the rest zero
  uint16_t w2t[64][HD_LD];   // W2^T: row = hidden1 unit, 64 hidden2 columns
  uint16_t w3t[64][16];      // W3^T: row = hidden2 unit, columns 0-2 the outputs
  float b1[64], b2[64], b3[4];
  uint16_t tr[4][16][16];    // per-wave transpose tile
};

__device__ void stage_weights(const float* __restrict__ theta, HeadLds& s) {
  for (int k = threadIdx.x; k < 1024; k += blockDim.x) s.w1[k >> 4][k & 15] = f2bf(theta[HD_OFF_W1 + k]);
  for (int k = threadIdx.x; k < 4096; k += blockDim.x) {
    const uint16_t v = f2bf(theta[HD_OFF_W2 + k]);
    s.w2[k >> 6][k & 63] = v;
    s.w2t[k & 63][k >> 6] = v;
  }
  for (int k = threadIdx.x; k < 16 * 64; k += blockDim.x) {
    const int o = k >> 6, i = k & 63;
    const uint16_t v = o < 3 ? f2bf(theta[HD_OFF_W3 + k]) : (uint16_t)0;
    s.w3[o][i] = v;
    s.w3t[i][o] = v;
  }
  for (int k = threadIdx.x; k < 64; k += blockDim.x) {
    s.b1[k] = theta[HD_OFF_B1 + k];
    s.b2[k] = theta[HD_OFF_B2 + k];
  }
  if (threadIdx.x < 4) s.b3[threadIdx.x] = threadIdx.x < 3 ? theta[HD_OFF_B3 + threadIdx.x] : 0.f;
  __syncthreads();
}

// Forward of one tile of 16 Gaussians [g0, g0 + 16) for lane (a, b).
struct HeadFwd {
  bf16x4 x;          // B operand: features 4b..4b+3 of Gaussian a
  f32x4 z1[4], z2[4];
  bf16x4 h1[4], h2[4];
  f32x4 out;         // rows 4b..4b+3 of the (16-padded) output, Gaussian a
};

__device__ __forceinline__ void head_forward(const HeadLds& s, const uint16_t* __restrict__ feat, int64_t n,
                                             int64_t g0, int a, int b, HeadFwd& f) {
  const int64_t gi = g0 + a;
  if (gi < n) {
    f.x = ld4(feat + gi * KGS_HEAD_FEATURES + 4 * b);
  } else {
    f.x = bf16x4{0, 0, 0, 0};
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 c = {s.b1[16 * t + 4 * b], s.b1[16 * t + 4 * b + 1], s.b1[16 * t + 4 * b + 2], s.b1[16 * t + 4 * b + 3]};
    c = mfma(ld4(&s.w1[16 * t + a][4 * b]), f.x, c);
    f.z1[t] = c;
    f.h1[t] = pack4(fmaxf(c[0], 0.f), fmaxf(c[1], 0.f), fmaxf(c[2], 0.f), fmaxf(c[3], 0.f));
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 c = {s.b2[16 * t + 4 * b], s.b2[16 * t + 4 * b + 1], s.b2[16 * t + 4 * b + 2], s.b2[16 * t + 4 * b + 3]};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) c = mfma(ld4(&s.w2[16 * t + a][16 * kk + 4 * b]), f.h1[kk], c);
    f.z2[t] = c;
    f.h2[t] = pack4(fmaxf(c[0], 0.f), fmaxf(c[1], 0.f), fmaxf(c[2], 0.f), fmaxf(c[3], 0.f));
  }
  f32x4 c = {0.f, 0.f, 0.f, 0.f};
  if (b == 0) c = f32x4{s.b3[0], s.b3[1], s.b3[2], 0.f};
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) c = mfma(ld4(&s.w3[a][16 * kk + 4 * b]), f.h2[kk], c);
  f.out = c;
}

__global__ __launch_bounds__(256) void k_head_forward(const float* __restrict__ theta,
                                                      const uint16_t* __restrict__ feat, int64_t n,
                                                      float* __restrict__ logits, uint8_t* __restrict__ decision) {
  __shared__ HeadLds s;
  stage_weights(theta, s);
  const int l = threadIdx.x & 63, a = l & 15, b = l >> 4;
  const int64_t tiles = (n + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < tiles; tile += (int64_t)gridDim.x * 4) {
    HeadFwd f;
    head_forward(s, feat, n, tile * 16, a, b, f);
    const int64_t gi = tile * 16 + a;
    if (b == 0 && gi < n) {
      if (logits) {
        logits[gi * 3] = f.out[0];
        logits[gi * 3 + 1] = f.out[1];
        logits[gi * 3 + 2] = f.out[2];
      }
      if (decision) {
        // argmax, the lower class on ties
        uint8_t d = 0;
        float best = f.out[0];
        if (f.out[1] > best) { d = 1; best = f.out[1]; }
        if (f.out[2] > best) d = 2;
        decision[gi] = d;
      }
    }
  }
}

// sum of the class weights over the labels: per-block partials, then one block
__global__ __launch_bounds__(256) void k_head_wsum(const uint8_t* __restrict__ labels, int64_t n,
                                                   const float* __restrict__ cw, double* __restrict__ part) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    acc += (double)cw[min((int)labels[i], 2)];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void k_head_wsum_final(const double* __restrict__ part, int nparts, float* __restrict__ wsum) {
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < nparts; ++k) t += part[k];
    wsum[0] = (float)t;
  }
}

// lane (a, b) holds Y[4b + j][a] (j = 0..3, a layer-output tile); returns the
// lane's A / B operand of the transposed use: Y[a][4b .. 4b + 3].
__device__ __forceinline__ bf16x4 transpose_tile(uint16_t (*tr)[16], bf16x4 y, int a, int b) {
#pragma unroll
  for (int j = 0; j < 4; ++j) tr[4 * b + j][a] = (uint16_t)y[j];
  __builtin_amdgcn_wave_barrier();   // LDS requests of one wave complete in order
  const bf16x4 r = ld4(&tr[a][4 * b]);
  __builtin_amdgcn_wave_barrier();
  return r;
}

__device__ __forceinline__ float row16_sum(float v) {
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One training pass: forward, weighted cross-entropy, backward, per-wave
// gradient partials (normalised by the weight sum, as the loss is).
__global__ __launch_bounds__(256) void k_head_train(const float* __restrict__ theta,
                                                    const uint16_t* __restrict__ feat,
                                                    const uint8_t* __restrict__ labels, int64_t n,
                                                    const float* __restrict__ cw, const float* __restrict__ wsum,
                                                    float* __restrict__ partial) {
  __shared__ HeadLds s;
  stage_weights(theta, s);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, a = l & 15, b = l >> 4;
  uint16_t (*tr)[16] = s.tr[w];
  const float inv_w = 1.0f / wsum[0];
  const float cw0 = cw[0], cw1 = cw[1], cw2 = cw[2];
  f32x4 gW1[4], gW2[4][4], gW3[4];
  f32x4 gb1[4], gb2[4], gb3;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    gW1[t] = zero;
    gW3[t] = zero;
    gb1[t] = zero;
    gb2[t] = zero;
#pragma unroll
    for (int u = 0; u < 4; ++u) gW2[t][u] = zero;
  }
  gb3 = zero;
  float lsum = 0.f;
  const int64_t tiles = (n + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + w; tile < tiles; tile += (int64_t)gridDim.x * 4) {
    HeadFwd f;
    head_forward(s, feat, n, tile * 16, a, b, f);
    const int64_t gi = tile * 16 + a;
    // dL/dlogits = w_y (softmax - onehot) / sum w, in the lanes holding the logits
    float d0 = 0.f, d1 = 0.f, d2 = 0.f;
    if (b == 0 && gi < n) {
      const int y = min((int)labels[gi], 2);
      const float wy = y == 0 ? cw0 : (y == 1 ? cw1 : cw2);
      const float m = fmaxf(fmaxf(f.out[0], f.out[1]), f.out[2]);
      const float e0 = expf(f.out[0] - m), e1 = expf(f.out[1] - m), e2 = expf(f.out[2] - m);
      const float se = e0 + e1 + e2, is = 1.0f / se;
      const float zy = y == 0 ? f.out[0] : (y == 1 ? f.out[1] : f.out[2]);
      lsum += wy * (logf(se) + m - zy);
      const float sc = wy * inv_w;
      d0 = (e0 * is - (y == 0 ? 1.f : 0.f)) * sc;
      d1 = (e1 * is - (y == 1 ? 1.f : 0.f)) * sc;
      d2 = (e2 * is - (y == 2 ? 1.f : 0.f)) * sc;
    }
    const bf16x4 dl = pack4(d0, d1, d2, 0.f);
    // data gradients: dz2 = (W3^T dl) * [z2 > 0], dz1 = (W2^T dz2) * [z1 > 0]
    bf16x4 dz2[4], dz1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const f32x4 c = mfma(ld4(&s.w3t[16 * t + a][4 * b]), dl, zero);
      dz2[t] = pack4(f.z2[t][0] > 0.f ? c[0] : 0.f, f.z2[t][1] > 0.f ? c[1] : 0.f, f.z2[t][2] > 0.f ? c[2] : 0.f,
                     f.z2[t][3] > 0.f ? c[3] : 0.f);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 c = zero;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) c = mfma(ld4(&s.w2t[16 * t + a][16 * kk + 4 * b]), dz2[kk], c);
      dz1[t] = pack4(f.z1[t][0] > 0.f ? c[0] : 0.f, f.z1[t][1] > 0.f ? c[1] : 0.f, f.z1[t][2] > 0.f ? c[2] : 0.f,
                     f.z1[t][3] > 0.f ? c[3] : 0.f);
    }
    // bias gradients: the same rounded values, summed over Gaussians later
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      gb3[j] += bf2f((uint16_t)dl[j]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        gb2[t][j] += bf2f((uint16_t)dz2[t][j]);
        gb1[t][j] += bf2f((uint16_t)dz1[t][j]);
      }
    }
    // weight gradients: dW = sum_g d[:, g] h[:, g]^T with Gaussians as K
    const bf16x4 At3 = transpose_tile(tr, dl, a, b);
    bf16x4 Bh2[4], Bh1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) Bh2[u] = transpose_tile(tr, f.h2[u], a, b);
#pragma unroll
    for (int u = 0; u < 4; ++u) gW3[u] = mfma(At3, Bh2[u], gW3[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) Bh1[u] = transpose_tile(tr, f.h1[u], a, b);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bf16x4 A2 = transpose_tile(tr, dz2[t], a, b);
#pragma unroll
      for (int u = 0; u < 4; ++u) gW2[t][u] = mfma(A2, Bh1[u], gW2[t][u]);
    }
    const bf16x4 Bx = transpose_tile(tr, f.x, a, b);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bf16x4 A1 = transpose_tile(tr, dz1[t], a, b);
      gW1[t] = mfma(A1, Bx, gW1[t]);
    }
  }
  // this wave's partial: D tiles hold rows 4b..4b+3, column a
  float* out = partial + ((int64_t)blockIdx.x * 4 + w) * HD_STRIDE;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      out[HD_OFF_W1 + (16 * t + 4 * b + j) * 16 + a] = gW1[t][j];
#pragma unroll
      for (int u = 0; u < 4; ++u) out[HD_OFF_W2 + (16 * t + 4 * b + j) * 64 + 16 * u + a] = gW2[t][u][j];
      if (b == 0 && j < 3) out[HD_OFF_W3 + j * 64 + 16 * t + a] = gW3[t][j];
    }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float s3 = row16_sum(gb3[j]);
    if (a == 0 && b == 0 && j < 3) out[HD_OFF_B3 + j] = s3;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float s1 = row16_sum(gb1[t][j]), s2 = row16_sum(gb2[t][j]);
      if (a == 0) {
        out[HD_OFF_B1 + 16 * t + 4 * b + j] = s1;
        out[HD_OFF_B2 + 16 * t + 4 * b + j] = s2;
      }
    }
  }
  const float ls = row16_sum(lsum);
  if (l == 0) out[KGS_HEAD_PARAMS] = ls;
}

// grad[k] = sum over the per-wave partials in wave order; loss = weighted sum / sum w
__global__ __launch_bounds__(256) void k_head_reduce(const float* __restrict__ partial, const float* __restrict__ wsum,
                                                     float* __restrict__ grad, float* __restrict__ loss) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k > KGS_HEAD_PARAMS) return;
  float acc = 0.f;
  for (int p = 0; p < HD_WAVES; ++p) acc += partial[(int64_t)p * HD_STRIDE + k];
  if (k < KGS_HEAD_PARAMS) grad[k] = acc;
  else if (loss) loss[0] = acc / wsum[0];
}

__global__ __launch_bounds__(256) void k_head_adam(float* __restrict__ theta, float* __restrict__ m,
                                                   float* __restrict__ v, const float* __restrict__ g, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= KGS_HEAD_PARAMS) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  theta[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// Features of the head from a chunk's statistics (the layout is documented
// with kgs_head_features in kgs.h).
__global__ __launch_bounds__(KGS_BLOCK) void k_head_features(kgs_gaussians g, kgs_view_stats st, int n_views,
                                                             const double* __restrict__ mm,
                                                             const uint8_t* __restrict__ densify,
                                                             const double* __restrict__ prune_score,
                                                             uint16_t* __restrict__ feat) {
  const int64_t i = (int64_t)blockIdx.x * KGS_BLOCK + threadIdx.x;
  const int64_t n = g.n;
  if (i >= n) return;
  const float kap = (float)st.kappa_sum[i], om = (float)st.omega_sum[i];
  const double gam = st.gamma_sum[i];
  const float vc = (float)st.view_count[i];
  const double L = log1p(gam);
  const double lo = mm[0], hi = mm[1];
  const double sp = (om > 0.f && hi > lo) ? (L - lo) / (hi - lo) : 0.0;
  float ls[3] = {g.log_scales[i], g.log_scales[n + i], g.log_scales[2 * n + i]};
  if (ls[0] < ls[1]) { const float t = ls[0]; ls[0] = ls[1]; ls[1] = t; }
  if (ls[1] < ls[2]) { const float t = ls[1]; ls[1] = ls[2]; ls[2] = t; }
  if (ls[0] < ls[1]) { const float t = ls[0]; ls[0] = ls[1]; ls[1] = t; }
  float f[KGS_HEAD_FEATURES];
  // S_d^(i,c) as the FP64 quotient rounded once (no float reciprocal of |V_c|)
  f[0] = (float)((double)st.kappa_sum[i] / (double)n_views);
  f[1] = (float)L;
  f[2] = (float)sp;
  f[3] = log1pf(om);
  f[4] = om > 0.f ? kap / om : 0.f;
  f[5] = (float)((double)st.view_count[i] / (double)n_views);
  f[6] = st.grad_norm_sum[i] / fmaxf(vc, 1.0f);
  f[7] = log1pf((float)max(st.max_radius[i], 0));
  f[8] = 1.0f / (1.0f + __expf(-g.opacity_logits[i]));
  f[9] = ls[0];
  f[10] = ls[1];
  f[11] = ls[2];
  f[12] = prune_score ? (float)prune_score[i] : 0.f;
  f[13] = densify ? (float)densify[i] : 0.f;
  f[14] = om > 0.f ? (float)(gam / (double)om) : 0.f;
  f[15] = om > 0.f ? 1.f : 0.f;
  uint32_t packed[KGS_HEAD_FEATURES / 2];
#pragma unroll
  for (int k = 0; k < KGS_HEAD_FEATURES / 2; ++k) {
    const float x0 = fminf(fmaxf(f[2 * k], -3.0e38f), 3.0e38f), x1 = fminf(fmaxf(f[2 * k + 1], -3.0e38f), 3.0e38f);
    packed[k] = (uint32_t)f2bf(x0) | ((uint32_t)f2bf(x1) << 16);
  }
  uint4* o = reinterpret_cast<uint4*>(feat + i * KGS_HEAD_FEATURES);
  o[0] = make_uint4(packed[0], packed[1], packed[2], packed[3]);
  o[1] = make_uint4(packed[4], packed[5], packed[6], packed[7]);
}

// ---------------------------------------------------------------- host side
size_t kgs_head_ws_bytes() { return (size_t)HD_WAVES * HD_STRIDE * 4 + 8 * 1024 + 256; }

kgs_status kgs_launch_head_forward(const float* theta, const uint16_t* feat, int64_t n, float* logits,
                                   uint8_t* decision, hipStream_t st) {
  if (n <= 0) return KGS_OK;
  const int64_t tiles = (n + 15) / 16;
  const unsigned grid = (unsigned)std::min<int64_t>((tiles + 3) / 4, 2048);
  hipLaunchKernelGGL(k_head_forward, dim3(grid), dim3(256), 0, st, theta, feat, n, logits, decision);
  return kgs_check_launch();
}

kgs_status kgs_launch_head_train(const float* theta, const uint16_t* feat, const uint8_t* labels, int64_t n,
                                 const float* cw, char* ws, float* grad, float* loss, hipStream_t st) {
  float* partial = reinterpret_cast<float*>(ws);
  double* wpart = reinterpret_cast<double*>(ws + (size_t)HD_WAVES * HD_STRIDE * 4);
  float* wsum = reinterpret_cast<float*>(ws + (size_t)HD_WAVES * HD_STRIDE * 4 + 8 * 1024);
  hipLaunchKernelGGL(k_head_wsum, dim3(1024), dim3(256), 0, st, labels, n, cw, wpart);
  hipLaunchKernelGGL(k_head_wsum_final, dim3(1), dim3(64), 0, st, (const double*)wpart, 1024, wsum);
  hipLaunchKernelGGL(k_head_train, dim3(HD_BLOCKS), dim3(256), 0, st, theta, feat, labels, n, cw,
                     (const float*)wsum, partial);
  hipLaunchKernelGGL(k_head_reduce, dim3((KGS_HEAD_PARAMS + 1 + 255) / 256), dim3(256), 0, st,
                     (const float*)partial, (const float*)wsum, grad, loss);
  return kgs_check_launch();
}

kgs_status kgs_launch_head_adam(float* theta, float* m, float* v, const float* grad, int32_t step, float lr,
                                float b1, float b2, float eps, hipStream_t st) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_head_adam, dim3((KGS_HEAD_PARAMS + 255) / 256), dim3(256), 0, st, theta, m, v, grad, lr, b1, b2,
                     eps, c1, c2);
  return kgs_check_launch();
}

kgs_status kgs_launch_head_features(kgs_ctx* ctx, const kgs_gaussians* g, const kgs_view_stats* stats, int V,
                                    const kgs_lifecycle_state* before, uint16_t* feat, hipStream_t st) {
  const int64_t n = g->n, nb = (n + KGS_BLOCK - 1) / KGS_BLOCK;
  if (nb == 0) return KGS_OK;
  const double* mm = kgs_launch_chunk_minmax(ctx, stats, n, st);
  hipLaunchKernelGGL(k_head_features, dim3((unsigned)nb), dim3(KGS_BLOCK), 0, st, *g, *stats, V, mm,
                     before ? (const uint8_t*)before->densify : (const uint8_t*)nullptr,
                     before ? (const double*)before->prune_score : (const double*)nullptr, feat);
  return kgs_check_launch();
}
