// Anchors: decoding a view's Gaussians from voxel anchors and the per-anchor
// footprint statistics.
//
// Decoding (appendix, "Voxelized Representation and MLP Decoding" and
// "Level-of-Detail (LoD) Mask Computation"): for anchor i and a camera centre
// c, d = |p_i - c|, d^ = (p_i - c) / d, and one network
//   36 inputs (f_i in R^32, d^, d) -> 32 ReLU -> 14 K outputs
// gives every child k (alpha, colour, rotation, ds, dO); then
//   x_k = p_i + (O_k + dO_k) * l_i,  s_k = l_i * sigmoid(ds_k),
//   alpha~ = tanh(alpha) * M_l(d)   (1 inside the level's distance band, else 0),
//   colour = sigmoid(.)  written as a degree-0 SH coefficient (c - 0.5) / Y_00,
//   opacity logit ln(alpha~ / (1 - alpha~)) (formed from the raw output, see tanh_logit),
//   -100 when alpha~ <= 0.
// Both products run on the matrix cores (v_mfma_f32_16x16x16_bf16, BF16
// operands, FP32 accumulation); anchors are the N dimension, so the hidden
// tile is directly the second product's B operand.  A wave decodes 16 anchors
// at a time and composes their children from an LDS copy of the output tile.
// Bound: the decoded parameters it writes (56 bytes per child) -- HBM.
//
// Footprint statistics (appendix, "Densification Score" / "Pruning Score": the
// footprint of an anchor is the set of pixels where any of its decoded
// Gaussians contributes).  A workgroup per (view, tile) walks every 8x8
// sub-block's sequence as the compositing forward does (same staging, same
// FP32 evaluation, so the same Gaussians blend), and each wave ORs the 64-bit
// ballot of "blended here" of every entry into an LDS hash table keyed by the
// entry's anchor: a pixel then counts once per anchor however many of its
// children blend there.  The ballots of a batch's entries are kept one per
// lane and inserted together after the batch (lane j inserts entry j: a key
// claimed by compare-and-swap, the ballot ORed in atomically), so the table
// probes of a batch overlap instead of following one another.  At the end of
// the walk each table entry adds the popcount of its union (and of the union
// with the error mask) to the anchor's counters -- integer atomics, so the sums
// do not depend on their order.  A sub-block whose distinct anchors do not fit
// the table is walked again for each half of the anchors (split by hash bits)
// until every part fits.
#include <cmath>

#include "kgs_internal.h"

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

#define AD_IN 36
#define AD_HID 32
#define AD_OUT 14
#define AD_MAXK 16
#define AD_OUTPAD (AD_OUT * AD_MAXK)   // 224 output rows at most (14 tiles)
#define AD_LDO (AD_OUTPAD + 1)

__device__ __forceinline__ uint16_t ad_f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x4_t ad_pack4(float v0, float v1, float v2, float v3) {
  bf16x4_t r;
  r[0] = (short)ad_f2bf(v0);
  r[1] = (short)ad_f2bf(v1);
  r[2] = (short)ad_f2bf(v2);
  r[3] = (short)ad_f2bf(v3);
  return r;
}

__device__ __forceinline__ f32x4_t ad_mfma(bf16x4_t a, bf16x4_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ln sigmoid(z) = min(z, 0) - ln(1 + e^{-|z|}), branch-free; the hardware exp2 / log2 (a few ulp) are far
// inside the decoded values' tolerance
__device__ __forceinline__ float log_sigmoid(float z) {
  return fminf(z, 0.f) - __logf(1.0f + __expf(-fabsf(z)));
}

__device__ __forceinline__ float sigmoid(float z) { return __fdividef(1.0f, 1.0f + __expf(-z)); }

// ln(tanh y / (1 - tanh y)) for y > 0, without forming 1 - tanh y (which cancels as tanh y -> 1): the ratio
// is (e^{2y} - 1) / 2, so the logit is ln(expm1(2y) / 2), or 2y - ln 2 + ln(1 - e^{-2y}) once e^{2y} is large.
__device__ __forceinline__ float tanh_logit(float y) {
  return y < 0.5f ? __logf(0.5f * expm1f(2.0f * y)) : 2.0f * y - 0.69314718055994531f + __logf(1.0f - __expf(-2.0f * y));
}

struct DecodeParams {
  double cx, cy, cz;          // camera centre
  double dmin[5], dmax[5];    // level bands
  int64_t n;                  // anchors
  int K;
};

struct DecodeLds {
  uint16_t w1[AD_HID][48];            // row = hidden unit, inputs padded to 48 with zeros
  uint16_t w2[AD_OUTPAD][AD_HID];     // row = output, rows past 14 K zero
  float b1[AD_HID];
  float b2[AD_OUTPAD];
  float out[4][16][AD_LDO];           // per-wave output tile, anchor-major
  float anc[4][16][10];               // per wave and anchor: p, log l, l (3 each), band flag
};

__global__ __launch_bounds__(256) void k_anchor_decode(DecodeParams P, const float* __restrict__ theta,
                                                       kgs_anchors A, kgs_gaussians_out G) {
  __shared__ DecodeLds s;
  const int K = P.K, NO = AD_OUT * K;
  const int n_tiles_out = (NO + 15) / 16;
  const float* W1 = theta;
  const float* B1 = W1 + AD_HID * AD_IN;
  const float* W2 = B1 + AD_HID;
  const float* B2 = W2 + NO * AD_HID;
  for (int k = threadIdx.x; k < AD_HID * 48; k += 256) {
    const int r = k / 48, c = k - r * 48;
    s.w1[r][c] = c < AD_IN ? ad_f2bf(W1[r * AD_IN + c]) : (uint16_t)0;
  }
  for (int k = threadIdx.x; k < n_tiles_out * 16 * AD_HID; k += 256) {
    const int r = k / AD_HID, c = k - r * AD_HID;
    s.w2[r][c] = r < NO ? ad_f2bf(W2[r * AD_HID + c]) : (uint16_t)0;
  }
  for (int k = threadIdx.x; k < AD_HID; k += 256) s.b1[k] = B1[k];
  for (int k = threadIdx.x; k < n_tiles_out * 16; k += 256) s.b2[k] = k < NO ? B2[k] : 0.f;
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, a = l & 15, b = l >> 4;
  const int64_t n = P.n, N = G.n;
  const int64_t tiles = (n + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + w; tile < tiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t g = tile * 16 + a;
    const bool ok = g < n;
    // inputs of anchor a: f, then the direction and distance from the camera centre (FP64, then BF16)
    bf16x4_t x0 = {0, 0, 0, 0}, x1 = {0, 0, 0, 0}, x2 = {0, 0, 0, 0};
    double d = 0.0;
    if (ok) {
      const float4 f0 = *reinterpret_cast<const float4*>(A.feat + g * 32 + 4 * b);
      const float4 f1 = *reinterpret_cast<const float4*>(A.feat + g * 32 + 16 + 4 * b);
      x0 = ad_pack4(f0.x, f0.y, f0.z, f0.w);
      x1 = ad_pack4(f1.x, f1.y, f1.z, f1.w);
      const double e0 = (double)A.p[g] - P.cx, e1 = (double)A.p[n + g] - P.cy, e2 = (double)A.p[2 * n + g] - P.cz;
      d = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
      if (b == 0) x2 = ad_pack4((float)(e0 / d), (float)(e1 / d), (float)(e2 / d), (float)d);
    }
    // what the children of anchor a share, once per anchor: position, local scale and the band test
    if (b == 0) {
      float* q = s.anc[w][a];
      const int lev = ok ? A.level[g] : -1;
      const bool in_band = ok && lev >= 0 && lev < 5 && d >= P.dmin[lev] && d < P.dmax[lev];
#pragma unroll
      for (int dim = 0; dim < 3; ++dim) {
        const float ll = ok ? A.log_l[dim * n + g] : 0.f;
        q[dim] = ok ? A.p[dim * n + g] : 0.f;
        q[3 + dim] = ll;
        q[6 + dim] = expf(ll);
      }
      q[9] = in_band ? 1.f : 0.f;
    }
    bf16x4_t h[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      f32x4_t c = {s.b1[16 * t + 4 * b], s.b1[16 * t + 4 * b + 1], s.b1[16 * t + 4 * b + 2], s.b1[16 * t + 4 * b + 3]};
      c = ad_mfma(*reinterpret_cast<const bf16x4_t*>(&s.w1[16 * t + a][4 * b]), x0, c);
      c = ad_mfma(*reinterpret_cast<const bf16x4_t*>(&s.w1[16 * t + a][16 + 4 * b]), x1, c);
      c = ad_mfma(*reinterpret_cast<const bf16x4_t*>(&s.w1[16 * t + a][32 + 4 * b]), x2, c);
      h[t] = ad_pack4(fmaxf(c[0], 0.f), fmaxf(c[1], 0.f), fmaxf(c[2], 0.f), fmaxf(c[3], 0.f));
    }
    for (int t2 = 0; t2 < n_tiles_out; ++t2) {
      f32x4_t c = {s.b2[16 * t2 + 4 * b], s.b2[16 * t2 + 4 * b + 1], s.b2[16 * t2 + 4 * b + 2],
                   s.b2[16 * t2 + 4 * b + 3]};
      c = ad_mfma(*reinterpret_cast<const bf16x4_t*>(&s.w2[16 * t2 + a][4 * b]), h[0], c);
      c = ad_mfma(*reinterpret_cast<const bf16x4_t*>(&s.w2[16 * t2 + a][16 + 4 * b]), h[1], c);
#pragma unroll
      for (int r = 0; r < 4; ++r) s.out[w][a][16 * t2 + 4 * b + r] = c[r];
    }
    __builtin_amdgcn_wave_barrier();
    // compose the 16 K children of this tile, child c = anchor (c / K), k = c % K
    for (int c = l; c < 16 * K; c += 64) {
      const int aa = c / K, k = c - aa * K;
      const int64_t ga = tile * 16 + aa;
      if (ga >= n) continue;
      const int64_t j = ga * K + k;
      if (j >= N) continue;
      const float* y = &s.out[w][aa][AD_OUT * k];
      const float* q = s.anc[w][aa];
      G.opacity_logits[j] = q[9] != 0.f && y[0] > 0.f ? tanh_logit(y[0]) : -100.0f;
      for (int ch = 0; ch < 3; ++ch) {
        const float col = sigmoid(y[1 + ch]);
        G.sh[(int64_t)ch * N + j] = (col - 0.5f) / 0.28209479177387814f;
      }
      for (int q = 0; q < 4; ++q) G.quats[(int64_t)q * N + j] = y[4 + q];
      for (int dim = 0; dim < 3; ++dim) {
        G.log_scales[(int64_t)dim * N + j] = q[3 + dim] + log_sigmoid(y[8 + dim]);
        const float off = A.offsets[((int64_t)k * 3 + dim) * n + ga] + y[11 + dim];
        G.means[(int64_t)dim * N + j] = q[dim] + off * q[6 + dim];
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// ---------------------------------------------------------------- footprint statistics
#define AS_TCAP 512
#define AS_EMPTY 0xffffffffu

struct AnchorStatParams {
  RenderParams R;
  float tau_err;
};

__device__ __forceinline__ uint32_t as_mix(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// One workgroup per (view, tile), NW waves of 8x8 sub-blocks.
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_anchor_footprint(AnchorStatParams AP, const uint2* __restrict__ ranges,
                                                              const uint32_t* __restrict__ sorted_slot,
                                                              const float4* __restrict__ slot_rec,
                                                              const uint32_t* __restrict__ slot_gid,
                                                              const uint32_t* __restrict__ anchor_of,
                                                              const float* __restrict__ color,
                                                              const float* __restrict__ target, int64_t n_anchor,
                                                              uint32_t* __restrict__ omega, uint32_t* __restrict__ kappa,
                                                              uint32_t* __restrict__ status) {
  const RenderParams& P = AP.R;
  __shared__ float4 s_rec[NW][64][3];
  __shared__ uint32_t s_key[NW][AS_TCAP];
  __shared__ uint64_t s_mask[NW][AS_TCAP];
  __shared__ uint32_t s_stack[NW][64];
  __shared__ uint32_t s_used[NW];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int gt = blockIdx.x;
  const int v = gt / P.n_tiles, t = gt - v * P.n_tiles;
  const int tx = t % P.tiles_x, ty = t / P.tiles_x;
  int sx, sy;
  tile_subblock(P.tile_w, w, sx, sy);
  const int bx = tx * P.tile_w + sx, by = ty * P.tile_h + sy;
  const int px = bx + (l & 7), py = by + (l >> 3);
  const bool inside = px < P.W && py < P.H;
  const int ox = pix_origin(P.W), oy = pix_origin(P.H);
  const float fpx = (float)(px - ox), fpy = (float)(py - oy);
  const uint2 rg = ranges[gt];
  const uint32_t start = rg.x, end = rg.y;
  // the error mask of the wave's pixels: sum over the channels of |I - I^| > tau_err
  bool M = false;
  if (inside) {
    const size_t npix = (size_t)P.W * P.H;
    const size_t c0 = (size_t)v * 3 * npix + (size_t)py * P.W + px;
    const float e = (fabsf(target[c0] - color[c0]) + fabsf(target[c0 + npix] - color[c0 + npix])) +
                    fabsf(target[c0 + 2 * npix] - color[c0 + 2 * npix]);
    M = e > AP.tau_err;
  }
  const uint64_t mmask = ballot64(M);
  // work stack of (part, bits): the anchors whose hash has `bits` low bits equal to part
  int sp = 0;
  if (l == 0) s_stack[w][0] = 0u;
  ++sp;
  __builtin_amdgcn_wave_barrier();
  while (sp > 0) {
    --sp;
    const uint32_t item = s_stack[w][sp];
    const uint32_t part = item & 0xffffu, bits = item >> 16;
    const uint32_t pmask = bits >= 32 ? 0xffffffffu : ((1u << bits) - 1u);
    for (int q = l; q < AS_TCAP; q += 64) {
      s_key[w][q] = AS_EMPTY;
      s_mask[w][q] = 0ull;
    }
    if (l == 0) s_used[w] = 0u;
    __builtin_amdgcn_wave_barrier();
    bool overflow = false;
    float T = inside ? 1.0f : -1.0f;
    for (uint32_t base = start; base < end && !overflow; base += 64) {
      if (!__any(T > 0.f)) break;
      const uint32_t k = base + (uint32_t)l;
      bool keep = false;
      float4 r0, r1, r2;
      uint32_t an = AS_EMPTY;
      if (k < end) {
        const uint32_t slot = sorted_slot[k];
        const float4* rec = slot_rec + (size_t)slot * 4;
        r0 = rec[0];
        r1 = rec[1];
        r2 = rec[2];
        const uint32_t xb = __float_as_uint(r1.w), yb = __float_as_uint(r2.w);
        const int xlo = (int)(int16_t)(xb & 0xffffu), xhi = (int)(int16_t)(xb >> 16);
        const int ylo = (int)(int16_t)(yb & 0xffffu), yhi = (int)(int16_t)(yb >> 16);
        if (xlo <= bx + 7 && xhi >= bx && ylo <= by + 7 && yhi >= by) {
          const float fx0 = (float)(bx - ox) - r0.x, fy0 = (float)(by - oy) - r0.y;
          keep = footprint_meets_box(fx0, fx0 + 7.0f, fy0, fy0 + 7.0f, r0, r1, P.log2_amin);
        }
        if (keep) an = anchor_of[slot_gid[slot]];
      }
      const uint64_t bal = ballot64(keep);
      if (keep) {
        const uint32_t q = mask_lt_count(bal);
        s_rec[w][q][0] = r0;
        s_rec[w][q][1] = r1;
        s_rec[w][q][2] = make_float4(r2.x, r2.y, r2.z, __uint_as_float(an));
      }
      __builtin_amdgcn_wave_barrier();
      const uint32_t len = (uint32_t)__popcll(bal);
      // lane j keeps the ballot of entry j (the pixels where it blends)
      uint64_t my_tb = 0ull;
      uint32_t nd = 0;
      for (uint32_t j = 0; j < len; ++j) {
        if (!__any(T > 0.f)) break;
        const float4 a0 = s_rec[w][j][0], a1 = s_rec[w][j][1];
        float dy, u;
        const float e = log2_alpha(fpx, fpy, a0, a1.x, a1.y, dy, u);
        const bool hit = T > 0.f && e >= P.log2_amin;
        const float a = hit ? fminf(exp2_approx(e), P.amax) : 0.f;
        const float Tn = T * (1.0f - a);
        const bool stop = hit && Tn < P.tmin;
        const bool take = hit && !stop;
        T = stop ? -T : Tn;   // a pixel that does not blend has a = 0, so Tn = T exactly
        const uint64_t tb = ballot64(take);
        my_tb = (uint32_t)l == j ? tb : my_tb;
        nd = j + 1;
      }
      // the batch's entries into the table, one per lane
      bool over = false;
      if ((uint32_t)l < nd && my_tb != 0ull) {
        const uint32_t anc = __float_as_uint(s_rec[w][l][2].w);
        if (anc < (uint32_t)n_anchor && (as_mix(anc) & pmask) == part) {
          uint32_t h = (as_mix(anc) >> bits) & (AS_TCAP - 1);
          for (int probe = 0; probe < AS_TCAP; ++probe) {
            const uint32_t key = atomicCAS(&s_key[w][h], AS_EMPTY, anc);
            if (key == AS_EMPTY || key == anc) {
              // a new key counts against the table's fill limit; at most 64
              // claims per batch past the limit still leave free slots
              if (key == AS_EMPTY && atomicAdd(&s_used[w], 1u) >= AS_TCAP * 3 / 4) over = true;
              atomicOr(reinterpret_cast<unsigned long long*>(&s_mask[w][h]), (unsigned long long)my_tb);
              break;
            }
            h = (h + 1) & (AS_TCAP - 1);
          }
        }
      }
      overflow = __any(over);
      __builtin_amdgcn_wave_barrier();
    }
    if (overflow) {
      // split this part by one more hash bit and walk each half again
      if (bits >= 16 || sp + 2 > 64) {
        if (l == 0) atomicOr(status, 4u);
        continue;
      }
      if (l == 0) {
        s_stack[w][sp] = part | ((bits + 1) << 16);
        s_stack[w][sp + 1] = (part | (1u << bits)) | ((bits + 1) << 16);
      }
      sp += 2;
      if (l == 0) atomicAdd(status + 1, 1u);   // counts the re-walks
      __builtin_amdgcn_wave_barrier();
      continue;
    }
    // flush the unions of this part
    for (int q = l; q < AS_TCAP; q += 64) {
      const uint32_t key = s_key[w][q];
      if (key == AS_EMPTY) continue;
      const uint64_t m = s_mask[w][q];
      const uint32_t om = (uint32_t)__popcll(m), ka = (uint32_t)__popcll(m & mmask);
      atomicAdd(omega + (size_t)v * n_anchor + key, om);
      if (ka) atomicAdd(kappa + (size_t)v * n_anchor + key, ka);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// per anchor: the chunk sums gain the views' counts; gamma with each view's loss (FP64, views in order)
__global__ __launch_bounds__(256) void k_anchor_accumulate(int V, int64_t n, const uint32_t* __restrict__ omega,
                                                           const uint32_t* __restrict__ kappa,
                                                           const float* __restrict__ view_loss,
                                                           kgs_view_stats st) {
  const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (a >= n) return;
  uint32_t om = 0, ka = 0;
  double gam = 0.0;
  for (int v = 0; v < V; ++v) {
    const uint32_t o = omega[(size_t)v * n + a];
    om += o;
    ka += kappa[(size_t)v * n + a];
    if (view_loss) gam += (double)view_loss[v] * (double)o;
  }
  if (st.omega_sum) st.omega_sum[a] += om;
  if (st.kappa_sum) st.kappa_sum[a] += ka;
  if (st.gamma_sum && view_loss) st.gamma_sum[a] += gam;
}

__global__ __launch_bounds__(256) void k_fill_zero_u32(uint32_t* __restrict__ p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) p[i] = 0u;
}

// ---------------------------------------------------------------- host side
kgs_status kgs_launch_anchor_decode(const kgs_anchors* a, const float* theta, const kgs_camera& cam,
                                    const kgs_gaussians_out* out, hipStream_t st) {
  DecodeParams P;
  double c[3];
  for (int i = 0; i < 3; ++i)
    c[i] = -((double)cam.R[i] * cam.t[0] + (double)cam.R[3 + i] * cam.t[1] + (double)cam.R[6 + i] * cam.t[2]);
  P.cx = c[0];
  P.cy = c[1];
  P.cz = c[2];
  const double eps[5] = {0.1, 0.25, 1.0, 5.0, 25.0};
  for (int l = 0; l < 5; ++l) {
    P.dmin[l] = l == 0 ? 0.0 : 100.0 * eps[l - 1];
    P.dmax[l] = l == 4 ? INFINITY : 100.0 * eps[l];
  }
  P.n = a->n;
  P.K = a->k;
  if (a->n == 0) return KGS_OK;
  const int64_t tiles = (a->n + 15) / 16;
  // each block stages the weights once; a few blocks per CU, each wave looping over tiles of 16 anchors
  const unsigned grid = (unsigned)std::min<int64_t>((tiles + 3) / 4, 1024);
  hipLaunchKernelGGL(k_anchor_decode, dim3(grid), dim3(256), 0, st, P, theta, *a, *out);
  return kgs_check_launch();
}

kgs_status kgs_launch_anchor_stats(kgs_ctx* ctx, const kgs_image* fwd, const uint32_t* anchor_of, int64_t n_anchor,
                                   const float* target, float tau_err, const float* view_loss, uint32_t* counts,
                                   const kgs_view_stats* stats, uint32_t* status, hipStream_t st) {
  const int V = ctx->last_views;
  const uint64_t nc = 2ull * V * (uint64_t)n_anchor;
  hipLaunchKernelGGL(k_fill_zero_u32, dim3((unsigned)std::max<uint64_t>(std::min<uint64_t>((nc + 255) / 256, 4096), 1)),
                     dim3(256), 0, st, counts, nc);
  AnchorStatParams AP;
  AP.R = render_params(ctx);
  AP.tau_err = tau_err;
  uint32_t* omega = counts;
  uint32_t* kappa = counts + (size_t)V * n_anchor;
  const unsigned grid = (unsigned)(V * ctx->n_tiles);
  if (grid > 0) {
    const uint32_t* sorted = ctx->sorted_slot;
    if (tile_waves(ctx) == 8)
      hipLaunchKernelGGL(k_anchor_footprint<8>, dim3(grid), dim3(512), 0, st, AP, (const uint2*)ctx->ranges, sorted,
                         (const float4*)ctx->slot_rec, (const uint32_t*)ctx->slot_gid, anchor_of,
                         (const float*)fwd->color, target, n_anchor, omega, kappa, status);
    else
      hipLaunchKernelGGL(k_anchor_footprint<4>, dim3(grid), dim3(256), 0, st, AP, (const uint2*)ctx->ranges, sorted,
                         (const float4*)ctx->slot_rec, (const uint32_t*)ctx->slot_gid, anchor_of,
                         (const float*)fwd->color, target, n_anchor, omega, kappa, status);
  }
  if (n_anchor > 0)
    hipLaunchKernelGGL(k_anchor_accumulate, dim3((unsigned)((n_anchor + 255) / 256)), dim3(256), 0, st, V, n_anchor,
                       (const uint32_t*)omega, (const uint32_t*)kappa, view_loss, *stats);
  return kgs_check_launch();
}
