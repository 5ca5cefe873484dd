// Front-to-back compositing (forward), the L1 loss harness and the
// compositing backward.
//
// One workgroup per (view, tile); each wave owns an 8x8 sub-block of the tile
// (four waves for 256-pixel tiles, eight for 512-pixel ones), or in a launch
// large enough to fill the device a 16x8 block with two pixels per lane (half
// the waves).  Every wave
// reads the tile's depth-sorted records itself, a batch at a time, tests each
// against its own sub-block (the integer rectangle, then the exact minimum of
// the conic over the sub-block's pixel-centre box, with a margin that keeps the
// test conservative) and keeps a compacted list of those that can reach its
// pixels, so a wave only evaluates Gaussians that can blend there and no
// result changes.  The forward shares nothing between waves; a wave stops as
// soon as all its pixels are saturated.
//
// The backward recomputes the same per-pixel sequence front to back (nothing
// per pixel is stored but T_final and the last blended position), reduces the
// per-pair gradient terms across the wave with a reduce-scatter butterfly (in
// a large launch a wave owns a 16x8 block, two pixels per lane, and sums a
// lane's two pixels before the reduction, which then serves 128 pixels), and
// after each batch the first wave adds the waves' partials in wave order and
// writes one 48-byte record per pair at the pair's emission position, which
// keeps each slot's pairs contiguous for the deterministic segmented sum that
// follows.  It stops each tile at the last batch any of its pixels reaches;
// the pairs behind it are never written, and a flag byte per pair tells the
// segmented sum which ones were.
#include "kgs_internal.h"

// Forward: every wave stages the tile's records itself, 64 at a time (one per
// lane), keeps those that reach its sub-block (rectangle, then the exact
// footprint test) compacted in its own LDS rows, and composites them; no
// workgroup barrier, so each wave stops as soon as its own pixels saturate.
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_render_fwd(RenderParams P, const uint2* __restrict__ ranges,
                                                        const uint32_t* __restrict__ tile_order,
                                                        const uint32_t* __restrict__ sorted_slot,
                                                        const float4* __restrict__ slot_rec,
                                                        float* __restrict__ color, float* __restrict__ depth,
                                                        float* __restrict__ tfinal, int32_t* __restrict__ last) {
  // each kept record's three float4 side by side: one address, three offsets;
  // r1.w (the x-bounds, used only by the staging test) holds the record's
  // position in the tile list, plus one.  Row 64 is never written: a round
  // reads entry j + 1 even when it does not exist (and ignores it).
  __shared__ float4 s_rec[NW][65][3];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int gt = (int)tile_order[blockIdx.x];
  const int v = gt / P.n_tiles, t = gt - v * P.n_tiles;
  const int tx = t % P.tiles_x, ty = t / P.tiles_x;
  const int tile_x0 = tx * P.tile_w, tile_y0 = ty * P.tile_h;
  int sx, sy;
  tile_subblock(P.tile_w, w, sx, sy);
  const int bx = tile_x0 + sx, by = tile_y0 + sy;
  const int px = bx + (l & 7), py = by + (l >> 3);
  const bool inside = px < P.W && py < P.H;
  const int ox = pix_origin(P.W), oy = pix_origin(P.H);
  const float fpx = (float)(px - ox), fpy = (float)(py - oy);
  const uint2 rg = ranges[gt];
  const uint32_t start = rg.x, end = rg.y;
  // the rows start as zeros: an absent second entry reads finite values, which
  // its zero weight then leaves out of the sums
  {
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    s_rec[w][l][0] = z;
    s_rec[w][l][1] = z;
    s_rec[w][l][2] = z;
    if (l < 3) s_rec[w][64][l] = z;
  }
  __builtin_amdgcn_wave_barrier();
  // T > 0 while the pixel composites; a pixel that saturates (or lies outside
  // the image) keeps -T, its final transmittance negated
  float T = inside ? 1.0f : -1.0f, c0 = 0.f, c1 = 0.f, c2 = 0.f, D = 0.f;
  int lst = 0;
  for (uint32_t base = start; base < end; base += 64) {
    if (!__any(T > 0.f)) break;
    // stage: lane l takes record base + l and keeps it if it reaches this sub-block
    const uint32_t k = base + (uint32_t)l;
    bool keep = false;
    float4 r0, r1, r2;
    if (k < end) {
      const float4* rec = slot_rec + (size_t)sorted_slot[k] * 4;
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
    }
    const uint64_t bal = ballot64(keep);
    if (keep) {
      const uint32_t q = mask_lt_count(bal);
      s_rec[w][q][0] = r0;
      s_rec[w][q][1] = make_float4(r1.x, r1.y, r1.z, __int_as_float((int)(k - start) + 1));
      s_rec[w][q][2] = r2;
    }
    __builtin_amdgcn_wave_barrier();
    const uint32_t len = (uint32_t)__popcll(bal);
    auto blend = [&](uint32_t q, bool present) {
      const float4 a0 = s_rec[w][q][0], a1 = s_rec[w][q][1], a2 = s_rec[w][q][2];
      float dy, u;
      const float e = log2_alpha(fpx, fpy, a0, a1.x, a1.y, dy, u);
      const bool hit = present && T > 0.f && e >= P.log2_amin;
      const float a = hit ? fminf(exp2_approx(e), P.amax) : 0.f;
      const float Tn = T * (1.0f - a);
      const bool stop = hit && Tn < P.tmin;
      const bool take = hit && !stop;
      const float wgt = take ? a * T : 0.f;
      c0 = fmaf(wgt, a2.x, c0);
      c1 = fmaf(wgt, a2.y, c1);
      c2 = fmaf(wgt, a2.z, c2);
      D = fmaf(wgt, a1.z, D);
      T = stop ? -T : Tn;   // a lane that does not blend has a = 0, so Tn = T exactly
      lst = take ? __float_as_int(a1.w) : lst;
    };
    // two entries per round (one saturation check for both)
    for (uint32_t j = 0; j < len; j += 2) {
      if (!__any(T > 0.f)) break;
      blend(j, true);
      blend(j + 1, j + 1 < len);
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (inside) {
    const size_t npix = (size_t)P.W * P.H;
    const size_t pix = (size_t)v * npix + (size_t)py * P.W + px;
    const size_t cpix = (size_t)v * 3 * npix + (size_t)py * P.W + px;
    T = fabsf(T);
    color[cpix] = c0 + T * P.bg0;
    color[cpix + npix] = c1 + T * P.bg1;
    color[cpix + 2 * npix] = c2 + T * P.bg2;
    depth[pix] = D;
    tfinal[pix] = T;
    last[pix] = lst;
  }
}

// Forward with PPL pixels per lane: a wave composites an (8 PPL)x8 block, lane l
// the pixels (8 p + l % 8, l / 8), p < PPL, of it, so one staging round, one
// record read from LDS and one loop step serve PPL pixels.  Each pixel's
// arithmetic is that of k_render_fwd, so the images are the same bits; the
// wave stops when all of every lane's pixels have saturated.
template <int NW, int PPL>
__global__ __launch_bounds__(64 * NW) void k_render_fwdn(RenderParams P, const uint2* __restrict__ ranges,
                                                         const uint32_t* __restrict__ tile_order,
                                                         const uint32_t* __restrict__ sorted_slot,
                                                         const float4* __restrict__ slot_rec,
                                                         float* __restrict__ color, float* __restrict__ depth,
                                                         float* __restrict__ tfinal, int32_t* __restrict__ last) {
  __shared__ float4 s_rec[NW][65][3];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int gt = (int)tile_order[blockIdx.x];
  const int v = gt / P.n_tiles, t = gt - v * P.n_tiles;
  const int tx = t % P.tiles_x, ty = t / P.tiles_x;
  constexpr int BW = 8 * PPL;        // block width
  const int nsx = P.tile_w / BW;     // blocks per tile row, in row-major order
  const int bx = tx * P.tile_w + (w % nsx) * BW, by = ty * P.tile_h + (w / nsx) * 8;
  const int py = by + (l >> 3);
  const int ox = pix_origin(P.W), oy = pix_origin(P.H);
  const float fpy = (float)(py - oy);
  int px[PPL];
  float fpx[PPL], T[PPL], c0[PPL], c1[PPL], c2[PPL], D[PPL];
  int lst[PPL];
  auto any_open = [&]() {
    bool o = false;
#pragma unroll
    for (int p = 0; p < PPL; ++p) o = o || T[p] > 0.f;
    return __any(o);
  };
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    px[p] = bx + 8 * p + (l & 7);
    fpx[p] = (float)(px[p] - ox);
    T[p] = px[p] < P.W && py < P.H ? 1.0f : -1.0f;
    c0[p] = c1[p] = c2[p] = D[p] = 0.f;
    lst[p] = 0;
  }
  const uint2 rg = ranges[gt];
  const uint32_t start = rg.x, end = rg.y;
  {
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    s_rec[w][l][0] = z;
    s_rec[w][l][1] = z;
    s_rec[w][l][2] = z;
    if (l < 3) s_rec[w][64][l] = z;
  }
  __builtin_amdgcn_wave_barrier();
  for (uint32_t base = start; base < end; base += 64) {
    if (!any_open()) break;
    const uint32_t k = base + (uint32_t)l;
    bool keep = false;
    float4 r0, r1, r2;
    if (k < end) {
      const float4* rec = slot_rec + (size_t)sorted_slot[k] * 4;
      r0 = rec[0];
      r1 = rec[1];
      r2 = rec[2];
      const uint32_t xb = __float_as_uint(r1.w), yb = __float_as_uint(r2.w);
      const int xlo = (int)(int16_t)(xb & 0xffffu), xhi = (int)(int16_t)(xb >> 16);
      const int ylo = (int)(int16_t)(yb & 0xffffu), yhi = (int)(int16_t)(yb >> 16);
      if (xlo <= bx + BW - 1 && xhi >= bx && ylo <= by + 7 && yhi >= by) {
        const float fx0 = (float)(bx - ox) - r0.x, fy0 = (float)(by - oy) - r0.y;
        keep = footprint_meets_box(fx0, fx0 + (float)(BW - 1), fy0, fy0 + 7.0f, r0, r1, P.log2_amin);
      }
    }
    const uint64_t bal = ballot64(keep);
    if (keep) {
      const uint32_t q = mask_lt_count(bal);
      s_rec[w][q][0] = r0;
      s_rec[w][q][1] = make_float4(r1.x, r1.y, r1.z, __int_as_float((int)(k - start) + 1));
      s_rec[w][q][2] = r2;
    }
    __builtin_amdgcn_wave_barrier();
    const uint32_t len = (uint32_t)__popcll(bal);
    auto blend = [&](uint32_t q, bool present) {
      const float4 a0 = s_rec[w][q][0], a1 = s_rec[w][q][1], a2 = s_rec[w][q][2];
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        float dy, u;
        const float e = log2_alpha(fpx[p], fpy, a0, a1.x, a1.y, dy, u);
        const bool hit = present && T[p] > 0.f && e >= P.log2_amin;
        const float a = hit ? fminf(exp2_approx(e), P.amax) : 0.f;
        const float Tn = T[p] * (1.0f - a);
        const bool stop = hit && Tn < P.tmin;
        const bool take = hit && !stop;
        const float wgt = take ? a * T[p] : 0.f;
        c0[p] = fmaf(wgt, a2.x, c0[p]);
        c1[p] = fmaf(wgt, a2.y, c1[p]);
        c2[p] = fmaf(wgt, a2.z, c2[p]);
        D[p] = fmaf(wgt, a1.z, D[p]);
        T[p] = stop ? -T[p] : Tn;   // a pixel that does not blend has a = 0, so Tn = T exactly
        lst[p] = take ? __float_as_int(a1.w) : lst[p];
      }
    };
    for (uint32_t j = 0; j < len; j += 2) {
      if (!any_open()) break;
      blend(j, true);
      blend(j + 1, j + 1 < len);
    }
    __builtin_amdgcn_wave_barrier();
  }
  const size_t npix = (size_t)P.W * P.H;
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    if (px[p] < P.W && py < P.H) {
      const size_t pix = (size_t)v * npix + (size_t)py * P.W + px[p];
      const size_t cpix = (size_t)v * 3 * npix + (size_t)py * P.W + px[p];
      const float Tf = fabsf(T[p]);
      color[cpix] = c0[p] + Tf * P.bg0;
      color[cpix + npix] = c1[p] + Tf * P.bg1;
      color[cpix + 2 * npix] = c2[p] + Tf * P.bg2;
      depth[pix] = D[p];
      tfinal[pix] = Tf;
      last[pix] = lst[p];
    }
  }
}

// ---------------------------------------------------------------- L1 loss harness
// One workgroup per (view, tile), pixels mapped to lanes as in the
// compositing kernels.  Per pixel |dR| + |dG| + |dB| in FP32, summed over the
// wave by a fixed butterfly, the waves in order in FP64, one partial per
// (view, tile); k_loss_final adds the partials of a view in tile order.  The
// chunk's fused backward forms the same partials in the same order, so both
// routes give the same bits.
__device__ __forceinline__ void l1_pixel(const float* __restrict__ color, const float* __restrict__ target,
                                         size_t cpix, size_t npix, float scale, float& g0, float& g1, float& g2,
                                         float& acc) {
  const float d0 = color[cpix] - target[cpix];
  const float d1 = color[cpix + npix] - target[cpix + npix];
  const float d2 = color[cpix + 2 * npix] - target[cpix + 2 * npix];
  acc = (fabsf(d0) + fabsf(d1)) + fabsf(d2);
  g0 = d0 > 0.f ? scale : (d0 < 0.f ? -scale : 0.f);
  g1 = d1 > 0.f ? scale : (d1 < 0.f ? -scale : 0.f);
  g2 = d2 > 0.f ? scale : (d2 < 0.f ? -scale : 0.f);
}

// the block's per-pixel values acc -> partial[gt] (uses sh[NW PPL] and one
// barrier).  A wave holds PPL pixels per lane, the p-th of each lane in the
// p-th 8x8 sub-block of its block; each sub-block is summed by a fixed
// butterfly, and the NW PPL sub-blocks, in row-major order, are added pairwise
// in FP64.  With either pixel layout the partial has the same bits.
template <int NW, int PPL>
__device__ __forceinline__ void l1_partial(const float (&acc)[PPL], float* sh, double* __restrict__ partial,
                                           int gt) {
  constexpr int NS = NW * PPL;
  static_assert(NS == 4 || NS == 8, "four or eight sub-blocks per tile");
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    const float a = wave_sum(acc[p]);
    if ((threadIdx.x & 63) == 0) sh[w * PPL + p] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double d = ((double)sh[0] + (double)sh[1]) + ((double)sh[2] + (double)sh[3]);
    if (NS == 8) d += ((double)sh[4] + (double)sh[5]) + ((double)sh[6] + (double)sh[7]);
    partial[gt] = d;
  }
}

template <int NW>
__global__ __launch_bounds__(64 * NW) void k_loss_l1(RenderParams P, const float* __restrict__ color,
                                                       const float* __restrict__ target, float* __restrict__ grad,
                                                       double* __restrict__ partial) {
  __shared__ float sh[NW];
  const int gt = blockIdx.x;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int v = gt / P.n_tiles, t = gt - v * P.n_tiles;
  const int tx = t % P.tiles_x, ty = t / P.tiles_x;
  int sx, sy;
  tile_subblock(P.tile_w, w, sx, sy);
  const int px = tx * P.tile_w + sx + (l & 7), py = ty * P.tile_h + sy + (l >> 3);
  const size_t npix = (size_t)P.W * P.H;
  const float scale = 1.0f / (float)(3 * npix);
  float acc[1] = {0.f};
  if (px < P.W && py < P.H) {
    const size_t cpix = (size_t)v * 3 * npix + (size_t)py * P.W + px;
    float g0, g1, g2;
    l1_pixel(color, target, cpix, npix, scale, g0, g1, g2, acc[0]);
    grad[cpix] = g0;
    grad[cpix + npix] = g1;
    grad[cpix + 2 * npix] = g2;
  }
  l1_partial<NW, 1>(acc, sh, partial, gt);
}

// one workgroup of KGS_FINAL_THREADS per view: thread l adds tiles l, l + 256,
// ... in order, then a fixed butterfly over each wave and the four wave sums
// in a fixed tree (a single wave walking all the tiles was latency-bound)
__global__ __launch_bounds__(KGS_FINAL_THREADS) void k_loss_final(int n_tiles, double inv_n,
                                                                  const double* __restrict__ partial,
                                                                  float* __restrict__ view_loss) {
  __shared__ double sh[KGS_FINAL_THREADS / 64];
  const int v = blockIdx.x, l = threadIdx.x;
  double s = 0.0;
  for (int b = l; b < n_tiles; b += KGS_FINAL_THREADS) s += partial[(size_t)v * n_tiles + b];
  s = block_sum_fixed(s, sh);
  if (l == 0) view_loss[v] = (float)(s * inv_n);
}

// ---------------------------------------------------------------- backward
// Reduce-scatter of 10 values over a wave: after the call lane L holds, in
// x[0], the wave sum of value 5 b5 + 3 b4 + 2 b3 + b2 (b_k = bit k of L) when
// `valid` is set.
__device__ __forceinline__ float f_swap_sum32(float lo_keep, float hi_keep) {
  // lanes 0-31 end with the wave-half sum of lo_keep, lanes 32-63 of hi_keep
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo_keep), __float_as_uint(hi_keep), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float f_swap_sum16(float even_keep, float odd_keep) {
  // 16-lane rows 0 and 2 end with even_keep summed over row pairs, rows 1 and 3 with odd_keep
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(even_keep), __float_as_uint(odd_keep), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

template <int CTRL>
__device__ __forceinline__ float f_dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// Reduce-scatter of ten per-lane values over the wave.  Each step pairs every
// lane with a partner whose lane bit b differs (lane halves, row pairs, the
// mirrored lane of a 16-lane row, the mirrored lane of an 8-lane half-row);
// the lane keeps the values its bit selects and adds the partner's copy.  The
// two pairings inside a quad then complete the sums.  Lanes with valid set
// hold the full wave sum of value idx.
__device__ __forceinline__ void wave_reduce10(float (&x)[10], int lane, int& idx, bool& valid) {
  const bool u4 = lane & 16, u3 = lane & 8, u2 = lane & 4;
#pragma unroll
  for (int k = 0; k < 5; ++k) x[k] = f_swap_sum32(x[k], x[k + 5]);
  x[0] = f_swap_sum16(x[0], x[3]);
  x[1] = f_swap_sum16(x[1], x[4]);
  x[2] = f_swap_sum16(x[2], 0.f);
  {
    const float s0 = u3 ? x[0] : x[2], k0 = u3 ? x[2] : x[0];
    const float s1 = u3 ? x[1] : 0.f, k1 = u3 ? 0.f : x[1];
    x[0] = k0 + f_dpp<0x140>(s0);  // row_mirror: lane 15 - i of the row
    x[1] = k1 + f_dpp<0x140>(s1);
  }
  {
    const float s0 = u2 ? x[0] : x[1], k0 = u2 ? x[1] : x[0];
    x[0] = k0 + f_dpp<0x141>(s0);  // row_half_mirror: lane 7 - i of the half-row
  }
  x[0] += f_dpp<0xB1>(x[0]);       // quad_perm [1, 0, 3, 2]
  x[0] += f_dpp<0x4E>(x[0]);       // quad_perm [2, 3, 0, 1]
  const int k = (u3 ? 2 : 0) + (u2 ? 1 : 0);
  const int rel = (u4 ? 3 : 0) + k;
  valid = (k < 3) && (rel < 5) && ((lane & 3) == 0);
  idx = ((lane & 32) ? 5 : 0) + rel;
}

// The same for twenty values (two pairs): lane halves, row pairs, mirrored
// lanes of a row (five values to three), of a half-row (three to two), then
// the lane pair inside a quad (two to one) and the other quad pair.  Lanes
// with valid set hold the full wave sum of value idx.  With NV = 9 the tenth
// value of each half is known to be zero and its first step is skipped.
template <int NV>
__device__ __forceinline__ void wave_reduce20(float (&x)[20], int lane, int& idx, bool& valid) {
  static_assert(NV == 9 || NV == 10, "nine or ten values per entry");
  const bool u4 = lane & 16, u3 = lane & 8, u2 = lane & 4, u0 = lane & 1;
#pragma unroll
  for (int k = 0; k < 10; ++k) x[k] = k < NV ? f_swap_sum32(x[k], x[k + 10]) : 0.f;
#pragma unroll
  for (int k = 0; k < 5; ++k) x[k] = f_swap_sum16(x[k], x[k + 5]);
  {
    const float s0 = u3 ? x[0] : x[3], k0 = u3 ? x[3] : x[0];
    const float s1 = u3 ? x[1] : x[4], k1 = u3 ? x[4] : x[1];
    const float s2 = u3 ? x[2] : 0.f, k2 = u3 ? 0.f : x[2];
    x[0] = k0 + f_dpp<0x140>(s0);
    x[1] = k1 + f_dpp<0x140>(s1);
    x[2] = k2 + f_dpp<0x140>(s2);
  }
  {
    const float s0 = u2 ? x[0] : x[2], k0 = u2 ? x[2] : x[0];
    const float s1 = u2 ? x[1] : 0.f, k1 = u2 ? 0.f : x[1];
    x[0] = k0 + f_dpp<0x141>(s0);
    x[1] = k1 + f_dpp<0x141>(s1);
  }
  {
    const float s0 = u0 ? x[0] : x[1], k0 = u0 ? x[1] : x[0];
    x[0] = k0 + f_dpp<0xB1>(s0);
  }
  x[0] += f_dpp<0x4E>(x[0]);
  const int rel = (u3 ? 3 : 0) + (u2 ? 2 : 0) + (u0 ? 1 : 0);
  valid = (u3 ? rel <= 4 : rel <= 2) && ((lane & 2) == 0);
  idx = ((lane & 32) ? 10 : 0) + (u4 ? 5 : 0) + rel;
}

// Per-pixel terms of one blended pair in the backward.  Lanes that do not blend
// come with e = -inf: exp2 gives alpha = 0, which zeroes every term and leaves
// T and Rj unchanged (the blend mask is applied to e once, so no lane mask has
// to live across the reduction's branches).
//   dL/dalpha_j = T_j (g . c_j) + Rj / (1 - alpha_j)
// with Rj = gAT - g . C + g . C_j (C the final colour and depth, C_j its part
// from Gaussians up to j).  x[0..5] are the moments (ge u, ge dy, ge u^2,
// ge u dy, ge dy^2, ge) with ge = dL/d(log2 alpha) / ln 2 (zero where alpha is
// clamped at alpha_max): with log2 alpha = log2 o + P' u^2 + E' dy^2 and
// u = dx + k dy, the pair's P', k, E' and ln 2 turn their sums into the
// record-space derivatives.  x[6..9] = alpha_j T_j g (colour and depth).
template <bool DEPTH, bool CLAMP>
__device__ __forceinline__ void blend_terms(float e, float u, float dy, const float4& r1, const float4& r2,
                                            float amax, float g0, float g1, float g2, float gD, float& T, float& Rj,
                                            float* __restrict__ x) {
  const float raw = exp2_approx(e);
  const float a = CLAMP ? fminf(raw, amax) : raw;
  const float wgt = a * T;
  // without a depth gradient (gD = 0) the depth terms are zero and left out
  const float gcc = fmaf(g2, r2.z, fmaf(g1, r2.y, g0 * r2.x));
  const float gc = DEPTH ? fmaf(gD, r1.z, gcc) : gcc;
  Rj = fmaf(wgt, gc, Rj);
  const float oma = 1.0f - a;
  const float dLda = fmaf(T, gc, Rj * __builtin_amdgcn_rcpf(oma));
  x[6] = wgt * g0;
  x[7] = wgt * g1;
  x[8] = wgt * g2;
  x[9] = DEPTH ? wgt * gD : 0.f;
  const float ge = !CLAMP || raw < amax ? dLda * a : 0.f;
  const float gu = ge * u, gd = ge * dy;
  x[0] = gu;
  x[1] = gd;
  x[2] = gu * u;
  x[3] = gu * dy;
  x[4] = gd * dy;
  x[5] = ge;
  T = T * oma;
}

// The same terms summed over a lane's two pixels, which share a row and so dy:
// the moments with a factor dy are formed once from the pixel sums,
// sum ge dy = dy sum ge and so on, instead of per pixel.  Without CLAMP the
// caller knows that no record of the batch reaches alpha_max, and the clamp
// and its zero derivative are left out (the same values).
template <bool DEPTH, bool CLAMP>
__device__ __forceinline__ void blend_terms2(const float (&e)[2], const float (&u)[2], float dy,
                                             const float4& r1, const float4& r2, float amax, const float (&g0)[2],
                                             const float (&g1)[2], const float (&g2)[2], const float (&gD)[2],
                                             float (&T)[2], float (&Rj)[2], float* __restrict__ x) {
  float ge[2], gu[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const float raw = exp2_approx(e[p]);
    const float a = CLAMP ? fminf(raw, amax) : raw;
    const float wgt = a * T[p];
    const float gcc = fmaf(g2[p], r2.z, fmaf(g1[p], r2.y, g0[p] * r2.x));
    const float gc = DEPTH ? fmaf(gD[p], r1.z, gcc) : gcc;
    Rj[p] = fmaf(wgt, gc, Rj[p]);
    const float oma = 1.0f - a;
    const float dLda = fmaf(T[p], gc, Rj[p] * __builtin_amdgcn_rcpf(oma));
    if (p == 0) {
      x[6] = wgt * g0[p];
      x[7] = wgt * g1[p];
      x[8] = wgt * g2[p];
      x[9] = DEPTH ? wgt * gD[p] : 0.f;
    } else {
      x[6] = fmaf(wgt, g0[p], x[6]);
      x[7] = fmaf(wgt, g1[p], x[7]);
      x[8] = fmaf(wgt, g2[p], x[8]);
      x[9] = DEPTH ? fmaf(wgt, gD[p], x[9]) : 0.f;
    }
    ge[p] = !CLAMP || raw < amax ? dLda * a : 0.f;
    gu[p] = ge[p] * u[p];
    T[p] = T[p] * oma;
  }
  x[5] = ge[0] + ge[1];
  x[0] = gu[0] + gu[1];
  x[1] = x[5] * dy;
  x[2] = fmaf(gu[1], u[1], gu[0] * u[0]);
  x[3] = x[0] * dy;
  x[4] = x[1] * dy;
}

// Emission position of the pair (slot, tile (tx, ty)): the slot's first pair
// plus the tile's row-major rank in the slot's tile rectangle, which is
// recovered from the record's packed pixel bounds.
__device__ __forceinline__ uint32_t pair_position(uint32_t first, float xb_f, float yb_f, int tx, int ty,
                                                  const RenderParams& P) {
  const uint32_t xb = __float_as_uint(xb_f), yb = __float_as_uint(yb_f);
  const int xlo = (int)(int16_t)(xb & 0xffffu), xhi = (int)(int16_t)(xb >> 16);
  const int ylo = (int)(int16_t)(yb & 0xffffu);
  const int x0 = max(floordiv_pow2(xlo, P.tile_w), 0), x1 = min(floordiv_pow2(xhi, P.tile_w) + 1, P.tiles_x);
  const int y0 = max(floordiv_pow2(ylo, P.tile_h), 0);
  return first + (uint32_t)((ty - y0) * (x1 - x0) + (tx - x0));
}

// PPL pixels per lane: a wave covers a block of 8 PPL x 8 pixels, lane l the
// pixels (8 p + l % 8, l / 8), p < PPL, of its block.  With two pixels per
// lane a list entry's ten terms are summed over the lane's two pixels before
// the one reduction over the wave, so the reductions per pixel halve; the
// block is tested against the footprint as a whole.
template <int PPL>
__device__ __forceinline__ void wave_block(int tile_w, int w, int& sx, int& sy) {
  const int nsx = tile_w / (8 * PPL);  // blocks per tile row, in row-major order
  sx = (w % nsx) * (8 * PPL);
  sy = (w / nsx) * 8;
}

template <int B, int NW, bool DEPTH, int PPL>
__global__ __launch_bounds__(64 * NW) void k_render_bwd(
    RenderParams P, const uint2* __restrict__ ranges, const uint32_t* __restrict__ tile_order,
    const uint32_t* __restrict__ sorted_slot,
    const float4* __restrict__ slot_rec, const float* __restrict__ color,
    const float* __restrict__ depth, const float* __restrict__ tfinal, const int32_t* __restrict__ last,
    const float* __restrict__ dl_dcolor, const float* __restrict__ dl_ddepth, const float* __restrict__ dl_dtfinal,
    const float* __restrict__ target, float tau_err, float4* __restrict__ pair_grad,
    uint8_t* __restrict__ pair_live, int fuse_l1,
    float* __restrict__ dl_out, double* __restrict__ loss_partial) {
  // B records per batch, R = B / 64 per lane (B = 32: the first half of the lanes)
  constexpr int R = B >= 64 ? B / 64 : 1;
  constexpr int BW = 8 * PPL;  // width of a wave's block
  static_assert(B == 32 || B == 64 || B == 128, "batch of 32, 64 or 128 records");
  static_assert(PPL == 1 || PPL == 2, "one or two pixels per lane");
  // each wave's kept records of the batch, compacted, and their batch indices
  __shared__ float4 s_rec[NW][B][3];
  __shared__ __align__(16) uint8_t s_id[NW][B];
  __shared__ uint64_t s_keep[NW][R];
  __shared__ float s_part[NW][B][12];
  __shared__ int s_wmax[NW];
  __shared__ float s_loss[NW * PPL];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int gt = (int)tile_order[blockIdx.x];
  const int v = gt / P.n_tiles, t = gt - v * P.n_tiles;
  const int tx = t % P.tiles_x, ty = t / P.tiles_x;
  const int tile_x0 = tx * P.tile_w, tile_y0 = ty * P.tile_h;
  int sx, sy;
  wave_block<PPL>(P.tile_w, w, sx, sy);
  const int bx = tile_x0 + sx, by = tile_y0 + sy;
  const int py = by + (l >> 3);
  const int ox = pix_origin(P.W), oy = pix_origin(P.H);
  const float fpy = (float)(py - oy);
  const uint2 rg = ranges[gt];
  const uint32_t start = rg.x, end = rg.y;
  // per-pixel inputs
  // dL/dalpha_j = T_j (g . c_j) - (g . (C - C_j)) / (1 - alpha_j) + gAT / (1 - alpha_j)
  // with C the final colour (and depth) and C_j its part from Gaussians up to j;
  // Rj = gAT - g . C + g . C_j is kept as one running scalar per pixel
  int lastp[PPL];
  float fpx[PPL], g0[PPL], g1[PPL], g2[PPL], gD[PPL], T[PPL], Rj[PPL], l1acc[PPL];
  uint64_t Mbal[PPL];  // the error mask of the wave's pixels
  int wmax = 0;
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    const int px = bx + 8 * p + (l & 7);
    fpx[p] = (float)(px - ox);
    lastp[p] = 0;
    float Co0 = 0.f, Co1 = 0.f, Co2 = 0.f, Do = 0.f, gAT = 0.f;
    g0[p] = g1[p] = g2[p] = gD[p] = 0.f;
    l1acc[p] = 0.f;
    bool M = false;
    if (px < P.W && py < P.H) {
      const size_t npix = (size_t)P.W * P.H;
      const size_t pix = (size_t)v * npix + (size_t)py * P.W + px;
      const size_t cpix = (size_t)v * 3 * npix + (size_t)py * P.W + px;
      lastp[p] = last[pix];
      Co0 = color[cpix];
      Co1 = color[cpix + npix];
      Co2 = color[cpix + 2 * npix];
      Do = depth[pix];
      if (fuse_l1) {
        // the L1 loss against target, its gradient and its per-tile partial,
        // exactly as the loss kernel forms them
        l1_pixel(color, target, cpix, npix, 1.0f / (float)(3 * npix), g0[p], g1[p], g2[p], l1acc[p]);
        if (dl_out) {
          dl_out[cpix] = g0[p];
          dl_out[cpix + npix] = g1[p];
          dl_out[cpix + 2 * npix] = g2[p];
        }
      } else {
        g0[p] = dl_dcolor[cpix];
        g1[p] = dl_dcolor[cpix + npix];
        g2[p] = dl_dcolor[cpix + 2 * npix];
      }
      if (dl_ddepth) gD[p] = dl_ddepth[pix];
      // the final transmittance: dT_final/dalpha_j = -T_final / (1 - alpha_j)
      if (dl_dtfinal) gAT = -dl_dtfinal[pix] * tfinal[pix];
      if (target) {
        const float err = fabsf(target[cpix] - Co0) + fabsf(target[cpix + npix] - Co1) +
                          fabsf(target[cpix + 2 * npix] - Co2);
        M = err > tau_err;
      }
    }
    Mbal[p] = ballot64(M);
    T[p] = 1.0f;
    Rj[p] = gAT - (g0[p] * Co0 + g1[p] * Co1 + g2[p] * Co2 + gD[p] * Do);
    wmax = max(wmax, lastp[p]);
  }
  if (fuse_l1) l1_partial<NW, PPL>(l1acc, s_loss, loss_partial, gt);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wmax = max(wmax, __shfl_xor(wmax, o, 64));
  wmax = __builtin_amdgcn_readfirstlane(wmax);
  if (l == 0) s_wmax[w] = wmax;
  __syncthreads();
  int bmax = s_wmax[0];
#pragma unroll
  for (int k = 1; k < NW; ++k) bmax = max(bmax, s_wmax[k]);
  const uint32_t pend = start + (uint32_t)bmax;
  uint32_t base = start;
  for (; base < pend; base += B) {
    // stage: every wave reads the batch's records (lane l: records l, l + 64,
    // ...) and keeps, compacted in order, those that reach its block; the
    // first wave also keeps what the pair records need
    uint32_t len = 0;
    float xbw[R], ybw[R];
    uint32_t firstp[R];
    uint64_t clamp_bal = 0ull;  // kept records that may reach alpha_max somewhere
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int bi = r * 64 + l;
      const uint32_t k = base + (uint32_t)bi;
      bool keep = false;
      // defined on every path: left unset where no record is read, the 64-record
      // variants kept r2 in scratch memory (a store and a reload per record)
      float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
      xbw[r] = 0.f;
      ybw[r] = 0.f;
      firstp[r] = 0u;
      if (bi < B && k < end) {
        const float4* rec = slot_rec + (size_t)sorted_slot[k] * 4;
        r0 = rec[0];
        r1 = rec[1];
        r2 = rec[2];
        if (w == 0) firstp[r] = __float_as_uint(rec[3].x);
        xbw[r] = r1.w;
        ybw[r] = r2.w;
        const uint32_t xb = __float_as_uint(r1.w), yb = __float_as_uint(r2.w);
        const int xlo = (int)(int16_t)(xb & 0xffffu), xhi = (int)(int16_t)(xb >> 16);
        const int ylo = (int)(int16_t)(yb & 0xffffu), yhi = (int)(int16_t)(yb >> 16);
        if (xlo <= bx + BW - 1 && xhi >= bx && ylo <= by + 7 && yhi >= by) {
          const float fx0 = (float)(bx - ox) - r0.x, fy0 = (float)(by - oy) - r0.y;
          keep = footprint_meets_box(fx0, fx0 + (float)(BW - 1), fy0, fy0 + 7.0f, r0, r1, P.log2_amin);
        }
      }
      const uint64_t bal = ballot64(keep);
      clamp_bal |= bal & ballot64(r1.y >= P.log2_amax_lo);
      if (keep) {
        const uint32_t q = len + mask_lt_count(bal);
        s_rec[w][q][0] = r0;
        s_rec[w][q][1] = r1;
        s_rec[w][q][2] = r2;
        s_id[w][q] = (uint8_t)bi;
      }
      if (l == 0) s_keep[w][r] = bal;
      len += (uint32_t)__popcll(bal);
    }
    __builtin_amdgcn_wave_barrier();
    const int rel0 = (int)(base - start);
    // the wave's list entries (batch indices), four to a lane, read by lane
    // index; the records of entry j sit at position j of the wave's rows
    const uint32_t packed = 4 * l < B ? reinterpret_cast<const uint32_t*>(s_id[w])[l] : 0u;
    auto entry = [&](uint32_t j) -> int {
      return (int)((__builtin_amdgcn_readlane(packed, (int)(j >> 2)) >> (8u * (j & 3u))) & 0xffu);
    };
    // list entries two at a time: a pair of entries that both blend shares one
    // reduction of twenty values; otherwise the one that blends is reduced alone.
    // Batches in which no kept record can reach alpha_max (nearly all) take the
    // variant without the clamp.
    auto entries = [&](auto clamp_tag) {
      constexpr bool CL = decltype(clamp_tag)::value;
      for (uint32_t j = 0; j < len;) {
        const int ta = entry(j);  // batch index, the same for the whole wave
        if (rel0 + ta >= wmax) break;
        const bool has_b = j + 1 < len;
        const uint32_t jb = has_b ? j + 1 : j;
        const int tb = entry(jb);
        const bool use_b = has_b && rel0 + tb < wmax;
        // both entries' records at once (the second is a repeat of the first when absent)
        const float4 ra0 = s_rec[w][j][0], ra1 = s_rec[w][j][1], rb0 = s_rec[w][jb][0], rb1 = s_rec[w][jb][1];
        float ea[PPL], ua[PPL], dya[PPL], eb[PPL], ub[PPL], dyb[PPL];
        // one ballot per entry and pixel of the lane; the entry blends in the wave if any of them is set
        uint64_t bal_a[PPL], bal_b[PPL], bba = 0ull, bbb = 0ull;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          ea[p] = log2_alpha(fpx[p], fpy, ra0, ra1.x, ra1.y, dya[p], ua[p]);
          eb[p] = log2_alpha(fpx[p], fpy, rb0, rb1.x, rb1.y, dyb[p], ub[p]);
          // each ballot of a single compare, the masks combined in scalar registers
          // (a ballot of a combined condition goes through a vector register)
          const bool ina = rel0 + ta < lastp[p], inb = rel0 + tb < lastp[p];
          const bool hta = ea[p] >= P.log2_amin, htb = eb[p] >= P.log2_amin;
          const bool bla = ina & hta, blb = use_b & inb & htb;
          bal_a[p] = ballot64(ina) & ballot64(hta);
          bal_b[p] = ballot64(inb) & ballot64(htb) & (0ull - (uint64_t)use_b);
          bba |= bal_a[p];
          bbb |= bal_b[p];
          // a pixel that does not blend the entry takes alpha = exp2(-inf) = 0 in the terms below
          ea[p] = bla ? ea[p] : -INFINITY;
          eb[p] = blb ? eb[p] : -INFINITY;
        }
        // blended pixels of the wave, and those under the error mask
        uint32_t na = 0u, nma = 0u, nb = 0u, nmb = 0u;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          na += (uint32_t)__popcll(bal_a[p]);
          nma += (uint32_t)__popcll(bal_a[p] & Mbal[p]);
          nb += (uint32_t)__popcll(bal_b[p]);
          nmb += (uint32_t)__popcll(bal_b[p] & Mbal[p]);
        }
        if (bba != 0ull && bbb != 0ull) {
          float x[20];
          const float4 ra2 = s_rec[w][j][2], rb2 = s_rec[w][jb][2];
          if constexpr (PPL == 2) {
            // entry a for both pixels, then entry b: each pixel's T and Rj still
            // see a before b
            blend_terms2<DEPTH, CL>(ea, ua, dya[0], ra1, ra2, P.amax, g0, g1, g2, gD, T, Rj, x);
            blend_terms2<DEPTH, CL>(eb, ub, dyb[0], rb1, rb2, P.amax, g0, g1, g2, gD, T, Rj, x + 10);
          } else {
            blend_terms<DEPTH, CL>(ea[0], ua[0], dya[0], ra1, ra2, P.amax, g0[0], g1[0], g2[0], gD[0], T[0],
                               Rj[0], x);
            blend_terms<DEPTH, CL>(eb[0], ub[0], dyb[0], rb1, rb2, P.amax, g0[0], g1[0], g2[0], gD[0], T[0],
                               Rj[0], x + 10);
          }
          int idx;
          bool valid;
          wave_reduce20<DEPTH ? 10 : 9>(x, l, idx, valid);
          if (valid) s_part[w][idx < 10 ? ta : tb][idx < 10 ? idx : idx - 10] = x[0];
          if (l == 0) {
            s_part[w][ta][10] = __uint_as_float(na);
            s_part[w][ta][11] = __uint_as_float(nma);
            s_part[w][tb][10] = __uint_as_float(nb);
            s_part[w][tb][11] = __uint_as_float(nmb);
          }
        } else if ((bba | bbb) != 0ull) {
          const bool first = bba != 0ull;
          const int tt = first ? ta : tb, tz = first ? tb : ta;
          const float4 q1 = first ? ra1 : rb1, q2 = s_rec[w][first ? j : jb][2];
          float x[10];
          if constexpr (PPL == 2) {
            float e2[2], u2[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
              e2[p] = first ? ea[p] : eb[p];
              u2[p] = first ? ua[p] : ub[p];
            }
            blend_terms2<DEPTH, CL>(e2, u2, first ? dya[0] : dyb[0], q1, q2, P.amax, g0, g1, g2, gD, T, Rj, x);
          } else {
            blend_terms<DEPTH, CL>(first ? ea[0] : eb[0], first ? ua[0] : ub[0], first ? dya[0] : dyb[0], q1, q2,
                               P.amax, g0[0], g1[0], g2[0], gD[0], T[0], Rj[0], x);
          }
          int idx;
          bool valid;
          wave_reduce10(x, l, idx, valid);
          if (valid) s_part[w][tt][idx] = x[0];
          if (l == 0) {
            s_part[w][tt][10] = __uint_as_float(first ? na : nb);
            s_part[w][tt][11] = __uint_as_float(first ? nma : nmb);
          }
          // the other entry blends nowhere in this wave: its partial is zero
          if (use_b && l < 12) s_part[w][tz][l] = 0.f;
        } else {
          if (l < 12) s_part[w][ta][l] = 0.f;
          if (use_b && l < 12) s_part[w][tb][l] = 0.f;
        }
        if (has_b && !use_b) break;
        j += use_b ? 2u : 1u;
      }
    };
    if (clamp_bal) entries(BoolC<true>{});
    else entries(BoolC<false>{});
    __syncthreads();
    // the first wave sums the waves' partials of every pair in wave order and
    // writes the pair's record
    if (w == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int bi = r * 64 + l;
        const uint32_t k = base + (uint32_t)bi;
        if (bi < B && k < end) {
          const int krel = (int)(k - start);
          float o[10];
          uint32_t c0 = 0u, c1 = 0u;
#pragma unroll
          for (int q = 0; q < 10; ++q) o[q] = 0.f;
#pragma unroll
          for (int ww = 0; ww < NW; ++ww) {
            if (((s_keep[ww][r] >> l) & 1ull) && krel < s_wmax[ww]) {
#pragma unroll
              for (int q = 0; q < 10; ++q) o[q] += s_part[ww][bi][q];
              c0 += __float_as_uint(s_part[ww][bi][10]);
              c1 += __float_as_uint(s_part[ww][bi][11]);
            }
          }
          const uint32_t pe = pair_position(firstp[r], xbw[r], ybw[r], tx, ty, P);
          const size_t p = (size_t)pe * 3;
          pair_grad[p] = make_float4(o[0], o[1], o[2], o[3]);
          pair_grad[p + 1] = make_float4(o[4], o[5], o[6], o[7]);
          pair_grad[p + 2] = make_float4(o[8], o[9], __uint_as_float(c0), __uint_as_float(c1));
          pair_live[pe] = 1u;
        }
      }
    }
    __syncthreads();
  }
  // pairs behind the tile's last batch are left unwritten: every pixel of the
  // tile has stopped before them, and their live flags stay clear
}

// ---------------------------------------------------------------- host side
// Two pixels per lane (a wave per 16x8 block) where the tile is at least 16
// wide and, unless the configuration asks for it, the launch still has waves
// to spare: at least 16 per CU (one view at 1242x375 has 3744, eight views
// 30k).  Otherwise one pixel per lane, a wave per 8x8 block, twice the waves.
static bool two_px_per_lane(const kgs_ctx* ctx, unsigned grid) {
  const uint64_t waves2 = (uint64_t)grid * (uint64_t)(ctx->cfg.tile_w * ctx->cfg.tile_h / 128);
  const int ppl = ctx->cfg.px_per_lane;
  return ctx->cfg.tile_w >= 16 && (ppl == 2 || (ppl == 0 && waves2 >= KGS_BWD_TWO_PX_MIN_WAVES));
}

// waves per compositing workgroup: one per 8x8 sub-block of the tile
kgs_status kgs_launch_render_fwd(kgs_ctx* ctx, const kgs_image* out, hipStream_t st) {
  const RenderParams P = render_params(ctx);
  const unsigned grid = (unsigned)(ctx->last_views * ctx->n_tiles);
#define KGS_FWD(NWV)                                                                                             \
  hipLaunchKernelGGL((k_render_fwd<NWV>), dim3(grid), dim3(64 * NWV), 0, st, P, (const uint2*)ctx->ranges,       \
                     (const uint32_t*)ctx->tile_order,                                                           \
                     (const uint32_t*)ctx->sorted_slot, (const float4*)ctx->slot_rec, out->color, out->depth,      \
                     out->t_final, out->last)
#define KGS_FWD2(NWV)                                                                                            \
  hipLaunchKernelGGL((k_render_fwdn<NWV, 2>), dim3(grid), dim3(64 * NWV), 0, st, P,                             \
                     (const uint2*)ctx->ranges,                                                                  \
                     (const uint32_t*)ctx->tile_order,                                                           \
                     (const uint32_t*)ctx->sorted_slot, (const float4*)ctx->slot_rec, out->color, out->depth,      \
                     out->t_final, out->last)
  // two pixels per lane on the same rule as the backward (tiles at least 16 wide, a launch with waves to spare)
  // (four pixels per lane, a wave per 32x8 block, measured 2.8x slower on the bench chunk)
  if (two_px_per_lane(ctx, grid)) {
    if (tile_waves(ctx) == 8) KGS_FWD2(4);
    else KGS_FWD2(2);
  } else {
    if (tile_waves(ctx) == 8) KGS_FWD(8);
    else KGS_FWD(4);
  }
#undef KGS_FWD
#undef KGS_FWD2
  return kgs_check_launch();
}

void kgs_launch_loss_final(kgs_ctx* ctx, float* view_loss, hipStream_t st);

kgs_status kgs_launch_loss(kgs_ctx* ctx, const float* target, const kgs_image* img, float* dl_dcolor,
                           float* view_loss, hipStream_t st) {
  const int V = ctx->last_views;
  const RenderParams P = render_params(ctx);
  if (tile_waves(ctx) == 8)
    hipLaunchKernelGGL(k_loss_l1<8>, dim3((unsigned)(V * ctx->n_tiles)), dim3(512), 0, st, P,
                       (const float*)img->color, target, dl_dcolor, ctx->loss_partial);
  else
    hipLaunchKernelGGL(k_loss_l1<4>, dim3((unsigned)(V * ctx->n_tiles)), dim3(256), 0, st, P,
                       (const float*)img->color, target, dl_dcolor, ctx->loss_partial);
  kgs_launch_loss_final(ctx, view_loss, st);
  return kgs_check_launch();
}

void kgs_launch_loss_final(kgs_ctx* ctx, float* view_loss, hipStream_t st) {
  const int V = ctx->last_views;
  const double inv_n = 1.0 / (3.0 * (double)ctx->cfg.width * (double)ctx->cfg.height);
  if (V > 0)
    hipLaunchKernelGGL(k_loss_final, dim3(V), dim3(KGS_FINAL_THREADS), 0, st, ctx->n_tiles, inv_n,
                       (const double*)ctx->loss_partial,
                       view_loss);
}

// Clears the pairs' live flags and the slots' blended-pixel counts (the counts
// are read on the device) before the compositing backward sets the flags of
// the pairs it writes; the segmented pair sums then write the counts of the
// slots with a written pair only.
__global__ __launch_bounds__(256) void k_clear_live(const uint32_t* __restrict__ counters, uint4* __restrict__ live,
                                                    uint32_t* __restrict__ slot_om) {
  const uint32_t n = (counters[1] + 15u) / 16u, ns = counters[0];
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) live[i] = make_uint4(0u, 0u, 0u, 0u);
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < ns; i += gridDim.x * 256) slot_om[i] = 0u;
}

// fuse_l1: the colour gradient is the L1 loss gradient against target, formed
// here (and written to dl_dcolor if it is not null) together with the loss
// partials; kgs_launch_loss_final then gives the per-view losses.
kgs_status kgs_launch_render_bwd(kgs_ctx* ctx, const kgs_image* fwd, const float* dl_dcolor, const float* dl_ddepth,
                                 const float* dl_dtfinal, const float* target, float tau_err, hipStream_t st,
                                 bool fuse_l1, float* dl_out) {
  const RenderParams P = render_params(ctx);
  const unsigned grid = (unsigned)(ctx->last_views * ctx->n_tiles);
  const uint64_t lw = ((uint64_t)ctx->cfg.pair_capacity + 15) / 16;
  hipLaunchKernelGGL(k_clear_live, dim3((unsigned)std::min<uint64_t>(std::max<uint64_t>((lw + 255) / 256, 1), 1024)),
                     dim3(256), 0, st, (const uint32_t*)ctx->counters, (uint4*)ctx->pair_live, ctx->slot_om);
#define KGS_BWD(BB, NWV, PX)                                                                                     \
  if (dl_ddepth) { KGS_BWD_D(BB, NWV, true, PX); } else { KGS_BWD_D(BB, NWV, false, PX); }
#define KGS_BWD_D(BB, NWV, DD, PX)                                                                               \
  hipLaunchKernelGGL((k_render_bwd<BB, NWV, DD, PX>), dim3(grid), dim3(64 * NWV), 0, st, P,                      \
                     (const uint2*)ctx->ranges, (const uint32_t*)ctx->tile_order,                                \
                     (const uint32_t*)ctx->sorted_slot,                                                           \
                     (const float4*)ctx->slot_rec,                                                                \
                     (const float*)fwd->color, (const float*)fwd->depth, (const float*)fwd->t_final,              \
                     (const int32_t*)fwd->last, dl_dcolor, dl_ddepth, dl_dtfinal, target, tau_err, ctx->pair_grad,  \
                     ctx->pair_live, fuse_l1 ? 1 : 0, dl_out, ctx->loss_partial)
  const bool two = two_px_per_lane(ctx, grid);
  if (!two) {
    if (tile_waves(ctx) == 8) {
      switch (ctx->cfg.batch) {
        case 32: KGS_BWD(32, 8, 1); break;
        default: KGS_BWD(64, 8, 1); break;
      }
    } else {
      switch (ctx->cfg.batch) {
        case 32: KGS_BWD(32, 4, 1); break;
        case 64: KGS_BWD(64, 4, 1); break;
        default: KGS_BWD(128, 4, 1); break;
      }
    }
  } else if (tile_waves(ctx) == 8) {
    switch (ctx->cfg.batch) {
      case 32: KGS_BWD(32, 4, 2); break;
      default: KGS_BWD(64, 4, 2); break;
    }
  } else {
    switch (ctx->cfg.batch) {
      case 32: KGS_BWD(32, 2, 2); break;
      case 64: KGS_BWD(64, 2, 2); break;
      default: KGS_BWD(128, 2, 2); break;
    }
  }
#undef KGS_BWD
#undef KGS_BWD_D
  return kgs_check_launch();
}
