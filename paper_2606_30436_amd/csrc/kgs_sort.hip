// Tile binning and depth sort.
//
// Pairs are emitted per slot at the slot's pair offset (so the pairs of one
// slot are contiguous in emission order), then sorted by a stable LSD radix
// sort over only the used key bits (32 depth bits + ceil(log2(views * tiles))
// tile bits), 8-bit digits, reduce-then-scan with a fixed grid: per pass a
// block histogram, a per-digit scan, and a stable in-block scatter whose ranks
// come from wave ballots.  Counts are read on the device, so the whole
// sequence can be captured in a graph.
#include "kgs_internal.h"

__global__ __launch_bounds__(KGS_BLOCK) void k_emit_pairs(const uint32_t* __restrict__ counters,
                                                          const float4* __restrict__ slot_rec,
                                                          const uint32_t* __restrict__ slot_view,
                                                          const int4* __restrict__ slot_pix,
                                                          const uint32_t* __restrict__ slot_pairoff,
                                                          const uint32_t* __restrict__ slot_ntiles, int tile_w,
                                                          int tile_h, int tiles_x, int tiles_y,
                                                          uint64_t pair_cap, uint64_t* __restrict__ keys,
                                                          uint32_t* __restrict__ vals,
                                                          uint32_t* __restrict__ pair_slot) {
  const uint32_t n = counters[0];
  const uint32_t tiles_per_view = (uint32_t)(tiles_x * tiles_y);
  for (uint32_t s = blockIdx.x * KGS_BLOCK + threadIdx.x; s < n; s += gridDim.x * KGS_BLOCK) {
    const int4 pix = slot_pix[s];
    const uint32_t depth_bits = __float_as_uint(slot_rec[(size_t)s * 3 + 1].z);
    const uint32_t v = slot_view[s];
    const uint32_t off = slot_pairoff[s];
    const uint32_t cnt = slot_ntiles[s];
    if ((uint64_t)off + cnt > pair_cap) continue;
    const int x0 = max(floordiv_i(pix.x - pix.z, tile_w), 0), x1 = min(floordiv_i(pix.x + pix.z, tile_w) + 1, tiles_x);
    const int y0 = max(floordiv_i(pix.y - pix.w, tile_h), 0), y1 = min(floordiv_i(pix.y + pix.w, tile_h) + 1, tiles_y);
    uint32_t k = 0;
    for (int ty = y0; ty < y1 && k < cnt; ++ty)
      for (int tx = x0; tx < x1 && k < cnt; ++tx, ++k) {
        const uint64_t tile = (uint64_t)v * tiles_per_view + (uint64_t)(ty * tiles_x + tx);
        keys[off + k] = (tile << 32) | depth_bits;
        vals[off + k] = off + k;
        pair_slot[off + k] = s;
      }
    // a re-projection that disagrees with the count leaves padding pairs
    for (; k < cnt; ++k) {
      keys[off + k] = ~0ull;
      vals[off + k] = off + k;
      pair_slot[off + k] = s;
    }
  }
}

__device__ __forceinline__ void sort_range(uint32_t n, int b, uint32_t& lo, uint32_t& hi) {
  const uint32_t per = ((n + KGS_SORT_BLOCKS - 1) / KGS_SORT_BLOCKS + 255u) & ~255u;
  lo = min(n, (uint32_t)b * per);
  hi = min(n, lo + per);
}

__global__ void k_radix_zero(uint32_t* __restrict__ total) {
  total[blockIdx.x * 256 + threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* __restrict__ counters,
                                                    const uint64_t* __restrict__ keys, int shift,
                                                    uint32_t* __restrict__ hist, uint32_t* __restrict__ total) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  uint32_t lo, hi;
  sort_range(counters[1], blockIdx.x, lo, hi);
  for (uint32_t i = lo + threadIdx.x; i < hi; i += 256) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  __syncthreads();
  const uint32_t c = h[threadIdx.x];
  hist[threadIdx.x * KGS_SORT_BLOCKS + blockIdx.x] = c;
  if (c) atomicAdd(&total[threadIdx.x], c);
}

// one block per digit: exclusive scan of its row of block counts, plus the
// counts of all smaller digits
__global__ __launch_bounds__(256) void k_radix_scan(uint32_t* __restrict__ hist,
                                                    const uint32_t* __restrict__ total) {
  __shared__ uint32_t sh[8];
  const int d = blockIdx.x, tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  uint32_t pre = 0;
  for (int k = tid; k < d; k += 256) pre += total[k];
  pre = wave_sum(pre);
  if (l == 0) sh[4 + w] = pre;
  constexpr int PER = KGS_SORT_BLOCKS / 256;
  uint32_t v[PER], s = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) { v[k] = hist[d * KGS_SORT_BLOCKS + tid * PER + k]; s += v[k]; }
  const uint32_t inc = wave_inclusive_scan(s);
  if (l == 63) sh[w] = inc;
  __syncthreads();
  uint32_t off = sh[4] + sh[5] + sh[6] + sh[7];
  for (int k = 0; k < w; ++k) off += sh[k];
  off += inc - s;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    hist[d * KGS_SORT_BLOCKS + tid * PER + k] = off;
    off += v[k];
  }
}

__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t* __restrict__ counters,
                                                       const uint64_t* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin, int shift,
                                                       const uint32_t* __restrict__ offsets,
                                                       uint64_t* __restrict__ kout, uint32_t* __restrict__ vout) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wc[4][256];
  const int tid = threadIdx.x, w = tid >> 6;
  run[tid] = offsets[tid * KGS_SORT_BLOCKS + blockIdx.x];
  uint32_t lo, hi;
  sort_range(counters[1], blockIdx.x, lo, hi);
  const uint64_t lt = (1ull << (tid & 63)) - 1ull;
  for (uint32_t base = lo; base < hi; base += 256) {
    const uint32_t i = base + tid;
    const bool valid = i < hi;
    uint64_t key = 0;
    uint32_t val = 0, d = 0;
    if (valid) {
      key = kin[i];
      val = vin[i];
      d = (uint32_t)(key >> shift) & 255u;
    }
    uint64_t peers = ballot64(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t b = ballot64((d >> bit) & 1u);
      peers &= ((d >> bit) & 1u) ? b : ~b;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    wc[0][tid] = 0; wc[1][tid] = 0; wc[2][tid] = 0; wc[3][tid] = 0;
    __syncthreads();
    if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int k = 0; k < w; ++k) pos += wc[k][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    run[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
    __syncthreads();
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(KGS_BLOCK) void k_ranges(const uint32_t* __restrict__ counters,
                                                      const uint64_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ vals,
                                                      const uint32_t* __restrict__ pair_slot, uint32_t n_tiles_all,
                                                      uint2* __restrict__ ranges, uint32_t* __restrict__ sorted_slot) {
  const uint32_t n = counters[1];
  for (uint32_t k = blockIdx.x * KGS_BLOCK + threadIdx.x; k < n; k += gridDim.x * KGS_BLOCK) {
    const uint64_t key = keys[k];
    sorted_slot[k] = pair_slot[vals[k]];
    const uint32_t t = (uint32_t)(key >> 32);
    if (t >= n_tiles_all) continue;  // padding pairs sort last
    if (k == 0 || (uint32_t)(keys[k - 1] >> 32) != t) ranges[t].x = k;
    if (k + 1 == n || (uint32_t)(keys[k + 1] >> 32) != t) ranges[t].y = k + 1;
  }
}

kgs_status kgs_launch_bin_sort(kgs_ctx* ctx, hipStream_t st) {
  const int V = ctx->last_views;
  const uint32_t n_tiles_all = (uint32_t)(V * ctx->n_tiles);
  const uint64_t S = (uint64_t)ctx->cfg.slot_capacity;
  const unsigned eg = (unsigned)std::min<uint64_t>(std::max<uint64_t>((S + KGS_BLOCK - 1) / KGS_BLOCK, 1), 4096);
  hipLaunchKernelGGL(k_emit_pairs, dim3(eg), dim3(KGS_BLOCK), 0, st, (const uint32_t*)ctx->counters,
                     (const float4*)ctx->slot_rec, (const uint32_t*)ctx->slot_view, (const int4*)ctx->slot_pix,
                     (const uint32_t*)ctx->slot_pairoff, (const uint32_t*)ctx->slot_ntiles, ctx->cfg.tile_w,
                     ctx->cfg.tile_h, ctx->tiles_x, ctx->tiles_y, (uint64_t)ctx->cfg.pair_capacity, ctx->keys[0],
                     ctx->vals[0], ctx->pair_slot);
  // key bits: 32 depth bits + tile bits
  int tile_bits = 0;
  while ((1u << tile_bits) < n_tiles_all) ++tile_bits;
  const int passes = (32 + tile_bits + 7) / 8;
  ctx->passes = passes;
  hipLaunchKernelGGL(k_radix_zero, dim3(passes), dim3(256), 0, st, ctx->radix_total);
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(k_radix_hist, dim3(KGS_SORT_BLOCKS), dim3(256), 0, st, (const uint32_t*)ctx->counters,
                       (const uint64_t*)ctx->keys[cur], 8 * p, ctx->radix_hist, ctx->radix_total + 256 * p);
    hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(256), 0, st, ctx->radix_hist,
                       (const uint32_t*)(ctx->radix_total + 256 * p));
    hipLaunchKernelGGL(k_radix_scatter, dim3(KGS_SORT_BLOCKS), dim3(256), 0, st, (const uint32_t*)ctx->counters,
                       (const uint64_t*)ctx->keys[cur], (const uint32_t*)ctx->vals[cur], 8 * p,
                       (const uint32_t*)ctx->radix_hist, ctx->keys[cur ^ 1], ctx->vals[cur ^ 1]);
    cur ^= 1;
  }
  ctx->sorted_buf = cur;
  const uint64_t nr = (uint64_t)n_tiles_all * 2;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<uint64_t>((nr + 255) / 256, 1024)), dim3(256), 0, st,
                     (uint32_t*)ctx->ranges, nr, 0u);
  const uint64_t P = (uint64_t)ctx->cfg.pair_capacity;
  const unsigned rg = (unsigned)std::min<uint64_t>(std::max<uint64_t>((P + KGS_BLOCK - 1) / KGS_BLOCK, 1), 8192);
  hipLaunchKernelGGL(k_ranges, dim3(rg), dim3(KGS_BLOCK), 0, st, (const uint32_t*)ctx->counters,
                     (const uint64_t*)ctx->keys[cur], (const uint32_t*)ctx->vals[cur],
                     (const uint32_t*)ctx->pair_slot, n_tiles_all, ctx->ranges, ctx->sorted_slot);
  return kgs_check_launch();
}
