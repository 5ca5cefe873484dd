// Tile binning and depth sort.
//
// The order the compositing needs is (view, tile, depth, Gaussian index).  It
// is built in two small sorts instead of one wide one:
//   1. the projected records (slots, already in (view, Gaussian) order) are
//      sorted by (view, fp32 depth) -- 38-bit keys over S records;
//   2. pairs are emitted in that depth order (a scan of the records' tile
//      counts gives each record's first pair), one per tile of the record's
//      rectangle, keyed by the global tile index only;
//   3. the pairs are sorted stably by tile -- 14 bits at 1242x375 x 8 views,
//      two 8-bit passes over 4-byte keys and values.
// Stability makes the result identical to one sort by the full key.
//
// The radix sort is LSD, reduce-then-scan, with one partition per wave: each
// wave histograms and scatters its contiguous range on its own (ranks from
// ballots, running digit offsets in the wave's own LDS row), so the scatter
// needs no block barriers.  Counts stay on the device, so the sequence can be
// captured in a graph.
#include <algorithm>

#include "kgs_internal.h"

#define RS_WAVES 4
#define RS_PARTS (KGS_SORT_BLOCKS * RS_WAVES)

__device__ __forceinline__ void part_range(uint32_t n, uint32_t part, uint32_t& lo, uint32_t& hi) {
  const uint32_t per = ((n + RS_PARTS - 1) / RS_PARTS + 63u) & ~63u;
  lo = min(n, part * per);
  hi = min(n, lo + per);
}

__global__ void k_radix_zero(uint32_t* __restrict__ total) { total[blockIdx.x * 256 + threadIdx.x] = 0u; }

// per-wave digit histograms: hist[d][part]; each lane keeps RS_KPT loads in flight
#define RS_KPT 8
template <typename K>
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* __restrict__ count, const K* __restrict__ keys,
                                                    int shift, uint32_t* __restrict__ hist,
                                                    uint32_t* __restrict__ total) {
  __shared__ uint32_t h[RS_WAVES][256];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
#pragma unroll
  for (int k = 0; k < RS_WAVES; ++k) h[k][tid] = 0u;
  __syncthreads();
  const uint32_t part = blockIdx.x * RS_WAVES + w;
  uint32_t lo, hi;
  part_range(*count, part, lo, hi);
  for (uint32_t base = lo; base < hi; base += 64 * RS_KPT) {
    uint32_t d[RS_KPT];
#pragma unroll
    for (int q = 0; q < RS_KPT; ++q) {
      const uint32_t i = base + q * 64 + l;
      d[q] = i < hi ? (uint32_t)(keys[i] >> shift) & 255u : 256u;
    }
#pragma unroll
    for (int q = 0; q < RS_KPT; ++q)
      if (d[q] < 256u) atomicAdd(&h[w][d[q]], 1u);
  }
  __syncthreads();
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < RS_WAVES; ++k) {
    const uint32_t c = h[k][tid];
    hist[(size_t)tid * RS_PARTS + blockIdx.x * RS_WAVES + k] = c;
    sum += c;
  }
  if (sum) atomicAdd(&total[tid], sum);
}

// one block per digit: exclusive scan of its row of partition counts, plus the
// total of all smaller digits
__global__ __launch_bounds__(256) void k_radix_scan(uint32_t* __restrict__ hist, const uint32_t* __restrict__ total) {
  __shared__ uint32_t sh[8];
  const int d = blockIdx.x, tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  uint32_t pre = 0;
  for (int k = tid; k < d; k += 256) pre += total[k];
  pre = wave_sum(pre);
  if (l == 0) sh[4 + w] = pre;
  constexpr int PER = RS_PARTS / 256;
  uint32_t v[PER], s = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    v[k] = hist[(size_t)d * RS_PARTS + tid * PER + k];
    s += v[k];
  }
  const uint32_t inc = wave_inclusive_scan(s);
  if (l == 63) sh[w] = inc;
  __syncthreads();
  uint32_t off = sh[4] + sh[5] + sh[6] + sh[7];
  for (int k = 0; k < w; ++k) off += sh[k];
  off += inc - s;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    hist[(size_t)d * RS_PARTS + tid * PER + k] = off;
    off += v[k];
  }
}

// stable scatter: every wave walks its partition RS_KPT x 64 keys at a time
// (all loads issued first, then ranked in index order)
template <typename K>
__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t* __restrict__ count, const K* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin, int shift,
                                                       const uint32_t* __restrict__ offsets, K* __restrict__ kout,
                                                       uint32_t* __restrict__ vout) {
  __shared__ uint32_t run[RS_WAVES][256];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const uint32_t part = blockIdx.x * RS_WAVES + w;
#pragma unroll
  for (int k = 0; k < 4; ++k) run[w][l + 64 * k] = offsets[(size_t)(l + 64 * k) * RS_PARTS + part];
  __builtin_amdgcn_wave_barrier();
  uint32_t lo, hi;
  part_range(*count, part, lo, hi);
  const uint64_t lt = (1ull << l) - 1ull;
  for (uint32_t base = lo; base < hi; base += 64 * RS_KPT) {
    K kk[RS_KPT];
    uint32_t vv[RS_KPT];
#pragma unroll
    for (int q = 0; q < RS_KPT; ++q) {
      const uint32_t i = base + q * 64 + l;
      kk[q] = 0;
      vv[q] = 0;
      if (i < hi) {
        kk[q] = kin[i];
        vv[q] = vin[i];
      }
    }
#pragma unroll
    for (int q = 0; q < RS_KPT; ++q) {
      const bool valid = base + q * 64 + l < hi;
      const uint32_t d = valid ? (uint32_t)(kk[q] >> shift) & 255u : 0u;
      uint64_t peers = ballot64(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const uint64_t b = ballot64((d >> bit) & 1u);
        peers &= ((d >> bit) & 1u) ? b : ~b;
      }
      const uint32_t rank = (uint32_t)__popcll(peers & lt);
      uint32_t pos = 0;
      if (valid) pos = run[w][d] + rank;
      __builtin_amdgcn_wave_barrier();
      if (valid) {
        kout[pos] = kk[q];
        vout[pos] = vv[q];
        if (rank == 0) run[w][d] += (uint32_t)__popcll(peers);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// ---------------------------------------------------------------- group scan
// The depth-sorted slots are cut into groups of 64; a group's pairs are
// contiguous.  k_group_sum: tile count of every group (one wave per group);
// k_scan_mid: exclusive scan of the group sums (one block).
__global__ __launch_bounds__(256) void k_group_sum(const uint32_t* __restrict__ count,
                                                   const uint32_t* __restrict__ perm,
                                                   const uint32_t* __restrict__ ntiles, uint32_t n_groups,
                                                   uint32_t* __restrict__ part) {
  const uint32_t n = *count;
  const uint32_t l = threadIdx.x & 63;
  const uint32_t waves = gridDim.x * 4;
  for (uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6); g < n_groups; g += waves) {
    const uint32_t j = g * 64 + l;
    const uint32_t c = j < n ? ntiles[perm[j]] : 0u;
    const uint32_t t = wave_sum(c);
    if (l == 0) part[g] = t;
  }
}

__global__ __launch_bounds__(1024) void k_scan_mid(uint32_t nparts, uint32_t* __restrict__ part) {
  __shared__ uint32_t sh[16];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const uint32_t per = (nparts + 1023) / 1024;
  const uint32_t lo = min(nparts, tid * per), hi = min(nparts, lo + per);
  uint32_t a = 0;
  for (uint32_t b = lo; b < hi; ++b) a += part[b];
  const uint32_t ia = wave_inclusive_scan(a);
  if (l == 63) sh[w] = ia;
  __syncthreads();
  uint32_t off = 0;
  for (int k = 0; k < w; ++k) off += sh[k];
  uint32_t r = off + ia - a;
  for (uint32_t b = lo; b < hi; ++b) {
    const uint32_t c = part[b];
    part[b] = r;
    r += c;
  }
}

// ---------------------------------------------------------------- slot keys
__global__ __launch_bounds__(KGS_BLOCK) void k_slot_keys(const uint32_t* __restrict__ counters,
                                                         const float4* __restrict__ slot_rec,
                                                         const uint32_t* __restrict__ slot_view,
                                                         uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const uint32_t n = counters[0];
  for (uint32_t s = blockIdx.x * KGS_BLOCK + threadIdx.x; s < n; s += gridDim.x * KGS_BLOCK) {
    keys[s] = ((uint64_t)slot_view[s] << 32) | __float_as_uint(slot_rec[(size_t)s * 3 + 1].z);
    vals[s] = s;
  }
}

// ---------------------------------------------------------------- pair emission
// Waves take the 64-slot groups grid-stride (so the large near-camera
// Gaussians, which cluster at the start of every view's depth order, spread
// over the whole grid).  In a group the lanes load their slot's rectangle and
// scan the tile counts; then the wave writes the group's pairs together: pair
// k belongs to the lane whose inclusive count first exceeds k (binary search
// over the lanes with shuffles), so writes are contiguous.  A pair's key is its
// global tile index, its value the slot; its emission position is the slot's
// first pair plus its row-major rank in the slot's tile rectangle.
__device__ __forceinline__ uint32_t udiv_small(uint32_t a, uint32_t b) {
  uint32_t q = (uint32_t)((float)a * __frcp_rn((float)b));
  while (q * b > a) --q;
  while ((q + 1) * b <= a) ++q;
  return q;
}

__global__ __launch_bounds__(256) void k_emit_pairs(const uint32_t* __restrict__ counters,
                                                    const uint32_t* __restrict__ perm,
                                                    const uint32_t* __restrict__ part, uint32_t n_groups,
                                                    const uint32_t* __restrict__ slot_view,
                                                    const int4* __restrict__ slot_pix,
                                                    const uint32_t* __restrict__ slot_ntiles, int tile_w, int tile_h,
                                                    int tiles_x, int tiles_y, uint64_t pair_cap,
                                                    uint32_t* __restrict__ slot_pairoff, uint32_t* __restrict__ keys,
                                                    uint32_t* __restrict__ vals) {
  const uint32_t n = counters[0];
  const int l = threadIdx.x & 63;
  const uint32_t waves = gridDim.x * 4;
  const uint32_t tiles_per_view = (uint32_t)(tiles_x * tiles_y);
  for (uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6); g < n_groups; g += waves) {
    const uint32_t j = g * 64 + (uint32_t)l;
    if (g * 64 >= n) break;
    const uint32_t s = j < n ? perm[j] : 0u;
    const uint32_t c = j < n ? slot_ntiles[s] : 0u;
    const uint32_t incl = wave_inclusive_scan(c);
    const uint32_t excl = incl - c;
    const uint32_t tot = (uint32_t)__shfl((int)incl, 63, 64);
    const uint32_t rbase = part[g];
    if ((uint64_t)rbase + tot > pair_cap) continue;
    int x0 = 0, y0 = 0, rw = 1, ok = 0;
    uint32_t gbase = 0;
    if (c > 0) {
      const int4 pix = slot_pix[s];
      x0 = max(floordiv_i(pix.x - pix.z, tile_w), 0);
      const int x1 = min(floordiv_i(pix.x + pix.z, tile_w) + 1, tiles_x);
      y0 = max(floordiv_i(pix.y - pix.w, tile_h), 0);
      rw = max(x1 - x0, 1);
      ok = x1 > x0;
      gbase = slot_view[s] * tiles_per_view;
      slot_pairoff[s] = rbase + excl;
    }
    // wave-uniform loop: every lane takes part in the shuffles (a shuffle
    // from a lane that has left the loop would read an undefined value)
    for (uint32_t kb = 0; kb < tot; kb += 64) {
      const uint32_t k = kb + (uint32_t)l;
      int lo = 0, hi = 63;
#pragma unroll
      for (int step = 0; step < 6; ++step) {
        const int mid = (lo + hi) >> 1;
        const uint32_t im = (uint32_t)__shfl((int)incl, mid, 64);
        if (im > k) hi = mid; else lo = mid + 1;
      }
      const int o = lo;
      const uint32_t oexcl = (uint32_t)__shfl((int)excl, o, 64);
      const int ox0 = __shfl(x0, o, 64), oy0 = __shfl(y0, o, 64), orw = __shfl(rw, o, 64), ook = __shfl(ok, o, 64);
      const uint32_t ogb = (uint32_t)__shfl((int)gbase, o, 64), os = (uint32_t)__shfl((int)s, o, 64);
      if (k < tot) {
        const uint32_t rk = k - oexcl;
        const uint32_t qy = udiv_small(rk, (uint32_t)orw);
        const int ty = oy0 + (int)qy, tx = ox0 + (int)(rk - qy * (uint32_t)orw);
        const uint32_t p = rbase + k;
        keys[p] = (ook && ty < tiles_y) ? ogb + (uint32_t)(ty * tiles_x + tx) : 0xffffffffu;
        vals[p] = os;
      }
    }
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(KGS_BLOCK) void k_ranges(const uint32_t* __restrict__ counters,
                                                      const uint32_t* __restrict__ keys, uint32_t n_tiles_all,
                                                      uint2* __restrict__ ranges) {
  const uint32_t n = counters[1];
  for (uint32_t k = blockIdx.x * KGS_BLOCK + threadIdx.x; k < n; k += gridDim.x * KGS_BLOCK) {
    const uint32_t t = keys[k];
    const uint32_t tn = k + 1 < n ? keys[k + 1] : 0xffffffffu;
    if (t == tn) continue;
    // k is the last pair of tile t and k + 1 the first of tile tn
    if (t < n_tiles_all) ranges[t].y = k + 1;
    if (tn < n_tiles_all) ranges[tn].x = k + 1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && n > 0) {
    const uint32_t t0 = keys[0];
    if (t0 < n_tiles_all) ranges[t0].x = 0;
  }
}

// ---------------------------------------------------------------- host side
template <typename K>
static int radix_sort(kgs_ctx* ctx, const uint32_t* count, K* keys[2], uint32_t* vals[2], int bits, hipStream_t st) {
  const int passes = (bits + 7) / 8;
  hipLaunchKernelGGL(k_radix_zero, dim3(passes), dim3(256), 0, st, ctx->radix_total);
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(k_radix_hist<K>, dim3(KGS_SORT_BLOCKS), dim3(256), 0, st, count, (const K*)keys[cur], 8 * p,
                       ctx->radix_hist, ctx->radix_total + 256 * p);
    hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(256), 0, st, ctx->radix_hist,
                       (const uint32_t*)(ctx->radix_total + 256 * p));
    hipLaunchKernelGGL(k_radix_scatter<K>, dim3(KGS_SORT_BLOCKS), dim3(256), 0, st, count, (const K*)keys[cur],
                       (const uint32_t*)vals[cur], 8 * p, (const uint32_t*)ctx->radix_hist, keys[cur ^ 1],
                       vals[cur ^ 1]);
    cur ^= 1;
  }
  return cur;
}

kgs_status kgs_launch_bin_sort(kgs_ctx* ctx, hipStream_t st) {
  const int V = ctx->last_views;
  const uint32_t n_tiles_all = (uint32_t)(V * ctx->n_tiles);
  const uint64_t S = (uint64_t)ctx->cfg.slot_capacity, P = (uint64_t)ctx->cfg.pair_capacity;
  const unsigned sgrid = (unsigned)std::min<uint64_t>(std::max<uint64_t>((S + KGS_BLOCK - 1) / KGS_BLOCK, 1), 4096);
  // 1. records by (view, depth)
  hipLaunchKernelGGL(k_slot_keys, dim3(sgrid), dim3(KGS_BLOCK), 0, st, (const uint32_t*)ctx->counters,
                     (const float4*)ctx->slot_rec, (const uint32_t*)ctx->slot_view, ctx->slot_keys[0],
                     ctx->slot_vals[0]);
  int view_bits = 0;
  while ((1 << view_bits) < V) ++view_bits;
  const int sc = radix_sort<uint64_t>(ctx, ctx->counters, ctx->slot_keys, ctx->slot_vals, 32 + view_bits, st);
  const uint32_t* perm = ctx->slot_vals[sc];
  // 2. first pair of every record in that order, then the pairs
  const uint32_t n_groups = (uint32_t)((S + 63) / 64);
  const unsigned eg = (unsigned)std::min<uint64_t>(std::max<uint64_t>((n_groups + 3) / 4, 1), 2048);
  hipLaunchKernelGGL(k_group_sum, dim3(eg), dim3(256), 0, st, (const uint32_t*)ctx->counters, perm,
                     (const uint32_t*)ctx->slot_ntiles, n_groups, ctx->scan_part);
  hipLaunchKernelGGL(k_scan_mid, dim3(1), dim3(1024), 0, st, n_groups, ctx->scan_part);
  hipLaunchKernelGGL(k_emit_pairs, dim3(eg), dim3(256), 0, st, (const uint32_t*)ctx->counters, perm,
                     (const uint32_t*)ctx->scan_part, n_groups, (const uint32_t*)ctx->slot_view,
                     (const int4*)ctx->slot_pix, (const uint32_t*)ctx->slot_ntiles, ctx->cfg.tile_w, ctx->cfg.tile_h,
                     ctx->tiles_x, ctx->tiles_y, P, ctx->slot_pairoff, ctx->keys[0], ctx->vals[0]);
  // 3. pairs by tile (stable)
  // padding pairs carry key 0xffffffff; with n_tiles_all < 2^tile_bits they
  // sort after every real pair
  int tile_bits = 0;
  while ((1u << tile_bits) <= n_tiles_all) ++tile_bits;
  const int cur = radix_sort<uint32_t>(ctx, ctx->counters + 1, ctx->keys, ctx->vals, std::max(tile_bits, 1), st);
  ctx->sorted_buf = cur;
  ctx->passes = (tile_bits + 7) / 8;
  const uint64_t nr = (uint64_t)n_tiles_all * 2;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<uint64_t>((nr + 255) / 256, 1024)), dim3(256), 0, st,
                     (uint32_t*)ctx->ranges, nr, 0u);
  const unsigned rg = (unsigned)std::min<uint64_t>(std::max<uint64_t>((P + KGS_BLOCK - 1) / KGS_BLOCK, 1), 8192);
  hipLaunchKernelGGL(k_ranges, dim3(rg), dim3(KGS_BLOCK), 0, st, (const uint32_t*)ctx->counters,
                     (const uint32_t*)ctx->keys[cur], n_tiles_all, ctx->ranges);
  ctx->sorted_slot = ctx->vals[cur];
  return kgs_check_launch();
}
