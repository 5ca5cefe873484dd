// Device-wide exclusive scan of W interleaved u32 values per entry (W = 1 or
// 2), accumulated in u64 and clamped on output at a per-value cap.
// Reduce-then-scan in three launches: per 4096-entry tile the block sums, one
// block scans those sums, then every tile rescans itself from its offset.
// Loads and stores are coalesced (each thread four consecutive entries).
#include "kgs_internal.h"

#define SC_THREADS 1024
#define SC_PER 4
#define SC_TILE (SC_THREADS * SC_PER)

template <int W>
__device__ __forceinline__ void sc_load(const uint32_t* __restrict__ in, int64_t entries, int64_t e0,
                                        uint32_t (&v)[SC_PER][W], unsigned long long (&a)[W]) {
#pragma unroll
  for (int w = 0; w < W; ++w) a[w] = 0;
#pragma unroll
  for (int k = 0; k < SC_PER; ++k) {
    const bool ok = e0 + k < entries;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      v[k][w] = ok ? in[(e0 + k) * W + w] : 0u;
      a[w] += v[k][w];
    }
  }
}

// Block-wide exclusive scan of one u64 per thread; returns the block total.
__device__ __forceinline__ unsigned long long sc_block_scan(unsigned long long a, unsigned long long* sh,
                                                            unsigned long long& excl) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const unsigned long long ia = wave_inclusive_scan(a);
  if (l == 63) sh[w] = ia;
  __syncthreads();
  unsigned long long off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < SC_THREADS / 64; ++k) {
    if (k < w) off += sh[k];
    tot += sh[k];
  }
  excl = off + ia - a;
  __syncthreads();
  return tot;
}

template <int W>
__global__ __launch_bounds__(SC_THREADS) void k_sc_reduce(const uint32_t* __restrict__ in, int64_t entries,
                                                          unsigned long long* __restrict__ part) {
  __shared__ unsigned long long sh[SC_THREADS / 64];
  const int64_t e0 = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_PER;
  uint32_t v[SC_PER][W];
  unsigned long long a[W];
  sc_load<W>(in, entries, e0, v, a);
#pragma unroll
  for (int w = 0; w < W; ++w) {
    unsigned long long ex;
    const unsigned long long tot = sc_block_scan(a[w], sh, ex);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * W + w] = tot;
  }
}

// One block: exclusive scan of the tile sums (in place) and the totals.
template <int W>
__global__ __launch_bounds__(SC_THREADS) void k_sc_top(unsigned long long* __restrict__ part, int64_t tiles,
                                                       unsigned long long* __restrict__ totals) {
  __shared__ unsigned long long sh[SC_THREADS / 64];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    unsigned long long carry = 0;
    for (int64_t b = 0; b < tiles; b += SC_THREADS) {
      const int64_t t = b + threadIdx.x;
      const unsigned long long a = t < tiles ? part[t * W + w] : 0ull;
      unsigned long long ex;
      const unsigned long long tot = sc_block_scan(a, sh, ex);
      if (t < tiles) part[t * W + w] = carry + ex;
      carry += tot;
    }
    if (threadIdx.x == 0) totals[w] = carry;
  }
}

template <int W>
__global__ __launch_bounds__(SC_THREADS) void k_sc_apply(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                         int64_t entries, const unsigned long long* __restrict__ part,
                                                         unsigned long long cap0, unsigned long long cap1) {
  __shared__ unsigned long long sh[SC_THREADS / 64];
  const int64_t e0 = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_PER;
  uint32_t v[SC_PER][W];
  unsigned long long a[W];
  sc_load<W>(in, entries, e0, v, a);
#pragma unroll
  for (int w = 0; w < W; ++w) {
    unsigned long long ex;
    sc_block_scan(a[w], sh, ex);
    unsigned long long r = part[(int64_t)blockIdx.x * W + w] + ex;
    const unsigned long long cap = w == 0 ? cap0 : cap1;
#pragma unroll
    for (int k = 0; k < SC_PER; ++k) {
      if (e0 + k < entries) out[(e0 + k) * W + w] = (uint32_t)min(r, cap);
      r += v[k][w];
    }
  }
}

int64_t kgs_scan_tiles(int64_t entries) { return (entries + SC_TILE - 1) / SC_TILE; }

void kgs_launch_scan(const uint32_t* in, uint32_t* out, int64_t entries, int W, unsigned long long cap0,
                     unsigned long long cap1, unsigned long long* part, unsigned long long* totals, hipStream_t st) {
  const int64_t tiles = kgs_scan_tiles(entries);
  const unsigned g = (unsigned)std::max<int64_t>(tiles, 1);
  if (W == 1) {
    hipLaunchKernelGGL(k_sc_reduce<1>, dim3(g), dim3(SC_THREADS), 0, st, in, entries, part);
    hipLaunchKernelGGL(k_sc_top<1>, dim3(1), dim3(SC_THREADS), 0, st, part, tiles, totals);
    hipLaunchKernelGGL(k_sc_apply<1>, dim3(g), dim3(SC_THREADS), 0, st, in, out, entries,
                       (const unsigned long long*)part, cap0, cap1);
  } else {
    hipLaunchKernelGGL(k_sc_reduce<2>, dim3(g), dim3(SC_THREADS), 0, st, in, entries, part);
    hipLaunchKernelGGL(k_sc_top<2>, dim3(1), dim3(SC_THREADS), 0, st, part, tiles, totals);
    hipLaunchKernelGGL(k_sc_apply<2>, dim3(g), dim3(SC_THREADS), 0, st, in, out, entries,
                       (const unsigned long long*)part, cap0, cap1);
  }
}
