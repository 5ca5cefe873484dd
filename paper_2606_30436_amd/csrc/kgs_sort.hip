// Tile binning and depth sort.
//
// The compositing needs, for every (view, tile), the Gaussians that touch it
// in (depth, Gaussian index) order.  That is built in two small sorts instead
// of one wide one:
//   1. the projected records (slots, already in (view, Gaussian) order) are
//      sorted by (view, fp32 depth) -- 30-bit keys at near 0.2, far 80 and
//      8 views (the depth bits offset from near), over S records;
//   2. pairs are emitted in that depth order (a scan of the records' tile
//      counts gives each record's first pair), one per tile of the record's
//      rectangle, keyed by (view << tile_bits) | tile; the projection left
//      each record's tile rectangle and count in one 16-byte descriptor, the
//      only thing these steps gather per record;
//   3. the pairs are sorted stably by the tile bits only -- 936 tiles per view
//      at 1242x375 and 32x16 tiles, one 10-bit pass over 4-byte keys and
//      values.  Emission order is view-major, so every (view, tile) group
//      comes out contiguous and in depth order (the groups ordered by tile,
//      then view); stability makes each group identical to its run in one
//      sort by the full key.
//
// The radix sort is LSD, reduce-then-scan, with one contiguous partition per
// block; B key bits take the fewest passes of at most 10 bits, of equal
// width (three for the 30-bit record keys, one for the tile keys).  The first
// pass of the record sort takes the records' own indices as its values.  The
// scatter ranks a tile of
// 256 x KPT keys in index order (ballot matching inside a wave, running digit
// counts per wave, a digit-major prefix over the waves), places the tile in
// LDS in digit order, and writes it out so that consecutive lanes write
// consecutive addresses of a digit's run.  Counts stay on the device, so the
// sequence can be captured in a graph.
#include <algorithm>
#include <cstring>

#include "kgs_internal.h"

// widest digit of the record (depth) sort: 30-bit keys take three passes
#define KGS_DEPTH_DIGIT_BITS 10

// partition of block b of nb: a multiple of 256 keys
__device__ __forceinline__ void part_range(uint32_t n, uint32_t nb, uint32_t b, uint32_t& lo, uint32_t& hi) {
  const uint32_t per = ((n + nb - 1) / nb + 255u) & ~255u;
  lo = min(n, b * per);
  hi = min(n, lo + per);
}

// Partition of workgroup b of nb (a multiple of 8).  Workgroups are dealt to
// the eight XCDs in turn, so this gives each XCD a contiguous run of
// partitions: a digit's output runs from neighbouring partitions, written by
// workgroups in flight together, then meet in one L2 instead of eight.
__device__ __forceinline__ uint32_t xcd_part(uint32_t b, uint32_t nb) { return (b & 7u) * (nb >> 3) + (b >> 3); }

// Lanes of the wave whose valid keys share digit d (d < 2^DB): one ballot per
// bit, all DB unrolled (bits above the pass's digit width are zero in every
// lane and leave the mask alone).
template <int DB>
__device__ __forceinline__ uint64_t digit_peers(bool valid, uint32_t d) {
  const uint64_t v = ballot64(valid);
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int bit = 0; bit < DB; ++bit) {
    // m: all ones where this lane's bit is set; keep the lanes whose bit agrees
    const uint32_t m = (uint32_t)((int32_t)(d << (31 - bit)) >> 31);
    const uint64_t b = ballot64((d >> bit) & 1u);
    lo &= ~((uint32_t)b ^ m);
    hi &= ~((uint32_t)(b >> 32) ^ m);
  }
  return ((uint64_t)hi << 32) | lo;
}

// per-block digit histograms hist[d][block].  With AGG the lowest lane of each
// group of equal digits adds the group's size (one LDS add per distinct
// digit: for keys whose digits repeat across the wave, like the depth keys'
// upper digits); without, every key adds one (for keys of many distinct
// digits, like tiles).  DB is the widest digit the kernel takes (8 or 10
// bits), dbits the pass's own.
template <typename K, int DB, bool AGG>
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* __restrict__ count, const K* __restrict__ keys,
                                                    int shift, int dbits, uint32_t nb, uint32_t* __restrict__ hist) {
  constexpr int R = 1 << DB;
  __shared__ uint32_t h[R];
  const int tid = threadIdx.x, l = tid & 63;
  const uint32_t dmask = (1u << dbits) - 1u;
  const uint64_t lt = (1ull << l) - 1ull;
  for (int d = tid; d < R; d += 256) h[d] = 0u;
  __syncthreads();
  const uint32_t part = xcd_part(blockIdx.x, nb);
  uint32_t lo, hi;
  part_range(*count, nb, part, lo, hi);
  // 16-byte loads: VW keys per load, four loads per thread in flight
  constexpr int VW = 16 / sizeof(K), KPI = 4 * VW;
  for (uint32_t base = lo; base < hi; base += 256 * KPI) {
    K kk[KPI];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t i0 = base + (q * 256 + tid) * VW;
      if (i0 + VW <= hi) {
        const uint4 v = *reinterpret_cast<const uint4*>(keys + i0);
        if constexpr (VW == 4) {
          kk[q * 4] = (K)v.x; kk[q * 4 + 1] = (K)v.y; kk[q * 4 + 2] = (K)v.z; kk[q * 4 + 3] = (K)v.w;
        } else {
          kk[q * 2] = (K)(((uint64_t)v.y << 32) | v.x);
          kk[q * 2 + 1] = (K)(((uint64_t)v.w << 32) | v.z);
        }
      } else {
#pragma unroll
        for (int e = 0; e < VW; ++e) kk[q * VW + e] = i0 + e < hi ? keys[i0 + e] : (K)0;
      }
    }
#pragma unroll
    for (int q = 0; q < KPI; ++q) {
      const bool valid = base + ((q / VW) * 256 + tid) * VW + (q % VW) < hi;
      const uint32_t d = (uint32_t)(kk[q] >> shift) & dmask;
      if constexpr (AGG) {
        const uint64_t peers = digit_peers<DB>(valid, d);
        if (valid && (peers & lt) == 0ull) atomicAdd(&h[d], (uint32_t)__popcll(peers));
      } else {
        if (valid) atomicAdd(&h[d], 1u);
      }
    }
  }
  __syncthreads();
  for (uint32_t d = (uint32_t)tid; d <= dmask; d += 256) hist[(size_t)d * nb + part] = h[d];
}

// one block per digit: exclusive scan of its row of block counts (in place)
// and the row total
__global__ __launch_bounds__(256) void k_radix_scan(uint32_t* __restrict__ hist, uint32_t nb,
                                                    uint32_t* __restrict__ total) {
  __shared__ uint32_t sh[4];
  const int d = blockIdx.x, tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const uint32_t per = nb / 256;
  uint32_t* row = hist + (size_t)d * nb + tid * per;
  uint32_t v[4], s = 0;
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    v[k] = k < per ? row[k] : 0u;
    s += v[k];
  }
  const uint32_t inc = wave_inclusive_scan(s);
  if (l == 63) sh[w] = inc;
  __syncthreads();
  uint32_t off = inc - s;
  for (int k = 0; k < w; ++k) off += sh[k];
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    if (k < per) row[k] = off;
    off += v[k];
  }
  if (tid == 255) total[d] = off;
}

// Stable scatter of one block's partition, a tile of 256 x KPT keys at a time
// (IDV: no values in, the keys' input positions are the values; WK: the keys
// are written out, which the last pass of the tile sort skips).
// Wave w ranks keys [w * 64 KPT, (w + 1) * 64 KPT) of the tile in index order.
// For the block-wide prefixes each thread owns DPT = 2^DB / 256 consecutive
// digits.
template <typename K, int KPT, int DB, bool IDV, bool WK>
__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t* __restrict__ count, const K* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin, int shift, int dbits,
                                                       uint32_t nb, const uint32_t* __restrict__ offsets,
                                                       const uint32_t* __restrict__ total, K* __restrict__ kout,
                                                       uint32_t* __restrict__ vout) {
  constexpr uint32_t TILE = 256 * KPT;
  constexpr int R = 1 << DB, DPT = R / 256;
  __shared__ K lk[TILE];
  __shared__ uint32_t lv[TILE];
  __shared__ uint32_t wc[4][R];     // running digit counts of each wave, then the waves' digit prefixes
  __shared__ uint32_t dstart[R], gofs[R];
  __shared__ uint32_t sh[4];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const uint32_t nd = 1u << dbits, dmask = nd - 1u;
  const uint32_t d0 = (uint32_t)tid * DPT;
  const uint32_t part = xcd_part(blockIdx.x, nb);
  {
    // digit bases: exclusive scan of the digit totals
    uint32_t t[DPT], ts = 0;
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      t[k] = d0 + k < nd ? total[d0 + k] : 0u;
      ts += t[k];
    }
    const uint32_t inc = wave_inclusive_scan(ts);
    if (l == 63) sh[w] = inc;
    __syncthreads();
    uint32_t base = inc - ts;
    for (int k = 0; k < w; ++k) base += sh[k];
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      gofs[d0 + k] = d0 + k < nd ? base + offsets[(size_t)(d0 + k) * nb + part] : 0u;
      base += t[k];
    }
  }
#pragma unroll
  for (int k = 0; k < DPT; ++k) wc[0][d0 + k] = wc[1][d0 + k] = wc[2][d0 + k] = wc[3][d0 + k] = 0u;
  uint32_t lo, hi;
  part_range(*count, nb, part, lo, hi);
  const uint64_t lt = (1ull << l) - 1ull;
  __syncthreads();
  for (uint32_t tb = lo; tb < hi; tb += TILE) {
    const uint32_t tn = min(TILE, hi - tb);
    const uint32_t wb = tb + (uint32_t)w * (64u * KPT);
    K kk[KPT];
    uint32_t vv[KPT], rk[KPT];
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const uint32_t i = wb + q * 64 + l;
      kk[q] = 0;
      vv[q] = 0;
      if (i < hi) {
        kk[q] = kin[i];
        vv[q] = IDV ? i : vin[i];
      }
    }
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const bool valid = wb + q * 64 + l < hi;
      const uint32_t d = (uint32_t)(kk[q] >> shift) & dmask;
      const uint64_t peers = digit_peers<DB>(valid, d);
      const uint32_t r = (uint32_t)__popcll(peers & lt);
      const uint32_t before = valid ? wc[w][d] : 0u;
      __builtin_amdgcn_wave_barrier();
      if (valid && r == 0) wc[w][d] = before + (uint32_t)__popcll(peers);
      rk[q] = before + r;
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // digit-major prefix: digit start in the tile, then the waves in order
    uint32_t c0[DPT], c1[DPT], c2[DPT], tot[DPT], ts = 0;
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      c0[k] = wc[0][d0 + k];
      c1[k] = wc[1][d0 + k];
      c2[k] = wc[2][d0 + k];
      tot[k] = c0[k] + c1[k] + c2[k] + wc[3][d0 + k];
      ts += tot[k];
    }
    const uint32_t inc = wave_inclusive_scan(ts);
    if (l == 63) sh[w] = inc;
    __syncthreads();
    uint32_t ex = inc - ts;
    for (int k = 0; k < w; ++k) ex += sh[k];
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      dstart[d0 + k] = ex;
      wc[0][d0 + k] = ex;
      wc[1][d0 + k] = ex + c0[k];
      wc[2][d0 + k] = ex + c0[k] + c1[k];
      wc[3][d0 + k] = ex + c0[k] + c1[k] + c2[k];
      ex += tot[k];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      if (wb + q * 64 + l < hi) {
        const uint32_t d = (uint32_t)(kk[q] >> shift) & dmask;
        const uint32_t pos = wc[w][d] + rk[q];
        lk[pos] = kk[q];
        lv[pos] = vv[q];
      }
    }
    __syncthreads();
    for (uint32_t i = (uint32_t)tid; i < tn; i += 256) {
      const K key = lk[i];
      const uint32_t d = (uint32_t)(key >> shift) & dmask;
      const uint32_t g = gofs[d] + (i - dstart[d]);
      if (WK) kout[g] = key;
      vout[g] = lv[i];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      gofs[d0 + k] += tot[k];
      wc[0][d0 + k] = wc[1][d0 + k] = wc[2][d0 + k] = wc[3][d0 + k] = 0u;
    }
    __syncthreads();
  }
}

// pair emission works in chunks of EP_CHUNK pairs, EP_PPT per thread
#define EP_PPT 8
#define EP_CHUNK (256 * EP_PPT)

struct EmitSlot {
  uint32_t s, gbase;
  int x0, y0, rw;
};
// A record's emission descriptor (emit_rec): its index, its view shifted
// above the tile bits of the pair keys, the first tile column and row of its
// rectangle (16 bits each) and the rectangle's width in tiles.  The projection
// leaves the last three, with the tile count, in emit_desc in record order.
__device__ __forceinline__ EmitSlot unpack_emit(uint4 q) {
  EmitSlot e;
  e.s = q.x;
  e.gbase = q.y;
  e.x0 = (int)(q.z & 0xffffu);
  e.y0 = (int)(q.z >> 16);
  e.rw = (int)q.w;
  return e;
}

// ---------------------------------------------------------------- group scan
// The depth-sorted slots are cut into groups of 64; a group's pairs are
// contiguous.  k_group_sum: tile count of every group (one wave per group);
// then a device-wide exclusive scan of the group sums;
// k_slot_offsets: each record's first pair.
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

// First pair of every record in depth order: pref[j] = part[g] + the exclusive
// scan of the tile counts inside the 64-record group g = j / 64; the same value
// goes into the record's fourth float4.  A record whose pairs hold the first
// pair of an emission chunk also names itself the chunk's first record, and
// every record leaves its emission descriptor at its depth-order position.
__global__ __launch_bounds__(256) void k_slot_offsets(const uint32_t* __restrict__ counters,
                                                      const uint32_t* __restrict__ perm,
                                                      const uint32_t* __restrict__ part, uint32_t n_groups,
                                                      const uint4* __restrict__ emit_desc, uint64_t pair_cap,
                                                      uint32_t* __restrict__ pref,
                                                      float4* __restrict__ slot_rec,
                                                      uint32_t* __restrict__ chunk_first,
                                                      uint4* __restrict__ emit_rec) {
  const uint32_t n = counters[0];
  const uint32_t l = threadIdx.x & 63;
  const uint32_t waves = gridDim.x * 4;
  for (uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6); g < n_groups; g += waves) {
    if (g * 64 >= n) break;
    const uint32_t j = g * 64 + l;
    const uint32_t s = j < n ? perm[j] : 0u;
    const uint4 d = j < n ? emit_desc[s] : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t c = d.w;
    const uint32_t incl = wave_inclusive_scan(c);
    const uint64_t off = min((uint64_t)part[g] + (incl - c), pair_cap);
    if (j < n) {
      pref[j] = (uint32_t)off;
      // the record's last 16 bytes, read with the record by the backward (the
      // debug view slot_pairoff is copied from here on request)
      slot_rec[(size_t)s * 4 + 3] = make_float4(__uint_as_float((uint32_t)off), 0.f, 0.f, 0.f);
      const uint64_t e = min(off + (uint64_t)c, pair_cap);
      for (uint64_t b = (off + EP_CHUNK - 1) / EP_CHUNK; b * EP_CHUNK < e; ++b) chunk_first[b] = j;
      emit_rec[j] = make_uint4(s, d.x, d.y, d.z);
    }
  }
}

// ---------------------------------------------------------------- slot keys
// (view, depth) key of every record.  Depths are positive FP32 values in
// [near, far], whose bit patterns are ordered like the values, so the bits
// minus those of a value just below near keep the order exactly in
// depth_bits bits (27 for near 0.2, far 80); the view sits above them.
// The keys are 4 bytes wide when view and depth bits fit in 32.  The view is
// the one the projection left above the tile bits of the emission descriptor.
template <typename K>
__global__ __launch_bounds__(KGS_BLOCK) void k_slot_keys(const uint32_t* __restrict__ counters,
                                                         const float4* __restrict__ slot_rec,
                                                         const uint4* __restrict__ emit_desc, int tile_bits,
                                                         uint32_t depth_lo, int depth_bits, K* __restrict__ keys) {
  const uint32_t n = counters[0];
  const uint32_t dmax = depth_bits >= 32 ? 0xffffffffu : (1u << depth_bits) - 1u;
  for (uint32_t s = blockIdx.x * KGS_BLOCK + threadIdx.x; s < n; s += gridDim.x * KGS_BLOCK) {
    const uint32_t b = __float_as_uint(slot_rec[(size_t)s * 4 + 1].z);
    const uint32_t d = b > depth_lo ? min(b - depth_lo, dmax) : 0u;
    keys[s] = (K)(((uint64_t)(emit_desc[s].x >> tile_bits) << depth_bits) | d);
  }
}

// ---------------------------------------------------------------- pair emission
// Balanced by pairs: each round a block takes the next EP_CHUNK pairs.  The
// chunk's first record and the next chunk's (named by k_slot_offsets) bound the
// records that own its pairs, the block stages those records' first-pair
// offsets in LDS, and each thread emits EP_PPT consecutive pairs, walking
// forward from a binary search in LDS.  A pair's key is (view << tile_bits) |
// tile, its value the record;
// pair k of a record is the k-th tile of its rectangle in row-major order, so
// its emission position is the record's first pair plus that rank.

__device__ __forceinline__ uint32_t udiv_small(uint32_t a, uint32_t b) {
  uint32_t q = (uint32_t)((float)a * __frcp_rn((float)b));
  while (q * b > a) --q;
  while ((q + 1) * b <= a) ++q;
  return q;
}

__global__ __launch_bounds__(256) void k_emit_pairs(const uint32_t* __restrict__ counters,
                                                    const uint4* __restrict__ emit_rec,
                                                    const uint32_t* __restrict__ pref,
                                                    const uint32_t* __restrict__ chunk_first,
                                                    int tiles_x, int tiles_y, uint32_t* __restrict__ keys,
                                                    uint32_t* __restrict__ vals) {
  __shared__ uint32_t s_pref[EP_CHUNK + 1];
  const uint32_t n = counters[0], np = counters[1];
  const int tid = threadIdx.x;
  const uint64_t nchunks = ((uint64_t)np + EP_CHUNK - 1) / EP_CHUNK;
  for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const uint64_t P0 = c * EP_CHUNK;
    const uint32_t p0 = (uint32_t)P0;
    const uint32_t p1 = (uint32_t)min<uint64_t>(P0 + EP_CHUNK, np) - 1u;
    // records jlo .. jhi: the owner of p0 up to the owner of the next chunk's
    // first pair (or the last record); every record owns a pair, so the owner
    // of p1 is among the first EP_CHUNK of them and the clamp drops none needed
    const uint32_t jlo = chunk_first[c];
    const uint32_t jhi = c + 1 < nchunks ? chunk_first[c + 1] : n - 1u;
    const uint32_t cnt = min(jhi - jlo + 1u, (uint32_t)EP_CHUNK);
    for (uint32_t k = tid; k < cnt; k += 256) s_pref[k] = pref[jlo + k];
    if (tid == 0) s_pref[cnt] = 0xffffffffu;
    __syncthreads();
    const uint32_t pa = p0 + (uint32_t)tid * EP_PPT;
    if (pa <= p1) {
      uint32_t a = 0, b = cnt;
      while (b - a > 1) {
        const uint32_t mid = (a + b) >> 1;
        if (s_pref[mid] <= pa) a = mid; else b = mid;
      }
      uint32_t jj = a, first = s_pref[jj], next = s_pref[jj + 1];
      EmitSlot e = unpack_emit(emit_rec[jlo + jj]);
      uint32_t ko[EP_PPT], vo[EP_PPT];
#pragma unroll
      for (int i = 0; i < EP_PPT; ++i) {
        const uint32_t p = pa + (uint32_t)i;
        ko[i] = 0xffffffffu;
        vo[i] = 0u;
        if (p <= p1) {
          if (p >= next) {
            while (p >= next) {
              ++jj;
              first = next;
              next = s_pref[jj + 1];
            }
            e = unpack_emit(emit_rec[jlo + jj]);
          }
          const uint32_t rk = p - first;
          const uint32_t qy = udiv_small(rk, (uint32_t)e.rw);
          const int ty = e.y0 + (int)qy, tx = e.x0 + (int)(rk - qy * (uint32_t)e.rw);
          ko[i] = ty < tiles_y ? e.gbase | (uint32_t)(ty * tiles_x + tx) : 0xffffffffu;
          vo[i] = e.s;
        }
      }
      if (pa + EP_PPT - 1 <= p1) {
        uint4* k4 = reinterpret_cast<uint4*>(keys + pa);
        uint4* v4 = reinterpret_cast<uint4*>(vals + pa);
        k4[0] = make_uint4(ko[0], ko[1], ko[2], ko[3]);
        k4[1] = make_uint4(ko[4], ko[5], ko[6], ko[7]);
        v4[0] = make_uint4(vo[0], vo[1], vo[2], vo[3]);
        v4[1] = make_uint4(vo[4], vo[5], vo[6], vo[7]);
      } else {
#pragma unroll
        for (int i = 0; i < EP_PPT; ++i)
          if (pa + (uint32_t)i <= p1) {
            keys[pa + i] = ko[i];
            vals[pa + i] = vo[i];
          }
      }
    }
    __syncthreads();
  }
}

// slot_pairoff[s]: the first pair of record s, copied from the record
__global__ __launch_bounds__(256) void k_pairoff_copy(const uint32_t* __restrict__ counters,
                                                      const float4* __restrict__ slot_rec,
                                                      uint32_t* __restrict__ slot_pairoff) {
  const uint32_t n = counters[0];
  for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256)
    slot_pairoff[s] = __float_as_uint(slot_rec[(size_t)s * 4 + 3].x);
}

// The sorted pair keys, for the debug view, when the single-pass tile sort did
// not write them: padding (all ones) everywhere, then (view << tile_bits) | tile
// over each (view, tile) range (one block per range).
__global__ __launch_bounds__(256) void k_keys_fill(const uint32_t* __restrict__ counters, uint32_t* __restrict__ keys) {
  const uint32_t n = counters[1];
  for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) keys[k] = 0xffffffffu;
}

__global__ __launch_bounds__(256) void k_keys_from_ranges(const uint2* __restrict__ ranges, uint32_t tiles_per_view,
                                                          int tile_bits, uint32_t* __restrict__ keys) {
  const uint32_t r = blockIdx.x, v = r / tiles_per_view, t = r - v * tiles_per_view;
  const uint2 g = ranges[r];
  for (uint32_t k = g.x + threadIdx.x; k < g.y; k += 256) keys[k] = (v << tile_bits) | t;
}

kgs_status kgs_launch_pair_keys(kgs_ctx* ctx, hipStream_t st) {
  if (ctx->pair_keys_written || !ctx->binned) return KGS_OK;
  uint32_t* keys = ctx->keys[ctx->sorted_buf];
  const uint64_t P = (uint64_t)ctx->cfg.pair_capacity;
  hipLaunchKernelGGL(k_keys_fill, dim3((unsigned)std::min<uint64_t>(std::max<uint64_t>((P + 255) / 256, 1), 4096)),
                     dim3(256), 0, st, (const uint32_t*)ctx->counters, keys);
  const uint32_t n_ranges = (uint32_t)(ctx->last_views * ctx->n_tiles);
  if (n_ranges > 0)
    hipLaunchKernelGGL(k_keys_from_ranges, dim3(n_ranges), dim3(256), 0, st, (const uint2*)ctx->ranges,
                       (uint32_t)ctx->n_tiles, ctx->tile_bits, keys);
  ctx->pair_keys_written = 1;
  return kgs_check_launch();
}

// slot_view[s] for the debug view: the projection keeps each slot's view only
// in its emission descriptor, above the tile bits.
__global__ __launch_bounds__(256) void k_slot_view_copy(const uint32_t* __restrict__ counters,
                                                        const uint4* __restrict__ emit_desc, int tile_bits,
                                                        uint32_t* __restrict__ slot_view) {
  const uint32_t n = counters[0];
  for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256) slot_view[s] = emit_desc[s].x >> tile_bits;
}

kgs_status kgs_launch_slot_view_copy(kgs_ctx* ctx, hipStream_t st) {
  const uint64_t S = (uint64_t)ctx->cfg.slot_capacity;
  hipLaunchKernelGGL(k_slot_view_copy, dim3((unsigned)std::min<uint64_t>(std::max<uint64_t>((S + 255) / 256, 1), 4096)),
                     dim3(256), 0, st, (const uint32_t*)ctx->counters, (const uint4*)ctx->emit_desc,
                     kgs_tile_bits(ctx->n_tiles), ctx->slot_view);
  return kgs_check_launch();
}

kgs_status kgs_launch_pairoff_copy(kgs_ctx* ctx, hipStream_t st) {
  const uint64_t S = (uint64_t)ctx->cfg.slot_capacity;
  hipLaunchKernelGGL(k_pairoff_copy, dim3((unsigned)std::min<uint64_t>(std::max<uint64_t>((S + 255) / 256, 1), 4096)),
                     dim3(256), 0, st, (const uint32_t*)ctx->counters, (const float4*)ctx->slot_rec,
                     ctx->slot_pairoff);
  return kgs_check_launch();
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(KGS_BLOCK) void k_ranges(const uint32_t* __restrict__ counters,
                                                      const uint32_t* __restrict__ keys, int tile_bits,
                                                      uint32_t tiles_per_view, uint32_t n_views,
                                                      uint2* __restrict__ ranges) {
  const uint32_t n = counters[1];
  const uint32_t tmask = (1u << tile_bits) - 1u;
  // view-major index of a key's (view, tile), or ~0 for padding
  auto dense = [&](uint32_t t) { return (t >> tile_bits) < n_views ? (t >> tile_bits) * tiles_per_view + (t & tmask)
                                                                   : 0xffffffffu; };
  for (uint32_t k = blockIdx.x * KGS_BLOCK + threadIdx.x; k < n; k += gridDim.x * KGS_BLOCK) {
    const uint32_t t = keys[k];
    const uint32_t tn = k + 1 < n ? keys[k + 1] : 0xffffffffu;
    if (t == tn) continue;
    // k is the last pair of group t and k + 1 the first of group tn
    const uint32_t a = dense(t), b = dense(tn);
    if (a != 0xffffffffu) ranges[a].y = k + 1;
    if (b != 0xffffffffu) ranges[b].x = k + 1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && n > 0) {
    const uint32_t t0 = dense(keys[0]);
    if (t0 != 0xffffffffu) ranges[t0].x = 0;
  }
}

// Launch order of the compositing workgroups: (view, tile) entries by
// decreasing pair count (log-spaced buckets, 8 per octave), so the longest
// tiles start first and the launch does not end on a few of them.  The order
// inside a bucket is whatever the atomics give; it changes only which
// workgroup runs when, never a result.
__device__ __forceinline__ uint32_t len_bucket(uint32_t n) {
  if (n == 0u) return 0u;
  const uint32_t lz = 31u - (uint32_t)__clz((int)n);
  const uint32_t frac = lz >= 3u ? (n >> (lz - 3u)) & 7u : (n << (3u - lz)) & 7u;
  return min(1u + lz * 8u + frac, 255u);
}

// Ranges of a single-pass tile sort, whose sorted keys are not written: tile
// t's pairs are the run [S_t, S_t + n_t) (S the exclusive sum of the digit
// totals, in digit order, as the scatter placed them), and inside the run the
// views come in order (emission is view-major and the sort stable).  A slot's
// view follows from its index, slots being view-major: view >= v exactly when
// the slot is at least view v's first slot.  So each (view, tile) range is two
// binary searches in its tile's run.  Every range is written (empty ones as
// (0, 0)).
__global__ __launch_bounds__(256) void k_ranges_by_slot(const uint32_t* __restrict__ counters,
                                                        const uint32_t* __restrict__ total, int n_digits,
                                                        const uint32_t* __restrict__ sorted_slot,
                                                        const uint32_t* __restrict__ blk_base, int64_t nb,
                                                        uint32_t tiles_per_view, uint32_t n_views,
                                                        uint2* __restrict__ ranges) {
  __shared__ uint32_t s_start[KGS_RADIX_BUCKETS];
  __shared__ uint32_t s_vb[KGS_MAX_VIEWS + 1];
  __shared__ uint32_t s_w[4];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const uint32_t n_slots = counters[0];
  // digit starts: exclusive scan of the totals, four digits per thread
  {
    uint32_t t[4], ts = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int d = 4 * tid + k;
      t[k] = d < n_digits ? total[d] : 0u;
      ts += t[k];
    }
    const uint32_t inc = wave_inclusive_scan(ts);
    if (l == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t ex = inc - ts;
    for (int k = 0; k < w; ++k) ex += s_w[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s_start[4 * tid + k] = ex;
      ex += t[k];
    }
  }
  for (uint32_t v = tid; v <= n_views; v += 256)
    s_vb[v] = v < n_views ? min(blk_base[((int64_t)v * nb) * 2], n_slots) : n_slots;
  __syncthreads();
  const uint32_t n_ranges = tiles_per_view * n_views;
  for (uint32_t r = blockIdx.x * 256 + tid; r < n_ranges; r += gridDim.x * 256) {
    const uint32_t v = r / tiles_per_view, t = r - v * tiles_per_view;
    const uint32_t a = s_start[t], e = a + total[t];
    // the first positions in [a, e) whose slot is at least view v's first slot
    // and at least view v + 1's: two binary searches, stepped together so that
    // their dependent loads overlap
    const uint32_t b0 = s_vb[v], b1 = s_vb[v + 1];
    uint32_t lo0 = a, hi0 = e, lo1 = a, hi1 = e;
    while (lo0 < hi0 || lo1 < hi1) {
      const bool go0 = lo0 < hi0, go1 = lo1 < hi1;
      const uint32_t m0 = lo0 + ((hi0 - lo0) >> 1), m1 = lo1 + ((hi1 - lo1) >> 1);
      const uint32_t x0 = go0 ? sorted_slot[m0] : 0u, x1 = go1 ? sorted_slot[m1] : 0u;
      if (go0) {
        if (x0 < b0) lo0 = m0 + 1; else hi0 = m0;
      }
      if (go1) {
        if (x1 < b1) lo1 = m1 + 1; else hi1 = m1;
      }
    }
    // an empty range is (0, 0), as k_ranges leaves it
    ranges[r] = lo0 < lo1 ? make_uint2(lo0, lo1) : make_uint2(0u, 0u);
  }
}


__global__ __launch_bounds__(1024) void k_tile_order(const uint2* __restrict__ ranges, uint32_t n_tiles_all,
                                                     uint32_t* __restrict__ order) {
  __shared__ uint32_t cnt[256], off[256];
  const int tid = threadIdx.x;
  if (tid < 256) cnt[tid] = 0u;
  __syncthreads();
  for (uint32_t i = tid; i < n_tiles_all; i += 1024) {
    const uint2 r = ranges[i];
    atomicAdd(&cnt[len_bucket(r.y - r.x)], 1u);
  }
  __syncthreads();
  if (tid < 64) {
    // buckets in decreasing order: bucket 255 - 4 tid - q
    uint32_t c[4], t = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      c[q] = cnt[255 - 4 * tid - q];
      t += c[q];
    }
    uint32_t ex = wave_inclusive_scan(t) - t;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      off[255 - 4 * tid - q] = ex;
      ex += c[q];
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < n_tiles_all; i += 1024) {
    const uint2 r = ranges[i];
    order[atomicAdd(&off[len_bucket(r.y - r.x)], 1u)] = i;
  }
}

// ---------------------------------------------------------------- host side
// Digit plan of a sort over `bits` key bits: the fewest passes of at most
// max_dbits (8 or 10) bits each, of equal width.
static void radix_plan(int bits, int max_dbits, int& passes, int& dbits) {
  passes = (bits + max_dbits - 1) / max_dbits;
  dbits = (bits + passes - 1) / passes;
}

// KPT keys per thread in a scatter tile: 16 (8 for 8-byte keys).
template <typename K, int KPT, int DB, bool AGG>
static void radix_pass(kgs_ctx* ctx, const uint32_t* count, uint32_t nb, const K* kin, const uint32_t* vin,
                       int shift, int dbits, uint32_t* total, K* kout, uint32_t* vout, bool write_keys,
                       hipStream_t st) {
  hipLaunchKernelGGL((k_radix_hist<K, DB, AGG>), dim3(nb), dim3(256), 0, st, count, kin, shift, dbits, nb,
                     ctx->radix_hist);
  hipLaunchKernelGGL(k_radix_scan, dim3(1u << dbits), dim3(256), 0, st, ctx->radix_hist, nb, total);
#define KGS_SCATTER(IDV, WK)                                                                                      \
  hipLaunchKernelGGL((k_radix_scatter<K, KPT, DB, IDV, WK>), dim3(nb), dim3(256), 0, st, count, kin, vin, shift,  \
                     dbits, nb, (const uint32_t*)ctx->radix_hist, (const uint32_t*)total, kout, vout)
  if (vin) {
    if (write_keys) KGS_SCATTER(false, true); else KGS_SCATTER(false, false);
  } else {
    if (write_keys) KGS_SCATTER(true, true); else KGS_SCATTER(true, false);
  }
#undef KGS_SCATTER
}

// vals_in: the values of the first pass (null: the key positions); agg: the
// histograms count runs of equal digits (keys whose digits repeat, like the
// depth keys' views and exponents) rather than single keys.
template <typename K>
static int radix_sort(kgs_ctx* ctx, const uint32_t* count, uint64_t cap, K* keys[2], uint32_t* vals[2], int bits,
                      int max_dbits, bool agg, hipStream_t st, const uint32_t* vals_in, bool last_keys = true) {
  int passes, dbits;
  radix_plan(bits, max_dbits, passes, dbits);
  // partitions: fewer for small sorts (a multiple of 256, at most KGS_SORT_BLOCKS): more would only add
  // histogram rows, the passes of a 2M-record sort being latency bound either way
  const uint32_t nb = cap >= (8u << 20) ? KGS_SORT_BLOCKS : std::min<uint32_t>(512u, KGS_SORT_BLOCKS);
  constexpr int KPT = sizeof(K) == 8 ? 8 : 16;
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    const K* kin = keys[cur];
    const uint32_t* vin = p == 0 ? vals_in : (const uint32_t*)vals[cur];
    uint32_t* total = ctx->radix_total + KGS_RADIX_BUCKETS * p;
    K* ko = keys[cur ^ 1];
    uint32_t* vo = vals[cur ^ 1];
    const bool wk = last_keys || p + 1 < passes;
#define KGS_RPASS(DB, AG) radix_pass<K, KPT, DB, AG>(ctx, count, nb, kin, vin, dbits * p, dbits, total, ko, vo, wk, st)
    if (dbits > 8) {
      if (agg) KGS_RPASS(10, true); else KGS_RPASS(10, false);
    } else {
      if (agg) KGS_RPASS(8, true); else KGS_RPASS(8, false);
    }
#undef KGS_RPASS
    cur ^= 1;
  }
  return cur;
}

kgs_status kgs_launch_bin_sort(kgs_ctx* ctx, hipStream_t st) {
  const int V = ctx->last_views;
  const uint32_t n_tiles_all = (uint32_t)(V * ctx->n_tiles);
  const uint64_t S = (uint64_t)ctx->cfg.slot_capacity, P = (uint64_t)ctx->cfg.pair_capacity;
  const unsigned sgrid = (unsigned)std::min<uint64_t>(std::max<uint64_t>((S + KGS_BLOCK - 1) / KGS_BLOCK, 1), 4096);
  // 1. records by (view, depth); the projection wrote the keys, unless a sort
  // since has used them
  const SlotKeyLayout KL = slot_key_layout(ctx->cfg.near_z, ctx->cfg.far_z, V);
  ctx->tile_bits = kgs_tile_bits(ctx->n_tiles);
  if (ctx->tile_bits + 7 > 32) return KGS_ERR_INVALID_ARG;  // 64 views above the tile bits, padding apart
  const int key_bits = KL.depth_bits + KL.view_bits;
  int sc;
  if (KL.key32()) {
    uint32_t* k32[2] = {reinterpret_cast<uint32_t*>(ctx->slot_keys[0]), reinterpret_cast<uint32_t*>(ctx->slot_keys[1])};
    if (!ctx->slot_keys_ready)
      hipLaunchKernelGGL(k_slot_keys<uint32_t>, dim3(sgrid), dim3(KGS_BLOCK), 0, st, (const uint32_t*)ctx->counters,
                         (const float4*)ctx->slot_rec, (const uint4*)ctx->emit_desc, ctx->tile_bits, KL.depth_lo,
                         KL.depth_bits, k32[0]);
    sc = radix_sort<uint32_t>(ctx, ctx->counters, S, k32, ctx->slot_vals, key_bits, KGS_DEPTH_DIGIT_BITS, true, st,
                              nullptr, false);
  } else {
    if (!ctx->slot_keys_ready)
      hipLaunchKernelGGL(k_slot_keys<uint64_t>, dim3(sgrid), dim3(KGS_BLOCK), 0, st, (const uint32_t*)ctx->counters,
                         (const float4*)ctx->slot_rec, (const uint4*)ctx->emit_desc, ctx->tile_bits, KL.depth_lo,
                         KL.depth_bits, ctx->slot_keys[0]);
    sc = radix_sort<uint64_t>(ctx, ctx->counters, S, ctx->slot_keys, ctx->slot_vals, key_bits, KGS_DEPTH_DIGIT_BITS,
                              true, st, nullptr, false);
  }
  // only the order is used: the last pass writes no keys (the buffer is scratch afterwards)
  ctx->slot_keys_ready = 0;
  const uint32_t* perm = ctx->slot_vals[sc];
  ctx->perm = perm;
  // 2. first pair of every record in that order, then the pairs
  const uint32_t n_groups = (uint32_t)((S + 63) / 64);
  const unsigned eg = (unsigned)std::min<uint64_t>(std::max<uint64_t>((n_groups + 3) / 4, 1), 2048);
  hipLaunchKernelGGL(k_group_sum, dim3(eg), dim3(256), 0, st, (const uint32_t*)ctx->counters, perm,
                     (const uint32_t*)ctx->slot_ntiles, n_groups, ctx->group_part);
  kgs_launch_scan(ctx->group_part, ctx->group_part, n_groups, 1, ~0ull, ~0ull, ctx->scan_part, ctx->scan_totals, st);
  uint32_t* pref = reinterpret_cast<uint32_t*>(ctx->slot_keys[sc ^ 1]);  // free after the record sort
  hipLaunchKernelGGL(k_slot_offsets, dim3(eg), dim3(256), 0, st, (const uint32_t*)ctx->counters, perm,
                     (const uint32_t*)ctx->group_part, n_groups, (const uint4*)ctx->emit_desc, P, pref,
                     ctx->slot_rec, ctx->chunk_first, ctx->emit_rec);
  const uint64_t chunks = (P + EP_CHUNK - 1) / EP_CHUNK;
  const unsigned pg = (unsigned)std::min<uint64_t>(std::max<uint64_t>(chunks, 1), 4096);
  hipLaunchKernelGGL(k_emit_pairs, dim3(pg), dim3(256), 0, st, (const uint32_t*)ctx->counters,
                     (const uint4*)ctx->emit_rec, (const uint32_t*)pref, (const uint32_t*)ctx->chunk_first,
                     ctx->tiles_x, ctx->tiles_y, ctx->keys[0], ctx->pair_slot);
  // 3. pairs by tile within the view (stable): the view bits above stay in the
  // keys but out of the sort, so a (view, tile) group stays in emission order
  // With one pass (tile bits <= 10) the sorted keys are not written: the
  // ranges come from the digit totals and the slots; with two, from the keys.
  int tpasses, tdbits;
  radix_plan(ctx->tile_bits, 10, tpasses, tdbits);
  const bool one_pass = tpasses == 1;
  const int cur = radix_sort<uint32_t>(ctx, ctx->counters + 1, P, ctx->keys, ctx->vals, ctx->tile_bits, 10, false, st,
                                       ctx->pair_slot, !one_pass);
  ctx->sorted_buf = cur;
  ctx->pair_keys_written = one_pass ? 0 : 1;
  if (one_pass) {
    const int64_t nbp = (ctx->last_n + KGS_BLOCK - 1) / KGS_BLOCK;   // the projection's blocks per view
    const unsigned rg = (unsigned)std::min<uint64_t>(std::max<uint64_t>((n_tiles_all + 255) / 256, 1), 1024);
    hipLaunchKernelGGL(k_ranges_by_slot, dim3(rg), dim3(256), 0, st, (const uint32_t*)ctx->counters,
                       (const uint32_t*)ctx->radix_total, 1 << tdbits, (const uint32_t*)ctx->vals[cur],
                       (const uint32_t*)ctx->blk_base, nbp, (uint32_t)ctx->n_tiles, (uint32_t)V, ctx->ranges);
  } else {
    const uint64_t nr = (uint64_t)n_tiles_all * 2;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<uint64_t>((nr + 255) / 256, 1024)), dim3(256), 0, st,
                       (uint32_t*)ctx->ranges, nr, 0u);
    const unsigned rg = (unsigned)std::min<uint64_t>(std::max<uint64_t>((P + KGS_BLOCK - 1) / KGS_BLOCK, 1), 8192);
    hipLaunchKernelGGL(k_ranges, dim3(rg), dim3(KGS_BLOCK), 0, st, (const uint32_t*)ctx->counters,
                       (const uint32_t*)ctx->keys[cur], ctx->tile_bits, (uint32_t)ctx->n_tiles, (uint32_t)V,
                       ctx->ranges);
  }
  hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, st, (const uint2*)ctx->ranges, n_tiles_all,
                     ctx->tile_order);
  ctx->sorted_slot = ctx->vals[cur];
  return kgs_check_launch();
}
