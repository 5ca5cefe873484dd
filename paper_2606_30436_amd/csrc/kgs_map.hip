// Map maintenance on the GPU: the spatial hash of occupied voxels and the
// anchors it creates (appendix, "Dynamic Map Expansion"), the densify and prune
// decisions of Sec. 3.3 acting on the map, and the rigid re-alignment after loop
// closure with the re-voxelisation that merges overlapping anchors (appendix,
// "Global Map Alignment").
//
// Hash: open addressing with linear probing over 2^k slots of 16 bytes (key,
// anchor, first candidate).  A batch insertion is deterministic although the
// slots are claimed by racing compare-and-swaps: every candidate first finds or
// claims its key's slot and, if the key is new in this batch (its anchor is still
// pending), lowers the slot's "first candidate" to its own index; the candidates
// that are their key's first then take consecutive anchor numbers through a scan
// in candidate order, and write them; finally every candidate reads its key's
// anchor.  Which slot a key lands in can differ between runs, but no output
// depends on it.  Bound: scattered 16-byte slot accesses and the scan (HBM / L2
// latency).  The per-Gaussian passes (spawn, compaction, alignment, densify
// points) stream structure-of-arrays parameters: HBM bound.
//
// Every integer decision (voxel floor, level band, argmax of the scales) is
// taken in FP64.
#include <cmath>

#include "kgs_internal.h"

#define MP_EMPTY 0xffffffffffffffffull
#define MP_PENDING 0xffffffffu
#define MP_OFF (1 << 19)

struct MapSlot {
  unsigned long long key;
  uint32_t anchor;
  uint32_t first;
};

struct MapEps {
  double eps[5], dmax[4];
};

static MapEps map_eps() {
  MapEps E;
  const double e[5] = {0.1, 0.25, 1.0, 5.0, 25.0};
  for (int l = 0; l < 5; ++l) E.eps[l] = e[l];
  for (int l = 0; l < 4; ++l) E.dmax[l] = 100.0 * e[l];
  return E;
}

__device__ __forceinline__ int level_of_dist(const MapEps& E, double d) {
  int lev = 4;
  for (int l = 3; l >= 0; --l)
    if (d < E.dmax[l]) lev = l;
  return lev;
}

// (level, idx) -> key; MP_EMPTY when an index leaves the 20-bit range
__device__ __forceinline__ unsigned long long pack_key(int level, long long x, long long y, long long z) {
  x += MP_OFF;
  y += MP_OFF;
  z += MP_OFF;
  if (level < 0 || level > 7 || x < 0 || y < 0 || z < 0 || x >= (1 << 20) || y >= (1 << 20) || z >= (1 << 20))
    return MP_EMPTY;
  return ((unsigned long long)level << 60) | ((unsigned long long)x << 40) | ((unsigned long long)y << 20) |
         (unsigned long long)z;
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long k) {
  k ^= k >> 30;
  k *= 0xbf58476d1ce4e5b9ull;
  k ^= k >> 27;
  k *= 0x94d049bb133111ebull;
  k ^= k >> 31;
  return k;
}

__global__ __launch_bounds__(256) void k_map_clear(MapSlot* __restrict__ t, uint64_t cap) {
  for (uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x; s < cap; s += (uint64_t)gridDim.x * 256) {
    t[s].key = MP_EMPTY;
    t[s].anchor = MP_PENDING;
    t[s].first = 0xffffffffu;
  }
}

__global__ __launch_bounds__(256) void k_map_keys(const int32_t* __restrict__ level, const int32_t* __restrict__ vox,
                                                  int64_t n, unsigned long long* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) keys[i] = pack_key(level[i], vox[3 * i], vox[3 * i + 1], vox[3 * i + 2]);
}

// Pass 1: find or claim the slot; a key still pending (new in this batch) records its first candidate.
__global__ __launch_bounds__(256) void k_map_probe(MapSlot* __restrict__ t, uint64_t mask,
                                                   const unsigned long long* __restrict__ keys, int64_t n,
                                                   uint32_t* __restrict__ cand_slot, uint32_t* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const unsigned long long key = keys[i];
  uint32_t found = 0xffffffffu;
  if (key != MP_EMPTY) {
    uint64_t s = mix64(key) & mask;
    for (uint64_t p = 0; p <= mask; ++p) {
      const unsigned long long old = atomicCAS(&t[s].key, MP_EMPTY, key);
      if (old == MP_EMPTY || old == key) {
        found = (uint32_t)s;
        break;
      }
      s = (s + 1) & mask;
    }
    if (found == 0xffffffffu) atomicOr(status, 1u);   // table full
    else if (t[found].anchor == MP_PENDING) atomicMin(&t[found].first, (uint32_t)i);
  }
  cand_slot[i] = found;
}

__device__ __forceinline__ bool map_is_first(const MapSlot* t, const uint32_t* cand_slot, int64_t i, int64_t n) {
  if (i >= n) return false;
  const uint32_t s = cand_slot[i];
  return s != 0xffffffffu && t[s].anchor == MP_PENDING && t[s].first == (uint32_t)i;
}

// Pass 2: per 256 candidates, how many are their key's first.
__global__ __launch_bounds__(256) void k_map_count(const MapSlot* __restrict__ t, const uint32_t* __restrict__ cand_slot,
                                                   int64_t n, uint32_t* __restrict__ counts) {
  __shared__ uint32_t sc[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t c = (uint32_t)__popcll(ballot64(map_is_first(t, cand_slot, i, n)));
  if ((threadIdx.x & 63) == 0) sc[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = (sc[0] + sc[1]) + (sc[2] + sc[3]);
}

// Pass 3: the firsts take anchors n_in + rank (candidate order) and free their slot's first field.
__global__ __launch_bounds__(256) void k_map_assign(MapSlot* __restrict__ t, const uint32_t* __restrict__ cand_slot,
                                                    int64_t n, const uint32_t* __restrict__ offsets,
                                                    const unsigned long long* __restrict__ total,
                                                    const uint32_t* __restrict__ n_in, uint32_t* __restrict__ created,
                                                    uint32_t* __restrict__ n_out) {
  __shared__ uint32_t sc[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool f = map_is_first(t, cand_slot, i, n);
  const uint64_t b = ballot64(f);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sc[w] = (uint32_t)__popcll(b);
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = *n_in + (uint32_t)*total;
  if (!f) return;
  uint32_t rank = offsets[blockIdx.x] + mask_lt_count(b);
  for (int k = 0; k < w; ++k) rank += sc[k];
  const uint32_t s = cand_slot[i];
  t[s].anchor = *n_in + rank;
  t[s].first = 0xffffffffu;
  if (created) created[rank] = (uint32_t)i;
}

// Pass 4: every candidate's anchor.
__global__ __launch_bounds__(256) void k_map_lookup(const MapSlot* __restrict__ t, const uint32_t* __restrict__ cand_slot,
                                                    int64_t n, uint32_t* __restrict__ anchor) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = cand_slot[i];
  anchor[i] = s == 0xffffffffu ? 0xffffffffu : t[s].anchor;
}

// ---- new Gaussians for created anchors
__global__ __launch_bounds__(256) void k_map_spawn(MapEps E, const uint32_t* __restrict__ created,
                                                   const uint32_t* __restrict__ n_in, const uint32_t* __restrict__ n_out,
                                                   const int32_t* __restrict__ level, const int32_t* __restrict__ vox,
                                                   const float* __restrict__ color, kgs_gaussians_out g,
                                                   uint32_t* __restrict__ status) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t a = *n_in, b = *n_out;
  if (k >= (int64_t)(b - a)) return;
  const int64_t j = (int64_t)a + k;   // the new Gaussian's index
  if (j >= g.n) {
    atomicOr(status, 2u);             // the parameter arrays are full
    return;
  }
  const uint32_t c = created[k];
  const int lev = level[c];
  const double eps = E.eps[lev];
  const int64_t N = g.n;
  for (int d = 0; d < 3; ++d) {
    g.means[d * N + j] = (float)((double)vox[3 * c + d] * eps);
    g.log_scales[d * N + j] = (float)log(eps);
  }
  g.quats[j] = 1.f;
  g.quats[N + j] = 0.f;
  g.quats[2 * N + j] = 0.f;
  g.quats[3 * N + j] = 0.f;
  g.opacity_logits[j] = (float)log(0.1 / 0.9);
  const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
  for (int d = 0; d < 3; ++d) {
    g.sh[(int64_t)d * N + j] = (float)(((double)color[3 * c + d] - 0.5) / 0.28209479177387814);
    for (int q = 1; q < K; ++q) g.sh[((int64_t)q * 3 + d) * N + j] = 0.f;
  }
}

// ---- densify points: mu +- s_max a_max of each Gaussian marked DENSIFY
__device__ __forceinline__ void quat_rot_d(const double q[4], double R[9]) {
  const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

__global__ __launch_bounds__(256) void k_densify_count(const uint8_t* __restrict__ decision, int64_t n,
                                                       uint32_t* __restrict__ counts) {
  __shared__ uint32_t sc[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t c = (uint32_t)__popcll(ballot64(i < n && decision[i] == KGS_DENSIFY));
  if ((threadIdx.x & 63) == 0) sc[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = (sc[0] + sc[1]) + (sc[2] + sc[3]);
}

__global__ __launch_bounds__(256) void k_densify_emit(MapEps E, kgs_gaussians g, const uint8_t* __restrict__ decision,
                                                      double cx, double cy, double cz,
                                                      const uint32_t* __restrict__ offsets,
                                                      const unsigned long long* __restrict__ total, int64_t cap,
                                                      int32_t* __restrict__ level, int32_t* __restrict__ vox,
                                                      float* __restrict__ point, uint32_t* __restrict__ source,
                                                      uint32_t* __restrict__ count) {
  __shared__ uint32_t sc[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = g.n;
  const bool f = i < n && decision[i] == KGS_DENSIFY;
  const uint64_t b = ballot64(f);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sc[w] = (uint32_t)__popcll(b);
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = (uint32_t)min(2ull * *total, 0xffffffffull);
  if (!f) return;
  uint64_t r = offsets[blockIdx.x] + mask_lt_count(b);
  for (int k = 0; k < w; ++k) r += sc[k];
  const double s[3] = {exp((double)g.log_scales[i]), exp((double)g.log_scales[n + i]),
                       exp((double)g.log_scales[2 * n + i])};
  int k = 0;
  if (s[1] > s[k]) k = 1;
  if (s[2] > s[k]) k = 2;
  const double q[4] = {g.quats[i], g.quats[n + i], g.quats[2 * n + i], g.quats[3 * n + i]};
  double R[9];
  quat_rot_d(q, R);
  const double mu[3] = {g.means[i], g.means[n + i], g.means[2 * n + i]};
  for (int h = 0; h < 2; ++h) {
    const uint64_t o = 2 * r + h;
    if (o >= (uint64_t)cap) return;
    const double sg = h == 0 ? 1.0 : -1.0;
    double p[3];
    for (int d = 0; d < 3; ++d) p[d] = mu[d] + sg * s[k] * R[3 * d + k];
    const double e0 = p[0] - cx, e1 = p[1] - cy, e2 = p[2] - cz;
    const int lev = level_of_dist(E, sqrt(e0 * e0 + e1 * e1 + e2 * e2));
    level[o] = lev;
    source[o] = (uint32_t)i;
    for (int d = 0; d < 3; ++d) {
      vox[3 * o + d] = (int32_t)floor(p[d] / E.eps[lev]);
      point[3 * o + d] = (float)p[d];
    }
  }
}

// ---- prune compaction: survivors gathered to their keep-map index
__global__ __launch_bounds__(256) void k_map_compact(kgs_gaussians g, const uint8_t* __restrict__ decision,
                                                     const uint32_t* __restrict__ keep_map, kgs_gaussians_out o) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = g.n;
  if (i >= n || decision[i] == KGS_PRUNE) return;
  const int64_t j = keep_map[i], M = o.n;
  if (j >= M) return;
  for (int d = 0; d < 3; ++d) {
    o.means[d * M + j] = g.means[d * n + i];
    o.log_scales[d * M + j] = g.log_scales[d * n + i];
  }
  for (int d = 0; d < 4; ++d) o.quats[d * M + j] = g.quats[d * n + i];
  o.opacity_logits[j] = g.opacity_logits[i];
  const int K3 = 3 * (g.sh_degree + 1) * (g.sh_degree + 1);
  for (int q = 0; q < K3; ++q) o.sh[q * M + j] = g.sh[q * n + i];
}

// ---- rigid alignment: p' = R_new^T (R_old p + t_old - t_new), q' = quat(R_new^T R_old) q
__device__ __forceinline__ void rot_to_quat_d(const double R[9], double q[4]) {
  const double tr = R[0] + R[4] + R[8];
  const double c[4] = {1 + tr, 1 + 2 * R[0] - tr, 1 + 2 * R[4] - tr, 1 + 2 * R[8] - tr};
  int k = 0;
  for (int j = 1; j < 4; ++j)
    if (c[j] > c[k]) k = j;
  const double r = sqrt(c[k]), h = 0.5 * r, f = 0.5 / r;
  if (k == 0) { q[0] = h; q[1] = (R[7] - R[5]) * f; q[2] = (R[2] - R[6]) * f; q[3] = (R[3] - R[1]) * f; }
  else if (k == 1) { q[0] = (R[7] - R[5]) * f; q[1] = h; q[2] = (R[1] + R[3]) * f; q[3] = (R[2] + R[6]) * f; }
  else if (k == 2) { q[0] = (R[2] - R[6]) * f; q[1] = (R[1] + R[3]) * f; q[2] = h; q[3] = (R[5] + R[7]) * f; }
  else { q[0] = (R[3] - R[1]) * f; q[1] = (R[2] + R[6]) * f; q[2] = (R[5] + R[7]) * f; q[3] = h; }
  if (q[0] < 0) for (int j = 0; j < 4; ++j) q[j] = -q[j];
}

__global__ __launch_bounds__(256) void k_map_align(float* __restrict__ means, float* __restrict__ quats, int64_t n,
                                                   const int32_t* __restrict__ keyframe_of,
                                                   const kgs_camera* __restrict__ old_pose,
                                                   const kgs_camera* __restrict__ new_pose, int n_kf) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int m = keyframe_of[i];
  if (m < 0 || m >= n_kf) return;
  const kgs_camera A = old_pose[m], B = new_pose[m];
  double p[3], y[3];
  for (int d = 0; d < 3; ++d) p[d] = means[d * n + i];
  for (int r = 0; r < 3; ++r)
    y[r] = (double)A.R[3 * r] * p[0] + (double)A.R[3 * r + 1] * p[1] + (double)A.R[3 * r + 2] * p[2] +
           (double)A.t[r] - (double)B.t[r];
  double Rr[9];
  for (int r = 0; r < 3; ++r) {
    means[r * n + i] = (float)((double)B.R[r] * y[0] + (double)B.R[3 + r] * y[1] + (double)B.R[6 + r] * y[2]);
    for (int c = 0; c < 3; ++c)
      Rr[3 * r + c] = (double)B.R[r] * A.R[c] + (double)B.R[3 + r] * A.R[3 + c] + (double)B.R[6 + r] * A.R[6 + c];
  }
  double a[4];
  rot_to_quat_d(Rr, a);
  const double b0 = quats[i], b1 = quats[n + i], b2 = quats[2 * n + i], b3 = quats[3 * n + i];
  quats[i] = (float)(a[0] * b0 - a[1] * b1 - a[2] * b2 - a[3] * b3);
  quats[n + i] = (float)(a[0] * b1 + a[1] * b0 + a[2] * b3 - a[3] * b2);
  quats[2 * n + i] = (float)(a[0] * b2 - a[1] * b3 + a[2] * b0 + a[3] * b1);
  quats[3 * n + i] = (float)(a[0] * b3 + a[1] * b2 - a[2] * b1 + a[3] * b0);
}

// ---- voxel keys of anchors at their level, from their means (re-voxelisation)
__global__ __launch_bounds__(256) void k_map_anchor_keys(MapEps E, const float* __restrict__ means,
                                                         const int32_t* __restrict__ level, int64_t n,
                                                         unsigned long long* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int lev = level[i];
  if (lev < 0 || lev > 4) {
    keys[i] = MP_EMPTY;
    return;
  }
  const double e = E.eps[lev];
  keys[i] = pack_key(lev, (long long)floor((double)means[i] / e), (long long)floor((double)means[n + i] / e),
                     (long long)floor((double)means[2 * n + i] / e));
}

// an anchor survives the re-voxelisation if it is the first (lowest index) of its voxel
__global__ __launch_bounds__(256) void k_map_keep(const uint32_t* __restrict__ anchor,
                                                  const uint32_t* __restrict__ created, int64_t n,
                                                  uint8_t* __restrict__ keep) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t a = anchor[i];
  keep[i] = a != 0xffffffffu && created[a] == (uint32_t)i;
}

__global__ void k_map_zero(uint32_t* __restrict__ p) {
  if (threadIdx.x == 0) *p = 0u;
}

// ---------------------------------------------------------------- host side
namespace {
size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
struct MapLayout {
  size_t slot, counts, offsets, part, tot, keys, created, zero, total;
};
MapLayout map_layout(int64_t n) {
  const int64_t nb = (n + 255) / 256 + 1;
  MapLayout L;
  size_t off = 0;
  L.slot = off; off = al256(off + 4 * (size_t)std::max<int64_t>(n, 1));
  L.counts = off; off = al256(off + 4 * (size_t)nb);
  L.offsets = off; off = al256(off + 4 * (size_t)nb);
  L.part = off; off = al256(off + 16 * (size_t)(kgs_scan_tiles(nb) + 1));
  L.tot = off; off = al256(off + 16);
  L.keys = off; off = al256(off + 8 * (size_t)std::max<int64_t>(n, 1));
  L.created = off; off = al256(off + 4 * (size_t)std::max<int64_t>(n, 1));
  L.zero = off; off = al256(off + 16);
  L.total = off;
  return L;
}
}  // namespace

size_t kgs_map_ws_bytes(int64_t n) { return map_layout(n).total; }
size_t kgs_map_slot_bytes() { return sizeof(MapSlot); }

void kgs_launch_map_clear(void* table, uint64_t cap, hipStream_t st) {
  const unsigned g = (unsigned)std::min<uint64_t>((cap + 255) / 256, 4096);
  hipLaunchKernelGGL(k_map_clear, dim3(std::max(g, 1u)), dim3(256), 0, st, (MapSlot*)table, cap);
}

kgs_status kgs_launch_map_insert(void* table, uint64_t cap, const unsigned long long* keys, int64_t n,
                                 const uint32_t* n_in, uint32_t* anchor, uint32_t* created, uint32_t* n_out,
                                 uint32_t* status, char* ws, hipStream_t st) {
  const MapLayout L = map_layout(n);
  uint32_t* cand_slot = (uint32_t*)(ws + L.slot);
  uint32_t* counts = (uint32_t*)(ws + L.counts);
  uint32_t* offsets = (uint32_t*)(ws + L.offsets);
  unsigned long long* tot = (unsigned long long*)(ws + L.tot);
  const int64_t nb = std::max<int64_t>((n + 255) / 256, 1);
  MapSlot* t = (MapSlot*)table;
  hipLaunchKernelGGL(k_map_probe, dim3((unsigned)nb), dim3(256), 0, st, t, cap - 1, keys, n, cand_slot, status);
  hipLaunchKernelGGL(k_map_count, dim3((unsigned)nb), dim3(256), 0, st, (const MapSlot*)t, (const uint32_t*)cand_slot,
                     n, counts);
  kgs_launch_scan(counts, offsets, nb, 1, 0xffffffffull, 0xffffffffull, (unsigned long long*)(ws + L.part), tot, st);
  hipLaunchKernelGGL(k_map_assign, dim3((unsigned)nb), dim3(256), 0, st, t, (const uint32_t*)cand_slot, n,
                     (const uint32_t*)offsets, (const unsigned long long*)tot, n_in, created, n_out);
  if (anchor)
    hipLaunchKernelGGL(k_map_lookup, dim3((unsigned)nb), dim3(256), 0, st, (const MapSlot*)t,
                       (const uint32_t*)cand_slot, n, anchor);
  return kgs_check_launch();
}

kgs_status kgs_launch_map_voxel_keys(const int32_t* level, const int32_t* vox, int64_t n, unsigned long long* keys,
                                     hipStream_t st) {
  if (n == 0) return KGS_OK;
  hipLaunchKernelGGL(k_map_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, level, vox, n, keys);
  return kgs_check_launch();
}

kgs_status kgs_launch_map_spawn(const uint32_t* created, const uint32_t* n_in, const uint32_t* n_out,
                                const int32_t* level, const int32_t* vox, const float* color, int64_t n_cand,
                                const kgs_gaussians_out* g, uint32_t* status, hipStream_t st) {
  if (n_cand == 0) return KGS_OK;
  hipLaunchKernelGGL(k_map_spawn, dim3((unsigned)((n_cand + 255) / 256)), dim3(256), 0, st, map_eps(), created, n_in,
                     n_out, level, vox, color, *g, status);
  return kgs_check_launch();
}

kgs_status kgs_launch_map_densify(const kgs_gaussians* g, const uint8_t* decision, const double centre[3],
                                  int64_t cap, int32_t* level, int32_t* vox, float* point, uint32_t* source,
                                  uint32_t* count, char* ws, hipStream_t st) {
  const int64_t n = g->n;
  const MapLayout L = map_layout(n);
  uint32_t* counts = (uint32_t*)(ws + L.counts);
  uint32_t* offsets = (uint32_t*)(ws + L.offsets);
  unsigned long long* tot = (unsigned long long*)(ws + L.tot);
  const int64_t nb = std::max<int64_t>((n + 255) / 256, 1);
  hipLaunchKernelGGL(k_densify_count, dim3((unsigned)nb), dim3(256), 0, st, decision, n, counts);
  kgs_launch_scan(counts, offsets, nb, 1, 0xffffffffull, 0xffffffffull, (unsigned long long*)(ws + L.part), tot, st);
  hipLaunchKernelGGL(k_densify_emit, dim3((unsigned)nb), dim3(256), 0, st, map_eps(), *g, decision, centre[0],
                     centre[1], centre[2], (const uint32_t*)offsets, (const unsigned long long*)tot, cap, level, vox,
                     point, source, count);
  return kgs_check_launch();
}

kgs_status kgs_launch_map_compact(const kgs_gaussians* g, const uint8_t* decision, const uint32_t* keep_map,
                                  const kgs_gaussians_out* out, hipStream_t st) {
  if (g->n == 0) return KGS_OK;
  hipLaunchKernelGGL(k_map_compact, dim3((unsigned)((g->n + 255) / 256)), dim3(256), 0, st, *g, decision, keep_map,
                     *out);
  return kgs_check_launch();
}

kgs_status kgs_launch_map_align(float* means, float* quats, int64_t n, const int32_t* keyframe_of,
                                const kgs_camera* old_pose, const kgs_camera* new_pose, int n_kf, hipStream_t st) {
  if (n == 0) return KGS_OK;
  hipLaunchKernelGGL(k_map_align, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, means, quats, n, keyframe_of,
                     old_pose, new_pose, n_kf);
  return kgs_check_launch();
}

kgs_status kgs_launch_map_revoxelize(const float* means, const int32_t* level, int64_t n, void* table, uint64_t cap,
                                     uint8_t* keep, uint32_t* anchor, uint32_t* n_keep, uint32_t* status, char* ws,
                                     hipStream_t st) {
  const MapLayout L = map_layout(n);
  unsigned long long* keys = (unsigned long long*)(ws + L.keys);
  uint32_t* created = (uint32_t*)(ws + L.created);
  uint32_t* zero = (uint32_t*)(ws + L.zero);
  kgs_launch_map_clear(table, cap, st);
  hipLaunchKernelGGL(k_map_zero, dim3(1), dim3(64), 0, st, zero);
  if (n == 0) {
    hipLaunchKernelGGL(k_map_zero, dim3(1), dim3(64), 0, st, n_keep);
    return kgs_check_launch();
  }
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_map_anchor_keys, dim3(nb), dim3(256), 0, st, map_eps(), means, level, n, keys);
  const kgs_status s = kgs_launch_map_insert(table, cap, keys, n, zero, anchor, created, n_keep, status, ws, st);
  if (s != KGS_OK) return s;
  hipLaunchKernelGGL(k_map_keep, dim3(nb), dim3(256), 0, st, (const uint32_t*)anchor, (const uint32_t*)created, n,
                     keep);
  return kgs_check_launch();
}
