// Chunk scores, their global merge and the densify / prune decision
// (appendix, "Densification Score" and "Pruning Score"; Sec. 3.3 global rules).
// Per-Gaussian streams over [N] arrays: HBM bound.  L, S_p and the min / max
// over the active set are FP64 so the prune threshold test is decided far
// below any FP32 rounding.
#include <mutex>

#include "kgs_internal.h"

__global__ __launch_bounds__(KGS_BLOCK) void k_chunk_scores(int64_t n, int n_views, double tau_d,
                                                            const uint32_t* __restrict__ kappa_sum,
                                                            const uint32_t* __restrict__ omega_sum,
                                                            const double* __restrict__ gamma_sum,
                                                            uint8_t* __restrict__ densify,
                                                            double* __restrict__ mm_partial) {
  __shared__ double smin[4], smax[4];
  const int64_t i = (int64_t)blockIdx.x * KGS_BLOCK + threadIdx.x;
  double lo = INFINITY, hi = -INFINITY;
  if (i < n) {
    // S_d^(i,c) = (1/|V_c|) sum_v kappa_v(i);  S_d(i) |= S_d^(i,c) > tau_d.  The quotient is
    // taken in FP64 (exact for kappa = tau_d |V_c|, where a float reciprocal of |V_c| rounds
    // 5 |V_c| / |V_c| up past 5 for |V_c| = 15, 30, 60, 63), so the strict test is the oracle's.
    if (densify && (double)kappa_sum[i] / (double)n_views > tau_d) densify[i] = 1;
    if (omega_sum[i] > 0) {
      const double L = log1p(gamma_sum[i]);
      lo = L;
      hi = L;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { smin[w] = lo; smax[w] = hi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    mm_partial[2 * blockIdx.x] = fmin(fmin(smin[0], smin[1]), fmin(smin[2], smin[3]));
    mm_partial[2 * blockIdx.x + 1] = fmax(fmax(smax[0], smax[1]), fmax(smax[2], smax[3]));
  }
}

__global__ __launch_bounds__(1024) void k_minmax_final(int64_t nb, double* __restrict__ mm) {
  __shared__ double smin[16], smax[16];
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t b = threadIdx.x; b < nb; b += 1024) {
    lo = fmin(lo, mm[2 * b]);
    hi = fmax(hi, mm[2 * b + 1]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { smin[w] = lo; smax[w] = hi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 16; ++k) { lo = fmin(lo, smin[k]); hi = fmax(hi, smax[k]); }
    mm[2 * nb] = lo;
    mm[2 * nb + 1] = hi;
  }
}

// S_p^(i,c) = (L - min_A L) / (max_A L - min_A L) on the active set A;
// S_p(i) = max_c S_p^(i,c).
__global__ __launch_bounds__(KGS_BLOCK) void k_chunk_prune(int64_t n, int64_t nb, uint32_t* __restrict__ kappa_sum,
                                                           uint32_t* __restrict__ omega_sum,
                                                           double* __restrict__ gamma_sum,
                                                           const double* __restrict__ mm,
                                                           double* __restrict__ prune_score, int reset) {
  const int64_t i = (int64_t)blockIdx.x * KGS_BLOCK + threadIdx.x;
  if (i >= n) return;
  const double lo = mm[2 * nb], hi = mm[2 * nb + 1];
  double sp = 0.0;
  if (omega_sum[i] > 0 && hi > lo) sp = (log1p(gamma_sum[i]) - lo) / (hi - lo);
  if (sp > prune_score[i]) prune_score[i] = sp;
  if (reset) {
    kappa_sum[i] = 0u;
    omega_sum[i] = 0u;
    gamma_sum[i] = 0.0;
  }
}

__global__ __launch_bounds__(KGS_BLOCK) void k_decide(int64_t n, double tau_p, const uint8_t* __restrict__ densify,
                                                      const double* __restrict__ prune_score,
                                                      uint8_t* __restrict__ decision,
                                                      uint32_t* __restrict__ keep_partial) {
  const int64_t i = (int64_t)blockIdx.x * KGS_BLOCK + threadIdx.x;
  uint8_t d = KGS_KEEP;
  bool keep = false;
  if (i < n) {
    if (prune_score[i] > tau_p) d = KGS_PRUNE;
    else if (densify[i]) d = KGS_DENSIFY;
    decision[i] = d;
    keep = d != KGS_PRUNE;
  }
  __shared__ uint32_t sh[4];
  const uint32_t c = (uint32_t)__popcll(ballot64(keep));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0 && keep_partial) keep_partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ __launch_bounds__(1024) void k_keep_scan(int64_t nb, uint32_t* __restrict__ part,
                                                    uint32_t* __restrict__ n_keep) {
  __shared__ uint32_t sh[16];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t lo = tid * per, hi = min(nb, lo + per);
  uint32_t a = 0;
  for (int64_t b = lo; b < hi; ++b) a += part[b];
  const uint32_t ia = wave_inclusive_scan(a);
  if (l == 63) sh[w] = ia;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int k = 0; k < 16; ++k) {
    if (k < w) off += sh[k];
    tot += sh[k];
  }
  uint32_t r = off + ia - a;
  for (int64_t b = lo; b < hi; ++b) {
    const uint32_t c = part[b];
    part[b] = r;
    r += c;
  }
  if (tid == 0 && n_keep) *n_keep = tot;
}

__global__ __launch_bounds__(KGS_BLOCK) void k_keep_map(int64_t n, const uint8_t* __restrict__ decision,
                                                        const uint32_t* __restrict__ base,
                                                        uint32_t* __restrict__ keep_map) {
  __shared__ uint32_t sh[16];
  const int64_t i = (int64_t)blockIdx.x * KGS_BLOCK + threadIdx.x;
  const uint32_t keep = (i < n && decision[i] != KGS_PRUNE) ? 1u : 0u;
  uint32_t ea, eb, ta, tb;
  block_scan2(keep, 0u, sh, ea, eb, ta, tb);
  if (i < n) keep_map[i] = base[blockIdx.x] + ea;
}

// The chunk close with its min / max partials in mm (2 nb + 2 doubles, nb = blocks of 256 over n).  Every
// partial is written before it is read, so mm needs no clearing.
static kgs_status launch_accumulate_mm(const kgs_view_stats* s, int64_t n, int V, const kgs_lifecycle_state* state,
                                       float tau_d, int reset, double* mm, hipStream_t st) {
  const int64_t nb = (n + KGS_BLOCK - 1) / KGS_BLOCK;
  if (nb == 0) return KGS_OK;
  hipLaunchKernelGGL(k_chunk_scores, dim3((unsigned)nb), dim3(KGS_BLOCK), 0, st, n, V, (double)tau_d,
                     (const uint32_t*)s->kappa_sum, (const uint32_t*)s->omega_sum, (const double*)s->gamma_sum,
                     state->densify, mm);
  hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(1024), 0, st, nb, mm);
  hipLaunchKernelGGL(k_chunk_prune, dim3((unsigned)nb), dim3(KGS_BLOCK), 0, st, n, nb, s->kappa_sum, s->omega_sum,
                     s->gamma_sum, (const double*)mm, state->prune_score, reset);
  return kgs_check_launch();
}

kgs_status kgs_launch_accumulate(kgs_ctx* ctx, const kgs_view_stats* s, int64_t n, int V,
                                 const kgs_lifecycle_state* state, float tau_d, int reset, hipStream_t st) {
  return launch_accumulate_mm(s, n, V, state, tau_d, reset, ctx->mm_partial, st);
}

// ------------------------------------------------------------------------------------------------
// The chunk close for callers that cannot allocate (graph capture, serving loops): its min / max
// partials live in a library-owned static device array instead of a workspace.  Each GPU holds its
// own copy for the life of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the array's name is a host-side stand-in there).
#define KGS_STATIC_MAX_BLOCKS 65535
#define KGS_STATIC_MAX_DEVICES 64
static __device__ __align__(256) double scratch[2 * KGS_STATIC_MAX_BLOCKS + 2];

static std::mutex g_scratch_mu;
static double* g_scratch_dev[KGS_STATIC_MAX_DEVICES];

// Device address of this GPU's copy of `scratch`, looked up once per device with it current.
static kgs_status static_scratch(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return KGS_ERR_HIP;
  if (dev < 0 || dev >= KGS_STATIC_MAX_DEVICES) return KGS_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return KGS_ERR_HIP;
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return KGS_OK;
}

extern "C" kgs_status kgs_accumulate_stats_static(const kgs_view_stats* stats, int64_t n, int32_t n_views,
                                                  const kgs_lifecycle_state* state, float tau_d, int32_t reset,
                                                  void* stream) {
  if (!stats || !state || n < 0 || n > KGS_ACCUMULATE_STATIC_MAX_N || n_views < 1) return KGS_ERR_INVALID_ARG;
  if (!stats->kappa_sum || !stats->omega_sum || !stats->gamma_sum || !state->densify || !state->prune_score)
    return KGS_ERR_INVALID_ARG;
  if (n == 0) return KGS_OK;
  double* mm = nullptr;
  const kgs_status e = static_scratch(&mm);
  if (e != KGS_OK) return e;
  return launch_accumulate_mm(stats, n, n_views, state, tau_d, reset, mm, (hipStream_t)stream);
}

kgs_status kgs_launch_decide(kgs_ctx* ctx, const kgs_lifecycle_state* state, int64_t n, double tau_p,
                             uint8_t* decision, uint32_t* keep_map, uint32_t* n_keep, hipStream_t st) {
  const int64_t nb = (n + KGS_BLOCK - 1) / KGS_BLOCK;
  if (nb == 0) return KGS_OK;
  const bool need_scan = keep_map || n_keep;
  hipLaunchKernelGGL(k_decide, dim3((unsigned)nb), dim3(KGS_BLOCK), 0, st, n, tau_p,
                     (const uint8_t*)state->densify, (const double*)state->prune_score, decision,
                     need_scan ? ctx->keep_partial : (uint32_t*)nullptr);
  if (need_scan) {
    hipLaunchKernelGGL(k_keep_scan, dim3(1), dim3(1024), 0, st, nb, ctx->keep_partial, n_keep);
    if (keep_map)
      hipLaunchKernelGGL(k_keep_map, dim3((unsigned)nb), dim3(KGS_BLOCK), 0, st, n, (const uint8_t*)decision,
                         (const uint32_t*)ctx->keep_partial, keep_map);
  }
  return kgs_check_launch();
}

// min / max of L = ln(1 + gamma) over the active set of a chunk, without
// touching any state; returns the device address of (min, max).
const double* kgs_launch_chunk_minmax(kgs_ctx* ctx, const kgs_view_stats* s, int64_t n, hipStream_t st) {
  const int64_t nb = (n + KGS_BLOCK - 1) / KGS_BLOCK;
  hipLaunchKernelGGL(k_chunk_scores, dim3((unsigned)nb), dim3(KGS_BLOCK), 0, st, n, 1, 0.0,
                     (const uint32_t*)s->kappa_sum, (const uint32_t*)s->omega_sum, (const double*)s->gamma_sum,
                     (uint8_t*)nullptr, ctx->mm_partial);
  hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(1024), 0, st, nb, ctx->mm_partial);
  return ctx->mm_partial + 2 * nb;
}
