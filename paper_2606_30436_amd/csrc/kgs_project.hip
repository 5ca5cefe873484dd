// Projection: pose application, per-(view, Gaussian) visibility and tile
// counts, the block-offset scan, and the compact record emission.
//
// Layout: one thread per Gaussian, looping over the views of the call, so the
// 44 bytes of geometry of a Gaussian are read once per call (not once per
// view); cameras are read with uniform addresses (scalar loads).  Records are
// compacted in (view, Gaussian index) order by a deterministic two-pass scan
// (per-block counts, then block bases), so slot and pair order never depend on
// scheduling.
#include "kgs_internal.h"

// ---------------------------------------------------------------- camera setup
// T' = Exp(xi) T with the closed-form SE(3) exponential:
//   R_phi = I + (sin t / t) K + ((1 - cos t) / t^2) K^2,
//   V     = I + ((1 - cos t) / t^2) K + ((t - sin t) / t^3) K^2,   K = [phi]x,
//   R' = R_phi R,  t' = R_phi t + V rho.
// Also the SE(3) left Jacobian [[J, Q], [0, J]] (J = V) used to turn the
// left-perturbation gradient into d/dxi.
namespace {
struct M3 {
  double a[9];
};
__device__ M3 m3_mul(const M3& A, const M3& B) {
  M3 C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.a[i * 3 + j] = A.a[i * 3] * B.a[j] + A.a[i * 3 + 1] * B.a[3 + j] + A.a[i * 3 + 2] * B.a[6 + j];
  return C;
}
__device__ M3 m3_skew(double x, double y, double z) {
  M3 K = {{0, -z, y, z, 0, -x, -y, x, 0}};
  return K;
}
__device__ M3 m3_lin(double a, const M3& A, double b, const M3& B) {
  M3 C;
  for (int k = 0; k < 9; ++k) C.a[k] = a * A.a[k] + b * B.a[k];
  return C;
}
}  // namespace

__global__ void k_cam_setup(const kgs_camera* __restrict__ cams, const float* __restrict__ xi, int V, float guard,
                            CamDev* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const kgs_camera c = cams[v];
  double r[3] = {0, 0, 0}, p[3] = {0, 0, 0};
  if (xi) {
    for (int k = 0; k < 3; ++k) { r[k] = xi[v * 6 + k]; p[k] = xi[v * 6 + 3 + k]; }
  }
  const double th2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2], th = sqrt(th2);
  double A, B, Cc, c2, c3;
  if (th < 1e-3) {
    A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    Cc = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    c2 = 1.0 / 24.0 - th2 / 720.0 + th2 * th2 / 40320.0;
    c3 = 1.0 / 120.0 - th2 / 2520.0 + th2 * th2 / 120960.0;
  } else {
    const double s = sin(th), co = cos(th);
    A = s / th;
    B = (1.0 - co) / th2;
    Cc = (th - s) / (th2 * th);
    c2 = (th2 + 2.0 * co - 2.0) / (2.0 * th2 * th2);
    c3 = (2.0 * th - 3.0 * s + th * co) / (2.0 * th2 * th2 * th);
  }
  const M3 I = {{1, 0, 0, 0, 1, 0, 0, 0, 1}};
  const M3 K = m3_skew(p[0], p[1], p[2]);
  const M3 K2 = m3_mul(K, K);
  M3 Rphi = m3_lin(1.0, I, A, K);
  Rphi = m3_lin(1.0, Rphi, B, K2);
  M3 Vm = m3_lin(1.0, I, B, K);
  Vm = m3_lin(1.0, Vm, Cc, K2);
  M3 R0;
  for (int k = 0; k < 9; ++k) R0.a[k] = c.R[k];
  const M3 Rp = m3_mul(Rphi, R0);
  double tp[3];
  for (int i = 0; i < 3; ++i)
    tp[i] = Rphi.a[i * 3] * c.t[0] + Rphi.a[i * 3 + 1] * c.t[1] + Rphi.a[i * 3 + 2] * c.t[2] +
            Vm.a[i * 3] * r[0] + Vm.a[i * 3 + 1] * r[1] + Vm.a[i * 3 + 2] * r[2];
  CamDev d;
  for (int k = 0; k < 9; ++k) d.R[k] = (float)Rp.a[k];
  for (int j = 0; j < 3; ++j) {
    const double cj = -(Rp.a[j] * tp[0] + Rp.a[3 + j] * tp[1] + Rp.a[6 + j] * tp[2]);
    d.ctr[j] = (float)cj;
    d.ctr_lo[j] = (float)(cj - (double)d.ctr[j]);
  }
  for (int k = 0; k < 9; ++k) d.Rd[k] = Rp.a[k];
  for (int i = 0; i < 3; ++i) d.td[i] = tp[i];
  d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
  const double hx = 0.5 * c.width / c.fx, hy = 0.5 * c.height / c.fy;
  const double mx = (0.5 * c.width - c.cx) / c.fx, my = (0.5 * c.height - c.cy) / c.fy;
  d.lox = (float)(mx - guard * hx); d.hix = (float)(mx + guard * hx);
  d.loy = (float)(my - guard * hy); d.hiy = (float)(my + guard * hy);
  d.W = c.width; d.H = c.height;
  d.pad0 = d.pad1 = 0;
  // Q(rho, phi) of the SE(3) left Jacobian
  const M3 P = K, Rr = m3_skew(r[0], r[1], r[2]);
  const M3 PR = m3_mul(P, Rr), RP = m3_mul(Rr, P), PRP = m3_mul(PR, P);
  const M3 PPR = m3_mul(P, PR), RPP = m3_mul(RP, P), PRPP = m3_mul(PRP, P), PPRP = m3_mul(P, PRP);
  M3 Q;
  for (int k = 0; k < 9; ++k)
    Q.a[k] = 0.5 * Rr.a[k] + Cc * (PR.a[k] + RP.a[k] + PRP.a[k]) + c2 * (PPR.a[k] + RPP.a[k] - 3.0 * PRP.a[k]) +
             c3 * (PRPP.a[k] + PPRP.a[k]);
  for (int k = 0; k < 36; ++k) d.Jl[k] = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      d.Jl[i * 6 + j] = Vm.a[i * 3 + j];
      d.Jl[(i + 3) * 6 + (j + 3)] = Vm.a[i * 3 + j];
      d.Jl[i * 6 + (j + 3)] = Q.a[i * 3 + j];
    }
  out[v] = d;
}

// ---------------------------------------------------------------- counting
struct ProjParams {
  float alpha_min, log_alpha_min, near_z, far_z, eps2d, rect_margin;
  int tile_w, tile_h, tiles_x, tiles_y;
  uint32_t depth_lo;        // record depth-sort key layout
  int depth_bits, key32;
};

__global__ __launch_bounds__(KGS_BLOCK) void k_count(kgs_gaussians g, const CamDev* __restrict__ cams, int V,
                                                     ProjParams P, uint32_t* __restrict__ vis,
                                                     uint32_t* __restrict__ blk_cnt, int64_t nb,
                                                     uint32_t* __restrict__ status) {
  __shared__ uint32_t sc[KGS_MAX_VIEWS][4], st[KGS_MAX_VIEWS][4];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * KGS_BLOCK + threadIdx.x;
  const bool valid = i < g.n;
  GaussLocal G;
  bool bad = false;
  G.ok = false;
  if (valid) load_gaussian(g, i, P.alpha_min, G, bad);
  if (bad) atomicOr(status, KGS_FLAG_NONFINITE);
  for (int v = 0; v < V; ++v) {
    uint32_t tiles = 0;
    if (G.ok) {
      ProjCore p;
      if (project_core(cams[v], G.mu, G.Rq, G.s, G.o, P.near_z, P.far_z, P.eps2d, P.rect_margin, P.log_alpha_min, P.tile_w,
                       P.tile_h, P.tiles_x, P.tiles_y, p))
        tiles = (uint32_t)((p.x1 - p.x0) * (p.y1 - p.y0));
    }
    if (valid) vis[(int64_t)v * g.n + i] = tiles;
    const uint32_t c = (uint32_t)__popcll(ballot64(tiles > 0));
    const uint32_t t = wave_sum(tiles);
    if (l == 0) { sc[v][w] = c; st[v][w] = t; }
  }
  __syncthreads();
  for (int v = threadIdx.x; v < V; v += KGS_BLOCK) {
    const int64_t e = ((int64_t)v * nb + blockIdx.x) * 2;
    blk_cnt[e] = sc[v][0] + sc[v][1] + sc[v][2] + sc[v][3];
    blk_cnt[e + 1] = st[v][0] + st[v][1] + st[v][2] + st[v][3];
  }
}

// ---------------------------------------------------------------- block scan
// The (visible, tiles) pairs of all (view, block) entries are scanned in
// (view, block) order by the device-wide scan (bases saturate at the
// capacities); this sets the record and pair totals, or on overflow zero
// totals and a status bit, so that every later stage sees nothing.
__global__ void k_scan_finish(const unsigned long long* __restrict__ totals, uint64_t slot_cap, uint64_t pair_cap,
                              uint32_t* __restrict__ counters) {
  const unsigned long long ta = totals[0], tb = totals[1];
  uint32_t f = 0;
  if (ta > slot_cap) f |= KGS_FLAG_SLOT_OVERFLOW;
  if (tb > pair_cap) f |= KGS_FLAG_PAIR_OVERFLOW;
  counters[0] = f ? 0u : (uint32_t)ta;
  counters[1] = f ? 0u : (uint32_t)tb;
  if (f) atomicOr(&counters[2], f);
}

// ---------------------------------------------------------------- emission
// Pixel bounds [lo, hi] of the rectangle packed as two int16 (clamped; the
// image is narrower than 32767 pixels, so clamping keeps every overlap test).
__device__ __forceinline__ float pack_bounds(int lo, int hi) {
  lo = min(max(lo, -32768), 32767);
  hi = min(max(hi, -32768), 32767);
  return __uint_as_float(((uint32_t)lo & 0xffffu) | ((uint32_t)hi << 16));
}

template <int DEG>
__global__ __launch_bounds__(KGS_BLOCK) void k_emit(kgs_gaussians g, const CamDev* __restrict__ cams, int V,
                                                    ProjParams P, uint32_t* __restrict__ vis,
                                                    const uint32_t* __restrict__ blk_base, int64_t nb,
                                                    uint64_t slot_cap,
                                                    float4* __restrict__ slot_rec, uint32_t* __restrict__ slot_gid,
                                                    int4* __restrict__ slot_pix, uint32_t* __restrict__ slot_ntiles,
                                                    void* __restrict__ slot_keys, uint4* __restrict__ emit_desc,
                                                    int tile_bits) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  // visible lanes of each wave, per view: a slot's index is the (view, block)
  // base plus the visible lanes before it (one barrier for all views)
  __shared__ uint32_t wcnt[KGS_MAX_VIEWS][4];
  const int w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * KGS_BLOCK + threadIdx.x;
  const bool valid = i < g.n;
  // the tile counts of views v0 .. v0 + 7, loaded together; those of the first
  // eight views (all of them in most calls) stay in registers for the emission
  auto load8 = [&](int v0, uint32_t (&t)[8]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) t[j] = (valid && v0 + j < V) ? vis[(int64_t)(v0 + j) * g.n + i] : 0u;
  };
  uint32_t t8[8];
  for (int v0 = 0; v0 < V; v0 += 8) {
    uint32_t t[8];
    load8(v0, t);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (v0 + j < V) {
        const uint64_t bal = ballot64(t[j] > 0u);
        if ((threadIdx.x & 63) == 0) wcnt[v0 + j][w] = (uint32_t)__popcll(bal);
      }
      if (v0 == 0) t8[j] = t[j];
    }
  }
  __syncthreads();
  GaussLocal G;
  bool bad = false;
  G.ok = false;
  if (valid) load_gaussian(g, i, P.alpha_min, G, bad);
  const float hl2e = 0.5f * 1.4426950408889634f;
  for (int v0 = 0; v0 < V; v0 += 8) {
    uint32_t tg[8];
    if (v0 == 0) {
#pragma unroll
      for (int j = 0; j < 8; ++j) tg[j] = t8[j];
    } else {
      load8(v0, tg);
    }
    const int nv = min(8, V - v0);
    for (int j = 0; j < nv; ++j) {
      const int v = v0 + j;
      // view v's count is tg[0]: the group's counts shift down one register per view
      const uint32_t tiles = tg[0];
#pragma unroll
      for (int k = 0; k < 7; ++k) tg[k] = tg[k + 1];
      const uint64_t bal = ballot64(tiles > 0u);
      if (tiles == 0u) continue;
      uint32_t below = mask_lt_count(bal);
      for (int k = 0; k < w; ++k) below += wcnt[v][k];
      const uint64_t s = (uint64_t)blk_base[((int64_t)v * nb + blockIdx.x) * 2] + below;
      // from here on vis[v][i] names the slot (index + 1), for the backward gather
      vis[(int64_t)v * g.n + i] = s < slot_cap ? (uint32_t)(s + 1) : 0u;
      // past the slot capacity nothing is written; the pair capacity needs no
      // check here: an overflow of either zeroes every count after the scan, and
      // otherwise every slot's pairs fit
      if (s >= slot_cap) continue;
      const CamDev& c = cams[v];
      ProjCore p;
      const bool vis_ok = G.ok && project_core(c, G.mu, G.Rq, G.s, G.o, P.near_z, P.far_z, P.eps2d, P.rect_margin,
                                               P.log_alpha_min, P.tile_w, P.tile_h, P.tiles_x, P.tiles_y, p);
      float4 r0, r1, r2;
      int4 pix;
      uint4 desc;   // the pair emission's view of the record: key base, first tile, rectangle width, tile count
      if (vis_ok) {
        r0 = make_float4(p.rmx, p.rmy, -hl2e * p.Pc, p.kc);
        r1 = make_float4(-hl2e * p.Ec, __log2f(G.o), p.tz, pack_bounds(p.fxi - p.rx, p.fxi + p.rx));
        pix = make_int4(p.fxi, p.fyi, p.rx, p.ry);
        desc = make_uint4((uint32_t)v << tile_bits, (uint32_t)p.x0 | ((uint32_t)p.y0 << 16), (uint32_t)(p.x1 - p.x0),
                          tiles);
        // the colour from the view direction (Gaussian mean minus camera centre),
        // so the record is written in three whole float4 stores; the SH
        // coefficients are read per visible view (the later views' reads hit
        // the cache), which overlaps their latency with the projections at the
        // cost of registers (two waves per SIMD: faster than a separate colour
        // pass at four)
        float dv[3];
        cam_offset(c, G.mu, dv);
        const float inv = 1.0f / sqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        float Y[16];
        sh_basis(DEG, dv[0] * inv, dv[1] * inv, dv[2] * inv, Y);
        float col[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          float acc = 0.5f;
#pragma unroll
          for (int k = 0; k < K; ++k) acc += Y[k] * g.sh[(int64_t)(k * 3 + ch) * g.n + i];
          col[ch] = fmaxf(acc, 0.0f);
        }
        r2 = make_float4(col[0], col[1], col[2], pack_bounds(p.fyi - p.ry, p.fyi + p.ry));
      } else {
        // the counting pass saw this Gaussian visible but the re-projection does
        // not: write a record that never blends and an empty rectangle
        r0 = make_float4(0.f, 0.f, 0.f, 0.f);
        r1 = make_float4(0.f, -INFINITY, 1.0f, pack_bounds(32767, -32768));
        r2 = make_float4(0.f, 0.f, 0.f, pack_bounds(32767, -32768));
        pix = make_int4(-(1 << 30), -(1 << 30), 0, 0);
        // its pairs (as many as the count gave) go down the first tile column; they never blend
        desc = make_uint4((uint32_t)v << tile_bits, 0u, 1u, tiles);
      }
      slot_rec[s * 4 + 0] = r0;
      slot_rec[s * 4 + 1] = r1;
      slot_rec[s * 4 + 2] = r2;
      slot_gid[s] = (uint32_t)i;
      slot_pix[s] = pix;
      slot_ntiles[s] = tiles;   // dense, for the group sums' gather in depth order
      emit_desc[s] = desc;      // also the slot's view (above the tile bits) and tile count for the later steps
      // the record's (view, depth) key for the depth sort, from its depth r1.z
      const uint32_t db = __float_as_uint(r1.z);
      const uint32_t dmax = P.depth_bits >= 32 ? 0xffffffffu : (1u << P.depth_bits) - 1u;
      const uint64_t key = ((uint64_t)v << P.depth_bits) | (db > P.depth_lo ? min(db - P.depth_lo, dmax) : 0u);
      if (P.key32)
        reinterpret_cast<uint32_t*>(slot_keys)[s] = (uint32_t)key;
      else
        reinterpret_cast<uint64_t*>(slot_keys)[s] = key;
      // the sort's values start as the record indices themselves (its first pass generates them)
    }
  }
}

// ---------------------------------------------------------------- host side
kgs_status kgs_launch_project(kgs_ctx* ctx, const kgs_gaussians* g, const kgs_camera* cams, int V,
                              const float* pose_xi, hipStream_t st) {
  const kgs_config& cfg = ctx->cfg;
  hipLaunchKernelGGL(k_cam_setup, dim3(1), dim3(64), 0, st, cams, pose_xi, V, cfg.guard, ctx->cams);
  ProjParams P;
  P.alpha_min = cfg.alpha_min;
  P.log_alpha_min = logf(cfg.alpha_min);
  P.near_z = cfg.near_z;
  P.far_z = cfg.far_z;
  P.eps2d = cfg.eps2d;
  P.rect_margin = cfg.rect_margin;
  P.tile_w = cfg.tile_w;
  P.tile_h = cfg.tile_h;
  P.tiles_x = ctx->tiles_x;
  P.tiles_y = ctx->tiles_y;
  const SlotKeyLayout KL = slot_key_layout(cfg.near_z, cfg.far_z, V);
  P.depth_lo = KL.depth_lo;
  P.depth_bits = KL.depth_bits;
  P.key32 = KL.key32() ? 1 : 0;
  const int64_t nb = (g->n + KGS_BLOCK - 1) / KGS_BLOCK;
  if (nb > 0)
    hipLaunchKernelGGL(k_count, dim3((unsigned)nb), dim3(KGS_BLOCK), 0, st, *g, (const CamDev*)ctx->cams, V, P,
                       ctx->vis, ctx->blk_cnt, nb, ctx->counters + 2);
  kgs_launch_scan(ctx->blk_cnt, ctx->blk_base, (int64_t)V * nb, 2, (unsigned long long)cfg.slot_capacity,
                  (unsigned long long)cfg.pair_capacity, ctx->scan_part, ctx->scan_totals, st);
  hipLaunchKernelGGL(k_scan_finish, dim3(1), dim3(1), 0, st, (const unsigned long long*)ctx->scan_totals,
                     (uint64_t)cfg.slot_capacity, (uint64_t)cfg.pair_capacity, ctx->counters);
  if (nb > 0) {
#define KGS_EMIT(D)                                                                                              \
  hipLaunchKernelGGL(k_emit<D>, dim3((unsigned)nb), dim3(KGS_BLOCK), 0, st, *g, (const CamDev*)ctx->cams, V, P,   \
                     ctx->vis, (const uint32_t*)ctx->blk_base, nb, (uint64_t)cfg.slot_capacity,                \
                     ctx->slot_rec, ctx->slot_gid, ctx->slot_pix, ctx->slot_ntiles, (void*)ctx->slot_keys[0],  \
                     ctx->emit_desc, kgs_tile_bits(ctx->n_tiles))
    switch (g->sh_degree) {
      case 0: KGS_EMIT(0); break;
      case 1: KGS_EMIT(1); break;
      case 2: KGS_EMIT(2); break;
      default: KGS_EMIT(3); break;
    }
#undef KGS_EMIT
  }
  ctx->slot_keys_ready = 1;
  return kgs_check_launch();
}
