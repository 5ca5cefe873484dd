// Backward of the projection: per Gaussian, the deterministic segmented sum of
// its pairs' gradients in every view, the chain rule to the 3D parameters and
// to the camera pose, and the per-view footprint statistics.
//
// One thread per Gaussian looping over the views of the call (same block
// structure as the emission kernel, so the block-local scan recovers each
// record's slot and pair offset without storing a map).  Views are summed in
// view order, so a batched call and a per-view loop produce identical bits.
// The pose gradient is accumulated as the left-perturbation gradient
// (rho, phi) of T' = Exp(delta) T', reduced per block into a [V][blocks][6]
// array, and turned into d/dxi by the SE(3) left Jacobian in a final pass.
#include "kgs_internal.h"

struct BwdParams {
  float alpha_min, log_alpha_min, near_z, eps2d, rect_margin;
  int tile_w, tile_h, tiles_x, tiles_y;
};

template <int DEG>
__global__ __launch_bounds__(KGS_BLOCK) void k_project_bwd(
    kgs_gaussians g, const CamDev* __restrict__ cams, int V, BwdParams P, const uint32_t* __restrict__ vis,
    const uint32_t* __restrict__ blk_base, int64_t nb, uint64_t slot_cap, uint64_t pair_cap,
    const float4* __restrict__ pair_grad, const float* __restrict__ view_loss, kgs_grads gr, kgs_view_stats st,
    float* __restrict__ pose_partial) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  __shared__ uint32_t scan_sh[16];
  __shared__ float pose_sh[4][6];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * KGS_BLOCK + threadIdx.x;
  const int64_t n = g.n;
  const bool valid = i < n;
  GaussLocal G;
  bool bad = false;
  G.ok = false;
  if (valid) load_gaussian(g, i, P.alpha_min, G, bad);
  float gm[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f}, glg = 0.f;
  float gsh[K][3];
#pragma unroll
  for (int k = 0; k < K; ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.f;
  uint32_t s_kap = 0, s_om = 0, s_vc = 0;
  double s_gam = 0.0;
  float s_gn = 0.f;
  int s_mr = 0;
  bool any = false;
  const float h = 0.5f * 1.4426950408889634f;
  const float LN2 = 0.69314718055994531f;
  for (int v = 0; v < V; ++v) {
    const uint32_t tiles = valid ? vis[(int64_t)v * n + i] : 0u;
    const uint32_t flag = tiles > 0 ? 1u : 0u;
    uint32_t ea, eb, ta, tb;
    block_scan2(flag, tiles, scan_sh, ea, eb, ta, tb);
    float pose[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (flag) {
      const int64_t e = ((int64_t)v * nb + blockIdx.x) * 2;
      const uint64_t s = (uint64_t)blk_base[e] + ea;
      const uint64_t po = (uint64_t)blk_base[e + 1] + eb;
      const CamDev& c = cams[v];
      ProjCore p;
      if (s < slot_cap && po + tiles <= pair_cap && G.ok &&
          project_core(c, G.mu, G.cw, G.o, P.near_z, P.eps2d, P.rect_margin, P.log_alpha_min, P.tile_w, P.tile_h,
                       P.tiles_x, P.tiles_y, p)) {
        // segmented sum of the record-space gradients of this record's pairs
        float r[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        uint32_t om = 0, kap = 0;
        for (uint32_t k = 0; k < tiles; ++k) {
          const float4 a = pair_grad[(po + k) * 3], b = pair_grad[(po + k) * 3 + 1],
                       cc = pair_grad[(po + k) * 3 + 2];
          r[0] += a.x; r[1] += a.y; r[2] += a.z; r[3] += a.w;
          r[4] += b.x; r[5] += b.y; r[6] += b.z; r[7] += b.w;
          r[8] += cc.x; r[9] += cc.y;
          om += __float_as_uint(cc.z);
          kap += __float_as_uint(cc.w);
        }
        any = true;
        // statistics of this view
        s_om += om;
        s_kap += kap;
        if (view_loss) s_gam += (double)view_loss[v] * (double)om;
        s_gn += sqrtf(r[0] * r[0] + r[1] * r[1]);
        s_vc += 1u;
        s_mr = max(s_mr, max(p.rx, p.ry));
        // record space -> conic (a, b, c) and opacity
        const float idet = 1.0f / p.det;
        const float ca = p.S11 * idet, cb = -p.S01 * idet, cc = p.S00 * idet;
        const float ga = -h * r[2], gb = -2.0f * h * r[3], gc = -h * r[4];
        glg += r[5] * (1.0f - G.o) / LN2;
        // dL/dSigma2D = -M G_M M, M the conic matrix, G_M = [[ga, gb/2], [gb/2, gc]]
        const float X00 = ga * ca + 0.5f * gb * cb, X01 = ga * cb + 0.5f * gb * cc;
        const float X10 = 0.5f * gb * ca + gc * cb, X11 = 0.5f * gb * cb + gc * cc;
        const float GS00 = -(ca * X00 + cb * X10);
        const float GS01 = -0.5f * ((ca * X01 + cb * X11) + (cb * X00 + cc * X10));
        const float GS11 = -(cb * X01 + cc * X11);
        // Y = G_S T (2x3); dL/dT = 2 Y Sigma_w; dL/dSigma_w = T^T Y
        float Y0[3], Y1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          Y0[k] = GS00 * p.T0[k] + GS01 * p.T1[k];
          Y1[k] = GS01 * p.T0[k] + GS11 * p.T1[k];
        }
        const float* cw = G.cw;  // xx xy xz yy yz zz
        float GT0[3], GT1[3];
        GT0[0] = 2.f * (Y0[0] * cw[0] + Y0[1] * cw[1] + Y0[2] * cw[2]);
        GT0[1] = 2.f * (Y0[0] * cw[1] + Y0[1] * cw[3] + Y0[2] * cw[4]);
        GT0[2] = 2.f * (Y0[0] * cw[2] + Y0[1] * cw[4] + Y0[2] * cw[5]);
        GT1[0] = 2.f * (Y1[0] * cw[0] + Y1[1] * cw[1] + Y1[2] * cw[2]);
        GT1[1] = 2.f * (Y1[0] * cw[1] + Y1[1] * cw[3] + Y1[2] * cw[4]);
        GT1[2] = 2.f * (Y1[0] * cw[2] + Y1[1] * cw[4] + Y1[2] * cw[5]);
        float GW[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) GW[a * 3 + b] = p.T0[a] * Y0[b] + p.T1[a] * Y1[b];
        // dL/dJ = dL/dT R'^T (full 2x3)
        float GJ0[3], GJ1[3];
#pragma unroll
        for (int cidx = 0; cidx < 3; ++cidx) {
          GJ0[cidx] = GT0[0] * c.R[cidx * 3] + GT0[1] * c.R[cidx * 3 + 1] + GT0[2] * c.R[cidx * 3 + 2];
          GJ1[cidx] = GT1[0] * c.R[cidx * 3] + GT1[1] * c.R[cidx * 3 + 1] + GT1[2] * c.R[cidx * 3 + 2];
        }
        // pose, rotation acting on J R':  A = J^T dL/dJ, g_phi += (A21 - A12, A02 - A20, A10 - A01)
        {
          const float A01 = p.J00 * GJ0[1], A02 = p.J00 * GJ0[2];
          const float A10 = p.J11 * GJ1[0], A12 = p.J11 * GJ1[2];
          const float A20 = p.J02 * GJ0[0] + p.J12 * GJ1[0], A21 = p.J02 * GJ0[1] + p.J12 * GJ1[1];
          pose[3] += A21 - A12;
          pose[4] += A02 - A20;
          pose[5] += A10 - A01;
        }
        // camera-frame point gradient
        const float tx = p.tx, ty = p.ty, tz = p.tz, iz = 1.0f / tz, iz2 = iz * iz;
        float gtx = r[0] * c.fx * iz, gty = r[1] * c.fy * iz;
        float gtz = -(r[0] * c.fx * tx + r[1] * c.fy * ty) * iz2 + r[9];
        gtz += GJ0[0] * (-c.fx * iz2) + GJ1[1] * (-c.fy * iz2);
        if (p.clx == 0) {
          gtx += GJ0[2] * (-c.fx * iz2);
          gtz += GJ0[2] * (2.0f * c.fx * tx * iz2 * iz);
        } else {
          gtz += GJ0[2] * (c.fx * p.ux * iz2);
        }
        if (p.cly == 0) {
          gty += GJ1[2] * (-c.fy * iz2);
          gtz += GJ1[2] * (2.0f * c.fy * ty * iz2 * iz);
        } else {
          gtz += GJ1[2] * (c.fy * p.uy * iz2);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) gm[k] += c.R[k] * gtx + c.R[3 + k] * gty + c.R[6 + k] * gtz;
        pose[0] += gtx;
        pose[1] += gty;
        pose[2] += gtz;
        pose[3] += ty * gtz - tz * gty;
        pose[4] += tz * gtx - tx * gtz;
        pose[5] += tx * gty - ty * gtx;
        // Sigma_w = M M^T, M = Rq diag(s)
        {
          float GM[9];
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int k = 0; k < 3; ++k)
              GM[a * 3 + k] = 2.f * (GW[a * 3] * G.Rq[k] + GW[a * 3 + 1] * G.Rq[3 + k] + GW[a * 3 + 2] * G.Rq[6 + k]) *
                              G.s[k];
          float GR[9];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            gls[k] += (GM[k] * G.Rq[k] + GM[3 + k] * G.Rq[3 + k] + GM[6 + k] * G.Rq[6 + k]) * G.s[k];
            GR[k] = GM[k] * G.s[k];
            GR[3 + k] = GM[3 + k] * G.s[k];
            GR[6 + k] = GM[6 + k] * G.s[k];
          }
          const float qw = G.qn[0], qx = G.qn[1], qy = G.qn[2], qz = G.qn[3];
          const float gw = 2.f * (-qz * GR[1] + qy * GR[2] + qz * GR[3] - qx * GR[5] - qy * GR[6] + qx * GR[7]);
          const float gx = 2.f * (qy * GR[1] + qz * GR[2] + qy * GR[3] - 2.f * qx * GR[4] - qw * GR[5] + qz * GR[6] +
                                  qw * GR[7] - 2.f * qx * GR[8]);
          const float gy = 2.f * (-2.f * qy * GR[0] + qx * GR[1] + qw * GR[2] + qx * GR[3] + qz * GR[5] - qw * GR[6] +
                                  qz * GR[7] - 2.f * qy * GR[8]);
          const float gz = 2.f * (-2.f * qz * GR[0] - qw * GR[1] + qx * GR[2] + qw * GR[3] - 2.f * qz * GR[4] +
                                  qy * GR[5] + qx * GR[6] + qy * GR[7]);
          const float dot = qw * gw + qx * gx + qy * gy + qz * gz;
          const float iq = 1.0f / G.qnorm;
          gq[0] += (gw - qw * dot) * iq;
          gq[1] += (gx - qx * dot) * iq;
          gq[2] += (gy - qy * dot) * iq;
          gq[3] += (gz - qz * dot) * iq;
        }
        // colour: SH coefficients and the view direction
        {
          float dv[3] = {G.mu[0] - c.ctr[0], G.mu[1] - c.ctr[1], G.mu[2] - c.ctr[2]};
          const float dist = sqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]), idist = 1.0f / dist;
          const float dx = dv[0] * idist, dy = dv[1] * idist, dz = dv[2] * idist;
          float Yb[16];
          sh_basis(DEG, dx, dy, dz, Yb);
          float gdir[3] = {0.f, 0.f, 0.f};
          float dYb[16][3];
          if (DEG > 0) sh_basis_grad(DEG, dx, dy, dz, dYb);
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            float raw = 0.5f;
            float coef[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
              coef[k] = g.sh[((int64_t)k * 3 + ch) * n + i];
              raw += Yb[k] * coef[k];
            }
            if (raw > 0.f) {
              const float gc_ = r[6 + ch];
#pragma unroll
              for (int k = 0; k < K; ++k) gsh[k][ch] += Yb[k] * gc_;
              if (DEG > 0) {
#pragma unroll
                for (int k = 1; k < K; ++k) {
                  gdir[0] += gc_ * coef[k] * dYb[k][0];
                  gdir[1] += gc_ * coef[k] * dYb[k][1];
                  gdir[2] += gc_ * coef[k] * dYb[k][2];
                }
              }
            }
          }
          if (DEG > 0) {
            const float dd = gdir[0] * dx + gdir[1] * dy + gdir[2] * dz;
            const float gv0 = (gdir[0] - dx * dd) * idist, gv1 = (gdir[1] - dy * dd) * idist,
                        gv2 = (gdir[2] - dz * dd) * idist;
            gm[0] += gv0;
            gm[1] += gv1;
            gm[2] += gv2;
            // the camera centre moves by -R'^T rho under a left perturbation
#pragma unroll
            for (int k = 0; k < 3; ++k) pose[k] += c.R[k * 3] * gv0 + c.R[k * 3 + 1] * gv1 + c.R[k * 3 + 2] * gv2;
          }
        }
      }
    }
    // block reduction of the pose gradient of this view
    if (pose_partial) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const float s_ = wave_sum(pose[k]);
        if (l == 0) pose_sh[w][k] = s_;
      }
      __syncthreads();
      if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        pose_partial[((int64_t)v * nb + blockIdx.x) * 6 + k] =
            (pose_sh[0][k] + pose_sh[1][k]) + (pose_sh[2][k] + pose_sh[3][k]);
      }
      __syncthreads();
    }
  }
  if (!valid || !any) return;
  if (gr.means)
    for (int k = 0; k < 3; ++k) gr.means[k * n + i] += gm[k];
  if (gr.log_scales)
    for (int k = 0; k < 3; ++k) gr.log_scales[k * n + i] += gls[k];
  if (gr.quats)
    for (int k = 0; k < 4; ++k) gr.quats[k * n + i] += gq[k];
  if (gr.opacity_logits) gr.opacity_logits[i] += glg;
  if (gr.sh)
#pragma unroll
    for (int k = 0; k < K; ++k)
      for (int ch = 0; ch < 3; ++ch) gr.sh[((int64_t)k * 3 + ch) * n + i] += gsh[k][ch];
  if (st.kappa_sum) st.kappa_sum[i] += s_kap;
  if (st.omega_sum) st.omega_sum[i] += s_om;
  if (st.gamma_sum) st.gamma_sum[i] += s_gam;
  if (st.grad_norm_sum) st.grad_norm_sum[i] += s_gn;
  if (st.view_count) st.view_count[i] += s_vc;
  if (st.max_radius) st.max_radius[i] = max(st.max_radius[i], s_mr);
}

// d/dxi = J_l(xi)^T (dL/drho, dL/dphi), summed over the blocks in fixed order.
__global__ void k_pose_final(int V, int64_t nb, const float* __restrict__ partial, const CamDev* __restrict__ cams,
                             float* __restrict__ grad) {
  const int v = blockIdx.x;
  __shared__ double sh[6][64];
  const int tid = threadIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t b = tid; b < nb; b += 64)
    for (int k = 0; k < 6; ++k) acc[k] += (double)partial[((int64_t)v * nb + b) * 6 + k];
  for (int k = 0; k < 6; ++k) sh[k][tid] = acc[k];
  __syncthreads();
  if (tid == 0) {
    double gd[6];
    for (int k = 0; k < 6; ++k) {
      double s = 0.0;
      for (int t = 0; t < 64; ++t) s += sh[k][t];
      gd[k] = s;
    }
    const CamDev& c = cams[v];
    for (int j = 0; j < 6; ++j) {
      double s = 0.0;
      for (int k = 0; k < 6; ++k) s += c.Jl[k * 6 + j] * gd[k];
      grad[v * 6 + j] += (float)s;
    }
  }
}

kgs_status kgs_launch_project_bwd(kgs_ctx* ctx, const kgs_gaussians* g, const kgs_camera* cams, int V,
                                  const float* pose_xi, const float* view_loss, const kgs_grads* gr,
                                  const kgs_view_stats* stats, hipStream_t st) {
  (void)cams;
  (void)pose_xi;
  const kgs_config& cfg = ctx->cfg;
  BwdParams P;
  P.alpha_min = cfg.alpha_min;
  P.log_alpha_min = logf(cfg.alpha_min);
  P.near_z = cfg.near_z;
  P.eps2d = cfg.eps2d;
  P.rect_margin = cfg.rect_margin;
  P.tile_w = cfg.tile_w;
  P.tile_h = cfg.tile_h;
  P.tiles_x = ctx->tiles_x;
  P.tiles_y = ctx->tiles_y;
  const int64_t nb = (g->n + KGS_BLOCK - 1) / KGS_BLOCK;
  kgs_grads G = *gr;
  kgs_view_stats S = stats ? *stats : kgs_view_stats{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  float* pp = G.pose_xi ? ctx->pose_partial : nullptr;
  if (nb > 0) {
#define KGS_PB(D)                                                                                               \
  hipLaunchKernelGGL(k_project_bwd<D>, dim3((unsigned)nb), dim3(KGS_BLOCK), 0, st, *g, (const CamDev*)ctx->cams, \
                     V, P, (const uint32_t*)ctx->vis, (const uint32_t*)ctx->blk_base, nb,                        \
                     (uint64_t)cfg.slot_capacity, (uint64_t)cfg.pair_capacity, (const float4*)ctx->pair_grad,    \
                     view_loss, G, S, pp)
    switch (g->sh_degree) {
      case 0: KGS_PB(0); break;
      case 1: KGS_PB(1); break;
      case 2: KGS_PB(2); break;
      default: KGS_PB(3); break;
    }
#undef KGS_PB
    if (G.pose_xi)
      hipLaunchKernelGGL(k_pose_final, dim3(V), dim3(64), 0, st, V, nb, (const float*)ctx->pose_partial,
                         (const CamDev*)ctx->cams, G.pose_xi);
  }
  return kgs_check_launch();
}
