// Backward of the projection, deterministic throughout:
//   k_pair_segsum   per slot, the sum of its pairs' gradient records (they
//   k_pair_fixup    are contiguous in emission order), segmented by slot;
//   k_slot_split    queues the slots that blended in some pixel (the others
//                   have zero sums, and slot_om tells the later kernels so);
//   k_slot_live     per queued slot, from its pair sum, the chain rule to the
//                   Gaussian's parameters and to the view's pose, and the
//                   view's footprint statistics, as one 96-byte record;
//   k_gauss_gather  per Gaussian, the sum of its records over the views in
//                   view order (the emission left each (view, Gaussian) slot
//                   index in vis), added into the gradients and statistics;
//   k_pose_reduce   per view, the pose contributions of its slots (contiguous,
//                   slots are in (view, Gaussian) order) in a fixed tree.
// Views are summed in view order; a per-view loop sums the same terms, in
// another order only where a slot's pairs fall into other scan windows.  The pose gradient is accumulated as the left-perturbation
// gradient (rho, phi) of T' = Exp(delta) T' and turned into d/dxi by the SE(3)
// left Jacobian at the end.
#include <algorithm>

#include "kgs_internal.h"

struct BwdParams {
  float alpha_min, log_alpha_min, near_z, far_z, eps2d, rect_margin;
  int tile_w, tile_h, tiles_x, tiles_y;
};


// Slot record (24 words): 0-2 dL/dmean, 3-5 dL/dlog_scale, 6-9 dL/dquat,
// 10 dL/dlogit, 11-16 pose (rho, phi), 17 |Omega| (u32), 18 kappa (u32),
// 19 ||dL/dmu2D||, 20 pixel radius (i32), 21-23 dL/dcolour where the colour is
// not clamped (0 where it is).  The SH basis at the view direction, which the
// SH gradient needs, is evaluated again by the gather from the mean and the
// camera rather than stored (16 words per slot written and read back).
// ---------------------------------------------------------------- pair sums
// Per-slot sums of the 12-word pair records (10 record-space gradient terms
// and the two footprint counts), three float4 per slot, by a segmented
// reduction over the pairs in emission order, where each slot's pairs are
// contiguous.  One wave takes a window of 64 consecutive pairs (one per lane,
// coalesced), scans them segmented by slot with DPP row shifts and the two
// row broadcasts, and the last lane of every segment holds the segment's sum
// within the window.  A segment wholly inside the window is final; one that
// crosses a window edge leaves its partial in the window's head / tail record,
// and k_pair_fixup adds the partials of such a slot in window order.  The
// adds follow a fixed tree, so the sums are deterministic.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp0(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, true));
}

// inclusive scan of x over lanes [sst, l] (sst: first lane of l's segment)
__device__ __forceinline__ float seg_scan(float x, int l, int sst) {
  float t;
  t = dpp0<0x111, 0xf>(x);                 // row_shr:1
  x = (l - 1 >= sst) ? x + t : x;
  t = dpp0<0x112, 0xf>(x);                 // row_shr:2
  x = (l - 2 >= sst) ? x + t : x;
  t = dpp0<0x114, 0xf>(x);                 // row_shr:4
  x = (l - 4 >= sst) ? x + t : x;
  t = dpp0<0x118, 0xf>(x);                 // row_shr:8
  x = (l - 8 >= sst) ? x + t : x;
  t = dpp0<0x142, 0xa>(x);                 // row_bcast:15 into rows 1 and 3
  x = (sst < (l & ~15)) ? x + t : x;
  t = dpp0<0x143, 0xc>(x);                 // row_bcast:31 into rows 2 and 3
  x = (sst < 32 && l >= 32) ? x + t : x;
  return x;
}

__device__ __forceinline__ void put_rec(float4* __restrict__ rec, const float x[12], uint32_t slot, uint32_t flag) {
  rec[0] = make_float4(x[0], x[1], x[2], x[3]);
  rec[1] = make_float4(x[4], x[5], x[6], x[7]);
  rec[2] = make_float4(x[8], x[9], x[10], x[11]);
  rec[3] = make_float4(__uint_as_float(slot), __uint_as_float(flag), 0.f, 0.f);
}

__device__ __forceinline__ void store_sum(float4* __restrict__ rec, const float x[12]) {
  // the two counts travelled as floats (exact below 2^24)
  rec[0] = make_float4(x[0], x[1], x[2], x[3]);
  rec[1] = make_float4(x[4], x[5], x[6], x[7]);
  rec[2] = make_float4(x[8], x[9], __uint_as_float((uint32_t)x[10]), __uint_as_float((uint32_t)x[11]));
}

#define SEG_NONE 0xffffffffu

struct SegWindow {
  uint32_t s, s_before, s_after;
  bool any;   // some pair of the window was written (else every sum in it is zero)
  float x[12];
};

__device__ __forceinline__ void seg_load(SegWindow& W, uint32_t w, uint32_t np, int l,
                                         const uint32_t* __restrict__ pair_slot, const float4* __restrict__ pair_grad,
                                         const uint8_t* __restrict__ pair_live) {
  const uint32_t p = w * 64 + (uint32_t)l;
  const bool valid = p < np;
  W.s = valid ? pair_slot[p] : SEG_NONE;
  // a pair the compositing backward did not reach adds nothing (its record is not written)
  const bool live = valid && pair_live[p] != 0u;
  W.any = ballot64(live) != 0ull;
  if (live) {
    const float4 a = pair_grad[(size_t)p * 3], b = pair_grad[(size_t)p * 3 + 1], c = pair_grad[(size_t)p * 3 + 2];
    W.x[0] = a.x; W.x[1] = a.y; W.x[2] = a.z; W.x[3] = a.w;
    W.x[4] = b.x; W.x[5] = b.y; W.x[6] = b.z; W.x[7] = b.w;
    W.x[8] = c.x; W.x[9] = c.y;
    W.x[10] = (float)__float_as_uint(c.z);
    W.x[11] = (float)__float_as_uint(c.w);
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) W.x[k] = 0.f;
  }
  // slots just before and just after the window (SEG_NONE - 1: none)
  W.s_before = w > 0 ? pair_slot[w * 64 - 1] : SEG_NONE - 1u;
  W.s_after = w * 64 + 64 < np ? pair_slot[w * 64 + 64] : SEG_NONE - 1u;
}

__device__ __forceinline__ void seg_window(SegWindow& W, uint32_t w, uint32_t np, int l,
                                           float4* __restrict__ slot_sum, uint32_t* __restrict__ slot_om,
                                           float4* __restrict__ seg_head, float4* __restrict__ seg_tail) {
  const uint32_t s = W.s;
  const bool valid = w * 64 + (uint32_t)l < np;
  // both shuffles run in every lane (a lane-conditional shuffle reads 0
  // from the lanes that skip it)
  const uint32_t s_up_raw = (uint32_t)__shfl_up((int)s, 1, 64);
  const uint32_t s_dn_raw = (uint32_t)__shfl_down((int)s, 1, 64);
  const uint32_t s_up = l > 0 ? s_up_raw : W.s_before;
  const uint32_t s_dn = l < 63 ? s_dn_raw : W.s_after;
  const bool head = l == 0 || s != s_up;
  const uint64_t H = ballot64(head);
  const uint64_t le = l == 63 ? ~0ull : ((1ull << (l + 1)) - 1ull);
  const int sst = 63 - __clzll((long long)(H & le));
  if (W.any) {
#pragma unroll
    for (int k = 0; k < 12; ++k) W.x[k] = seg_scan(W.x[k], l, sst);
  }
  const bool tail = valid && s != s_dn;
  const bool started = sst > 0 || s != W.s_before;   // the slot's first pair lies in this window
  if (tail) {
    if (started) {
      // a segment that ends in a window without written pairs lies wholly in
      // it: its slot blended nowhere, and its count keeps the zero the
      // compositing backward cleared it to (nothing reads the sums of such a
      // slot)
      if (W.any) {
        store_sum(slot_sum + (size_t)s * (KGS_SLOT_WORDS / 4), W.x);
        slot_om[s] = (uint32_t)W.x[10];
      }
    } else {
      put_rec(seg_head + (size_t)w * 4, W.x, s, 1u);  // continued from before, ends here
    }
  }
  if (l == 63) {
    // the window's last segment goes on past the window
    const bool open = valid && s == s_dn;
    if (open && !started) put_rec(seg_head + (size_t)w * 4, W.x, s, 0u);   // covers the whole window
    put_rec(seg_tail + (size_t)w * 4, W.x, (open && started) ? s : SEG_NONE, 0u);
  }
}

// Two windows per wave and round, both loaded before either is scanned.
__global__ __launch_bounds__(256) void k_pair_segsum(const uint32_t* __restrict__ counters,
                                                     const uint32_t* __restrict__ pair_slot,
                                                     const float4* __restrict__ pair_grad,
                                                     const uint8_t* __restrict__ pair_live,
                                                     float4* __restrict__ slot_sum, uint32_t* __restrict__ slot_om,
                                                     float4* __restrict__ seg_head, float4* __restrict__ seg_tail) {
  const uint32_t np = counters[1];
  const int l = threadIdx.x & 63;
  const uint32_t nwin = (np + 63) / 64;
  const uint32_t stride = gridDim.x * 4;
  for (uint32_t w0 = blockIdx.x * 4 + (threadIdx.x >> 6); w0 < nwin; w0 += 2 * stride) {
    const uint32_t w1 = w0 + stride;
    SegWindow A, B;
    seg_load(A, w0, np, l, pair_slot, pair_grad, pair_live);
    if (w1 < nwin) seg_load(B, w1, np, l, pair_slot, pair_grad, pair_live);
    seg_window(A, w0, np, l, slot_sum, slot_om, seg_head, seg_tail);
    if (w1 < nwin) seg_window(B, w1, np, l, slot_sum, slot_om, seg_head, seg_tail);
  }
}

// For every window whose last segment starts in it and goes on: add the head
// partials of the following windows, in window order, up to the one where the
// slot's pairs end.
__global__ __launch_bounds__(256) void k_pair_fixup(const uint32_t* __restrict__ counters,
                                                    const float4* __restrict__ seg_head,
                                                    const float4* __restrict__ seg_tail,
                                                    float4* __restrict__ slot_sum, uint32_t* __restrict__ slot_om,
                                                    uint32_t* __restrict__ live_count) {
  // the live-slot queue of the chain rule starts empty (nothing reads it before)
  if (blockIdx.x == 0 && threadIdx.x == 0) *live_count = 0u;
  const uint32_t np = counters[1];
  const uint32_t nwin = (np + 63) / 64;
  for (uint32_t w = blockIdx.x * 256 + threadIdx.x; w < nwin; w += gridDim.x * 256) {
    const float4* t = seg_tail + (size_t)w * 4;
    const uint32_t slot = __float_as_uint(t[3].x);
    if (slot == SEG_NONE) continue;
    float x[12];
    const float4 a = t[0], b = t[1], c = t[2];
    x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
    x[8] = c.x; x[9] = c.y; x[10] = c.z; x[11] = c.w;
    for (uint32_t v = w + 1; v < nwin; ++v) {
      const float4* h = seg_head + (size_t)v * 4;
      const float4 d = h[3];
      if (__float_as_uint(d.x) != slot) break;
      const float4 e = h[0], f = h[1], g = h[2];
      x[0] += e.x; x[1] += e.y; x[2] += e.z; x[3] += e.w;
      x[4] += f.x; x[5] += f.y; x[6] += f.z; x[7] += f.w;
      x[8] += g.x; x[9] += g.y; x[10] += g.z; x[11] += g.w;
      if (__float_as_uint(d.y) != 0u) break;
    }
    store_sum(slot_sum + (size_t)slot * (KGS_SLOT_WORDS / 4), x);
    slot_om[slot] = (uint32_t)x[10];
  }
}

template <int DEG>
__device__ __forceinline__ void slot_record(uint32_t s, uint32_t v, const kgs_gaussians& g,
                                            const CamDev* __restrict__ cams, const BwdParams& P,
                                            const uint32_t* __restrict__ slot_gid, uint32_t tiles, const float r[10],
                                            uint32_t om, uint32_t kap, float4* __restrict__ slot_bwd,
                                            float2* __restrict__ slot_pose) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int64_t n = g.n;
  const float h = 0.5f * 1.4426950408889634f;
  const float LN2 = 0.69314718055994531f;
  {
    float out[KGS_SLOT_WORDS];
#pragma unroll
    for (int k = 0; k < KGS_SLOT_WORDS; ++k) out[k] = 0.f;
    const int64_t i = slot_gid[s];
    GaussLocal G;
    bool bad = false;
    load_gaussian(g, i, P.alpha_min, G, bad);
    const CamDev& c = cams[v];
    ProjCore p;
    if (tiles > 0 && G.ok &&
        project_core(c, G.mu, G.Rq, G.s, G.o, P.near_z, P.far_z, P.eps2d, P.rect_margin, P.log_alpha_min, P.tile_w,
                     P.tile_h, P.tiles_x, P.tiles_y, p)) {
      float gm[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
      float pose[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      // pixel moments (ge u, ge dy, ge u^2, ge u dy, ge dy^2, ge) summed over
      // the slot's pixels -> derivatives of log2 alpha = log2 o + P' u^2 +
      // E' dy^2, u = dx + k dy, in the record's mean, P', k, E' and log2 o
      // (dx, dy fall with the mean); ge is dL/d(log2 alpha) / ln 2
      float rr[6];
      {
        const float Pq = -h * p.Pc, Eq = -h * p.Ec;
        const float m0 = r[0] * LN2, m1 = r[1] * LN2;
        rr[0] = -2.0f * Pq * m0;
        rr[1] = -2.0f * (Pq * p.kc * m0 + Eq * m1);
        rr[2] = r[2] * LN2;
        rr[3] = 2.0f * Pq * (r[3] * LN2);
        rr[4] = r[4] * LN2;
        rr[5] = r[5] * LN2;
      }
      out[17] = __uint_as_float(om);
      out[18] = __uint_as_float(kap);
      out[19] = sqrtf(rr[0] * rr[0] + rr[1] * rr[1]);
      out[20] = __int_as_float(max(p.rx, p.ry));
        float Yb_out[16];
        // record space -> pivoted conic (P, k, E) and opacity
        const float gP = -h * rr[2], gk = rr[3], gE = -h * rr[4];
        out[10] = r[5] * (1.0f - G.o);
        // P = S11 / det, k = -S01 / S11, E = 1 / S11
        const float gS11 = gP / p.det - (gk * p.kc + gE * p.Ec) * p.Ec;
        const float gS01 = -gk * p.Ec;
        const float gdet = -gP * p.Pc / p.det;
        // det = K^2 |cof(s) v|^2 + eps (S'00 + S'11) + eps^2,  S11 = S'11 + eps
        const float gSp00 = P.eps2d * gdet, gSp11 = gS11 + P.eps2d * gdet;
        const float c0 = G.s[1] * G.s[2], c1 = G.s[0] * G.s[2], c2 = G.s[0] * G.s[1];
        const float hv0 = c0 * p.v[0], hv1 = c1 * p.v[1], hv2 = c2 * p.v[2];
        const float gK = 2.0f * p.K * (hv0 * hv0 + hv1 * hv1 + hv2 * hv2) * gdet;
        const float k2g = 2.0f * p.K * p.K * gdet;
        const float gh0 = k2g * hv0, gh1 = k2g * hv1, gh2 = k2g * hv2;
        float gs[3];
        gs[0] = G.s[2] * p.v[1] * gh1 + G.s[1] * p.v[2] * gh2;
        gs[1] = G.s[2] * p.v[0] * gh0 + G.s[0] * p.v[2] * gh2;
        gs[2] = G.s[1] * p.v[0] * gh0 + G.s[0] * p.v[1] * gh1;
        const float gv[3] = {c0 * gh0, c1 * gh1, c2 * gh2};
        // S'00 = |m0|^2, S'11 = |m1|^2, S01 = m0 . m1 with m = s * a
        float ga0[3], ga1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const float m0 = G.s[k] * p.a0[k], m1 = G.s[k] * p.a1[k];
          const float gm0 = 2.0f * m0 * gSp00 + m1 * gS01, gm1 = 2.0f * m1 * gSp11 + m0 * gS01;
          gs[k] += p.a0[k] * gm0 + p.a1[k] * gm1;
          ga0[k] = G.s[k] * gm0;
          ga1[k] = G.s[k] * gm1;
        }
        // v = Rq^T w, a0 = Rq^T T0, a1 = Rq^T T1 with w = R'^T (ux, uy, 1)
        float w[3], gw[3], gT0[3], gT1[3], GR[9];
#pragma unroll
        for (int j = 0; j < 3; ++j) w[j] = c.R[j] * p.ux + c.R[3 + j] * p.uy + c.R[6 + j];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
#pragma unroll
          for (int k = 0; k < 3; ++k) GR[j * 3 + k] = w[j] * gv[k] + p.T0[j] * ga0[k] + p.T1[j] * ga1[k];
          gw[j] = G.Rq[j * 3] * gv[0] + G.Rq[j * 3 + 1] * gv[1] + G.Rq[j * 3 + 2] * gv[2];
          gT0[j] = G.Rq[j * 3] * ga0[0] + G.Rq[j * 3 + 1] * ga0[1] + G.Rq[j * 3 + 2] * ga0[2];
          gT1[j] = G.Rq[j * 3] * ga1[0] + G.Rq[j * 3 + 1] * ga1[1] + G.Rq[j * 3 + 2] * ga1[2];
        }
        // T0 = J00 R'_0 + J02 R'_2, T1 = J11 R'_1 + J12 R'_2, w = ux R'_0 + uy R'_1 + R'_2 (rows of R')
        float gJ00 = 0.f, gJ02 = 0.f, gJ11 = 0.f, gJ12 = 0.f, gux = 0.f, guy = 0.f;
        float gRr[9];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          gJ00 += c.R[j] * gT0[j];
          gJ02 += c.R[6 + j] * gT0[j];
          gJ11 += c.R[3 + j] * gT1[j];
          gJ12 += c.R[6 + j] * gT1[j];
          gux += c.R[j] * gw[j];
          guy += c.R[3 + j] * gw[j];
          gRr[j] = p.J00 * gT0[j] + p.ux * gw[j];
          gRr[3 + j] = p.J11 * gT1[j] + p.uy * gw[j];
          gRr[6 + j] = p.J02 * gT0[j] + p.J12 * gT1[j] + gw[j];
        }
        // pose, rotation acting on R' where it enters T and w: M = R' (dL/dR')^T,
        // g_phi += (M12 - M21, M20 - M02, M01 - M10)
        {
          float M[9];
#pragma unroll
          for (int a2 = 0; a2 < 3; ++a2)
#pragma unroll
            for (int b2 = 0; b2 < 3; ++b2)
              M[a2 * 3 + b2] = c.R[a2 * 3] * gRr[b2 * 3] + c.R[a2 * 3 + 1] * gRr[b2 * 3 + 1] +
                               c.R[a2 * 3 + 2] * gRr[b2 * 3 + 2];
          pose[3] += M[5] - M[7];
          pose[4] += M[6] - M[2];
          pose[5] += M[1] - M[3];
        }
        // camera-frame point gradient
        const float tx = p.tx, ty = p.ty, tz = p.tz, iz = 1.0f / tz, iz2 = iz * iz;
        float gtx = rr[0] * c.fx * iz, gty = rr[1] * c.fy * iz;
        float gtz = -(rr[0] * c.fx * tx + rr[1] * c.fy * ty) * iz2 + r[9];
        gtz += -2.0f * gK * p.K * iz;
        gtz += -(gJ00 * c.fx + gJ11 * c.fy) * iz2;
        gux += -gJ02 * c.fx * iz;
        gtz += gJ02 * c.fx * p.ux * iz2;
        guy += -gJ12 * c.fy * iz;
        gtz += gJ12 * c.fy * p.uy * iz2;
        if (p.clx == 0) {
          gtx += gux * iz;
          gtz -= gux * tx * iz2;
        }
        if (p.cly == 0) {
          gty += guy * iz;
          gtz -= guy * ty * iz2;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) gm[k] += c.R[k] * gtx + c.R[3 + k] * gty + c.R[6 + k] * gtz;
        pose[0] += gtx;
        pose[1] += gty;
        pose[2] += gtz;
        pose[3] += ty * gtz - tz * gty;
        pose[4] += tz * gtx - tx * gtz;
        pose[5] += tx * gty - ty * gtx;
        // s = exp(log_s); Rq from the normalised quaternion
#pragma unroll
        for (int k = 0; k < 3; ++k) gls[k] += gs[k] * G.s[k];
        {
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
        // colour: SH basis at the view direction, masked colour gradient, and
        // the direction gradient sum_k w_k grad Y_k with w_k = sum_ch g_ch c_k,ch
        {
          float dv[3];
          cam_offset(c, G.mu, dv);
          const float dist = sqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]), idist = 1.0f / dist;
          const float dx = dv[0] * idist, dy = dv[1] * idist, dz = dv[2] * idist;
          sh_basis(DEG, dx, dy, dz, Yb_out);
          float gcm[3];
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            float raw = 0.5f;
#pragma unroll
            for (int k = 0; k < K; ++k) raw += Yb_out[k] * g.sh[((int64_t)k * 3 + ch) * n + i];
            gcm[ch] = raw > 0.f ? r[6 + ch] : 0.f;
            out[21 + ch] = gcm[ch];
          }
          if (DEG > 0) {
            float wk[16];
#pragma unroll
            for (int k = 0; k < K; ++k)
              wk[k] = gcm[0] * g.sh[((int64_t)k * 3) * n + i] + gcm[1] * g.sh[((int64_t)k * 3 + 1) * n + i] +
                      gcm[2] * g.sh[((int64_t)k * 3 + 2) * n + i];
            float gdir[3];
            sh_dir_grad(DEG, dx, dy, dz, wk, gdir);
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
      out[0] = gm[0]; out[1] = gm[1]; out[2] = gm[2];
      out[3] = gls[0]; out[4] = gls[1]; out[5] = gls[2];
      out[6] = gq[0]; out[7] = gq[1]; out[8] = gq[2]; out[9] = gq[3];
#pragma unroll
      for (int k = 0; k < 6; ++k) out[11 + k] = pose[k];
    }
    float4* o4 = slot_bwd + (size_t)s * (KGS_SLOT_WORDS / 4);
#pragma unroll
    for (int k = 0; k < KGS_SLOT_WORDS / 4; ++k)
      o4[k] = make_float4(out[4 * k], out[4 * k + 1], out[4 * k + 2], out[4 * k + 3]);
    // the pose contributions again, packed, for the per-view reduction
    float2* p2 = slot_pose + (size_t)s * 3;
    p2[0] = make_float2(out[11], out[12]);
    p2[1] = make_float2(out[13], out[14]);
    p2[2] = make_float2(out[15], out[16]);
  }
}

// Slots whose pixels blended nowhere have a zero sum (every pixel term is a
// zero at alpha = 0), so zero gradients and pose terms, and nothing reads their
// records: the gather and the pose reduction look at slot_om first.
// k_slot_split queues the others: a block takes 2048 consecutive slots, eight
// per thread (two 16-byte loads), ranks them with a block scan and claims its
// share of the queue with one atomic (the queue's order does not matter, since
// every result is written at its slot); k_slot_live takes the queue with full
// waves.  counters[KGS_CNT_LIVE] is cleared by k_pair_fixup.
__global__ __launch_bounds__(KGS_BLOCK) void k_slot_split(uint32_t* __restrict__ counters,
                                                          const uint32_t* __restrict__ slot_om,
                                                          uint32_t* __restrict__ slot_live) {
  __shared__ uint32_t s_wave[KGS_BLOCK / 64];
  __shared__ uint32_t s_base;
  const uint32_t n_slots = counters[0];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  constexpr uint32_t PER_BLOCK = KGS_BLOCK * 8u;
  for (uint64_t bb = (uint64_t)blockIdx.x * PER_BLOCK; bb < n_slots; bb += (uint64_t)gridDim.x * PER_BLOCK) {
    const uint64_t s0 = bb + (uint64_t)tid * 8u;
    uint32_t m = 0u;
    if (s0 + 8u <= n_slots) {
      const uint4* q = reinterpret_cast<const uint4*>(slot_om + s0);
      const uint4 a = q[0], b = q[1];
      m = (a.x != 0u ? 1u : 0u) | (a.y != 0u ? 2u : 0u) | (a.z != 0u ? 4u : 0u) | (a.w != 0u ? 8u : 0u) |
          (b.x != 0u ? 16u : 0u) | (b.y != 0u ? 32u : 0u) | (b.z != 0u ? 64u : 0u) | (b.w != 0u ? 128u : 0u);
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (s0 + k < n_slots && slot_om[s0 + k] != 0u) m |= 1u << k;
    }
    const uint32_t c = (uint32_t)__popc(m);
    const uint32_t inc = wave_inclusive_scan(c);
    if (l == 63) s_wave[w] = inc;
    __syncthreads();
    if (tid == 0) {
      uint32_t tot = 0u;
#pragma unroll
      for (int k = 0; k < KGS_BLOCK / 64; ++k) tot += s_wave[k];
      s_base = tot ? atomicAdd(&counters[KGS_CNT_LIVE], tot) : 0u;
    }
    __syncthreads();
    uint32_t pos = s_base + inc - c;
    for (int k = 0; k < w; ++k) pos += s_wave[k];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if ((m >> k) & 1u) slot_live[pos++] = (uint32_t)(s0 + k);
    __syncthreads();   // s_wave and s_base are rewritten by the next round
  }
}

// Chain rule of every queued slot: its pair sum (words 0-11 of its record)
// becomes the full backward record.
template <int DEG>
__global__ __launch_bounds__(KGS_BLOCK) void k_slot_live(kgs_gaussians g, const CamDev* __restrict__ cams,
                                                         BwdParams P, const uint32_t* __restrict__ counters,
                                                         const uint32_t* __restrict__ slot_live,
                                                         const uint32_t* __restrict__ slot_gid,
                                                         const uint4* __restrict__ emit_desc, int tile_bits,
                                                         float4* __restrict__ slot_bwd,
                                                         float2* __restrict__ slot_pose) {
  const uint32_t n_live = counters[KGS_CNT_LIVE];
  for (uint32_t j = blockIdx.x * KGS_BLOCK + threadIdx.x; j < n_live; j += gridDim.x * KGS_BLOCK) {
    const uint32_t s = slot_live[j];
    const float4* q = slot_bwd + (size_t)s * (KGS_SLOT_WORDS / 4);
    const float4 a = q[0], b = q[1], c = q[2];
    const float r[10] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y};
    // the slot's view and tile count, from the projection's emission descriptor;
    // one view at a time across the wave, so that its camera is read with
    // scalar loads; queued slots keep view order within a wave's share
    const uint4 dsc = emit_desc[s];
    const uint32_t v = dsc.x >> tile_bits;
    bool pending = true;
    while (pending) {
      const uint32_t vu = __builtin_amdgcn_readfirstlane(v);
      if (v == vu) {
        slot_record<DEG>(s, vu, g, cams, P, slot_gid, dsc.w, r, __float_as_uint(c.z), __float_as_uint(c.w),
                         slot_bwd, slot_pose);
        pending = false;
      }
    }
  }
}

// Per Gaussian, the sum of its slot records over the views in view order
// (vis names each view's slot), added into the gradients and statistics.
template <int DEG>
__global__ __launch_bounds__(KGS_BLOCK) void k_gauss_gather(kgs_gaussians g, int V, const CamDev* __restrict__ cams,
                                                            const uint32_t* __restrict__ vis,
                                                            const uint32_t* __restrict__ counters,
                                                            const float4* __restrict__ slot_bwd,
                                                            const uint32_t* __restrict__ slot_om,
                                                            const int4* __restrict__ slot_pix,
                                                            const float* __restrict__ view_loss, kgs_grads gr,
                                                            kgs_view_stats st, int overwrite) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int64_t n = g.n;
  const int64_t i = (int64_t)blockIdx.x * KGS_BLOCK + threadIdx.x;
  if (i >= n) return;
  const uint32_t n_slots = counters[0];
  float mu[3] = {0.f, 0.f, 0.f};
  if (DEG > 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) mu[k] = g.means[k * n + i];
  }
  float acc[11];
#pragma unroll
  for (int k = 0; k < 11; ++k) acc[k] = 0.f;
  float gsh[K][3];
#pragma unroll
  for (int k = 0; k < K; ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.f;
  uint32_t s_kap = 0, s_om = 0, s_vc = 0;
  double s_gam = 0.0;
  float s_gn = 0.f;
  int s_mr = 0;
  // views in groups of eight: the slot indices of a group, then their counts,
  // are loaded together, so a Gaussian waits on two loads per group instead
  // of two per view
  for (int v0 = 0; v0 < V; v0 += 8) {
    uint32_t uu[8], oo[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t u = v0 + j < V ? vis[(int64_t)(v0 + j) * n + i] : 0u;
      uu[j] = (u == 0u || u > n_slots) ? 0u : u;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) oo[j] = uu[j] ? slot_om[uu[j] - 1u] : 0u;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t u = uu[j];
      if (u == 0u) continue;
      const int v = v0 + j;
      s_vc += 1u;
      if (oo[j] == 0u) {
        // a slot that blended nowhere adds nothing but its radius, which the
        // projection stored (every slot has a tile, so the radius stands)
        const int4 pix = slot_pix[u - 1u];
        s_mr = max(s_mr, max(pix.z, pix.w));
        continue;
      }
      const float4* r4 = slot_bwd + (size_t)(u - 1u) * (KGS_SLOT_WORDS / 4);
      // words 16-23: counts, gradient norm, radius, masked colour gradient
      const float4 q4 = r4[4], q5 = r4[5];
      const uint32_t om = __float_as_uint(q4.y);
      s_mr = max(s_mr, __float_as_int(q5.x));
      float r[16];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float4 q = r4[k];
        r[4 * k] = q.x; r[4 * k + 1] = q.y; r[4 * k + 2] = q.z; r[4 * k + 3] = q.w;
      }
#pragma unroll
      for (int k = 0; k < 11; ++k) acc[k] += r[k];
      // SH basis at this view's direction (as in the chain rule per slot)
      float Y[16];
      Y[0] = 0.f;
      if (DEG > 0) {
        float dv[3];
        cam_offset(cams[v], mu, dv);
        const float idist = 1.0f / sqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        sh_basis(DEG, dv[0] * idist, dv[1] * idist, dv[2] * idist, Y);
      } else {
        sh_basis(0, 0.f, 0.f, 1.f, Y);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        gsh[k][0] += Y[k] * q5.y;
        gsh[k][1] += Y[k] * q5.z;
        gsh[k][2] += Y[k] * q5.w;
      }
      s_om += om;
      s_kap += __float_as_uint(q4.z);
      if (view_loss) s_gam += (double)view_loss[v] * (double)om;
      s_gn += q4.w;
    }
  }
  if (overwrite) {
    // the outputs start from zero: every Gaussian is written, seen or not
    if (gr.means)
      for (int k = 0; k < 3; ++k) gr.means[k * n + i] = acc[k];
    if (gr.log_scales)
      for (int k = 0; k < 3; ++k) gr.log_scales[k * n + i] = acc[3 + k];
    if (gr.quats)
      for (int k = 0; k < 4; ++k) gr.quats[k * n + i] = acc[6 + k];
    if (gr.opacity_logits) gr.opacity_logits[i] = acc[10];
    if (gr.sh)
#pragma unroll
      for (int k = 0; k < K; ++k)
        for (int ch = 0; ch < 3; ++ch) gr.sh[((int64_t)k * 3 + ch) * n + i] = gsh[k][ch];
    if (st.kappa_sum) st.kappa_sum[i] = s_kap;
    if (st.omega_sum) st.omega_sum[i] = s_om;
    if (st.gamma_sum) st.gamma_sum[i] = s_gam;
    if (st.grad_norm_sum) st.grad_norm_sum[i] = s_gn;
    if (st.view_count) st.view_count[i] = s_vc;
    if (st.max_radius) st.max_radius[i] = s_mr;
    return;
  }
  if (s_vc == 0) return;
  if (gr.means)
    for (int k = 0; k < 3; ++k) gr.means[k * n + i] += acc[k];
  if (gr.log_scales)
    for (int k = 0; k < 3; ++k) gr.log_scales[k * n + i] += acc[3 + k];
  if (gr.quats)
    for (int k = 0; k < 4; ++k) gr.quats[k * n + i] += acc[6 + k];
  if (gr.opacity_logits) gr.opacity_logits[i] += acc[10];
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

// Pose contributions of view v's slots (blockIdx.y = v), in KGS_POSE_BLOCKS
// contiguous pieces, FP64, fixed reduction tree.
__global__ __launch_bounds__(256) void k_pose_reduce(const uint32_t* __restrict__ counters,
                                                     const uint32_t* __restrict__ blk_base, int64_t nb, int V,
                                                     const float2* __restrict__ slot_pose,
                                                     const uint32_t* __restrict__ slot_om,
                                                     double* __restrict__ partial) {
  __shared__ double sh[4][6];
  const int v = blockIdx.y, b = blockIdx.x, tid = threadIdx.x;
  const uint32_t n_slots = counters[0];
  uint32_t lo = blk_base[((int64_t)v * nb) * 2];
  uint32_t hi = (v + 1 < V) ? blk_base[((int64_t)(v + 1) * nb) * 2] : n_slots;
  lo = min(lo, n_slots);
  hi = min(max(hi, lo), n_slots);
  const uint32_t per = (hi - lo + KGS_POSE_BLOCKS - 1) / KGS_POSE_BLOCKS;
  const uint32_t a = lo + b * per, e = min(hi, a + per);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (uint32_t s = a + tid; s < e; s += 256) {
    if (slot_om[s] == 0u) continue;   // no pose terms (and none written)
    const float2* p2 = slot_pose + (size_t)s * 3;
    const float2 a = p2[0], b = p2[1], c = p2[2];
    acc[0] += a.x; acc[1] += a.y; acc[2] += b.x; acc[3] += b.y; acc[4] += c.x; acc[5] += c.y;
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double t = wave_sum(acc[k]);
    if ((tid & 63) == 0) sh[tid >> 6][k] = t;
  }
  __syncthreads();
  if (tid < 6) partial[((size_t)v * KGS_POSE_BLOCKS + b) * 6 + tid] = (sh[0][tid] + sh[1][tid]) + (sh[2][tid] + sh[3][tid]);
}

// d/dxi = J_l(xi)^T (dL/drho, dL/dphi), the pieces summed by a fixed tree
// (one block per view, one piece per thread).
__global__ __launch_bounds__(KGS_POSE_BLOCKS) void k_pose_final(const double* __restrict__ partial,
                                                                const CamDev* __restrict__ cams,
                                                                float* __restrict__ grad, int overwrite) {
  static_assert(KGS_POSE_BLOCKS == 256, "one thread per piece, four waves");
  __shared__ double sh[4][6];
  const int v = blockIdx.x, tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double t = wave_sum(partial[((size_t)v * KGS_POSE_BLOCKS + tid) * 6 + k]);
    if ((tid & 63) == 0) sh[tid >> 6][k] = t;
  }
  __syncthreads();
  if (tid < 6) {
    const int j = tid;
    double gd[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) gd[k] = (sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]);
    const CamDev& c = cams[v];
    double s = 0.0;
    for (int k = 0; k < 6; ++k) s += c.Jl[k * 6 + j] * gd[k];
    grad[v * 6 + j] = overwrite ? (float)s : grad[v * 6 + j] + (float)s;
  }
}

kgs_status kgs_launch_project_bwd(kgs_ctx* ctx, const kgs_gaussians* g, const kgs_camera* cams, int V,
                                  const float* pose_xi, const float* view_loss, const kgs_grads* gr,
                                  const kgs_view_stats* stats, hipStream_t st, bool overwrite) {
  (void)cams;
  (void)pose_xi;
  const kgs_config& cfg = ctx->cfg;
  BwdParams P;
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
  const int64_t nb = (g->n + KGS_BLOCK - 1) / KGS_BLOCK;
  kgs_grads G = *gr;
  kgs_view_stats S = stats ? *stats : kgs_view_stats{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  const uint64_t cap = (uint64_t)cfg.slot_capacity;
  if (nb > 0) {
    const unsigned sg = (unsigned)std::min<uint64_t>(std::max<uint64_t>((cap + 255) / 256, 1), 4096);
    const uint64_t wins = ((uint64_t)cfg.pair_capacity + 63) / 64;
    const unsigned wg = (unsigned)std::min<uint64_t>(std::max<uint64_t>((wins + 7) / 8, 1), 4096);
    hipLaunchKernelGGL(k_pair_segsum, dim3(wg), dim3(256), 0, st, (const uint32_t*)ctx->counters,
                       (const uint32_t*)ctx->pair_slot, (const float4*)ctx->pair_grad,
                       (const uint8_t*)ctx->pair_live, ctx->slot_bwd, ctx->slot_om, ctx->seg_head,
                       ctx->seg_tail);
    hipLaunchKernelGGL(k_pair_fixup, dim3((unsigned)std::min<uint64_t>(std::max<uint64_t>((wins + 255) / 256, 1), 2048)),
                       dim3(256), 0, st, (const uint32_t*)ctx->counters, (const float4*)ctx->seg_head,
                       (const float4*)ctx->seg_tail, ctx->slot_bwd, ctx->slot_om, ctx->counters + KGS_CNT_LIVE);
    const unsigned spg = (unsigned)std::min<uint64_t>(std::max<uint64_t>((cap + 8 * KGS_BLOCK - 1) / (8 * KGS_BLOCK), 1),
                                                      4096);
    hipLaunchKernelGGL(k_slot_split, dim3(spg), dim3(KGS_BLOCK), 0, st, ctx->counters,
                       (const uint32_t*)ctx->slot_om, ctx->slot_live);
#define KGS_PB(D)                                                                                                  \
  hipLaunchKernelGGL(k_slot_live<D>, dim3(sg), dim3(KGS_BLOCK), 0, st, *g, (const CamDev*)ctx->cams, P,            \
                     (const uint32_t*)ctx->counters, (const uint32_t*)ctx->slot_live,                               \
                     (const uint32_t*)ctx->slot_gid, (const uint4*)ctx->emit_desc, kgs_tile_bits(ctx->n_tiles),   \
                     ctx->slot_bwd, ctx->slot_pose);                                                               \
  hipLaunchKernelGGL(k_gauss_gather<D>, dim3((unsigned)nb), dim3(KGS_BLOCK), 0, st, *g, V,                        \
                     (const CamDev*)ctx->cams, (const uint32_t*)ctx->vis, (const uint32_t*)ctx->counters,          \
                     (const float4*)ctx->slot_bwd, (const uint32_t*)ctx->slot_om,                                \
                     (const int4*)ctx->slot_pix, view_loss, G, S, overwrite ? 1 : 0)
    switch (g->sh_degree) {
      case 0: KGS_PB(0); break;
      case 1: KGS_PB(1); break;
      case 2: KGS_PB(2); break;
      default: KGS_PB(3); break;
    }
#undef KGS_PB
    if (G.pose_xi) {
      hipLaunchKernelGGL(k_pose_reduce, dim3(KGS_POSE_BLOCKS, V), dim3(256), 0, st, (const uint32_t*)ctx->counters,
                         (const uint32_t*)ctx->blk_base, nb, V, (const float2*)ctx->slot_pose,
                         (const uint32_t*)ctx->slot_om, ctx->pose_partial);
      hipLaunchKernelGGL(k_pose_final, dim3(V), dim3(KGS_POSE_BLOCKS), 0, st, (const double*)ctx->pose_partial,
                         (const CamDev*)ctx->cams, G.pose_xi, overwrite ? 1 : 0);
    }
  }
  return kgs_check_launch();
}
