// Front-to-back alpha compositing of colour, depth and the low-dimensional
// feature (UP-SLAM Sec. 3.1 Eq. 3, Sec. 3.3 Eq. 10) and its backward.
//
// One 256-thread workgroup per 16x16 screen tile, one pixel per thread. The
// tile's depth-ordered list is staged through LDS in batches of records; each
// pixel walks the batch, skips alpha < alpha_min, stops before the
// transmittance would fall below T_min, and accumulates w = alpha * T times
// (rgb, z, feature). The workgroup leaves as soon as every pixel has stopped.
//
// The backward replays each pixel's list back to front from its last
// composited Gaussian, recovering T_k = T_{k+1} / (1 - alpha_k). Per list entry
// the 26 gradient values (u, v, conic, opacity, channels) of the 256 pixels are
// summed over each 16-lane row with DPP (skipped by ballot when no lane of the
// wave touches the Gaussian), the 16 row sums of the workgroup are combined in
// LDS and written once to the entry's gradient slot; no global atomics. The
// projection backward then sums each Gaussian's slots.
#include "internal.h"

namespace asgs {

namespace {

template <int CTRL>
ASGS_DEV float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Sum over each row of 16 lanes; every lane of a row receives its row's sum.
// All lanes must be active.
ASGS_DEV float row_sum(float x) {
  x += dpp<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp<0x124>(x);  // row_ror:4
  x += dpp<0x128>(x);  // row_ror:8
  return x;
}

ASGS_DEV int find_view(const ViewDev* views, int n_views, int tile) {
  int v = 0;
  for (int k = 1; k < n_views; ++k)
    if (tile >= views[k].tile_base) v = k;
  return v;
}

template <int NF>
__global__ void __launch_bounds__(kTilePix) k_blend_fwd(RenderConst rc, const ViewDev* __restrict__ views,
                                                        char* ctx, CtxLayout L, asgs_images out) {
  constexpr int CS = 4 + NF;
  constexpr int CS4 = CS / 4;
  const int tile = blockIdx.x;
  const int view = find_view(views, rc.n_views, tile);
  const ViewDev& V = views[view];
  const int lt = tile - V.tile_base;
  const int ty = lt / V.TX, tx = lt - ty * V.TX;
  const int t = threadIdx.x;
  const int px = tx * kTile + (t & (kTile - 1));
  const int py = ty * kTile + (t / kTile);
  const bool inside = px < V.W && py < V.H;
  const float pxf = (float)px, pyf = (float)py;
  const uint2 rg = ctx_ptr<const uint2>(ctx, L.ranges)[tile];
  const uint32_t* pairgid = ctx_ptr<const uint32_t>(ctx, L.pairgid);
  const float4* geom = ctx_ptr<const float4>(ctx, L.geom);
  const float4* chan4 = ctx_ptr<const float4>(ctx, L.chan);

  __shared__ float4 sg[kTilePix * 2];
  __shared__ float4 sc[kTilePix * CS4];

  float T = 1.f;
  float acc[CS];
#pragma unroll
  for (int c = 0; c < CS; ++c) acc[c] = 0.f;
  uint32_t last = 0;
  bool done = !inside;
  const float amin = rc.alpha_min, amax = rc.alpha_max, tmin = rc.T_min;
  for (uint32_t base = rg.x; base < rg.y; base += kTilePix) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t p = base + t;
    if (p < rg.y) {
      const uint32_t gid = pairgid[p];
      sg[2 * t] = geom[2 * (size_t)gid];
      sg[2 * t + 1] = geom[2 * (size_t)gid + 1];
#pragma unroll
      for (int c = 0; c < CS4; ++c) sc[t * CS4 + c] = chan4[(size_t)gid * CS4 + c];
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)kTilePix, rg.y - base);
    if (!done) {
      float4 n0 = sg[0], n1 = sg[1];
      for (int j = 0; j < cnt; ++j) {
        // geometry of the next entry is read before this one is evaluated
        const float4 g0 = n0;
        const float4 g1 = n1;
        const int jn = j + 1 < cnt ? j + 1 : j;
        n0 = sg[2 * jn];
        n1 = sg[2 * jn + 1];
        float dx, dy;
        const float power = eval_power(g0.x, g0.y, g0.z, g0.w, g1.x, pxf, pyf, dx, dy);
        if (power > 0.f) continue;
        const float alpha = fminf(amax, g1.y * __expf(power));
        if (alpha < amin) continue;
        const float Tn = T * (1.f - alpha);
        if (Tn < tmin) {
          done = true;
          break;
        }
        const float w = alpha * T;
#pragma unroll
        for (int c4 = 0; c4 < CS4; ++c4) {
          const float4 v = sc[j * CS4 + c4];
          acc[4 * c4 + 0] = fmaf(w, v.x, acc[4 * c4 + 0]);
          acc[4 * c4 + 1] = fmaf(w, v.y, acc[4 * c4 + 1]);
          acc[4 * c4 + 2] = fmaf(w, v.z, acc[4 * c4 + 2]);
          acc[4 * c4 + 3] = fmaf(w, v.w, acc[4 * c4 + 3]);
        }
        T = Tn;
        last = base - rg.x + (uint32_t)j + 1u;
      }
    }
  }
  if (!inside) return;
  const size_t HW = (size_t)V.W * V.H;
  const size_t pix = (size_t)py * V.W + px;
  const size_t pb = (size_t)V.pix_base;
  out.rgb[3 * pb + 0 * HW + pix] = acc[0] + T * rc.bg[0];
  out.rgb[3 * pb + 1 * HW + pix] = acc[1] + T * rc.bg[1];
  out.rgb[3 * pb + 2 * HW + pix] = acc[2] + T * rc.bg[2];
  out.depth[pb + pix] = acc[3];
  if (NF > 0) {
#pragma unroll
    for (int c = 0; c < NF; ++c) out.feat[NF * pb + c * HW + pix] = acc[4 + c];
  }
  out.alpha[pb + pix] = 1.f - T;
  ctx_ptr<float>(ctx, L.tfinal)[pb + pix] = T;
  ctx_ptr<uint32_t>(ctx, L.ncontrib)[pb + pix] = last;
}

constexpr int kBwdBatch = 16;

template <int NF>
__global__ void __launch_bounds__(kTilePix) k_blend_bwd(RenderConst rc, const ViewDev* __restrict__ views,
                                                        char* ctx, CtxLayout L, asgs_images dout) {
  constexpr int CS = 4 + NF;
  constexpr int CS4 = CS / 4;
  constexpr int GS = 6 + CS;
  constexpr int NW = kTilePix / 64;
  const int tile = blockIdx.x;
  const int view = find_view(views, rc.n_views, tile);
  const ViewDev& V = views[view];
  const int lt = tile - V.tile_base;
  const int ty = lt / V.TX, tx = lt - ty * V.TX;
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int px = tx * kTile + (t & (kTile - 1));
  const int py = ty * kTile + (t / kTile);
  const bool inside = px < V.W && py < V.H;
  const float pxf = (float)px, pyf = (float)py;
  const uint2 rg = ctx_ptr<const uint2>(ctx, L.ranges)[tile];
  const uint32_t len = rg.y - rg.x;
  const uint32_t* pairgid = ctx_ptr<const uint32_t>(ctx, L.pairgid);
  const uint32_t* pslot = ctx_ptr<const uint32_t>(ctx, L.pval_fin);
  const float4* geom = ctx_ptr<const float4>(ctx, L.geom);
  const float4* chan4 = ctx_ptr<const float4>(ctx, L.chan);
  float* gslot = ctx_ptr<float>(ctx, L.gslot);

  constexpr int NR = NW * 4;  // 16-lane rows per workgroup
  __shared__ float4 sg[kBwdBatch * 2];
  __shared__ float4 sc[kBwdBatch * CS4];
  // row partials, row index innermost (+1 pad) so the four row leaders of a
  // wave hit four different banks
  __shared__ float part[kBwdBatch][GS][NR + 1];
  __shared__ uint32_t smax;

  const size_t HW = (size_t)V.W * V.H;
  const size_t pix = (size_t)py * V.W + px;
  const size_t pb = (size_t)V.pix_base;
  float Tf = 1.f;
  uint32_t last = 0;
  float G[CS];
#pragma unroll
  for (int c = 0; c < CS; ++c) G[c] = 0.f;
  float GT = 0.f;
  if (inside) {
    Tf = ctx_ptr<const float>(ctx, L.tfinal)[pb + pix];
    last = ctx_ptr<const uint32_t>(ctx, L.ncontrib)[pb + pix];
    for (int c = 0; c < 3; ++c) G[c] = dout.rgb[3 * pb + c * HW + pix];
    G[3] = dout.depth[pb + pix];
#pragma unroll
    for (int c = 0; c < NF; ++c) G[4 + c] = dout.feat[NF * pb + c * HW + pix];
    const float ga = dout.alpha ? dout.alpha[pb + pix] : 0.f;
    GT = rc.bg[0] * G[0] + rc.bg[1] * G[1] + rc.bg[2] * G[2] - ga;
  }
  if (t == 0) smax = 0u;
  __syncthreads();
  atomicMax(&smax, last);
  __syncthreads();
  const uint32_t nproc = smax;
  // entries behind every pixel's last Gaussian get zero gradient
  for (uint32_t q = nproc + t; q < len; q += kTilePix) {
    float* dst = gslot + (size_t)pslot[rg.x + q] * GS;
#pragma unroll
    for (int c = 0; c < GS; ++c) dst[c] = 0.f;
  }
  float T = Tf;
  float sacc = 0.f;  // sum over later Gaussians of w_l (G . c_l)
  const float amin = rc.alpha_min, amax = rc.alpha_max;
  for (int hi = (int)nproc; hi > 0; hi -= kBwdBatch) {
    const int lo = hi - kBwdBatch > 0 ? hi - kBwdBatch : 0;
    const int cnt = hi - lo;
    __syncthreads();
    if (t < cnt) {
      const uint32_t gid = pairgid[rg.x + lo + t];
      sg[2 * t] = geom[2 * (size_t)gid];
      sg[2 * t + 1] = geom[2 * (size_t)gid + 1];
#pragma unroll
      for (int c = 0; c < CS4; ++c) sc[t * CS4 + c] = chan4[(size_t)gid * CS4 + c];
    }
    __syncthreads();
    for (int jj = cnt - 1; jj >= 0; --jj) {
      const int pos = lo + jj;
      float gv[GS];
#pragma unroll
      for (int c = 0; c < GS; ++c) gv[c] = 0.f;
      bool contrib = false;
      if ((uint32_t)pos < last) {
        const float4 g0 = sg[2 * jj];
        const float4 g1 = sg[2 * jj + 1];
        float dx, dy;
        const float power = eval_power(g0.x, g0.y, g0.z, g0.w, g1.x, pxf, pyf, dx, dy);
        if (power <= 0.f) {
          const float e = __expf(power);
          const float raw = g1.y * e;
          const float alpha = fminf(amax, raw);
          if (alpha >= amin) {
            contrib = true;
            const float oma = 1.f - alpha;
            const float ioma = __builtin_amdgcn_rcpf(oma);
            T = T * ioma;
            const float w = alpha * T;
            float dotg = 0.f;
#pragma unroll
            for (int c4 = 0; c4 < CS4; ++c4) {
              const float4 v = sc[jj * CS4 + c4];
              dotg = fmaf(G[4 * c4 + 0], v.x, dotg);
              dotg = fmaf(G[4 * c4 + 1], v.y, dotg);
              dotg = fmaf(G[4 * c4 + 2], v.z, dotg);
              dotg = fmaf(G[4 * c4 + 3], v.w, dotg);
            }
#pragma unroll
            for (int c = 0; c < CS; ++c) gv[6 + c] = w * G[c];
            const float dalpha = T * dotg - (sacc + GT * Tf) * ioma;
            sacc = fmaf(w, dotg, sacc);
            if (raw < amax) {
              const float dp = dalpha * alpha;
              gv[0] = -dp * (g0.z * dx + g0.w * dy);
              gv[1] = -dp * (g0.w * dx + g1.x * dy);
              gv[2] = -0.5f * dp * dx * dx;
              gv[3] = -dp * dx * dy;
              gv[4] = -0.5f * dp * dy * dy;
              gv[5] = dalpha * e;
            }
          }
        }
      }
      const int row = wv * 4 + (lane >> 4);
      if (__ballot(contrib) != 0ull) {
#pragma unroll
        for (int c = 0; c < GS; ++c) {
          const float s = row_sum(gv[c]);
          if ((lane & 15) == 0) part[jj][c][row] = s;
        }
      } else if ((lane & 15) < GS) {
        for (int c = lane & 15; c < GS; c += 16) part[jj][c][row] = 0.f;
      }
    }
    __syncthreads();
    for (int e = t; e < cnt * GS; e += kTilePix) {
      const int jj = e / GS, c = e - jj * GS;
      float s = 0.f;
#pragma unroll
      for (int r = 0; r < NR; ++r) s += part[jj][c][r];
      gslot[(size_t)pslot[rg.x + lo + jj] * GS + c] = s;
    }
  }
}

}  // namespace

void launch_blend_forward(const RenderConst& rc, const CtxLayout& L, char* ctx, const asgs_images& out,
                          hipStream_t s) {
  const ViewDev* views = reinterpret_cast<const ViewDev*>(ctx + L.views);
  if (rc.nf == 16)
    hipLaunchKernelGGL(k_blend_fwd<16>, dim3(rc.total_tiles), dim3(kTilePix), 0, s, rc, views, ctx, L, out);
  else
    hipLaunchKernelGGL(k_blend_fwd<0>, dim3(rc.total_tiles), dim3(kTilePix), 0, s, rc, views, ctx, L, out);
}

void launch_blend_backward(const RenderConst& rc, const CtxLayout& L, char* ctx, const asgs_images& dout,
                           hipStream_t s) {
  const ViewDev* views = reinterpret_cast<const ViewDev*>(ctx + L.views);
  if (rc.nf == 16)
    hipLaunchKernelGGL(k_blend_bwd<16>, dim3(rc.total_tiles), dim3(kTilePix), 0, s, rc, views, ctx, L, dout);
  else
    hipLaunchKernelGGL(k_blend_bwd<0>, dim3(rc.total_tiles), dim3(kTilePix), 0, s, rc, views, ctx, L, dout);
}

}  // namespace asgs
