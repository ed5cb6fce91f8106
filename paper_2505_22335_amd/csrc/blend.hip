// Front-to-back alpha compositing of colour, depth and the low-dimensional
// feature (UP-SLAM Sec. 3.1 Eq. 3, Sec. 3.3 Eq. 10) and its backward.
//
// One workgroup per 16x16 screen tile; each wave covers an 8x8 quarter of it
// (the forward has two waves per quarter, see k_blend_fwd). The tile's
// depth-ordered list is staged through LDS in rounds of records; a wave visits
// only the entries whose alpha >= alpha_min ellipse can reach its quarter;
// each pixel skips alpha < alpha_min, stops before the transmittance would
// fall below T_min, and accumulates w = alpha * T times (rgb, z, feature).
// The workgroup leaves as soon as every pixel has stopped.
//
// The backward replays each pixel's list back to front from its last
// composited Gaussian, recovering T_k = T_{k+1} / (1 - alpha_k), and sums each
// entry's gradient over the tile's pixels on the matrix cores (see
// k_blend_bwd); every entry's gradient slot is written once, without global
// atomics. The projection backward then sums each Gaussian's slots.
#include "internal.h"

namespace asgs {

namespace {

// Pixel of thread t: wave w covers the 8x8 quarter (w & 1, w >> 1) of the
// tile, lane l the pixel (l & 7, l >> 3) inside it. Square quarters keep the
// per-wave culling below tight.
ASGS_DEV int tile_lx(int t) { return ((t >> 6) & 1) * 8 + (t & 7); }
ASGS_DEV int tile_ly(int t) { return ((t >> 7) & 1) * 8 + ((t >> 3) & 7); }

// Issue priority of a tile's waves by its rank in the blend order (longest
// list first). The first workgroups of a launch spread over the compute units,
// so the longest list on each unit gets the highest priority, the next one the
// next level: the tiles on the critical path of the launch are preferred over
// the shorter ones sharing their SIMDs (the order of the results does not
// change).
ASGS_DEV void prioritise(uint32_t rank, int n_cu) {
  const uint32_t band = rank / (uint32_t)(n_cu > 0 ? n_cu : 1);
  if (band == 0u) __builtin_amdgcn_s_setprio(3);
  else if (band == 1u) __builtin_amdgcn_s_setprio(2);
  else if (band == 2u) __builtin_amdgcn_s_setprio(1);
}

// Which of the tile's four 8x8 quarters (bit w) hold a pixel centre that can
// pass the alpha test power >= ln(alpha_min / o) of an entry: a conservative
// test against the bounding box of the ellipse d^T Q d <= 2 L, Q = [[A, B],
// [B, C]], L = -ln(alpha_min / o), whose half extents are sqrt(2 L C / det Q)
// and sqrt(2 L A / det Q). The box is computed in FP64 from the stored FP32
// conic and widened by a relative 1e-3 + 2e-6 cond(Q) (covering the FP32
// rounding of the per-pixel power, whose error grows with the condition
// number) plus 0.01 px; entries too ill-conditioned for that bound are kept
// everywhere. Entries whose threshold no pixel can reach (o < alpha_min, or
// a NaN threshold) are dropped everywhere.
ASGS_DEV uint32_t quarter_mask(const float4& g0, const float4& g1, int x0, int y0) {
  const float lnthr = g1.z;
  if (!(lnthr <= 0.f)) return 0u;
  const double a = g0.z, b = g0.w, c = g1.x;
  const double det = a * c - b * b;
  if (!(det > 0.0) || !(a > 0.0) || !(c > 0.0)) return 0xFu;
  const double half_tr = 0.5 * (a + c);
  const double disc = sqrt(0.25 * (a - c) * (a - c) + b * b);
  const double lmax = half_tr + disc;
  const double cond = lmax * lmax / det;  // lmax / lmin
  const double rel = 1e-3 + 2e-6 * cond;
  if (!(rel < 0.25)) return 0xFu;
  const double L2 = -2.0 * (double)lnthr;
  const double hx = sqrt(L2 * c / det) * (1.0 + rel) + 0.01;
  const double hy = sqrt(L2 * a / det) * (1.0 + rel) + 0.01;
  const double u = g0.x, v = g0.y;
  uint32_t m = 0u;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const double sx = x0 + 8 * (w & 1), sy = y0 + 8 * (w >> 1);
    if (u + hx >= sx && u - hx <= sx + 7.0 && v + hy >= sy && v - hy <= sy + 7.0) m |= 1u << w;
  }
  return m;
}

constexpr int kFwdThreads = 2 * kTilePix;  // two waves per 8x8 quarter: front and back half of its list
constexpr int kSplitMin = 16;             // a round's quarter list shorter than this stays on the front wave

// Forward compositing, one 512-thread workgroup per tile. Each 8x8 quarter
// of the tile has two waves. Per round of staged list entries, the quarter's
// entries that can reach one of its pixels are split in list order: the
// front wave composites the first half onto the running state (T, channels,
// last contributor), the back wave the second half from T = 1 at the same
// time; then the front wave appends the back half's result,
//   C <- C + T C_back,  T <- T T_back,
// which equals compositing the two halves in order as long as the
// transmittance cannot have crossed T_min inside the back half
// (T T_back >= T_min, T being monotone). Pixels where it could re-run the
// back half on the front wave with the sequential rule.
//
// With L1, the output stage also forms the weighted L1 residual of the maps
// against the targets and its gradient (the terms of the L1 loss kernel, in
// the same arithmetic), and each quarter's loss partial.
ASGS_DEV float l1_sgn(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

template <int NF, bool L1>
__global__ void __launch_bounds__(kFwdThreads) k_blend_fwd(RenderConst rc, const ViewDev* __restrict__ views,
                                                           char* ctx, CtxLayout L, asgs_images out, BlendL1 l1) {
  constexpr int CS = 4 + NF;
  constexpr int CS4 = CS / 4;
  uint4* binfo = ctx_ptr<uint4>(ctx, L.binfo);
  const uint4 bi = binfo[blockIdx.x];  // longest lists first
  const int tile = (int)bi.x;
  const int view = find_view(views, rc.n_views, tile);
  const ViewDev& V = views[view];
  const int lt = tile - V.tile_base;
  const int ty = lt / V.TX, tx = lt - ty * V.TX;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int qd = wv & 3;         // quarter
  const bool back = wv >= 4;     // back half of the quarter's list
  const int tq = (qd << 6) | lane;
  const int x0 = tx * kTile, y0 = ty * kTile;
  const int px = x0 + tile_lx(tq);
  const int py = y0 + tile_ly(tq);
  const bool inside = px < V.W && py < V.H;
  const float pxf = (float)px, pyf = (float)py;
  const uint2 rg = make_uint2(bi.y, bi.z);
  prioritise(blockIdx.x, rc.n_cu);
  const uint32_t* pairgid = ctx_ptr<const uint32_t>(ctx, L.pairgid);
  const float4* geom = ctx_ptr<const float4>(ctx, L.geom);
  const float4* chan4 = ctx_ptr<const float4>(ctx, L.chan);
  uint8_t* pmask = ctx_ptr<uint8_t>(ctx, L.pmask);
  // lists walked by several backward workgroups: staged kSeg entries at a
  // time, with the pixel's state recorded at every segment boundary
  static_assert(kSeg * 2 == kTilePix && split_floats(CS) == ((kSegMax - 1) * split_first(CS) + split_final(CS)) * kTilePix,
                "segment layout");
  const uint32_t sl = ctx_ptr<const uint32_t>(ctx, L.bslot)[tile];  // 1 + split-record slot, or 0
  const int nseg = sl ? split_segments(rg.y - rg.x) : 1;
  const uint32_t rstep = nseg > 1 ? (uint32_t)kSeg : (uint32_t)kTilePix;  // entries staged per round
  constexpr int SA = split_first(CS), SF = split_final(CS);
  float* sp = ctx_ptr<float>(ctx, L.split) + (size_t)(sl ? sl - 1u : 0u) * split_floats(CS);

  __shared__ float4 sg[kTilePix * 2];
  __shared__ float4 sc[kTilePix * CS4];
  __shared__ uint8_t smask[kTilePix];
  __shared__ uint16_t swl[kFwdThreads / 64][kTilePix];
  __shared__ float xch[4][CS + 2][64];  // back-half state per quarter pixel: T, channels, last
  __shared__ uint64_t qdone[4];         // front lanes already stopped, per quarter

  // L1 targets and weight of the pixel, requested now and used in the output stage
  float tv[CS + 1], tw = 1.f;
  if (L1) {
#pragma unroll
    for (int c = 0; c <= CS; ++c) tv[c] = 0.f;
    if (!back && inside) {
      const size_t HW = (size_t)V.W * V.H;
      const size_t pix = (size_t)py * V.W + px;
      const size_t pb = (size_t)V.pix_base;
      if (l1.w) tw = l1.w[pix];
      if (l1.t[0])
        for (int c = 0; c < 3; ++c) tv[c] = l1.t[0][3 * pb + c * HW + pix];
      if (l1.t[1]) tv[3] = l1.t[1][pb + pix];
      if (NF > 0 && l1.t[2]) {
#pragma unroll
        for (int c = 0; c < NF; ++c) tv[4 + c] = l1.t[2][NF * pb + c * HW + pix];
      }
      if (l1.t[3]) tv[CS] = l1.t[3][pb + pix];
    }
  }

  float T = 1.f;
  float acc[CS];
#pragma unroll
  for (int c = 0; c < CS; ++c) acc[c] = 0.f;
  uint32_t last = 0;
  bool done = back || !inside;  // back lanes keep no running state
  const float amax = rc.alpha_max, tmin = rc.T_min;
  // Composite list positions [i0, i1) of this wave's round list. real: the
  // running state with the T_min stop; otherwise a local back-half state.
  // The next entry's index and geometry are read from LDS while the current
  // one is composited.
  auto run = [&](int i0, int i1, uint32_t base, bool act, bool real) {
    if (i0 >= i1) return;
    int jn = __builtin_amdgcn_readfirstlane(swl[wv][i0]);
    float4 g0n = sg[2 * jn], g1n = sg[2 * jn + 1];
    for (int i = i0; i < i1; ++i) {
      const int j = jn;
      const float4 g0 = g0n, g1 = g1n;
      if (i + 1 < i1) {
        jn = __builtin_amdgcn_readfirstlane(swl[wv][i + 1]);
        g0n = sg[2 * jn];
        g1n = sg[2 * jn + 1];
      }
      float dx, dy;
      const float power = eval_power(g0.x, g0.y, g0.z, g0.w, g1.x, pxf, pyf, dx, dy);
      // alpha >= alpha_min  <=>  power >= ln(alpha_min / o) (record slot 6)
      const bool take = act && power <= 0.f && power >= g1.z;
      if (!__ballot(take)) continue;
      const float alpha = fminf(amax, g1.y * __expf(power));
      const float Tn = T * (1.f - alpha);
      const bool stop = real && take && Tn < tmin;
      if (take && !stop) {
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
      if (real && __ballot(stop)) {
        done = done || stop;
        act = act && !stop;
        if (__ballot(act) == 0) break;
      }
    }
  };
  // the Gaussian ids of the next round are read while this round is staged
  uint32_t gid_next = t < rstep && rg.x + t < rg.y ? pairgid[rg.x + t] : 0u;
  for (uint32_t base = rg.x; base < rg.y; base += rstep) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t p = base + t;
    if (t < rstep && p < rg.y) {
      const uint32_t gid = gid_next;
      const float4 g0 = geom[2 * (size_t)gid];
      const float4 g1 = geom[2 * (size_t)gid + 1];
      sg[2 * t] = g0;
      sg[2 * t + 1] = g1;
#pragma unroll
      for (int c = 0; c < CS4; ++c) sc[t * CS4 + c] = chan4[(size_t)gid * CS4 + c];
      const uint8_t m = (uint8_t)quarter_mask(g0, g1, x0, y0);
      smask[t] = m;
      pmask[p] = m;  // reused by the backward
      if (p + rstep < rg.y) gid_next = pairgid[p + rstep];
    }
    {
      const uint64_t dm = __ballot(done);
      if (!back && lane == 0) qdone[qd] = dm;
    }
    __syncthreads();
    const int cnt = (int)min(rstep, rg.y - base);
    // the quarter's entries of the round (those that can reach one of its
    // pixels), in list order, compacted into swl (the same list on both waves)
    int n = 0;
    for (int c64 = 0; c64 < cnt; c64 += 64) {
      const bool mine = c64 + lane < cnt && ((smask[c64 + lane] >> qd) & 1u);
      const uint64_t bits = __ballot(mine);
      if (mine) swl[wv][n + __builtin_amdgcn_mbcnt_hi((uint32_t)(bits >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bits, 0u))] = (uint16_t)(c64 + lane);
      n += __builtin_popcountll(bits);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int nf = n < kSplitMin ? n : (n + 1) / 2;
    if (back) {
      T = 1.f;
#pragma unroll
      for (int c = 0; c < CS; ++c) acc[c] = 0.f;
      last = 0u;
      const bool skip = !inside || ((qdone[qd] >> lane) & 1u);
      run(nf, n, base, !skip, false);
      xch[qd][0][lane] = T;
#pragma unroll
      for (int c = 0; c < CS; ++c) xch[qd][1 + c][lane] = acc[c];
      xch[qd][CS + 1][lane] = __uint_as_float(last);
    } else if (__ballot(!done)) {
      run(0, nf, base, !done, true);
    }
    __syncthreads();
    if (!back && nf != n) {
      // append the back half
      const float Tb = xch[qd][0][lane];
      const uint32_t lastb = __float_as_uint(xch[qd][CS + 1][lane]);
      const bool fix = !done && T * Tb < tmin;
      if (!done && !fix) {
#pragma unroll
        for (int c = 0; c < CS; ++c) acc[c] = fmaf(T, xch[qd][1 + c][lane], acc[c]);
        T *= Tb;
        if (lastb) last = lastb;
      }
      if (__ballot(fix)) run(nf, n, base, fix, true);
    }
    const int bnd = (int)((base - rg.x) / kSeg) + 1;  // segment boundary after this round
    if (nseg > 1 && !back && bnd < nseg) {
      // state after the first bnd * kSeg entries
      float* rp = sp + ((size_t)(bnd - 1) * kTilePix + tq) * SA;
      float r[SA];
      r[0] = T;
#pragma unroll
      for (int c = 0; c < CS; ++c) r[1 + c] = acc[c];
#pragma unroll
      for (int c = 1 + CS; c < SA; ++c) r[c] = 0.f;
#pragma unroll
      for (int c4 = 0; c4 < SA / 4; ++c4)
        reinterpret_cast<float4*>(rp)[c4] = make_float4(r[4 * c4], r[4 * c4 + 1], r[4 * c4 + 2], r[4 * c4 + 3]);
    }
  }
  if (nseg > 1 && !back) {
    // the final channels (the entries after a boundary add C_final - C_boundary)
    float* rp = sp + (size_t)(kSegMax - 1) * kTilePix * SA + (size_t)tq * SF;
    float r[SF];
#pragma unroll
    for (int c = 0; c < SF; ++c) r[c] = c < CS ? acc[c < CS ? c : 0] : 0.f;
#pragma unroll
    for (int c4 = 0; c4 < SF / 4; ++c4)
      reinterpret_cast<float4*>(rp)[c4] = make_float4(r[4 * c4], r[4 * c4 + 1], r[4 * c4 + 2], r[4 * c4 + 3]);
  }
  // the list length the backward walks: the tile's largest last contributor
  if (!back) {
    uint32_t lm = inside ? last : 0u;
    for (int o = 32; o > 0; o >>= 1) lm = max(lm, (uint32_t)__shfl_xor((int)lm, o));
    if (lane == 0 && lm > 0u) {
      atomicMax(&binfo[blockIdx.x].w, lm);
      if (sl) atomicMax(&ctx_ptr<uint4>(ctx, L.sinfo)[sl - 1u].w, lm);
    }
  }
  if (back) return;
  float lsum = 0.f;  // this pixel's L1 loss terms
  if (inside) {
    const size_t HW = (size_t)V.W * V.H;
    const size_t pix = (size_t)py * V.W + px;
    const size_t pb = (size_t)V.pix_base;
    float map[CS + 1];  // rgb, depth, feature, opacity sum
    map[0] = acc[0] + T * rc.bg[0];
    map[1] = acc[1] + T * rc.bg[1];
    map[2] = acc[2] + T * rc.bg[2];
#pragma unroll
    for (int c = 3; c < CS; ++c) map[c] = acc[c];
    map[CS] = 1.f - T;
#pragma unroll
    for (int c = 0; c < 3; ++c) out.rgb[3 * pb + c * HW + pix] = map[c];
    out.depth[pb + pix] = map[3];
    if (NF > 0) {
#pragma unroll
      for (int c = 0; c < NF; ++c) out.feat[NF * pb + c * HW + pix] = map[4 + c];
    }
    out.alpha[pb + pix] = map[CS];
    ctx_ptr<float>(ctx, L.tfinal)[pb + pix] = T;
    ctx_ptr<uint32_t>(ctx, L.ncontrib)[pb + pix] = last;
    if (L1) {
      const float w = tw;
      // group q: channels [c0, c0 + nc) of the maps, plane base of view v
      auto group = [&](int q, int c0, int nc, size_t vbase) {
        float* g = l1.g[q];
        if (!l1.t[q]) {
          if (g)
            for (int c = 0; c < nc; ++c) g[vbase + c * HW + pix] = 0.f;
          return;
        }
        float l = 0.f;
        for (int c = 0; c < nc; ++c) {
          const float d = map[c0 + c] - tv[c0 + c];
          l += fabsf(d);
          if (g) g[vbase + c * HW + pix] = w * l1_sgn(d) * l1.s[q];
        }
        lsum += w * l * l1.s[q];
      };
      group(0, 0, 3, 3 * pb);
      group(1, 3, 1, pb);
      if (NF > 0) group(2, 4, NF, NF * pb);
      group(3, CS, 1, pb);
    }
  }
  if (L1) {
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
    if (lane == 0) ctx_ptr<float>(ctx, L.lpart)[4 * tile + qd] = lsum;
  }
}

// Per view: the fused forward's loss, a fixed-order sum of its tiles' quarter
// partials.
__global__ void __launch_bounds__(256) k_l1_tile_loss(const ViewDev* __restrict__ views, const float* lpart,
                                                      float* loss) {
  __shared__ float red[256 / 64];
  const ViewDev& V = views[blockIdx.x];
  const int nt = V.TX * V.TY;
  float s = 0.f;
  for (int t = threadIdx.x; t < nt; t += blockDim.x) {
    const float* p = lpart + 4 * (size_t)(V.tile_base + t);
    s += (p[0] + p[1]) + (p[2] + p[3]);
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) loss[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

constexpr int kBwdBatch = 16;  // list entries per MFMA tile (M = 16)

typedef float f4v __attribute__((ext_vector_type(4)));

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

ASGS_DEV f4v mfma_bf(const bf8v& a, const bf8v& b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// v = hi + lo with hi = bf16(v) and lo = bf16(v - hi), both rounded to nearest
// even: |v - hi - lo| <= 2^-17 |v| for finite v. With exact bf16 products and
// FP32 accumulation, a b ~ ah bh + ah bl + al bh to ~2^-15 relative.
// Round to nearest even bfloat16 (the hardware conversion of gfx950).
ASGS_DEV uint16_t bf_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
// v = hi + lo + O(2^-16 |v|), both bfloat16.
ASGS_DEV void bf_split(float v, uint16_t& hi, uint16_t& lo) {
  hi = bf_rne(v);
  lo = bf_rne(v - __uint_as_float((uint32_t)hi << 16));
}

// Backward compositing, one workgroup per tile (or per 128-entry segment of
// a split list), one pixel per thread.
//
// Per list entry k and pixel p the gradient contributions are
//   dL/dc_k      += w_kp G_p                 (w = alpha T, G = upstream channel gradients)
//   dL/dpower_kp  = dL/dalpha_kp * alpha_kp  (0 when alpha is clamped)
//   dL/do_k      += dL/dpower_kp / o_k
//   dL/du_k       = -sum_p dpow (A dx + B dy), ...  with dx = u - px, dy = v - py
// so the per-entry sums over the tile's pixels are dot products of two
// per-pixel coefficients (w, dpow) with fixed per-pixel features: the
// channel gradients G_p and the moments (1, lx, ly, lx^2, lx ly, ly^2) of the
// tile-local pixel coordinates, from which the conic and position gradients
// follow in closed form. The list is staged in rounds of 32 entries from the
// back. Each wave takes only the round's entries that one of its pixels uses
// (the quarter test of the forward, then a ballot), writes its pixels'
// coefficients for batches of up to 16 such entries to LDS and contracts them
// on the matrix cores (bf16 16x16x32 MFMAs with both operands split into
// hi + lo parts, K = pixels) into per-wave partial rows; the four waves' rows
// are summed in a fixed order and written once to each entry's gradient slot.
// A segment of a split list starts from the state the forward recorded at the
// segment's end: T there and the sum the later entries contribute,
// G . (C_final - C_boundary), instead of T_final and zero.
template <int NF>
__global__ void __launch_bounds__(kTilePix) __attribute__((amdgpu_waves_per_eu(3))) k_blend_bwd(RenderConst rc, const ViewDev* __restrict__ views,
                                                        char* ctx, CtxLayout L, asgs_images dout) {
  constexpr int CS = 4 + NF;
  constexpr int CS4 = CS / 4;
  constexpr int GS = 6 + CS;
  constexpr int NW = kTilePix / 64;
  constexpr int CP = 64;          // row of 64 pixel coefficients (bf16), 8-pixel groups XOR-swizzled by row
  // The first n_views kSplitPerView (kSegMax - 1) workgroups take the
  // segments but the last of the split lists, one split-record slot each
  // (and exit at once where there is none), the rest one blend position each
  // (longest lists first): the whole walked list, or its last segment.
  const uint32_t extra = (uint32_t)rc.n_views * kSplitPerView * (kSegMax - 1);
  const bool front = blockIdx.x < extra;
  uint4 bi;
  uint32_t slot;
  int nseg, seg;
  if (front) {
    slot = blockIdx.x / (kSegMax - 1);
    bi = ctx_ptr<const uint4>(ctx, L.sinfo)[slot];
    if (bi.x == ~0u) return;
    nseg = split_segments(bi.z - bi.y);
    seg = (int)(blockIdx.x % (kSegMax - 1));
    if (seg >= nseg - 1) return;
  } else {
    bi = ctx_ptr<const uint4>(ctx, L.binfo)[blockIdx.x - extra];
    const uint32_t sl = ctx_ptr<const uint32_t>(ctx, L.bslot)[bi.x];
    slot = sl ? sl - 1u : 0u;
    nseg = sl ? split_segments(bi.z - bi.y) : 1;
    seg = nseg - 1;
  }
  const int tile = (int)bi.x;
  const int view = find_view(views, rc.n_views, tile);
  const ViewDev& V = views[view];
  const int lt = tile - V.tile_base;
  const int ty = lt / V.TX, tx = lt - ty * V.TX;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int x0 = tx * kTile, y0 = ty * kTile;
  const int px = x0 + tile_lx(t);
  const int py = y0 + tile_ly(t);
  const bool inside = px < V.W && py < V.H;
  const float pxf = (float)px, pyf = (float)py;
  const uint2 rg = make_uint2(bi.y, bi.z);
  prioritise(blockIdx.x, rc.n_cu);
  const uint32_t len = rg.y - rg.x;
  const uint32_t nproc = bi.w;  // entries behind every pixel's last Gaussian are not walked
  // this workgroup's entries [elo, ehi) of the walked list
  const bool lastseg = seg == nseg - 1;
  const int elo = seg * kSeg;
  const int ehi = lastseg ? (int)nproc : min((int)nproc, (seg + 1) * kSeg);
  const uint32_t* pairgid = ctx_ptr<const uint32_t>(ctx, L.pairgid);
  const uint32_t* pslot = ctx_ptr<const uint32_t>(ctx, L.pslot);
  const float4* geom = ctx_ptr<const float4>(ctx, L.geom);
  const float4* chan4 = ctx_ptr<const float4>(ctx, L.chan);
  const uint8_t* pmask = ctx_ptr<const uint8_t>(ctx, L.pmask);
  float* gslot = ctx_ptr<float>(ctx, L.gslot);

  constexpr int kRecF4 = 2 + CS4;  // float4 per list entry: geometry (2) + channels
  constexpr int kRound = 32;       // list entries staged per round (one per lane of half a wave)
  constexpr int kPer = (kRound * kRecF4 + kTilePix - 1) / kTilePix;
  constexpr int PS = (GS + 3) & ~3;  // row of a partial-sum entry and of a gradient slot (whole float4)
  __shared__ float4 srec[kRound * kRecF4];
  // per wave, per batch position and pixel: w and dL/dpower as bf16 hi + lo
  // (one array: before the first batch it holds each wave's channel gradients
  // for the exchange into the MFMA operand layout)
  __shared__ __attribute__((aligned(16))) uint16_t acf[4][NW][kBwdBatch][CP];
  uint16_t (&awh)[NW][kBwdBatch][CP] = acf[0];
  uint16_t (&awl)[NW][kBwdBatch][CP] = acf[1];
  uint16_t (&aph)[NW][kBwdBatch][CP] = acf[2];
  uint16_t (&apl)[NW][kBwdBatch][CP] = acf[3];
  __shared__ __attribute__((aligned(16))) float part[NW][kRound][PS];  // per-wave partial rows of the round's entries
  __shared__ int sent[NW][kBwdBatch];     // round entry of each batch position
  __shared__ uint32_t sslot[2][kRound];   // gradient slot of each round entry (two rounds in flight)
  __shared__ uint8_t smk[kRound];         // quarter mask of each round entry (from the forward)

  // The Gaussian ids of the first round (the back kRound entries of the
  // walked list) are requested before anything else.
  uint32_t gid_next[kPer];
  auto fetch_gid = [&](int lo_r, int cnt_r) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int ent = (t + k * kTilePix) / kRecF4;
      gid_next[k] = ent < cnt_r ? pairgid[rg.x + lo_r + ent] : 0u;
    }
  };
  int rhi = ehi;
  int rlo = rhi - kRound > elo ? rhi - kRound : elo;
  if (rhi > elo) fetch_gid(rlo, rhi - rlo);
  const size_t HW = (size_t)V.W * V.H;
  const size_t pb = (size_t)V.pix_base;
  float Tf = 1.f;
  uint32_t last = 0;
  float G[CS];
#pragma unroll
  for (int c = 0; c < CS; ++c) G[c] = 0.f;
  float GT = 0.f;
  if (inside) {
    const size_t pix = (size_t)py * V.W + px;
    Tf = ctx_ptr<const float>(ctx, L.tfinal)[pb + pix];
    last = ctx_ptr<const uint32_t>(ctx, L.ncontrib)[pb + pix];
    for (int c = 0; c < 3; ++c) G[c] = dout.rgb[3 * pb + c * HW + pix];
    G[3] = dout.depth[pb + pix];
#pragma unroll
    for (int c = 0; c < NF; ++c) G[4 + c] = dout.feat[NF * pb + c * HW + pix];
    const float ga = dout.alpha ? dout.alpha[pb + pix] : 0.f;
    GT = rc.bg[0] * G[0] + rc.bg[1] * G[1] + rc.bg[2] * G[2] - ga;
  }
  // B operands of the MFMAs (v_mfma_f32_16x16x32_bf16): K block kb covers
  // pixels 32 kb .. 32 kb + 31 of this wave; lane l supplies feature l % 16 of
  // pixels 32 kb + 8 (l / 16) + i, i = 0..7: the channel gradients split into
  // bf16 hi + lo, the pixel-coordinate moments (small integers, exact). The
  // gradients reach that layout through the wave's rows of LDS (stride GXS,
  // so that the 16 channel rows of one read fall in different banks).
  constexpr int GXS = 68;
  static_assert(NW * CS * GXS * 4 <= (int)sizeof(acf), "exchange rows fit the coefficient array");
  float* gx = reinterpret_cast<float*>(&acf[0][0][0][0]) + wv * CS * GXS;
#pragma unroll
  for (int c = 0; c < CS; ++c) gx[c * GXS + lane] = G[c];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int fcol = lane & 15;
  bf8v bG0h[2], bG0l[2], bG1h[2], bG1l[2], bM[2];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) {
    const int q0 = 32 * kb + 8 * (lane >> 4);  // first of the lane's 8 pixels in the wave
    float g0[8], g1[8];
    if (fcol < CS) {
      const float4 a = *reinterpret_cast<const float4*>(&gx[fcol * GXS + q0]);
      const float4 b = *reinterpret_cast<const float4*>(&gx[fcol * GXS + q0 + 4]);
      g0[0] = a.x; g0[1] = a.y; g0[2] = a.z; g0[3] = a.w;
      g0[4] = b.x; g0[5] = b.y; g0[6] = b.z; g0[7] = b.w;
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) g0[i] = 0.f;
    }
    if (16 + fcol < CS) {
      const float4 a = *reinterpret_cast<const float4*>(&gx[(16 + fcol) * GXS + q0]);
      const float4 b = *reinterpret_cast<const float4*>(&gx[(16 + fcol) * GXS + q0 + 4]);
      g1[0] = a.x; g1[1] = a.y; g1[2] = a.z; g1[3] = a.w;
      g1[4] = b.x; g1[5] = b.y; g1[6] = b.z; g1[7] = b.w;
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) g1[i] = 0.f;
    }
    uint16_t h0[8], l0[8], h1[8], l1[8], m[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int q = 64 * wv + q0 + i;  // pixel of thread q
      bf_split(g0[i], h0[i], l0[i]);
      bf_split(g1[i], h1[i], l1[i]);
      const float fx = (float)tile_lx(q), fy = (float)tile_ly(q);
      m[i] = bf_rne(fcol == 0 ? 1.f : fcol == 1 ? fx : fcol == 2 ? fy : fcol == 3 ? fx * fx
                    : fcol == 4 ? fx * fy : fcol == 5 ? fy * fy : 0.f);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      bG0h[kb][i] = __builtin_bit_cast(__bf16, h0[i]);
      bG0l[kb][i] = __builtin_bit_cast(__bf16, l0[i]);
      bG1h[kb][i] = __builtin_bit_cast(__bf16, h1[i]);
      bG1l[kb][i] = __builtin_bit_cast(__bf16, l1[i]);
      bM[kb][i] = __builtin_bit_cast(__bf16, m[i]);
    }
  }

  // entries behind every pixel's last Gaussian get zero gradient
  for (uint32_t q = nproc + t; lastseg && q < len; q += kTilePix) {
    float4* dst = reinterpret_cast<float4*>(gslot + (size_t)pslot[rg.x + q] * PS);
#pragma unroll
    for (int c = 0; c < PS / 4; ++c) dst[c] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  float T = Tf;
  float sacc = 0.f;  // sum over later Gaussians of w_l (G . c_l)
  if (!lastseg && ehi == (seg + 1) * kSeg && inside) {
    // the state at the segment's end (a boundary the forward passed): T
    // there, and the later entries' sum, G . (C_final - C_boundary)
    constexpr int SA = split_first(CS), SF = split_final(CS);
    const float* sp = ctx_ptr<const float>(ctx, L.split) + (size_t)slot * split_floats(CS);
    const float4* rb = reinterpret_cast<const float4*>(sp + ((size_t)seg * kTilePix + t) * SA);
    const float4* rf = reinterpret_cast<const float4*>(sp + (size_t)(kSegMax - 1) * kTilePix * SA + (size_t)t * SF);
    float r[SA], f[SF];
#pragma unroll
    for (int c4 = 0; c4 < SA / 4; ++c4) {
      const float4 v = rb[c4];
      r[4 * c4] = v.x;
      r[4 * c4 + 1] = v.y;
      r[4 * c4 + 2] = v.z;
      r[4 * c4 + 3] = v.w;
    }
#pragma unroll
    for (int c4 = 0; c4 < SF / 4; ++c4) {
      const float4 v = rf[c4];
      f[4 * c4] = v.x;
      f[4 * c4 + 1] = v.y;
      f[4 * c4 + 2] = v.z;
      f[4 * c4 + 3] = v.w;
    }
    T = r[0];
#pragma unroll
    for (int c = 0; c < CS; ++c) sacc = fmaf(G[c], f[c] - r[1 + c], sacc);
  }
  const float amax = rc.alpha_max;
  // Records are staged in rounds of kRound entries, walking the list from the
  // back; the global loads of the next round are issued before the current
  // round is processed and land in LDS at the start of the next round.
  // The Gaussian ids of a round are read one round earlier still, so that
  // no load of the staging waits on another.
  float4 stage[kPer];
  uint32_t stage_slot = 0u, stage_mask = 0u;
  auto fetch = [&](int lo_r, int cnt_r) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = t + k * kTilePix;
      const int ent = e / kRecF4, f = e - ent * kRecF4;
      if (ent < cnt_r) {
        const uint32_t gid = gid_next[k];
        stage[k] = f < 2 ? geom[2 * (size_t)gid + f] : chan4[(size_t)gid * CS4 + (f - 2)];
      }
    }
    if (t < cnt_r) {
      stage_slot = pslot[rg.x + lo_r + t];
      stage_mask = pmask[rg.x + lo_r + t];
    }
  };
  auto rec_of = [&](int e) { return &srec[e * kRecF4]; };
  // Contract the wave's nb batched entries over its 64 pixels on the matrix
  // cores and store the rows of the partial sums under their round entries.
  auto flush = [&](int nb) {
    // the coefficients are read back by other lanes of this wave only
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    f4v c1 = {0.f, 0.f, 0.f, 0.f}, c2 = c1, c3 = c1;
    // A operands: batch position l % 16, pixels 32 kb + 8 (l / 16) .. + 7
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const int p0 = (32 * kb + 8 * (lane >> 4)) ^ ((fcol & 7) << 3);
      const bf8v wh = *reinterpret_cast<const bf8v*>(&awh[wv][fcol][p0]);
      const bf8v wl = *reinterpret_cast<const bf8v*>(&awl[wv][fcol][p0]);
      const bf8v ph = *reinterpret_cast<const bf8v*>(&aph[wv][fcol][p0]);
      const bf8v pl = *reinterpret_cast<const bf8v*>(&apl[wv][fcol][p0]);
      c1 = mfma_bf(wh, bG0h[kb], c1);
      c1 = mfma_bf(wh, bG0l[kb], c1);
      c1 = mfma_bf(wl, bG0h[kb], c1);
      if (CS > 16) {
        c2 = mfma_bf(wh, bG1h[kb], c2);
        c2 = mfma_bf(wh, bG1l[kb], c2);
        c2 = mfma_bf(wl, bG1h[kb], c2);
      }
      c3 = mfma_bf(ph, bM[kb], c3);
      c3 = mfma_bf(pl, bM[kb], c3);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pos = 4 * (lane >> 4) + r;
      if (pos < nb) {
        float* row = part[wv][sent[wv][pos]];
        if (fcol < CS) row[6 + fcol] = c1[r];
        if (CS > 16 && fcol < CS - 16) row[6 + 16 + fcol] = c2[r];
        if (fcol < 6) row[fcol] = c3[r];
      }
    }
    // the conic, position and opacity parts of the wave's rows in closed form
    // from its moment sums (linear in them, so the four waves' rows still add
    // up): all moments are read before any is overwritten
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float cf[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int it = lane + 64 * k;
      cf[k] = 0.f;
      if (it < nb * 6) {
        const int pos = it / 6, c = it - pos * 6;
        const int e = sent[wv][pos];
        const float* M = part[wv][e];
        const float4 g0 = rec_of(e)[0];
        const float4 g1 = rec_of(e)[1];
        const float uu = g0.x - (float)x0, vv = g0.y - (float)y0;  // tile-local centre
        const float Sdx = uu * M[0] - M[1];
        const float Sdy = vv * M[0] - M[2];
        if (c == 0) cf[k] = -(g0.z * Sdx + g0.w * Sdy);
        else if (c == 1) cf[k] = -(g0.w * Sdx + g1.x * Sdy);
        else if (c == 2) cf[k] = -0.5f * (uu * uu * M[0] - 2.f * uu * M[1] + M[3]);
        else if (c == 3) cf[k] = -(uu * vv * M[0] - uu * M[2] - vv * M[1] + M[4]);
        else if (c == 4) cf[k] = -0.5f * (vv * vv * M[0] - 2.f * vv * M[2] + M[5]);
        else cf[k] = M[0] / g1.y;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int it = lane + 64 * k;
      if (it < nb * 6) {
        const int pos = it / 6, c = it - pos * 6;
        part[wv][sent[wv][pos]][c] = cf[k];
      }
    }
    // the next batch overwrites the coefficients and the entry table
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  if (rhi > elo) {
    fetch(rlo, rhi - rlo);
    const int nrlo = rlo - kRound > elo ? rlo - kRound : elo;
    if (rlo > elo) fetch_gid(nrlo, rlo - nrlo);
  }
  // partial rows start at zero; the reduction of each round zeroes the rows
  // it has read
  for (int q = lane; q < kRound * PS; q += 64) (&part[wv][0][0])[q] = 0.f;
  int par = 0;  // sslot buffer of this round
  while (rhi > elo) {
    // Every wave has passed the previous round's candidate loop (the barrier
    // before its reduction), so the records and masks can be overwritten;
    // the slots the reduction still reads are in the other buffer.
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = t + k * kTilePix;
      if (e / kRecF4 < rhi - rlo) srec[e] = stage[k];
    }
    if (t < rhi - rlo) {
      sslot[par][t] = stage_slot;
      smk[t] = (uint8_t)stage_mask;
    }
    __syncthreads();  // staging visible; the previous reduction has zeroed its rows
    const int cnt = rhi - rlo;
    const int nrhi = rlo, nrlo = rlo - kRound > elo ? rlo - kRound : elo;
    if (nrhi > elo) {
      fetch(nrlo, nrhi - nrlo);
      const int n2lo = nrlo - kRound > elo ? nrlo - kRound : elo;
      if (nrlo > elo) fetch_gid(n2lo, nrlo - n2lo);
    }
    // entries of the round that can reach a pixel of this wave's quarter
    const bool mine = lane < cnt && ((smk[lane] >> wv) & 1u);
    uint64_t bits = __ballot(mine);
    int nb = 0;
    // back to front over this wave's entries; entries no pixel of the wave
    // uses are left out of the batches (their partial rows stay zero). Two
    // entries are taken at a time: everything that does not depend on T
    // (footprint, alpha, the channel dot product) is formed for both before
    // the T recursion consumes them in order, so the two chains overlap.
    struct Cand {
      int j;
      bool use;
      float raw, alpha, ioma, dotg;
    };
    auto prepare = [&](int j) {
      Cand c;
      c.j = j;
      const float4 g0 = srec[j * kRecF4];
      const float4 g1 = srec[j * kRecF4 + 1];
      float dx, dy;
      const float power = eval_power(g0.x, g0.y, g0.z, g0.w, g1.x, pxf, pyf, dx, dy);
      // same alpha threshold as the forward
      c.use = (uint32_t)(rlo + j) < last && power <= 0.f && power >= g1.z;
      c.raw = g1.y * __expf(power);
      c.alpha = fminf(amax, c.raw);
      c.ioma = __builtin_amdgcn_rcpf(1.f - c.alpha);
      float dot0 = 0.f, dot1 = 0.f;  // two independent chains
#pragma unroll
      for (int c4 = 0; c4 < CS4; ++c4) {
        const float4 v = srec[j * kRecF4 + 2 + c4];
        dot0 = fmaf(G[4 * c4 + 0], v.x, dot0);
        dot1 = fmaf(G[4 * c4 + 1], v.y, dot1);
        dot0 = fmaf(G[4 * c4 + 2], v.z, dot0);
        dot1 = fmaf(G[4 * c4 + 3], v.w, dot1);
      }
      c.dotg = dot0 + dot1;
      return c;
    };
    auto consume = [&](const Cand& c) {
      if (!__ballot(c.use)) return;
      float wgt = 0.f, dpow = 0.f;
      const float Tk = T * c.ioma;
      const float w_ = c.alpha * Tk;
      const float dalpha = Tk * c.dotg - (sacc + GT * Tf) * c.ioma;
      if (c.use) {
        T = Tk;
        wgt = w_;
        sacc = fmaf(w_, c.dotg, sacc);
        dpow = c.raw < amax ? dalpha * c.alpha : 0.f;
      }
      uint16_t hi, lo;
      const int sp = lane ^ ((nb & 7) << 3);  // swizzled position of this pixel in row nb
      bf_split(wgt, hi, lo);
      awh[wv][nb][sp] = hi;
      awl[wv][nb][sp] = lo;
      bf_split(dpow, hi, lo);
      aph[wv][nb][sp] = hi;
      apl[wv][nb][sp] = lo;
      if (lane == 0) sent[wv][nb] = c.j;
      ++nb;
    };
    while (bits) {
      const int j1 = 63 - __builtin_clzll(bits);
      bits &= ~(1ull << j1);
      if (nb > kBwdBatch - 2) {  // room for two more rows
        flush(nb);
        nb = 0;
      }
      const Cand c1 = prepare(j1);
      if (bits) {
        const int j2 = 63 - __builtin_clzll(bits);
        bits &= ~(1ull << j2);
        const Cand c2 = prepare(j2);
        consume(c1);
        consume(c2);
      } else {
        consume(c1);
      }
    }
    if (nb > 0) flush(nb);
    __syncthreads();
    // the four waves' rows -> one gradient slot per entry, a float4 per
    // thread; the rows read are zeroed for the next round
    constexpr int F4 = PS / 4;
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int q = t; q < cnt * F4; q += kTilePix) {
      const int e = q / F4, f = q - e * F4;
      const float4 a = reinterpret_cast<const float4*>(part[0][e])[f];
      const float4 b = reinterpret_cast<const float4*>(part[1][e])[f];
      const float4 c = reinterpret_cast<const float4*>(part[2][e])[f];
      const float4 d = reinterpret_cast<const float4*>(part[3][e])[f];
      reinterpret_cast<float4*>(gslot + (size_t)sslot[par][e] * PS)[f] =
          make_float4((a.x + b.x) + (c.x + d.x), (a.y + b.y) + (c.y + d.y), (a.z + b.z) + (c.z + d.z),
                      (a.w + b.w) + (c.w + d.w));
      reinterpret_cast<float4*>(part[0][e])[f] = z4;
      reinterpret_cast<float4*>(part[1][e])[f] = z4;
      reinterpret_cast<float4*>(part[2][e])[f] = z4;
      reinterpret_cast<float4*>(part[3][e])[f] = z4;
    }
    par ^= 1;
    rhi = nrhi;
    rlo = nrlo;
  }
}

}  // namespace

void launch_blend_forward(const RenderConst& rc, const CtxLayout& L, char* ctx, const asgs_images& out,
                          const BlendL1* l1, hipStream_t s) {
  const ViewDev* views = reinterpret_cast<const ViewDev*>(ctx + L.views);
  const BlendL1 a = l1 ? *l1 : BlendL1{};
  const dim3 grid(rc.total_tiles), block(kFwdThreads);
  if (rc.nf == 16) {
    if (l1) hipLaunchKernelGGL((k_blend_fwd<16, true>), grid, block, 0, s, rc, views, ctx, L, out, a);
    else hipLaunchKernelGGL((k_blend_fwd<16, false>), grid, block, 0, s, rc, views, ctx, L, out, a);
  } else {
    if (l1) hipLaunchKernelGGL((k_blend_fwd<0, true>), grid, block, 0, s, rc, views, ctx, L, out, a);
    else hipLaunchKernelGGL((k_blend_fwd<0, false>), grid, block, 0, s, rc, views, ctx, L, out, a);
  }
}

void launch_l1_tile_loss(const RenderConst& rc, const CtxLayout& L, char* ctx, float* loss, hipStream_t s) {
  const ViewDev* views = reinterpret_cast<const ViewDev*>(ctx + L.views);
  hipLaunchKernelGGL(k_l1_tile_loss, dim3(rc.n_views), dim3(256), 0, s, views,
                     reinterpret_cast<const float*>(ctx + L.lpart), loss);
}

void launch_blend_backward(const RenderConst& rc, const CtxLayout& L, char* ctx, const asgs_images& dout,
                           hipStream_t s) {
  const ViewDev* views = reinterpret_cast<const ViewDev*>(ctx + L.views);
  if (rc.nf == 16)
    hipLaunchKernelGGL(k_blend_bwd<16>, dim3(rc.total_tiles + rc.n_views * kSplitPerView * (kSegMax - 1)),
                       dim3(kTilePix), 0, s, rc,
                       views, ctx, L,
                       dout);
  else
    hipLaunchKernelGGL(k_blend_bwd<0>, dim3(rc.total_tiles + rc.n_views * kSplitPerView * (kSegMax - 1)),
                       dim3(kTilePix), 0, s, rc,
                       views, ctx, L,
                       dout);
}

}  // namespace asgs
