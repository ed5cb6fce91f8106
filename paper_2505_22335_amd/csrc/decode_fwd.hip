// Decoder forward on the matrix cores (UP-SLAM Eq. 8 and Eq. 9), FP32 or
// BF16. One
// workgroup of eight waves takes (16-anchor tile, view) items in turn: waves
// 0..3 each own one of the opacity, colour, scale and rotation heads, waves
// 4..7 share the feature head's output rows. Per item and head, with X the
// tile's inputs for the view (one row per anchor):
//   Z = X W1^T + b1, H = act(Z)                 (ReLU; SoftPlus for features)
//   Y = H W2^T + b2, decoded = out_act(Y)
// on FP32 16x16x4 MFMAs, with the operand layouts of the backward
// (decode_bwd.hip): Z is formed transposed (units x anchors), which is the B
// operand of Y without a transpose, and both layers' weights sit in registers
// for the whole kernel. The outputs are scattered into per-(head, component)
// plane runs in LDS and written as the tile's contiguous runs of 16 k values;
// the Gaussian means x_v + l_o O_i (view independent) go with the first view.
#include <math.h>

#include "decode_shared.h"

namespace asgs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kBW = 8;         // waves per workgroup
constexpr int kBT = 64 * kBW;  // threads per workgroup
constexpr int kXL = 52;        // LDS row of an anchor's inputs (35 + distance column, pad)
constexpr int kHB = 36;        // rows of the feature head's shared H (32 units + pad)
constexpr int kWL = 36;        // LDS rows of the weights in the prologue (35 or 32 + pad)
constexpr int kPlanes = 27;    // (head, component) planes: 1 + 3 + 3 + 4 + 16

// LDS carve (floats), for the largest k of an instantiation (12 with three
// row tiles per wave, else 16). The prologue's weight copy (first-layer rows
// of every head, second-layer rows, b1, b2) uses the output buffers' region.
constexpr int kOffX = 0;
constexpr int kOffHF = kOffX + 2 * 16 * kXL;
constexpr int kOffTW = kOffHF + 16 * kHB;  // temporal weights of every unit: [5 * 32][2]
constexpr int kOffOB = kOffTW + kHeads * kHid * 2;
template <int kR>
struct FwdLds {
  static constexpr int kK = kR == 3 ? 12 : ASGS_MAX_K;
  static constexpr int kOB = kPlanes * (16 * kK + 1);  // one output buffer: each plane's run + pad
  static constexpr int kWCopy = kHeads * kHid * kWL + 27 * kK * (kWL + 1) + 3 + kHeads * kHid;
  static constexpr int kFloats = kOffOB + (2 * kOB > kWCopy ? 2 * kOB : kWCopy);
};
static_assert(FwdLds<3>::kFloats * 4 <= 80 * 1024, "two workgroups per compute unit at k <= 12");

ASGS_DEV f4v mfma(float a, float b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// bfloat16 bits of a finite float, rounded to nearest even
ASGS_DEV unsigned f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
// eight floats as the bfloat16 operand of v_mfma_f32_16x16x32_bf16 (element j = K index 8 g + j)
ASGS_DEV bf8v pack_bf8(const float (&v)[8]) {
  u4v p;
#pragma unroll
  for (int i = 0; i < 4; ++i) p[i] = f2bf(v[2 * i]) | (f2bf(v[2 * i + 1]) << 16);
  return __builtin_bit_cast(bf8v, p);
}

// kBf: the BF16 decoder (operands of the feature columns of the first layer
// and of the second layer rounded to bfloat16, FP32 accumulation; the
// direction and distance columns, biases and activations in FP32)
template <int kR, bool kBf>
__global__ void __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(4, 4))) k_dec_fwd(DecodeConst dc, HeadTable ht, DecodeViews dv,
                                                    const float* __restrict__ xyz, const float* __restrict__ feat,
                                                    const float* __restrict__ off, const float* __restrict__ params,
                                                    asgs_gaussians out) {
  extern __shared__ __attribute__((aligned(16))) float smem[];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int fl = lane & 15, fg = lane >> 4;
  float (*const XB)[16][kXL] = reinterpret_cast<float (*)[16][kXL]>(smem + kOffX);
  float (*const HF)[kHB] = reinterpret_cast<float (*)[kHB]>(smem + kOffHF);
  float* const OB = smem + kOffOB;
  float* const TW = smem + kOffTW;
  // BF16: the feature columns 8 g .. 8 g + 7 of anchor f as the B operand of Z^T
  auto xbf = [&](int buf) {
    const f4v a = *reinterpret_cast<const f4v*>(&XB[buf][fl][8 * fg]);
    const f4v b = *reinterpret_cast<const f4v*>(&XB[buf][fl][8 * fg + 4]);
    const float v8[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    return pack_bf8(v8);
  };
  constexpr int kOB = FwdLds<kR>::kOB;
  const int A = (int)dc.A;
  const int k = dc.k;
  const int n = A * k;
  const int V = dc.n_views;
  const int nx = ht.nx;
  const bool has_feat = ht.m[4] > 0;
  // ---- this wave's head and output rows ----
  const int hd = wv < 4 ? wv : 4;
  const int q = wv - 4;  // index among the feature waves
  const bool active = wv < 4 || has_feat;
  const int m = ht.m[hd];
  const int rows = k * m;
  const int T = (rows + 15) / 16;
  int t0 = 0, nt = T;
  if (wv >= 4) {
    const int base = T / 4, extra = T - 4 * base;
    nt = base + (q < extra ? 1 : 0);
    t0 = q * base + (q < extra ? q : extra);
  }
  const int run = 16 * k, gstride = run + 1;  // output plane runs in LDS
  const int nplanes = has_feat ? kPlanes : 11;

  // ---- the weights into LDS (coalesced, every load of a thread before its
  // first store), then into registers ----
  float* const W1L = OB;                                   // [5 * 32][kWL]
  float* const W2L = W1L + kHeads * kHid * kWL;            // [all rows][kWL]
  const int nrows = ht.nrows;
  float* const B2L = W2L + nrows * kWL;
  float* const B1L = B2L + ((nrows + 3) & ~3);            // [5][32] (16-byte aligned)
  {
    constexpr int kK = FwdLds<kR>::kK;
    constexpr int kMs[kHeads] = {1, 3, 3, 4, 16};
    constexpr int kE1 = (kHid * kIn + kBT - 1) / kBT;
    constexpr int kE2m = (16 * kK * kHid + kBT - 1) / kBT;
    const int nh = has_feat ? kHeads : 4;
    float v1[kHeads][kE1], v2[kHeads][kE2m], vd[kHeads], vb1[kHeads], vb2[kHeads];
#pragma unroll
    for (int h = 0; h < kHeads; ++h) {
      if (h >= nh) break;
      const int o1 = (int)ht.off[h], rw = k * ht.m[h], w2 = o1 + kHid * kIn + kHid;
      const int ox = (int)ht.xoff[h];
#pragma unroll
      for (int qq = 0; qq < kE1; ++qq) {
        const int e = t + qq * kBT;
        v1[h][qq] = params[o1 + (e < kHid * kIn ? e : 0)];
      }
      const int ne2 = (kMs[h] * kK * kHid + kBT - 1) / kBT;  // a constant once unrolled
#pragma unroll
      for (int qq = 0; qq < kE2m; ++qq) {
        if (qq >= ne2) break;
        const int e = t + qq * kBT;
        v2[h][qq] = params[w2 + (e < rw * kHid ? e : 0)];
      }
      vd[h] = nx > 0 ? params[ox + (t & 31) * nx] : 0.f;
      vb1[h] = params[o1 + kHid * kIn + (t & 31)];
      vb2[h] = params[w2 + rw * kHid + (t < rw ? t : 0)];
    }
#pragma unroll
    for (int h = 0; h < kHeads; ++h) {
      if (h >= nh) break;
      const int rw = k * ht.m[h], r0 = ht.row0[h];
#pragma unroll
      for (int qq = 0; qq < kE1; ++qq) {
        const int e = t + qq * kBT;
        const int u = e / kIn, i = e - u * kIn;
        if (e < kHid * kIn) W1L[(h * kHid + u) * kWL + i] = v1[h][qq];
      }
      const int ne2 = (kMs[h] * kK * kHid + kBT - 1) / kBT;
#pragma unroll
      for (int qq = 0; qq < kE2m; ++qq) {
        if (qq >= ne2) break;
        const int e = t + qq * kBT;
        if (e < rw * kHid) W2L[(r0 + (e >> 5)) * kWL + (e & 31)] = v2[h][qq];
      }
      if (t < kHid) {
        W1L[(h * kHid + t) * kWL + kIn] = vd[h];  // the distance weight (zero without that input)
        B1L[h * kHid + t] = vb1[h];
        // the temporal weights (the time input is the same for every anchor of a view)
        TW[(h * kHid + t) * 2] = nx == 3 ? params[(int)ht.xoff[h] + t * 3 + 1] : 0.f;
        TW[(h * kHid + t) * 2 + 1] = nx == 3 ? params[(int)ht.xoff[h] + t * 3 + 2] : 0.f;
      }
      if (t < rw) B2L[r0 + t] = vb2[h];
    }
    // input columns past 35 are never read by the first layer; keep them finite
    for (int e = t; e < 2 * 16 * (kXL - 37); e += kBT) {
      const int row = e / (kXL - 37);
      XB[row >> 4][row & 15][37 + e - row * (kXL - 37)] = 0.f;
    }
  }
  __syncthreads();
  // first layer as the A operand of Z^T (unit 16 b + f, input 4 s + g); the
  // feature waves 0 and 1 form one unit block each
  float w1a[2][9], b1r[2][4];
  float w2y[kR][2][4], b2r[kR];
  // BF16: the feature columns as bfloat16 A operands (unit 16 b + f, inputs
  // 8 g .. 8 g + 7), the other four columns as FP32 (input 32 + g), and the
  // second layer as bfloat16 B operands with K index 8 g + j taken as unit
  // 4 g + j (j < 4) or 16 + 4 g + j - 4, the units the lane holds of H
  bf8v w1b[2], w2b[kR];
  float w1x[2];
  const int pb0 = hd == 0 ? 0 : hd == 1 ? 1 : hd == 2 ? 4 : hd == 3 ? 7 : 11;  // first plane of the head
  const int hr0 = ht.row0[hd];
  const int minv = (65536 + m - 1) / (m > 0 ? m : 1);  // o / m = (o * minv) >> 16, exact for o <= 256
  int ooff[kR];  // LDS output offset of the lane's row of row tile i (plus a k)
  bool rok[kR];
  {
    const int ub = wv < 4 ? 0 : (q & 1) * 16;  // unit offset of block 0
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const float* wrow = &W1L[(hd * kHid + ub + 16 * b + fl) * kWL];
      if constexpr (kBf) {
        float v8[8];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) v8[jj] = wrow[8 * fg + jj];
        w1b[b] = pack_bf8(v8);
        w1x[b] = wrow[32 + fg];
      } else {
#pragma unroll
        for (int s = 0; s < 9; ++s) w1a[b][s] = wrow[4 * s + fg];
      }
      const f4v v = *reinterpret_cast<const f4v*>(&B1L[hd * kHid + (ub + 16 * b + 4 * fg) % kHid]);
#pragma unroll
      for (int r = 0; r < 4; ++r) b1r[b][r] = v[r];
    }
  }
  const int tw0 = (hd * kHid + (wv < 4 ? 0 : (q & 1) * 16) + 4 * fg) * 2;  // the lane's first temporal pair
#pragma unroll
  for (int i = 0; i < kR; ++i) {
    const int o = 16 * (t0 + i) + fl;
    const bool ok = active && i < nt && o < rows;
    rok[i] = ok;
    const int oc = ok ? o : 0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const f4v v = *reinterpret_cast<const f4v*>(&W2L[(hr0 + oc) * kWL + 16 * b + 4 * fg]);
#pragma unroll
      for (int r = 0; r < 4; ++r) w2y[i][b][r] = ok ? v[r] : 0.f;
    }
    if constexpr (kBf) {
      float v8[8];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) v8[jj] = w2y[i][jj >> 2][jj & 3];
      w2b[i] = pack_bf8(v8);
    }
    b2r[i] = ok ? B2L[hr0 + oc] : 0.f;
    const int gi = (oc * minv) >> 16, gc = oc - gi * m;
    ooff[i] = (pb0 + gc) * gstride + gi;
  }
  __syncthreads();  // the weight copy is no longer read

  // ---- items (tile, view): inputs fetched an item ahead and staged through
  // LDS; the means of the tile's Gaussians fetched with the first view ----
  const int ngrid = (A + 15) / 16;
  float xv = 0.f, pv[3] = {0.f, 0.f, 0.f}, mx[2] = {0.f, 0.f}, mo[2] = {0.f, 0.f};
  // item j of this workgroup: tile blockIdx.x + (j / V) gridDim.x, view j % V
  auto fetch = [&](int tile, int view) {
    const int a0 = tile * 16, a = t >> 5, c = t & 31;
    const int ax = a0 + a < A ? a0 + a : 0, ap = a0 + (t & 15) < A ? a0 + (t & 15) : 0;
    xv = feat[(int64_t)ax * 32 + c];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) pv[cc] = xyz[(int64_t)cc * A + ap];
    if (view == 0) {
      // means: elements t and t + 512 of the tile's 3 x 16 k values (component-major)
#pragma unroll
      for (int c2 = 0; c2 < 2; ++c2) {
        const int e = t + c2 * kBT;
        const int cm = e / run, gl = e - cm * run;
        const int g = a0 * k + gl;
        const bool okm = cm < 3 && g < n;
        mo[c2] = off[okm ? (int64_t)cm * n + g : 0];
        mx[c2] = xyz[okm ? (int64_t)cm * A + g / k : 0];
      }
    }
  };
  auto put_x = [&](int buf, int tile, int view) {
    const int a0 = tile * 16;
    XB[buf][t >> 5][t & 31] = a0 + (t >> 5) < A ? xv : 0.f;
    if (t < 16) {
      float D[3] = {0.f, 0.f, 0.f}, dist = 1.f;
      if (a0 + t < A) {
        for (int c = 0; c < 3; ++c) D[c] = pv[c] - dv.c[view][c];
        dist = sqrtf(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
        for (int c = 0; c < 3; ++c) D[c] /= dist;
      }
      for (int c = 0; c < 3; ++c) XB[buf][t][32 + c] = D[c];
      XB[buf][t][35] = nx > 0 && a0 + t < A ? dist : 0.f;  // distance input (weight column 35)
      XB[buf][t][36] = 0.f;
    }
  };
  const int ntile_wg = (int)blockIdx.x < ngrid ? (ngrid - 1 - (int)blockIdx.x) / (int)gridDim.x + 1 : 0;
  const int nitems = ntile_wg * V;
  if (nitems > 0) {
    fetch(blockIdx.x, 0);
    put_x(0, blockIdx.x, 0);
  }
  __syncthreads();
  for (int j = 0; j < nitems; ++j) {
    const int tile = blockIdx.x + (j / V) * gridDim.x, view = j % V;
    const int a0 = tile * 16;
    const int buf = j & 1;
    const bool more = j + 1 < nitems;
    const int tile_n = blockIdx.x + ((j + 1) / V) * gridDim.x, view_n = (j + 1) % V;
    // the means of this tile (first view), held until the outputs are written
    const float mx0 = mx[0], mo0 = mo[0], mx1 = mx[1], mo1 = mo[1];
    if (more) fetch(tile_n, view_n);
    const float lt0 = dv.lt[view][0], lt1 = dv.lt[view][1];
    // the first-layer bias of the item's view (unit 16 b + 4 g + r of the lane)
    float bv[2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        bv[b][r] = b1r[b][r];
        if (nx == 3) {
          const int e = (tw0 + (16 * b + r) * 2) % (kHeads * kHid * 2);
          bv[b][r] += TW[e] * lt0 + TW[e + 1] * lt1;
        }
      }
    f4v h[2];
    if (wv < 4) {
      // Z^T (units x anchors) = W1 X^T, K = inputs
      f4v z0 = {0.f, 0.f, 0.f, 0.f}, z1 = z0;
      if constexpr (kBf) {
        const bf8v xb = xbf(buf);
        const float xr = XB[buf][fl][32 + fg];
        z0 = mfma(w1x[0], xr, __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1b[0], xb, z0, 0, 0, 0));
        z1 = mfma(w1x[1], xr, __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1b[1], xb, z1, 0, 0, 0));
      } else {
#pragma unroll
        for (int s = 0; s < 9; ++s) {
          const float xb = XB[buf][fl][4 * s + fg];
          z0 = mfma(w1a[0][s], xb, z0);
          z1 = mfma(w1a[1][s], xb, z1);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        h[0][r] = fmaxf(z0[r] + bv[0][r], 0.f);
        h[1][r] = fmaxf(z1[r] + bv[1][r], 0.f);
      }
    } else if (has_feat && q < 2) {
      // the feature head's hidden layer once: unit block q on feature wave q
      f4v z = {0.f, 0.f, 0.f, 0.f};
      if constexpr (kBf) {
        z = mfma(w1x[0], XB[buf][fl][32 + fg], __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1b[0], xbf(buf), z, 0, 0, 0));
      } else {
#pragma unroll
        for (int s = 0; s < 9; ++s) z = mfma(w1a[0][s], XB[buf][fl][4 * s + fg], z);
      }
      f4v hq;
#pragma unroll
      for (int r = 0; r < 4; ++r) hq[r] = fsoftplus(z[r] + bv[0][r]);
      *reinterpret_cast<f4v*>(&HF[fl][16 * q + 4 * fg]) = hq;
    }
    __syncthreads();  // the feature head's H is complete; the last item's outputs are written
    if (wv >= 4 && has_feat) {
#pragma unroll
      for (int b = 0; b < 2; ++b) h[b] = *reinterpret_cast<const f4v*>(&HF[fl][16 * b + 4 * fg]);
    }
    float* const ob = OB + buf * kOB;
    bf8v hb;  // BF16: H as the A operand of the second layer
    if constexpr (kBf) {
      float v8[8];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) v8[jj] = h[jj >> 2][jj & 3];
      hb = pack_bf8(v8);
    }
    if (active) {
#pragma unroll
      for (int i = 0; i < kR; ++i) {
        if (i >= nt) break;
        // Y (anchors x rows) = H W2^T, K = units; lane (f, g) holds Y[anchor 4 g + r][row 16 i + f]
        f4v y = {0.f, 0.f, 0.f, 0.f};
        if constexpr (kBf) {
          y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hb, w2b[i], y, 0, 0, 0);
        } else {
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) y = mfma(h[b][r], w2y[i][b][r], y);
        }
        if (rok[i]) {
#pragma unroll
          for (int r = 0; r < 4; ++r) ob[ooff[i] + (4 * fg + r) * k] = fout_act(hd, y[r] + b2r[i], dc.l_s);
        }
      }
    }
    if (more) put_x(buf ^ 1, tile_n, view_n);
    __syncthreads();  // the item's output runs are complete; the next item's inputs staged
    // ---- the tile's contiguous runs of every plane: wave w takes planes
    // w, w + 8, w + 16, w + 24 ----
    const int g0 = a0 * k;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = wv + 8 * i;
      if (p >= nplanes) break;
      const int ph = p < 1 ? 0 : p < 4 ? 1 : p < 7 ? 2 : p < 11 ? 3 : 4;
      const int pc = p - (ph == 0 ? 0 : ph == 1 ? 1 : ph == 2 ? 4 : ph == 3 ? 7 : 11);
      float* const dst = out_plane(out, view, ph, pc, n) + g0;
#pragma unroll
      for (int c = 0; c < kR; ++c) {
        const int idx = lane + 64 * c;
        if (idx < run && g0 + idx < n) dst[idx] = ob[p * gstride + idx];
      }
    }
    if (view == 0) {
#pragma unroll
      for (int c2 = 0; c2 < 2; ++c2) {
        const int e = t + c2 * kBT;
        const int cm = e / run, gl = e - cm * run;
        if (cm < 3 && g0 + gl < n) out.mean[(int64_t)cm * n + g0 + gl] = c2 ? mx1 + dc.l_o * mo1 : mx0 + dc.l_o * mo0;
      }
    }
  }
}

template <int kR, bool kBf>
void launch_k(const DecodeConst& dc, const HeadTable& ht, const DecodeViews& dv, const float* xyz, const float* feat,
              const float* off, const float* params, const asgs_gaussians& out, hipStream_t s) {
  static bool attr_set = false;  // more than 64 KiB of dynamic LDS
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_dec_fwd<kR, kBf>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, FwdLds<kR>::kFloats * (int)sizeof(float));
    attr_set = true;
  }
  // two workgroups per compute unit
  const int64_t tiles = (dc.A + 15) / 16;
  const unsigned nblk = (unsigned)(tiles < 512 ? tiles : 512);
  hipLaunchKernelGGL((k_dec_fwd<kR, kBf>), dim3(nblk), dim3(kBT), FwdLds<kR>::kFloats * sizeof(float), s, dc, ht, dv, xyz,
                     feat, off, params, out);
}

}  // namespace

void launch_dec_fwd(const DecodeConst& dc, const HeadTable& ht, const DecodeViews& dv, const float* xyz,
                    const float* feat, const float* off, const float* params, const asgs_gaussians& out,
                    hipStream_t s) {
  // second-layer row tiles per wave: the rotation head has ceil(4 k / 16),
  // each feature wave ceil(k / 4)
  const bool bf = dc.precision == 1;
  if (dc.k <= 12) {
    if (bf) launch_k<3, true>(dc, ht, dv, xyz, feat, off, params, out, s);
    else launch_k<3, false>(dc, ht, dv, xyz, feat, off, params, out, s);
  } else {
    if (bf) launch_k<4, true>(dc, ht, dv, xyz, feat, off, params, out, s);
    else launch_k<4, false>(dc, ht, dv, xyz, feat, off, params, out, s);
  }
}

}  // namespace asgs
