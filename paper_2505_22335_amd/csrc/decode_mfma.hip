// BF16 anchor decoding on the matrix cores (UP-SLAM Sec. 3.3, Eq. 8 and Eq. 9).
//
// The two layers of the five heads are dense contractions over anchors:
//   layer 1: Z[a][u] = X_f[a] . W1f[u] + delta[a] . W1d[u] + b1[u]   (u < 160 hidden units)
//            (+ dist[a] W1x[u] + lt . W1t[u] for the distance and temporal inputs)
//   layer 2: Y[a][r] = H_h[a] . W2[r] + b2[r]                        (rows r of head h)
// with X_f the 32-d anchor feature and H_h the 32 hidden activations of head
// h, so K = 32 for both: one v_mfma_f32_16x16x32_bf16 per 16x16 output tile.
// Operands (anchor features, first- and second-layer weights, hidden
// activations) are rounded to bfloat16 (nearest even); accumulation, the
// view-direction and distance terms (on the vector ALUs), biases (with the
// view's temporal term folded in) and activations are FP32. Means do not pass through the MLP and stay FP32.
//
// Persistent grid, one workgroup per CU: the workgroup stages both layers'
// weights once in LDS (padded rows against bank conflicts) together with a
// per-row output table, then its 12 waves loop over 16-anchor tiles of the
// grid-strided sequence (dealt out workgroup-first, so that every compute
// unit gets tiles also when there are fewer than 12 per unit). Everything a
// wave keeps per tile is bfloat16 in LDS so that 12 waves fit beside the
// weights. The backward always runs in FP32
// (decode.hip).
#include <math.h>

#include "decode_shared.h"

namespace asgs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kMT = 16;            // anchors per tile (M)
constexpr int kWaves = 12;
constexpr int kThreads = 64 * kWaves;
constexpr int kRow = 40;           // padded LDS row (bf16) of a 32-wide operand row
constexpr int kHRow = 168;         // padded LDS row (bf16) of the 160 hidden activations
constexpr int kMaxPRows = 432;     // second-layer rows, each head padded to a multiple of 16
constexpr int kMaxWG = 256;        // persistent workgroups (one per CU)
static_assert(kMaxPRows >= kMaxRows, "padded rows");

ASGS_DEV uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return (uint16_t)(u >> 16);
}

// v0 .. v4 selected by four ordered conditions (the last true one wins).
ASGS_DEV int sel5(bool c1, bool c2, bool c3, bool c4, int v0, int v1, int v2, int v3, int v4) {
  int x = v0;
  x = c1 ? v1 : x;
  x = c2 ? v2 : x;
  x = c3 ? v3 : x;
  x = c4 ? v4 : x;
  return x;
}

ASGS_DEV float fast_sigm(float y) { return __builtin_amdgcn_rcpf(1.f + __expf(-y)); }

ASGS_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(kThreads) k_decode_bf16(DecodeConst dc, HeadTable ht, DecodeViews dv,
                                                         const float* __restrict__ xyz,
                                                         const float* __restrict__ feat,
                                                         const float* __restrict__ off,
                                                         const float* __restrict__ params, asgs_gaussians out) {
  __shared__ __attribute__((aligned(16))) uint16_t w1[160 * kRow];
  __shared__ __attribute__((aligned(16))) uint16_t w2[kMaxPRows * kRow];
  __shared__ float w1d[160][5];        // direction weights (3), bias, distance weight of each hidden unit
  __shared__ float b2s[kMaxPRows];     // second-layer bias per padded row
  __shared__ int32_t epi[kMaxPRows];   // per padded row: comp * n + i (or -1 for padding)
  __shared__ __attribute__((aligned(16))) uint16_t Xs[kWaves][kMT][kRow];
  __shared__ float dls[kWaves][kMT][4];
  __shared__ __attribute__((aligned(16))) uint16_t Hs[kWaves][kMT][kHRow];
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int view = blockIdx.y;
  const int A = (int)dc.A;
  const int k = dc.k;
  const int n = A * k;
  const int nunits = ht.nunits;
  const int fl = lane & 15, fg = lane >> 4;
  int prow0[kHeads + 1];
  {
    int r = 0;
    for (int h = 0; h < kHeads; ++h) {
      prow0[h] = r;
      r += (k * ht.m[h] + 15) / 16 * 16;
    }
    prow0[kHeads] = r;
  }
  // ---- stage the weights and the output table ----
  // Every load is issued before the first store (one round trip to memory):
  // thread t takes the elements t + q * kThreads of the first layer's
  // 160 x 32 feature weights and of the padded second-layer rows. The source
  // of an element is selected from the heads' (uniform) offsets by
  // comparisons, without branches; elements of absent heads or of padding
  // rows load a valid address and are stored as zero or into rows that are
  // never read.
  constexpr int kQ1 = (kHeads * kHid * 32 + kThreads - 1) / kThreads;
  constexpr int kQ2 = kMaxPRows * 32 / kThreads;
  static_assert(kQ2 * kThreads == kMaxPRows * 32, "second-layer rounds cover the padded rows exactly");
  static_assert(kMaxPRows <= kThreads && kHeads * kHid <= kThreads, "one bias row per thread");
  const int nprows = prow0[kHeads];
  // per head (uniform): packed offset, source base of its padded-row
  // elements, end of its real rows, output components and source of b2
  int o1[kHeads], ob[kHeads], rend[kHeads], mm[kHeads], obb[kHeads];
  for (int h = 0; h < kHeads; ++h) {
    o1[h] = ht.off[h];
    ob[h] = ht.off[h] + kHid * kIn + kHid - kHid * prow0[h];
    rend[h] = prow0[h] + k * ht.m[h];
    mm[h] = ht.m[h];
    obb[h] = ht.off[h] + kHid * kIn + kHid + kHid * k * ht.m[h] - prow0[h];
  }
  // value of the head that hidden unit u (by unit) or padded row pr (by row)
  // belongs to; the arrays are read at constant indices only
#define ASGS_BY_UNIT(u, v) sel5((u) >= 32, (u) >= 64, (u) >= 96, (u) >= 128, v[0], v[1], v[2], v[3], v[4])
#define ASGS_BY_ROW(pr, v) \
  sel5((pr) >= prow0[1], (pr) >= prow0[2], (pr) >= prow0[3], (pr) >= prow0[4], v[0], v[1], v[2], v[3], v[4])
  float v1[kQ1], v2[kQ2];
#pragma unroll
  for (int q = 0; q < kQ1; ++q) {
    const int e = t + q * kThreads;
    int u = e >> 5;
    u = u < nunits ? u : nunits - 1;
    v1[q] = params[(unsigned)(ASGS_BY_UNIT(u, o1) + (u & 31) * kIn + (e & 31))];
  }
#pragma unroll
  for (int q = 0; q < kQ2; ++q) {
    const int e = t + q * kThreads;
    int pr = e >> 5;
    pr = pr < nprows ? pr : nprows - 1;
    const int re = ASGS_BY_ROW(pr, rend);
    const int prc = pr < re ? pr : re - 1;  // padding rows read the head's last row
    const float w = params[(unsigned)(ASGS_BY_ROW(pr, ob) + prc * kHid + (e & 31))];
    v2[q] = pr < re ? w : 0.f;
  }
  float wd[5];
  {
    const int u = t < nunits ? t : nunits - 1;
    const int src = ASGS_BY_UNIT(u, o1) + (u & 31) * kIn;
    wd[0] = params[(unsigned)(src + 32)];
    wd[1] = params[(unsigned)(src + 33)];
    wd[2] = params[(unsigned)(src + 34)];
    wd[3] = params[(unsigned)(ASGS_BY_UNIT(u, o1) + kHid * kIn + (u & 31))];
    wd[4] = 0.f;
    if (ht.nx > 0) {  // distance weight; temporal weights folded into the bias
      int xo[kHeads];
      for (int h = 0; h < kHeads; ++h) xo[h] = ht.xoff[h];
      const int xsrc = ASGS_BY_UNIT(u, xo) + (u & 31) * ht.nx;
      wd[4] = params[(unsigned)xsrc];
      if (ht.nx == 3)
        wd[3] += params[(unsigned)(xsrc + 1)] * dv.lt[view][0] + params[(unsigned)(xsrc + 2)] * dv.lt[view][1];
    }
  }
  // per padded row t: second-layer bias and output code (r % m) * n + r / m
  float bias2;
  int code;
  {
    const int pr = t < nprows ? t : nprows - 1;
    const int m = ASGS_BY_ROW(pr, mm);
    const int re = ASGS_BY_ROW(pr, rend);
    const int r = pr - (re - k * m);
    const bool real = pr < re;
    const float bv = params[(unsigned)(ASGS_BY_ROW(pr, obb) + (real ? pr : re - 1))];
    bias2 = real ? bv : 0.f;
    code = real ? (r % m) * n + r / m : -1;
  }
#undef ASGS_BY_UNIT
#undef ASGS_BY_ROW
#pragma unroll
  for (int q = 0; q < kQ1; ++q) {
    const int e = t + q * kThreads;
    if (e < kHeads * kHid * 32) w1[(e >> 5) * kRow + (e & 31)] = f2bf(v1[q]);
  }
#pragma unroll
  for (int q = 0; q < kQ2; ++q) {
    const int e = t + q * kThreads;
    w2[(e >> 5) * kRow + (e & 31)] = f2bf(v2[q]);
  }
  if (t < kHeads * kHid) {
#pragma unroll
    for (int c = 0; c < 5; ++c) w1d[t][c] = wd[c];
  }
  if (t < kMaxPRows) {
    b2s[t] = t < nprows ? bias2 : 0.f;
    epi[t] = t < nprows ? code : -1;
  }
  __syncthreads();
  float* hbase[kHeads];
  for (int h = 0; h < kHeads; ++h) hbase[h] = ht.m[h] ? out_plane(out, view, h, 0, n) : nullptr;
  const int ntiles = (A + kMT - 1) / kMT;
  const int tstride = (int)gridDim.x * kWaves;
  const float4* feat4 = reinterpret_cast<const float4*>(feat);
  float4 xf[2];
  float xd[3];
  // Loads of one tile's inputs, issued a tile ahead; anchors past the end are
  // clamped to the last one (their results are never stored).
  auto load_tile = [&](int tl) {
    const int a0n = tl * kMT;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = lane + 64 * q;
      int a = a0n + (e >> 3);
      a = a < A ? a : A - 1;
      xf[q] = feat4[a * 8 + (e & 7)];
    }
    int a = a0n + fl;
    a = a < A ? a : A - 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) xd[c] = xyz[c * A + a];
  };
  // tiles are dealt out workgroup-first (tile b + gridDim.x * (wv + kWaves * i)),
  // so that a short sequence still reaches every compute unit
  int tile = (int)blockIdx.x + (int)gridDim.x * wv;
  if (tile < ntiles) load_tile(tile);
  for (; tile < ntiles; tile += tstride) {
    const int a0 = tile * kMT;
    if (view == 0) {  // means (view independent)
      const int cnt = kMT * k;
      for (int e = lane; e < cnt * 3; e += 64) {
        const int c = e / cnt;
        const int r = e - c * cnt;
        const int gn = a0 * k + r;
        if (gn < n) out.mean[c * n + gn] = xyz[c * A + a0 + r / k] + dc.l_o * off[c * n + gn];
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = lane + 64 * q;
      const int a = e >> 3, c4 = (e & 7) * 4;
      Xs[wv][a][c4 + 0] = f2bf(xf[q].x);
      Xs[wv][a][c4 + 1] = f2bf(xf[q].y);
      Xs[wv][a][c4 + 2] = f2bf(xf[q].z);
      Xs[wv][a][c4 + 3] = f2bf(xf[q].w);
    }
    if (lane < kMT) {
      float D[3];
      for (int c = 0; c < 3; ++c) D[c] = xd[c] - dv.c[view][c];
      const float d = sqrtf(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
      for (int c = 0; c < 3; ++c) dls[wv][lane][c] = D[c] / d;
      dls[wv][lane][3] = d;
    }
    if (tile + tstride < ntiles) load_tile(tile + tstride);
    wave_sync();
    // ---- layer 1: 16 anchors x 160 hidden units, two column tiles at a time ----
    const bf8v xa = *reinterpret_cast<const bf8v*>(&Xs[wv][fl][8 * fg]);
    float dl[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) dl[r][c] = dls[wv][4 * fg + r][c];
    for (int nt = 0; nt < nunits / 16; nt += 2) {
      const int ua = 16 * nt + fl, ub = ua + 16;
      const bf8v ba = *reinterpret_cast<const bf8v*>(&w1[ua * kRow + 8 * fg]);
      const bf8v bb = *reinterpret_cast<const bf8v*>(&w1[ub * kRow + 8 * fg]);
      f4v ca = {0.f, 0.f, 0.f, 0.f}, cb = ca;
      ca = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa, ba, ca, 0, 0, 0);
      cb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa, bb, cb, 0, 0, 0);
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int u = half ? ub : ua;
        const f4v c4 = half ? cb : ca;
        const bool sp = (u >> 5) == 4;  // the feature head's hidden layer uses SoftPlus
        const float wd0 = w1d[u][0], wd1 = w1d[u][1], wd2 = w1d[u][2], b1 = w1d[u][3], wx = w1d[u][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float z = c4[r] + b1 + dl[r][0] * wd0 + dl[r][1] * wd1 + dl[r][2] * wd2 + dl[r][3] * wx;
          Hs[wv][4 * fg + r][u] = f2bf(sp ? softplus(z) : fmaxf(z, 0.f));
        }
      }
    }
    wave_sync();
    // ---- layer 2, head by head: (k * m) rows x 16 anchors ----
    // The weight rows are the A operand and the anchors the B operand, so
    // that lane (fl, fg) holds rows 4 fg + r of anchor fl: a store
    // instruction writes four rows of 16 consecutive anchors (stride k).
    const int a = a0 + fl;
    for (int h = 0; h < kHeads; ++h) {
      if (ht.m[h] == 0) continue;
      const bf8v ha = *reinterpret_cast<const bf8v*>(&Hs[wv][fl][32 * h + 8 * fg]);
      float* base = hbase[h];
      for (int pr0 = prow0[h]; pr0 < prow0[h + 1]; pr0 += 16) {
        const bf8v b = *reinterpret_cast<const bf8v*>(&w2[(pr0 + fl) * kRow + 8 * fg]);
        f4v c4 = {0.f, 0.f, 0.f, 0.f};
        c4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, ha, c4, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int pr = pr0 + 4 * fg + r;
          const int code = epi[pr];
          const float y = c4[r] + b2s[pr];
          const float v = h <= 1 ? fast_sigm(y) : (h == 2 ? dc.l_s * fast_sigm(y) : y);
          if (code >= 0 && a < A) base[code + a * k] = v;
        }
      }
    }
    wave_sync();
  }
}

}  // namespace

void launch_decode_mfma(const DecodeConst& dc, const HeadTable& ht, const DecodeViews& dv, const float* xyz,
                        const float* feat, const float* off, const float* params, const asgs_gaussians& out,
                        hipStream_t s) {
  const int64_t tiles = (dc.A + kMT - 1) / kMT;
  dim3 grid((unsigned)(tiles < kMaxWG ? tiles : kMaxWG), (unsigned)dc.n_views);
  hipLaunchKernelGGL(k_decode_bf16, grid, dim3(kThreads), 0, s, dc, ht, dv, xyz, feat, off, params, out);
}

}  // namespace asgs
