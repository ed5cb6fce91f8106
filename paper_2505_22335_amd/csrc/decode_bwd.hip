// Decoder backward on the matrix cores (VJP of UP-SLAM Eq. 8 and Eq. 9), per
// view. One workgroup of eight waves takes 16-anchor tiles in turn: waves
// 0..3 each own one of the opacity, colour, scale and rotation heads, waves
// 4..7 share the feature head's output rows. Per tile and head, with X the
// tile's inputs (one row per anchor):
//   Z = X W1^T + b1, H = act(Z)                 (ReLU; SoftPlus for features)
//   Y = H W2^T + b2, dY = dL/d(decoded) * act'(Y)
//   dW2 += dY^T H, db2 += sum_a dY, dH = dY W2, dZ = dH * act'(Z)
//   dW1 += dZ^T X, db1 += sum_a dZ, dX = dZ W1
// all on FP32 16x16x4 MFMAs. The heads' dX are summed per anchor in a fixed
// order inside the workgroup, which then forms the anchor gradients (feature
// part; view direction and distance through delta = (x - c)/|x - c|) and its
// share of the camera-centre gradient. Each workgroup writes one partial of
// every parameter gradient, reduced afterwards in a fixed order
// (deterministic, no atomics).
//
// Operand layouts. v_mfma_f32_16x16x4f32 (wave64): lane l = 16 g + f supplies
// A[f][g] and B[g][f] and receives D[4 g + r][f], r = 0..3. A 16x16 block
// held by rows in that way (lane (f, g) holds M[4 g + r][f]) is directly a B
// operand with K = its rows, and an A operand with K = its rows and M = its
// columns, when step r of lane group g takes K index 4 g + r (a contraction
// may visit K in any order that both operands share). Chained this way, H and
// dH stay in registers as (units x anchors) blocks and Y, dY as (anchors x
// rows) blocks; only H, dY and dZ pass once each through per-wave LDS rows to
// be transposed. Both layouts of the second-layer weights (B of Y, A of dH^T)
// sit in registers for the whole kernel; the first-layer weights (A of Z^T
// and of dX^T) are read from LDS, as are the tile's inputs and upstream
// gradients, which are loaded a tile ahead as coalesced runs.
#include <math.h>

#include "decode_shared.h"

namespace asgs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kBW = 8;         // waves per workgroup
constexpr int kBT = 64 * kBW;  // threads per workgroup
constexpr int kMaxWG = 256;    // one workgroup per compute unit
constexpr int kW1L = 36;       // LDS row of a first-layer weight row: 35 inputs + the distance column
constexpr int kW2L = 36;       // LDS row of a second-layer weight row in the prologue (32 units + pad)
constexpr int kXL = 52;        // LDS row of an anchor's inputs: 35 + distance column, |x - c| at 36
constexpr int kHB = 36;        // per-wave transpose rows of H and dZ (32 units + pad)
constexpr int kYB = 20;        // per-wave transpose rows of dY (16 rows + pad)
constexpr int kDXL = 36;       // dX row of an anchor in a head's slot
constexpr int kSlots = 5;      // dX slots: heads 0..3 and the feature head

// LDS carve (floats)
constexpr int kOffW1 = 0;
constexpr int kOffX = kOffW1 + kHeads * kHid * kW1L;
constexpr int kOffHB = kOffX + 2 * 16 * kXL;
constexpr int kOffYB = kOffHB + kBW * 16 * kHB;
constexpr int kOffHF = kOffYB + kBW * 16 * kYB;  // the feature head's H, shared by its waves
constexpr int kOffDH = kOffHF + 16 * kHB;
constexpr int kOffDX = kOffDH + 4 * 64 * 8;
constexpr int kOffG = kOffDX + 2 * kSlots * 16 * kDXL;
constexpr int kPlanes = 27;    // (head, component) planes of the upstream gradients: 1 + 3 + 3 + 4 + 16
constexpr int kGB = kPlanes * (16 * ASGS_MAX_K + 1);  // one buffer: each plane's run of 16 k values + pad
constexpr int kLdsFloats = kOffG + 2 * kGB;
// the second-layer weights (at most 27 k = 432 rows of kW2L), b2 and b1 are
// copied once into the region from kOffHB on
static_assert(kLdsFloats - kOffHB >= 27 * ASGS_MAX_K * (kW2L + 1) + 3 + kHeads * kHid, "weight copy does not fit");

ASGS_DEV f4v mfma(float a, float b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

ASGS_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Element i of a five-entry table with a lane-varying index, as selects (no
// private-memory copy of the table).
template <typename T>
ASGS_DEV T pick5(const T (&a)[kHeads], int i) {
  T v = a[0];
  v = i == 1 ? a[1] : v;
  v = i == 2 ? a[2] : v;
  v = i == 3 ? a[3] : v;
  v = i == 4 ? a[4] : v;
  return v;
}

template <int kR>
__global__ void __launch_bounds__(kBT, 1) k_dec_bwd(DecodeConst dc, HeadTable ht, DecodeViews dv,
                                                    const float* __restrict__ xyz, const float* __restrict__ feat,
                                                    const float* __restrict__ params, asgs_gaussians dg, int view,
                                                    DecWork w, float* d_xyz, float* d_feat, int want_params) {
  extern __shared__ __attribute__((aligned(16))) float smem[];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int fl = lane & 15, fg = lane >> 4;
  float* const W1L = smem + kOffW1;
  float (*const XB)[16][kXL] = reinterpret_cast<float (*)[16][kXL]>(smem + kOffX);
  float (*const HBw)[kHB] = reinterpret_cast<float (*)[kHB]>(smem + kOffHB + wv * 16 * kHB);
  float (*const YBw)[kYB] = reinterpret_cast<float (*)[kYB]>(smem + kOffYB + wv * 16 * kYB);
  float (*const HF)[kHB] = reinterpret_cast<float (*)[kHB]>(smem + kOffHF);
  float* const DH = smem + kOffDH;
  float (*const DX)[kSlots][16][kDXL] = reinterpret_cast<float (*)[kSlots][16][kDXL]>(smem + kOffDX);
  float* const GB = smem + kOffG;
  const int A = (int)dc.A;
  const int k = dc.k;
  const int n = A * k;
  const int nx = ht.nx;
  const float lt0 = dv.lt[view][0], lt1 = dv.lt[view][1];
  const bool has_feat = ht.m[4] > 0;
  // ---- this wave's head, output rows and duties ----
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
  // dX: waves 0..3 and feature wave 2. dW1, db1: waves 0..2 of their heads,
  // feature wave 0 of the rotation head (its wave has the most rows) and
  // feature wave 3 of the feature head
  const int hw1 = wv < 3 ? wv : wv == 4 ? 3 : (wv == 7 && has_feat) ? 4 : -1;
  const int w2o = (int)ht.off[hd] + kHid * kIn + kHid;  // the head's W2 [rows][32], then b2 [rows]
  // the tile's upstream gradients are staged per (head, component) plane as
  // runs of 16 k values (stride run + 1, odd, against bank conflicts)
  const int run = 16 * k, gstride = run + 1;
  // ---- per-tile inputs: features, positions and upstream gradients, fetched a
  // tile ahead into registers and staged through LDS ----
  // (loads are unconditional, from clamped indices, and masked when staged:
  // a load under a branch would be waited for at the branch's end)
  float xv = 0.f, pv[3] = {0.f, 0.f, 0.f};
  auto fetch_x = [&](int tile) {
    const int a0 = tile * 16, a = t >> 5, c = t & 31;
    const int ax = a0 + a < A ? a0 + a : 0, ap = a0 + (t & 15) < A ? a0 + (t & 15) : 0;
    xv = feat[(int64_t)ax * 32 + c];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) pv[cc] = xyz[(int64_t)cc * A + ap];
  };
  auto put_x = [&](int buf, int tile) {
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
      XB[buf][t][36] = dist;                                // |x - c| for the anchor gradients
    }
  };
  // wave w loads planes w, w + 8, w + 16, w + 24 (those present), each as
  // kR coalesced chunks of 64 values (16 k <= 64 kR)
  const int nplanes = has_feat ? kPlanes : 11;
  // the plane, or for an absent plane the first parameter as a stand-in
  // that is only ever read at index 0
  const float* pbase[4];
  int plim[4];  // indices below plim are read from the plane, others at 0
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int p = wv + 8 * i;
    const int ph = p < 1 ? 0 : p < 4 ? 1 : p < 7 ? 2 : p < 11 ? 3 : 4;
    const int pc = p - (ph == 0 ? 0 : ph == 1 ? 1 : ph == 2 ? 4 : ph == 3 ? 7 : 11);
    const bool present = p < nplanes;
    pbase[i] = present ? out_plane(dg, view, ph, pc, n) : params;
    plim[i] = present ? n : 0;
  }
  float gpre[4][kR];
  auto fetch_g = [&](int tile) {
    const int g0 = tile * run;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < kR; ++c) {
        const int gi = g0 + lane + 64 * c;
        gpre[i][c] = pbase[i][gi < plim[i] ? gi : 0];
      }
  };
  auto put_g = [&](int buf, int tile) {
    const int g0 = tile * run;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (wv + 8 * i >= nplanes) break;
#pragma unroll
      for (int c = 0; c < kR; ++c) {
        const int idx = lane + 64 * c;
        if (idx < run) GB[buf * kGB + (wv + 8 * i) * gstride + idx] = g0 + idx < n ? gpre[i][c] : 0.f;
      }
    }
  };
  const int ngrid = (A + 15) / 16;
  if ((int)blockIdx.x < ngrid) {
    fetch_x(blockIdx.x);
    fetch_g(blockIdx.x);
  }
  // ---- the weights into LDS (coalesced): the first-layer rows of every head
  // (kept for the whole kernel); the second-layer rows (36 floats: b128 reads
  // of four units and b32 reads across rows without bank conflicts), b2 and
  // b1 (with the view's temporal term), in the region past the input tiles,
  // which is free until the first tile is staged ----
  float* const W2L = smem + kOffHB;                         // [all rows][kW2L]
  const int nrows = ht.nrows;
  float* const B2L = W2L + nrows * kW2L;                    // [all rows]
  float* const B1L = B2L + ((nrows + 3) & ~3);             // [5 heads][32] (16-byte aligned)
  {
    // head by head, each a contiguous block of the packed parameters: every
    // load of the thread is issued before its first store
    constexpr int kK = kR == 3 ? 12 : ASGS_MAX_K;  // largest k of this instantiation
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
      for (int q = 0; q < kE1; ++q) {
        const int e = t + q * kBT;
        v1[h][q] = params[o1 + (e < kHid * kIn ? e : 0)];
      }
      const int ne2 = (kMs[h] * kK * kHid + kBT - 1) / kBT;  // a constant once unrolled
#pragma unroll
      for (int q = 0; q < kE2m; ++q) {
        if (q >= ne2) break;
        const int e = t + q * kBT;
        v2[h][q] = params[w2 + (e < rw * kHid ? e : 0)];
      }
      vd[h] = nx > 0 ? params[ox + (t & 31) * nx] : 0.f;
      vb1[h] = params[o1 + kHid * kIn + (t & 31)];
      if (nx == 3) vb1[h] += params[ox + (t & 31) * 3 + 1] * lt0 + params[ox + (t & 31) * 3 + 2] * lt1;
      vb2[h] = params[w2 + rw * kHid + (t < rw ? t : 0)];
    }
#pragma unroll
    for (int h = 0; h < kHeads; ++h) {
      if (h >= nh) break;
      const int rw = k * ht.m[h], r0 = ht.row0[h];
#pragma unroll
      for (int q = 0; q < kE1; ++q) {
        const int e = t + q * kBT;
        const int u = e / kIn, i = e - u * kIn;
        if (e < kHid * kIn) W1L[(h * kHid + u) * kW1L + i] = v1[h][q];
      }
      const int ne2 = (kMs[h] * kK * kHid + kBT - 1) / kBT;
#pragma unroll
      for (int q = 0; q < kE2m; ++q) {
        if (q >= ne2) break;
        const int e = t + q * kBT;
        if (e < rw * kHid) W2L[(r0 + (e >> 5)) * kW2L + (e & 31)] = v2[h][q];
      }
      if (t < kHid) {
        W1L[(h * kHid + t) * kW1L + kIn] = vd[h];  // the distance weight (zero without that input)
        B1L[h * kHid + t] = vb1[h];
      }
      if (t < rw) B2L[r0 + t] = vb2[h];
    }
    // input columns past 36 only meet discarded outputs of dW1; keep them finite
    for (int e = t; e < 2 * 16 * (kXL - 37); e += kBT) {
      const int row = e / (kXL - 37);
      XB[row >> 4][row & 15][37 + e - row * (kXL - 37)] = 0.f;
    }
  }
  __syncthreads();
  // ---- second-layer weights and biases in registers ----
  float b1r[2][4];
  float w2y[kR][2][4], w2h[kR][2][4], b2r[kR];
  // the lane's output row of row tile i reads plane offset goff[i] + a k
  const int pb0 = hd == 0 ? 0 : hd == 1 ? 1 : hd == 2 ? 4 : hd == 3 ? 7 : 11;  // first plane of the head
  const int hr0 = ht.row0[hd];  // the head's first row among all rows
  const int minv = (65536 + m - 1) / (m > 0 ? m : 1);  // o / m = (o * minv) >> 16, exact for o <= 256
  int goff[kR];
  bool rok[kR];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const f4v v = *reinterpret_cast<const f4v*>(&B1L[hd * kHid + 16 * b + 4 * fg]);
#pragma unroll
    for (int r = 0; r < 4; ++r) b1r[b][r] = active ? v[r] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < kR; ++i) {
    const int o = 16 * (t0 + i) + fl;
    const bool ok = active && i < nt && o < rows;
    rok[i] = ok;
    const int oc = ok ? o : 0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const f4v v = *reinterpret_cast<const f4v*>(&W2L[(hr0 + oc) * kW2L + 16 * b + 4 * fg]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int oh = 16 * (t0 + i) + 4 * fg + r;
        const bool okh = active && i < nt && oh < rows;
        w2y[i][b][r] = ok ? v[r] : 0.f;
        const float wh = W2L[(hr0 + (okh ? oh : 0)) * kW2L + 16 * b + fl];
        w2h[i][b][r] = okh ? wh : 0.f;
      }
    }
    b2r[i] = ok ? B2L[hr0 + oc] : 0.f;
    const int gi = (oc * minv) >> 16, gc = oc - gi * m;
    goff[i] = (pb0 + gc) * gstride + gi;
  }
  __syncthreads();  // the second-layer copy is no longer read
  if ((int)blockIdx.x < ngrid) {
    put_x(0, blockIdx.x);
    put_g(0, blockIdx.x);
  }
  __syncthreads();
  // ---- accumulators ----
  f4v dw2[kR][2];
  float db2[kR];
#pragma unroll
  for (int i = 0; i < kR; ++i) {
    dw2[i][0] = dw2[i][1] = f4v{0.f, 0.f, 0.f, 0.f};
    db2[i] = 0.f;
  }
  f4v dw1[2][3];
#pragma unroll
  for (int b = 0; b < 2; ++b) dw1[b][0] = dw1[b][1] = dw1[b][2] = f4v{0.f, 0.f, 0.f, 0.f};
  float db1[2] = {0.f, 0.f};
  float dcl[3] = {0.f, 0.f, 0.f};
  const float* w1l = W1L + hd * kHid * kW1L;

  // dZ from dH and H (registers, units x anchors), then the head's dX^T into
  // its slot; with publish, dZ also into the wave's transpose rows
  auto tail = [&](const f4v (&h)[2], const f4v (&dh)[2], int buf, bool dx_now, bool publish) {
    f4v dz[2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        dz[b][r] = hd == 4 ? dh[b][r] * (1.f - fexp(-h[b][r])) : (h[b][r] > 0.f ? dh[b][r] : 0.f);
    if (dx_now) {
      // dX^T (inputs x anchors) = W1^T dZ^T, K = units
      f4v dx[3];
#pragma unroll
      for (int ct = 0; ct < 3; ++ct) dx[ct] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float* wr = w1l + (16 * b + 4 * fg + r) * kW1L;
#pragma unroll
          for (int ct = 0; ct < 3; ++ct) {
            const int i = 16 * ct + fl;
            const float wv1 = wr[i < kW1L ? i : 0];
            dx[ct] = mfma(i < kW1L ? wv1 : 0.f, dz[b][r], dx[ct]);
          }
        }
      // lane (f, g) holds dX[anchor f][inputs 16 ct + 4 g + r]
#pragma unroll
      for (int ct = 0; ct < 3; ++ct)
        if (16 * ct + 4 * fg < kDXL) *reinterpret_cast<f4v*>(&DX[buf][wv < 4 ? wv : 4][fl][16 * ct + 4 * fg]) = dx[ct];
    }
    if (publish) {
#pragma unroll
      for (int b = 0; b < 2; ++b) *reinterpret_cast<f4v*>(&HBw[fl][16 * b + 4 * fg]) = dz[b];
    }
  };
  // dW1 += dZ^T X, db1 += sum_a dZ, with dZ read by rows of anchors from the
  // transpose rows src of the wave that formed it
  auto acc_dw1 = [&](const float (*src)[kHB], int buf) {
    float dzt[2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) dzt[b][r] = src[4 * fg + r][16 * b + fl];
    float xa[3][4];
#pragma unroll
    for (int ct = 0; ct < 3; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) xa[ct][r] = XB[buf][4 * fg + r][16 * ct + fl];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      db1[b] += (dzt[b][0] + dzt[b][1]) + (dzt[b][2] + dzt[b][3]);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int ct = 0; ct < 3; ++ct) dw1[b][ct] = mfma(dzt[b][r], xa[ct][r], dw1[b][ct]);
    }
  };
  float (*const HB3)[kHB] = reinterpret_cast<float (*)[kHB]>(smem + kOffHB + 3 * 16 * kHB);

  int j = 0;
  for (int tile = blockIdx.x; tile < ngrid; tile += gridDim.x, ++j) {
    const int a0 = tile * 16;
    const int buf = j & 1;
    const bool more = tile + (int)gridDim.x < ngrid;
    const float* gb = GB + buf * kGB;
    if (more) {
      fetch_x(tile + gridDim.x);
      fetch_g(tile + gridDim.x);
    }
    f4v h[2], dh[2];
    dh[0] = dh[1] = f4v{0.f, 0.f, 0.f, 0.f};
    float ht_[2][4];
    if (wv < 4) {
      // Z^T (units x anchors) = W1 X^T, K = inputs
      f4v z0 = {0.f, 0.f, 0.f, 0.f}, z1 = z0;
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        const float xb = XB[buf][fl][4 * s + fg];
        z0 = mfma(w1l[fl * kW1L + 4 * s + fg], xb, z0);
        z1 = mfma(w1l[(16 + fl) * kW1L + 4 * s + fg], xb, z1);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        h[0][r] = fmaxf(z0[r] + b1r[0][r], 0.f);
        h[1][r] = fmaxf(z1[r] + b1r[1][r], 0.f);
      }
      // H by rows of anchors (B operand of dW2)
#pragma unroll
      for (int b = 0; b < 2; ++b) *reinterpret_cast<f4v*>(&HBw[fl][16 * b + 4 * fg]) = h[b];
      wave_sync();
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) ht_[b][r] = HBw[4 * fg + r][16 * b + fl];
    } else if (has_feat && q < 2) {
      // the feature head's hidden layer once: unit block q on feature wave q
      f4v z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 9; ++s) z = mfma(w1l[(16 * q + fl) * kW1L + 4 * s + fg], XB[buf][fl][4 * s + fg], z);
      f4v hq;
#pragma unroll
      for (int r = 0; r < 4; ++r) hq[r] = fsoftplus(z[r] + (q ? b1r[1][r] : b1r[0][r]));
      *reinterpret_cast<f4v*>(&HF[fl][16 * q + 4 * fg]) = hq;
    }
    __syncthreads();  // the feature head's H is complete
    if (wv >= 4 && has_feat) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        h[b] = *reinterpret_cast<const f4v*>(&HF[fl][16 * b + 4 * fg]);
#pragma unroll
        for (int r = 0; r < 4; ++r) ht_[b][r] = HF[4 * fg + r][16 * b + fl];
      }
    }
    if (active) {
#pragma unroll
      for (int i = 0; i < kR; ++i) {
        if (i >= nt) break;
        // Y (anchors x rows) = H W2^T, K = units
        f4v y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) y = mfma(h[b][r], w2y[i][b][r], y);
        f4v dy;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float gv = gb[goff[i] + (4 * fg + r) * k];  // a valid location for every lane
          dy[r] = (rok[i] ? gv : 0.f) * fact_grad(hd, y[r] + b2r[i], dc.l_s);
        }
        db2[i] += (dy[0] + dy[1]) + (dy[2] + dy[3]);
        // dW2 (rows x units) += dY^T H, K = anchors
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) dw2[i][b] = mfma(dy[r], ht_[b][r], dw2[i][b]);
        // dH^T (units x anchors) += W2^T dY^T, K = rows (dY transposed through LDS)
#pragma unroll
        for (int r = 0; r < 4; ++r) YBw[4 * fg + r][fl] = dy[r];
        wave_sync();
        const f4v dyt = *reinterpret_cast<const f4v*>(&YBw[fl][4 * fg]);
        wave_sync();
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) dh[b] = mfma(w2h[i][b][r], dyt[r], dh[b]);
      }
    }
    if (wv < 4) {
      tail(h, dh, buf, true, true);
      if (hw1 >= 0) {
        wave_sync();
        acc_dw1(HBw, buf);
      }
    } else if (active) {
      // the feature waves' dH partials, summed below in a fixed order
#pragma unroll
      for (int b = 0; b < 2; ++b) *reinterpret_cast<f4v*>(&DH[(q * 64 + lane) * 8 + 4 * b]) = dh[b];
    }
    __syncthreads();  // feature dH partials and the rotation head's dZ written; every thread is past the last tile's anchor step
    if (wv == 4) acc_dw1(HB3, buf);  // the rotation head's dW1
    if (wv >= 4 && active && (q == 2 || q == 3)) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const f4v p0 = *reinterpret_cast<const f4v*>(&DH[(0 * 64 + lane) * 8 + 4 * b]);
        const f4v p1 = *reinterpret_cast<const f4v*>(&DH[(1 * 64 + lane) * 8 + 4 * b]);
        const f4v p2 = *reinterpret_cast<const f4v*>(&DH[(2 * 64 + lane) * 8 + 4 * b]);
        const f4v p3 = *reinterpret_cast<const f4v*>(&DH[(3 * 64 + lane) * 8 + 4 * b]);
        dh[b] = (p0 + p1) + (p2 + p3);
      }
      tail(h, dh, buf, q == 2, q == 3);
      if (q == 3) {
        wave_sync();
        acc_dw1(HBw, buf);
      }
    }
    if (more) {
      put_x(buf ^ 1, tile + gridDim.x);
      put_g(buf ^ 1, tile + gridDim.x);
    }
    __syncthreads();  // every head's dX of the tile is in its slot; the next tile's inputs staged
    // ---- anchor gradients of the tile ----
    {
      const int a = t >> 5, c = t & 31;
      if (d_feat && a0 + a < A) {
        float v = (DX[buf][0][a][c] + DX[buf][1][a][c]) + (DX[buf][2][a][c] + DX[buf][3][a][c]);
        if (has_feat) v += DX[buf][4][a][c];
        float* p = d_feat + (int64_t)(a0 + a) * 32 + c;
        *p = (view == 0 ? 0.f : *p) + v;
      }
      if (t < 16 && a0 + t < A) {
        float gd[3], del[3];
        for (int cc = 0; cc < 3; ++cc) {
          gd[cc] = (DX[buf][0][t][32 + cc] + DX[buf][1][t][32 + cc]) + (DX[buf][2][t][32 + cc] + DX[buf][3][t][32 + cc]);
          if (has_feat) gd[cc] += DX[buf][4][t][32 + cc];
          del[cc] = XB[buf][t][32 + cc];
        }
        float gdist = 0.f;
        if (nx > 0) {
          gdist = (DX[buf][0][t][35] + DX[buf][1][t][35]) + (DX[buf][2][t][35] + DX[buf][3][t][35]);
          if (has_feat) gdist += DX[buf][4][t][35];
        }
        const float dist = XB[buf][t][36];
        const float pr = del[0] * gd[0] + del[1] * gd[1] + del[2] * gd[2];
        for (int cc = 0; cc < 3; ++cc) {
          // through delta = D / |D| (projected, scaled by 1/|D|) and |D| (along delta)
          const float dD = (gd[cc] - del[cc] * pr) / dist + gdist * del[cc];
          if (d_xyz) {
            float* p = &d_xyz[(int64_t)cc * A + a0 + t];
            *p = (view == 0 ? 0.f : *p) + dD;
          }
          dcl[cc] -= dD;
        }
      }
    }
  }
  // ---- the workgroup's camera-centre partial (lanes 0..15 of wave 0) ----
  if (wv == 0) {
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      float x = dcl[cc];
      x += __shfl_xor(x, 8);
      x += __shfl_xor(x, 4);
      x += __shfl_xor(x, 2);
      x += __shfl_xor(x, 1);
      if (lane == 0) w.dcpart[((int64_t)blockIdx.x * dc.n_views + view) * 3 + cc] = x;
    }
  }
  if (!want_params) return;
  // ---- this workgroup's parameter partials ----
  float* P = w.part;
  const int64_t bk = blockIdx.x, nbk = w.nblk_w;
  const bool add = view > 0;
  auto put = [&](int64_t pi, float v) {
    float* dst = P + part_index(pi, bk, nbk);
    *dst = (add ? *dst : 0.f) + v;
  };
#pragma unroll
  for (int i = 0; i < kR; ++i) {
    if (!active || i >= nt) break;
    const int r0 = 16 * (t0 + i);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = r0 + 4 * fg + r;
      if (o < rows) {
        put(w2o + (int64_t)o * kHid + fl, dw2[i][0][r]);
        put(w2o + (int64_t)o * kHid + 16 + fl, dw2[i][1][r]);
      }
    }
    float sb = db2[i];
    sb += __shfl_xor(sb, 16);
    sb += __shfl_xor(sb, 32);
    if (fg == 0 && r0 + fl < rows) put(w2o + (int64_t)rows * kHid + r0 + fl, sb);
  }
  if (hw1 < 0) return;
  const int o1w = (int)ht.off[hw1], oxw = (int)ht.xoff[hw1];  // the head of this wave's dW1
  // extra input columns: the distance weight's gradient is column 35 of the
  // products with X; the temporal weights' gradients are the bias gradient
  // times the view's embedding (accumulated over views by put)
#pragma unroll
  for (int b = 0; b < 2; ++b) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int u = 16 * b + 4 * fg + r;
      put(o1w + u * kIn + fl, dw1[b][0][r]);
      put(o1w + u * kIn + 16 + fl, dw1[b][1][r]);
      if (fl < 3) put(o1w + u * kIn + 32 + fl, dw1[b][2][r]);
      if (fl == 3 && nx > 0) put(oxw + u * nx, dw1[b][2][r]);
    }
    float sb = db1[b];
    sb += __shfl_xor(sb, 16);
    sb += __shfl_xor(sb, 32);
    if (fg == 0) {
      const int u = 16 * b + fl;
      put(o1w + kHid * kIn + u, sb);
      if (nx == 3) {
        put(oxw + u * 3 + 1, sb * lt0);
        put(oxw + u * 3 + 2, sb * lt1);
      }
    }
  }
}

template <int kR>
void launch_k(const DecodeConst& dc, const HeadTable& ht, const DecodeViews& dv, const float* xyz, const float* feat,
              const float* params, const asgs_gaussians& dg, int view, const DecWork& w, float* d_xyz,
              float* d_feat, bool want_params, hipStream_t s) {
  static bool attr_set = false;  // more than 64 KiB of dynamic LDS
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_dec_bwd<kR>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kLdsFloats * (int)sizeof(float));
    attr_set = true;
  }
  hipLaunchKernelGGL(k_dec_bwd<kR>, dim3((unsigned)w.nblk_w), dim3(kBT), kLdsFloats * sizeof(float), s, dc, ht, dv,
                     xyz, feat, params, dg, view, w, d_xyz, d_feat, want_params ? 1 : 0);
}

}  // namespace

int64_t dec_bwd_blocks(int64_t n_anchors) {
  const int64_t tiles = (n_anchors + 15) / 16;
  return tiles < kMaxWG ? tiles : kMaxWG;
}

void launch_dec_bwd(const DecodeConst& dc, const HeadTable& ht, const DecodeViews& dv, const float* xyz,
                    const float* feat, const float* params, const asgs_gaussians& dg, int view, const DecWork& w,
                    float* d_xyz, float* d_feat, bool want_params, hipStream_t s) {
  // second-layer row tiles per wave: the rotation head has ceil(4 k / 16),
  // each feature wave ceil(k / 4)
  if (dc.k <= 12)
    launch_k<3>(dc, ht, dv, xyz, feat, params, dg, view, w, d_xyz, d_feat, want_params, s);
  else
    launch_k<4>(dc, ht, dv, xyz, feat, params, dg, view, w, d_xyz, d_feat, want_params, s);
}

}  // namespace asgs
