// Decoder backward, weight gradients, on the matrix cores (VJP of UP-SLAM
// Eq. 8 and Eq. 9 with respect to the head MLP parameters):
//   dW2_h = sum_a dY_h[a]^T H_h[a]     (rows of head h x 32 hidden units)
//   dW1   = sum_a dZ[a]^T X[a]         (160 hidden units x 35 inputs)
//   db2 = sum_a dY[a],  db1 = sum_a dZ[a]
// over the anchors, with X, H, dY and dZ written by the first backward kernel.
// Persistent workgroups (one per CU) each own a contiguous range of anchors.
// Per 16-anchor chunk the workgroup stages the chunk's rows in LDS (the next
// chunk's loads are in flight meanwhile) and each of its eight waves
// accumulates FP32 16x16x4 MFMAs (K = the chunk's anchors) into its fixed
// share of output tiles: second-layer row tiles w, w+8, ... (both hidden
// halves) and first-layer unit tiles w, w+8 (three input tiles). Each workgroup
// writes one partial of every parameter; a fixed-order reduction over
// workgroups follows (deterministic).
#include <math.h>

#include "decode_shared.h"

namespace asgs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8;
constexpr int kNT = 64 * kWaves;
constexpr int kYS = kMaxRows;  // LDS row strides, each = 16 mod 32 (conflict-free K rows)
constexpr int kHS = 176;
constexpr int kXS = 48;
constexpr int kRT = 4;         // second-layer row tiles per wave (27 at most over 8 waves)
constexpr int kUT = 2;         // first-layer unit tiles per wave (10 at most over 8 waves)
constexpr int kStageF4 = 7;    // float4 per thread staged for the next chunk
static_assert(kMaxRows % 32 == 16, "dY stride");
static_assert(16 * (kMaxRows + 2 * 160 + 36) / 4 <= kStageF4 * kNT, "staging capacity");
static_assert(kRT * kWaves >= 27 && kUT * kWaves >= 10, "tile shares");

ASGS_DEV f4v mfma(float a, float b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

__global__ void __launch_bounds__(kNT) k_dec_wgrad_mfma(DecodeConst dc, HeadTable ht, int view, DecWork w,
                                                        int chunks_per_wg) {
  __shared__ __attribute__((aligned(16))) float sY[16 * kYS];
  __shared__ __attribute__((aligned(16))) float sH[16 * kHS];
  __shared__ __attribute__((aligned(16))) float sZ[16 * kHS];
  __shared__ __attribute__((aligned(16))) float sX[16 * kXS];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);  // wave index, uniform across the wave
  const int fl = lane & 15, fg = lane >> 4;
  const int A = (int)dc.A;
  const int k = dc.k;
  const int nunits = ht.nunits;
  const int nrow4 = w.RP / 4;
  const int nY = 16 * nrow4, nH = 16 * 40, nX = 16 * 9;
  const int ntot = nY + 2 * nH + nX;
  // this wave's second-layer row tiles: LDS column of the tile's first row,
  // rows left in the head, hidden base of the head
  int ycol[kRT], yrows[kRT], hbase[kRT];
#pragma unroll
  for (int i = 0; i < kRT; ++i) ycol[i] = yrows[i] = hbase[i] = 0;
  int nrt_all = 0;
  {
    int rt = 0;
    for (int h = 0; h < kHeads; ++h) {
      const int rows = k * ht.m[h];
      for (int r0 = 0; r0 < rows; r0 += 16, ++rt) {
#pragma unroll
        for (int i = 0; i < kRT; ++i) {
          if (rt == wv + kWaves * i) {
            ycol[i] = ht.row0[h] + r0;
            yrows[i] = rows - r0;
            hbase[i] = 32 * h;
          }
        }
      }
    }
    nrt_all = rt;
  }
  f4v a2[kRT][2];
  f4v a1[kUT][3];
#pragma unroll
  for (int i = 0; i < kRT; ++i) a2[i][0] = a2[i][1] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < kUT; ++i) a1[i][0] = a1[i][1] = a1[i][2] = f4v{0.f, 0.f, 0.f, 0.f};
  float bacc[2] = {0.f, 0.f};
  const int nchunks = (A + 15) / 16;
  const int c_begin = blockIdx.x * chunks_per_wg;
  const int c_end = min(nchunks, c_begin + chunks_per_wg);
  const float4* Y4 = reinterpret_cast<const float4*>(w.dY);
  const float4* H4 = reinterpret_cast<const float4*>(w.H);
  const float4* Z4 = reinterpret_cast<const float4*>(w.dZ);
  const float4* X4 = reinterpret_cast<const float4*>(w.X);
  float4 stage[kStageF4];
  // element e of a chunk: dY rows, then H, dZ, X (row-major per anchor)
  auto fetch = [&](int c) {
    const int a0 = c * 16;
#pragma unroll
    for (int q = 0; q < kStageF4; ++q) {
      const int e = t + q * kNT;
      float4 v = {0.f, 0.f, 0.f, 0.f};
      if (e < nY) {
        const int a = e / nrow4, j = e - a * nrow4;
        if (a0 + a < A) v = Y4[(size_t)(a0 + a) * nrow4 + j];
      } else if (e < nY + nH) {
        const int f = e - nY, a = f / 40, j = f - a * 40;
        if (a0 + a < A) v = H4[(size_t)(a0 + a) * 40 + j];
      } else if (e < nY + 2 * nH) {
        const int f = e - nY - nH, a = f / 40, j = f - a * 40;
        if (a0 + a < A) v = Z4[(size_t)(a0 + a) * 40 + j];
      } else if (e < ntot) {
        const int f = e - nY - 2 * nH, a = f / 9, j = f - a * 9;
        if (a0 + a < A) v = X4[(size_t)(a0 + a) * 9 + j];
      }
      stage[q] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < kStageF4; ++q) {
      const int e = t + q * kNT;
      float* dst = nullptr;
      if (e < nY) {
        const int a = e / nrow4, j = e - a * nrow4;
        dst = &sY[a * kYS + 4 * j];
      } else if (e < nY + nH) {
        const int f = e - nY, a = f / 40, j = f - a * 40;
        dst = &sH[a * kHS + 4 * j];
      } else if (e < nY + 2 * nH) {
        const int f = e - nY - nH, a = f / 40, j = f - a * 40;
        dst = &sZ[a * kHS + 4 * j];
      } else if (e < ntot) {
        const int f = e - nY - 2 * nH, a = f / 9, j = f - a * 9;
        dst = &sX[a * kXS + 4 * j];
      }
      if (dst) *reinterpret_cast<float4*>(dst) = stage[q];
    }
  };
  if (c_begin < c_end) fetch(c_begin);
  for (int c = c_begin; c < c_end; ++c) {
    __syncthreads();  // the previous chunk's readers are done
    store();
    __syncthreads();
    if (c + 1 < c_end) fetch(c + 1);
    // second layer: A = dY^T (M = rows, K = anchors), B = H (K = anchors, N = hidden)
#pragma unroll
    for (int i = 0; i < kRT; ++i) {
      if (wv + kWaves * i < nrt_all) {
        const bool rok = fl < yrows[i];
        const int yc = rok ? ycol[i] + fl : 0;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int a = 4 * ks + fg;
          const float yv = sY[a * kYS + yc];
          const float av = rok ? yv : 0.f;
          a2[i][0] = mfma(av, sH[a * kHS + hbase[i] + fl], a2[i][0]);
          a2[i][1] = mfma(av, sH[a * kHS + hbase[i] + 16 + fl], a2[i][1]);
        }
      }
    }
    // first layer: A = dZ^T (M = units, K = anchors), B = X (K = anchors, N = inputs)
#pragma unroll
    for (int i = 0; i < kUT; ++i) {
      const int ut = wv + kWaves * i;
      if (16 * ut < nunits) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int a = 4 * ks + fg;
          const float av = sZ[a * kHS + 16 * ut + fl];
          a1[i][0] = mfma(av, sX[a * kXS + fl], a1[i][0]);
          a1[i][1] = mfma(av, sX[a * kXS + 16 + fl], a1[i][1]);
          const float x2 = sX[a * kXS + 32 + (fl & 3)];
          a1[i][2] = mfma(av, fl < 4 ? x2 : 0.f, a1[i][2]);
        }
      }
    }
    // bias sums: thread t owns entries t and t + 512 (rows, then hidden units)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = t + q * kNT;
      float s = 0.f;
      if (e < ht.nrows) {
        for (int a = 0; a < 16; ++a) s += sY[a * kYS + e];
      } else if (e < ht.nrows + nunits) {
        for (int a = 0; a < 16; ++a) s += sZ[a * kHS + e - ht.nrows];
      }
      bacc[q] += s;
    }
  }
  // ---- this workgroup's partial of every parameter ----
  float* P = w.part;
  const int64_t bk = blockIdx.x, nbk = w.nblk_w;
  const bool add = view > 0;
  auto put = [&](int64_t pi, float v) {
    float* dst = P + part_index(pi, bk, nbk);
    *dst = (add ? *dst : 0.f) + v;
  };
#pragma unroll
  for (int i = 0; i < kRT; ++i) {
    if (wv + kWaves * i >= nrt_all) continue;
    const int h = hbase[i] / 32;
    const int r_in_head = ycol[i] - ht.row0[h];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = 4 * fg + r;
      if (rr < yrows[i]) {
        const int64_t base = ht.off[h] + kHid * kIn + kHid + (int64_t)(r_in_head + rr) * kHid;
        put(base + fl, a2[i][0][r]);
        put(base + 16 + fl, a2[i][1][r]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kUT; ++i) {
    const int ut = wv + kWaves * i;
    if (16 * ut >= nunits) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int u = 16 * ut + 4 * fg + r;
      const int64_t base = ht.off[u >> 5] + (int64_t)(u & 31) * kIn;
      put(base + fl, a1[i][0][r]);
      put(base + 16 + fl, a1[i][1][r]);
      if (fl < 3) put(base + 32 + fl, a1[i][2][r]);
    }
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = t + q * kNT;
    if (e < ht.nrows) {
      const int h = row_head(ht, e);
      put(ht.off[h] + kHid * kIn + kHid + (int64_t)k * ht.m[h] * kHid + (e - ht.row0[h]), bacc[q]);
    } else if (e < ht.nrows + nunits) {
      const int u = e - ht.nrows;
      put(ht.off[u >> 5] + kHid * kIn + (u & 31), bacc[q]);
    }
  }
}

}  // namespace

int64_t wgrad_blocks(int64_t n_anchors) {
  const int64_t nchunks = (n_anchors + 15) / 16;
  return nchunks < kWgradMaxWG ? nchunks : kWgradMaxWG;
}

void launch_dec_wgrad_mfma(const DecodeConst& dc, const HeadTable& ht, int view, const DecWork& w, hipStream_t s) {
  const int64_t nchunks = (dc.A + 15) / 16;
  const int64_t nb = w.nblk_w;
  const int cpw = (int)((nchunks + nb - 1) / nb);
  hipLaunchKernelGGL(k_dec_wgrad_mfma, dim3((unsigned)nb), dim3(kNT), 0, s, dc, ht, view, w, cpw);
}

}  // namespace asgs
