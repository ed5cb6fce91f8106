// Decoder backward in one pass on the matrix cores (VJP of UP-SLAM Eq. 8 and
// Eq. 9): for each 16-anchor tile the workgroup recomputes the first layer
// and each head's outputs, then forms every gradient with FP32 16x16x4 MFMAs
// and keeps the parameter gradients in registers across its tiles:
//   Z_h = X W1_h^T + b1_h, H_h = act(Z_h)       (ReLU; SoftPlus for features)
//   Y_h = H_h W2_h^T + b2_h, dY = dL/d(decoded) * act'(Y_h)
//   dW2_h += dY^T H_h, db2_h += sum_a dY        (K = the tile's anchors)
//   dH_h = dY W2_h, dZ_h = dH_h * act'(Z_h)     (act' from H)
//   dW1_h += dZ_h^T X, db1_h += sum_a dZ_h
//   dX = sum_h dZ_h W1_h -> anchor feature and view-direction gradients
// The four waves of a workgroup split the heads (opacity + colour, scale +
// rotation, and the feature head's output rows in two halves whose dH
// partial sums are combined through LDS), so no intermediate leaves the CU.
// Each workgroup writes one partial of every parameter at the end; a
// fixed-order reduction over workgroups follows (deterministic).
//
// Layouts of v_mfma_f32_16x16x4f32 (wave64): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] and receives D rows 4 (l / 16) + r, column l % 16.
// With K-step ks taken as anchors 4 (l / 16) + ks, the D tiles of dY and dZ
// (rows = anchors) are directly the A operands of the weight-gradient
// products; products with K over rows or units go through a per-wave LDS
// transpose.
#include <math.h>

#include "decode_shared.h"

namespace asgs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kNT = 64 * kWaves;
constexpr int kW1S = 37;   // LDS row of a first-layer weight row (35 inputs + zero pad)
constexpr int kW2S = 33;   // LDS row of a second-layer weight row (32 hidden units)
constexpr int kXS = 37;
constexpr int kHW = 65;    // per-wave H / dZ rows: up to two heads (64 units)
constexpr int kTS = 33;
constexpr int kMaxG = 27 * 16 * ASGS_MAX_K;  // upstream gradients of one tile (all heads)
constexpr int kMaxWG = 256;

ASGS_DEV f4v mfma(float a, float b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

ASGS_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct Smem {
  float W1s[160 * kW1S];
  float b1s[160];
  float W2s[kMaxRows * kW2S];
  float b2s[kMaxRows];
  float X[16][kXS];
  float dir[16][4];            // unit view direction and distance of each anchor
  float G[kMaxG];              // dL/d(decoded) of the tile: per (head, component) a run of 16 k values
  float H[kWaves][16][kHW];    // per wave: H of its heads, then dZ
  float T[kWaves][16][kTS];    // per wave: transposes
  float DX[kWaves][16][kXS];   // per wave: dX partial
  float DH[2][16][33];         // feature head: dH partial of each half
  float red[kWaves][4];
};

// Per-head context shared by the steps below.
struct HeadCtx {
  int h, m, rows, row0, gbase, hcol;
};

// First layer of head h for the tile: H (D layout) into the wave's LDS rows.
ASGS_DEV void head_forward(const Smem& S, float (*Hw)[kHW], const HeadCtx& c, int fl, int fg) {
  f4v z0 = {0.f, 0.f, 0.f, 0.f}, z1 = z0;
#pragma unroll
  for (int ks = 0; ks < 9; ++ks) {
    const int kk = 4 * ks + fg;
    const float av = S.X[fl][kk];
    z0 = mfma(av, S.W1s[(32 * c.h + fl) * kW1S + kk], z0);
    z1 = mfma(av, S.W1s[(32 * c.h + 16 + fl) * kW1S + kk], z1);
  }
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int u = 16 * half + fl;
    const float b = S.b1s[32 * c.h + u];
    const f4v z = half ? z1 : z0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float zz = z[r] + b;
      Hw[4 * fg + r][c.hcol + u] = c.h == 4 ? softplus(zz) : fmaxf(zz, 0.f);
    }
  }
}

// Output row tiles [t0, t0 + nt) of head h (nt <= MAXT): dY, dW2, db2 and the
// partial dH over these rows.
constexpr int kAcc = 8;  // second-layer row tiles accumulated per wave

template <int MAXT, int OFF>
ASGS_DEV void head_rows(const Smem& S, float (*Hw)[kHW], float (*Tw)[kTS], const HeadCtx& c, int t0, int nt, int k,
                        float l_s, f4v (&dw2)[kAcc][2], float (&db2)[kAcc], f4v& dh0, f4v& dh1, int fl, int fg) {
  static_assert(OFF + MAXT <= kAcc, "accumulator slots");
#pragma unroll
  for (int i = 0; i < MAXT; ++i) {
    if (i >= nt) break;
    const int r0 = 16 * (t0 + i);
    const int orow = r0 + fl;
    const bool rok = orow < c.rows;
    const int wrow = c.row0 + (rok ? orow : 0);
    f4v y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int kk = 4 * ks + fg;
      y = mfma(Hw[fl][c.hcol + kk], S.W2s[wrow * kW2S + kk], y);
    }
    const float bias = S.b2s[wrow];
    const int gi = orow / c.m, gc = orow - gi * c.m;
    f4v dy;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = 4 * fg + r;
      const float g = S.G[c.gbase + gc * 16 * k + a * k + gi];
      dy[r] = rok ? g * act_grad(c.h, y[r] + bias, l_s) : 0.f;
      Tw[a][fl] = dy[r];
    }
    db2[OFF + i] += (dy[0] + dy[1]) + (dy[2] + dy[3]);
    // dW2 += dY^T H: A = own dY registers (K = anchors 4 fg + ks), B = H rows
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int a = 4 * fg + ks;
      dw2[OFF + i][0] = mfma(dy[ks], Hw[a][c.hcol + fl], dw2[OFF + i][0]);
      dw2[OFF + i][1] = mfma(dy[ks], Hw[a][c.hcol + 16 + fl], dw2[OFF + i][1]);
    }
    wave_sync();
    // dH += dY W2 (K = the tile's rows, through the transpose)
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kr = r0 + 4 * ks + fg;
      const bool kok = kr < c.rows;
      const int wr = c.row0 + (kok ? kr : 0);
      const float av = Tw[fl][4 * ks + fg];
      const float b0 = S.W2s[wr * kW2S + fl], b1 = S.W2s[wr * kW2S + 16 + fl];
      dh0 = mfma(av, kok ? b0 : 0.f, dh0);
      dh1 = mfma(av, kok ? b1 : 0.f, dh1);
    }
    wave_sync();
  }
}

// dZ of head h from the complete dH; optionally dW1/db1 and the dX partial.
ASGS_DEV void head_dz(const Smem& S, float (*Hw)[kHW], float (*Tw)[kTS], const HeadCtx& c, f4v dh0, f4v dh1,
                      bool do_w1, f4v (&dw1)[2][3], float (&db1)[2], bool do_dx, f4v (&dx)[3], int fl, int fg) {
  f4v dz[2];
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int u = 16 * half + fl;
    const f4v dh = half ? dh1 : dh0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = 4 * fg + r;
      const float hv = Hw[a][c.hcol + u];
      dz[half][r] = c.h == 4 ? dh[r] * (1.f - expf(-hv)) : (hv > 0.f ? dh[r] : 0.f);
      Tw[a][u] = dz[half][r];
    }
  }
  if (do_w1) {
    // dW1 += dZ^T X: A = own dZ registers (K = anchors 4 fg + ks), B = X rows
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      db1[half] += (dz[half][0] + dz[half][1]) + (dz[half][2] + dz[half][3]);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int a = 4 * fg + ks;
#pragma unroll
        for (int ct = 0; ct < 3; ++ct) {
          const int cc = 16 * ct + fl;
          dw1[half][ct] = mfma(dz[half][ks], cc < kXS ? S.X[a][cc] : 0.f, dw1[half][ct]);
        }
      }
    }
  }
  wave_sync();
  if (do_dx) {
    // dX += dZ W1_h (K = the head's 32 units, through the transpose)
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int u = 4 * ks + fg;
      const float av = Tw[fl][u];
      const float* w1 = &S.W1s[(32 * c.h + u) * kW1S];
#pragma unroll
      for (int ct = 0; ct < 3; ++ct) {
        const int cc = 16 * ct + fl;
        dx[ct] = mfma(av, cc < kW1S ? w1[cc] : 0.f, dx[ct]);
      }
    }
  }
  wave_sync();
}

__global__ void __launch_bounds__(kNT) k_dec_bwd_fused(DecodeConst dc, HeadTable ht, DecodeViews dv,
                                                      const float* __restrict__ xyz,
                                                      const float* __restrict__ feat,
                                                      const float* __restrict__ params, asgs_gaussians dg,
                                                      int view, DecWork w, float* d_xyz, float* d_feat,
                                                      int want_params) {
  __shared__ __attribute__((aligned(16))) Smem S;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int fl = lane & 15, fg = lane >> 4;
  const int A = (int)dc.A;
  const int k = dc.k;
  const int n = A * k;
  const int nunits = ht.nunits;
  const bool has_feat = ht.m[4] > 0;
  // ---- stage the weights ----
  for (int e0 = t; e0 < nunits * kW1S; e0 += 8 * kNT) {
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + q * kNT;
      const int u = e / kW1S, c = e - u * kW1S;
      v[q] = (e < nunits * kW1S && c < kIn) ? params[ht.off[u >> 5] + (u & 31) * kIn + c] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (e0 + q * kNT < nunits * kW1S) S.W1s[e0 + q * kNT] = v[q];
  }
  for (int u = t; u < nunits; u += kNT) S.b1s[u] = params[ht.off[u >> 5] + kHid * kIn + (u & 31)];
  for (int h = 0; h < kHeads; ++h) {
    if (ht.m[h] == 0) continue;
    const int rows = k * ht.m[h];
    const float* W2 = params + ht.off[h] + kHid * kIn + kHid;
    for (int e0 = t; e0 < rows * kHid; e0 += 8 * kNT) {
      float v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = e0 + q * kNT;
        v[q] = e < rows * kHid ? W2[e] : 0.f;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = e0 + q * kNT;
        if (e < rows * kHid) S.W2s[(ht.row0[h] + (e >> 5)) * kW2S + (e & 31)] = v[q];
      }
    }
    for (int r = t; r < rows; r += kNT) S.b2s[ht.row0[h] + r] = W2[rows * kHid + r];
  }
  // ---- this wave's heads ----
  HeadCtx hc[2];
  int nheads = 0;
  int ft0 = 0, fnt = 0;  // feature head: first row tile and count of this wave
  {
    auto mk = [&](int h, int slot) {
      HeadCtx c;
      c.h = h;
      c.m = ht.m[h];
      c.rows = k * c.m;
      c.row0 = ht.row0[h];
      int gb = 0;
      for (int q = 0; q < h; ++q) gb += ht.m[q] * 16 * k;
      c.gbase = gb;
      c.hcol = 32 * slot;
      return c;
    };
    if (wv < 2) {
      hc[0] = mk(2 * wv, 0);
      hc[1] = mk(2 * wv + 1, 1);
      nheads = 2;
    } else if (has_feat) {
      hc[0] = mk(4, 0);
      nheads = 1;
      const int T = (hc[0].rows + 15) / 16;
      const int half = (T + 1) / 2;
      ft0 = wv == 2 ? 0 : half;
      fnt = wv == 2 ? half : T - half;
    }
  }
  // accumulators: second-layer row tiles at static slots (wave 0: opacity 0,
  // colour 1..3; wave 1: scale 0..2, rotation 3..6; waves 2, 3: feature 0..7)
  f4v dw2[kAcc][2];
  float db2[kAcc];
#pragma unroll
  for (int i = 0; i < kAcc; ++i) {
    dw2[i][0] = dw2[i][1] = f4v{0.f, 0.f, 0.f, 0.f};
    db2[i] = 0.f;
  }
  f4v dw1[2][2][3];
  float db1[2][2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      dw1[j][q][0] = dw1[j][q][1] = dw1[j][q][2] = f4v{0.f, 0.f, 0.f, 0.f};
      db1[j][q] = 0.f;
    }
  float dcacc[3] = {0.f, 0.f, 0.f};
  float (*Hw)[kHW] = S.H[wv];
  float (*Tw)[kTS] = S.T[wv];
  const int ngrid = (A + 15) / 16;
  // features of a tile, fetched one tile ahead
  float xpre[2];
  auto fetch_x = [&](int tile) {
    const int a0 = tile * 16;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = t + q * kNT;
      const int a = e >> 5, c = e & 31;
      xpre[q] = a0 + a < A ? feat[(size_t)(a0 + a) * 32 + c] : 0.f;
    }
  };
  // upstream gradients of a tile straight into LDS: per (head, component) the
  // tile's run of 16 k values, coalesced; loads issued in batches of eight
  int gtot = 0;
  for (int h = 0; h < kHeads; ++h) gtot += ht.m[h] * 16 * k;
  const int run = 16 * k;
  auto load_g = [&](int tile) {
    const size_t a0k = (size_t)tile * 16 * k;
    for (int e0 = t; e0 < gtot; e0 += 8 * kNT) {
      float v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = e0 + q * kNT;
        v[q] = 0.f;
        if (e < gtot) {
          const int pl = e / run, o = e - pl * run;  // plane index over (head, component)
          int h = 0, rem = pl;
          while (rem >= ht.m[h]) {
            rem -= ht.m[h];
            ++h;
          }
          const size_t gidx = a0k + o;
          if (gidx < (size_t)n) v[q] = out_plane(dg, view, h, rem, n)[gidx];
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (e0 + q * kNT < gtot) S.G[e0 + q * kNT] = v[q];
    }
  };
  if ((int)blockIdx.x < ngrid) fetch_x(blockIdx.x);
  for (int tile = blockIdx.x; tile < ngrid; tile += gridDim.x) {
    const int a0 = tile * 16;
    __syncthreads();  // weights staged / the previous tile's readers are done
    load_g(tile);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = t + q * kNT;
      S.X[e >> 5][e & 31] = xpre[q];
    }
    if (t < 16) {
      float D[3] = {0.f, 0.f, 0.f}, dist = 1.f;
      if (a0 + t < A) {
        for (int c = 0; c < 3; ++c) D[c] = xyz[(size_t)c * A + a0 + t] - dv.c[view][c];
        dist = sqrtf(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
        for (int c = 0; c < 3; ++c) D[c] /= dist;
      }
      for (int c = 0; c < 3; ++c) {
        S.X[t][32 + c] = D[c];
        S.dir[t][c] = D[c];
      }
      S.X[t][35] = 0.f;
      S.X[t][36] = 0.f;
      S.dir[t][3] = dist;
    }
    __syncthreads();
    if (tile + (int)gridDim.x < ngrid) fetch_x(tile + gridDim.x);
    f4v dx[3];
#pragma unroll
    for (int ct = 0; ct < 3; ++ct) dx[ct] = f4v{0.f, 0.f, 0.f, 0.f};
    f4v fdh0 = {0.f, 0.f, 0.f, 0.f}, fdh1 = fdh0;
    if (wv < 2) {
#pragma unroll
      for (int j = 0; j < 2; ++j) head_forward(S, Hw, hc[j], fl, fg);
      wave_sync();
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        f4v dh0 = {0.f, 0.f, 0.f, 0.f}, dh1 = dh0;
        const HeadCtx& c = hc[j];
        const int T = (c.rows + 15) / 16;
        if (wv == 0) {
          if (j == 0) head_rows<1, 0>(S, Hw, Tw, c, 0, T, k, dc.l_s, dw2, db2, dh0, dh1, fl, fg);
          else head_rows<3, 1>(S, Hw, Tw, c, 0, T, k, dc.l_s, dw2, db2, dh0, dh1, fl, fg);
        } else {
          if (j == 0) head_rows<3, 0>(S, Hw, Tw, c, 0, T, k, dc.l_s, dw2, db2, dh0, dh1, fl, fg);
          else head_rows<4, 3>(S, Hw, Tw, c, 0, T, k, dc.l_s, dw2, db2, dh0, dh1, fl, fg);
        }
        head_dz(S, Hw, Tw, c, dh0, dh1, true, dw1[j], db1[j], true, dx, fl, fg);
      }
    } else if (nheads == 1) {
      head_forward(S, Hw, hc[0], fl, fg);
      wave_sync();
      head_rows<8, 0>(S, Hw, Tw, hc[0], ft0, fnt, k, dc.l_s, dw2, db2, fdh0, fdh1, fl, fg);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        S.DH[wv - 2][4 * fg + r][fl] = fdh0[r];
        S.DH[wv - 2][4 * fg + r][16 + fl] = fdh1[r];
      }
    }
    __syncthreads();  // feature-head dH halves visible
    if (nheads == 1) {
      // the full dH of the feature head, summed in a fixed order on both waves
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        fdh0[r] = S.DH[0][4 * fg + r][fl] + S.DH[1][4 * fg + r][fl];
        fdh1[r] = S.DH[0][4 * fg + r][16 + fl] + S.DH[1][4 * fg + r][16 + fl];
      }
      head_dz(S, Hw, Tw, hc[0], fdh0, fdh1, wv == 2, dw1[0], db1[0], wv == 3, dx, fl, fg);
    }
#pragma unroll
    for (int ct = 0; ct < 3; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (16 * ct + fl < kXS) S.DX[wv][4 * fg + r][16 * ct + fl] = dx[ct][r];
    __syncthreads();
    // ---- anchor gradients: the four waves' dX partials in a fixed order ----
    for (int e = t; e < 16 * 32; e += kNT) {
      const int a = e >> 5, c = e & 31;
      if (d_feat && a0 + a < A) {
        const float v = (S.DX[0][a][c] + S.DX[1][a][c]) + (S.DX[2][a][c] + S.DX[3][a][c]);
        float* p = &d_feat[(size_t)(a0 + a) * 32 + c];
        *p = (view == 0 ? 0.f : *p) + v;
      }
    }
    if (t < 64) {
      float dcl[3] = {0.f, 0.f, 0.f};
      if (t < 16 && a0 + t < A) {
        float gd[3];
        for (int c = 0; c < 3; ++c)
          gd[c] = (S.DX[0][t][32 + c] + S.DX[1][t][32 + c]) + (S.DX[2][t][32 + c] + S.DX[3][t][32 + c]);
        const float* del = S.dir[t];
        const float pr = del[0] * gd[0] + del[1] * gd[1] + del[2] * gd[2];
        for (int c = 0; c < 3; ++c) {
          const float dD = (gd[c] - del[c] * pr) / del[3];
          if (d_xyz) {
            float* p = &d_xyz[(size_t)c * A + a0 + t];
            *p = (view == 0 ? 0.f : *p) + dD;
          }
          dcl[c] = -dD;
        }
      }
      for (int c = 0; c < 3; ++c) {
        float x = dcl[c];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        dcacc[c] += x;
      }
    }
  }
  // ---- this workgroup's partials ----
  if (t < 3) {
    const float v = t == 0 ? dcacc[0] : (t == 1 ? dcacc[1] : dcacc[2]);
    w.dcpart[((int64_t)blockIdx.x * dc.n_views + view) * 3 + t] = v;
  }
  if (!want_params) return;
  float* P = w.part;
  const int64_t bk = blockIdx.x, nbk = w.nblk_w;
  const bool add = view > 0;
  auto put = [&](int64_t pi, float v) {
    float* dst = P + part_index(pi, bk, nbk);
    *dst = (add ? *dst : 0.f) + v;
  };
  // second-layer weights and biases of the row tiles this wave owns; slot
  // OFF + i holds row tile t0 + i of head c
  auto put_rows = [&](const HeadCtx& c, int t0, int nt, int off) {
    const int64_t wb = ht.off[c.h] + kHid * kIn + kHid;
#pragma unroll
    for (int slot = 0; slot < kAcc; ++slot) {
      const int i = slot - off;
      if (i < 0 || i >= nt) continue;
      const int r0 = 16 * (t0 + i);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + 4 * fg + r;
        if (row < c.rows) {
          put(wb + (int64_t)row * kHid + fl, dw2[slot][0][r]);
          put(wb + (int64_t)row * kHid + 16 + fl, dw2[slot][1][r]);
        }
      }
      // bias: lanes of row fl summed over the four anchor groups
      float sb = db2[slot];
      sb += __shfl_xor(sb, 16);
      sb += __shfl_xor(sb, 32);
      if (fg == 0 && r0 + fl < c.rows) put(wb + (int64_t)c.rows * kHid + r0 + fl, sb);
    }
  };
  auto put_units = [&](const HeadCtx& c, const f4v (&d)[2][3], const float (&b)[2]) {
    const int64_t w1b = ht.off[c.h];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int u = 16 * half + 4 * fg + r;
        put(w1b + (int64_t)u * kIn + fl, d[half][0][r]);
        put(w1b + (int64_t)u * kIn + 16 + fl, d[half][1][r]);
        if (fl < 3) put(w1b + (int64_t)u * kIn + 32 + fl, d[half][2][r]);
      }
      float sb = b[half];
      sb += __shfl_xor(sb, 16);
      sb += __shfl_xor(sb, 32);
      if (fg == 0) put(w1b + kHid * kIn + 16 * half + fl, sb);
    }
  };
  if (wv < 2) {
    put_rows(hc[0], 0, (hc[0].rows + 15) / 16, 0);
    put_rows(hc[1], 0, (hc[1].rows + 15) / 16, wv == 0 ? 1 : 3);
    put_units(hc[0], dw1[0], db1[0]);
    put_units(hc[1], dw1[1], db1[1]);
  } else if (nheads == 1) {
    put_rows(hc[0], ft0, fnt, 0);
    if (wv == 2) put_units(hc[0], dw1[0], db1[0]);
  }
}

}  // namespace

int64_t dec_bwd_fused_blocks(int64_t n_anchors) {
  const int64_t tiles = (n_anchors + 15) / 16;
  return tiles < kMaxWG ? tiles : kMaxWG;
}

void launch_dec_bwd_fused(const DecodeConst& dc, const HeadTable& ht, const DecodeViews& dv, const float* xyz,
                          const float* feat, const float* params, const asgs_gaussians& dg, int view,
                          const DecWork& w, float* d_xyz, float* d_feat, bool want_params, hipStream_t s) {
  hipLaunchKernelGGL(k_dec_bwd_fused, dim3((unsigned)w.nblk_w), dim3(kNT), 0, s, dc, ht, dv, xyz, feat, params, dg,
                     view, w, d_xyz, d_feat, want_params ? 1 : 0);
}

}  // namespace asgs
