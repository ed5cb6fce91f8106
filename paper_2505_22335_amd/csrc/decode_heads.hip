// Decoder forward on the matrix cores (UP-SLAM Eq. 8 and Eq. 9), per view and
// head group. For each 16-anchor tile a workgroup forms the first layer and
// the second-layer rows of its heads with FP32 16x16x4 MFMAs:
//   Z_h = X W1_h^T + b1_h, H_h = act(Z_h)       (ReLU; SoftPlus for features)
//   Y_h = H_h W2_h^T + b2_h, decoded = out_act(Y_h)
// The heads are split over two kinds of workgroup that run side by side
// (blockIdx.y): group 0 takes opacity, colour, scale and rotation, one head
// per wave; group 1 takes the feature head: its hidden layer is formed once
// (one 16-unit half on each of waves 0 and 1) and its output rows are split
// over the four waves.
//
// Layouts of v_mfma_f32_16x16x4f32 (wave64): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] and receives D rows 4 (l / 16) + r, column l % 16.
#include <math.h>

#include "decode_shared.h"

namespace asgs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kNT = 64 * kWaves;
constexpr int kW1S = 37;   // LDS row of a first-layer weight row (35 inputs + zero pad)
constexpr int kW2S = 33;   // LDS row of a second-layer weight row (32 hidden units)
constexpr int kXS = 37;    // LDS row of an anchor input (35 + distance column + pad)
constexpr int kHS = 37;    // per-wave H rows (32 units + pad)
constexpr int kAcc = 4;    // second-layer row tiles accumulated per wave
constexpr int kMaxFwdWG = 384;

ASGS_DEV f4v mfma(float a, float b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

ASGS_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Float offsets of the LDS arrays of one group (dynamic shared memory).
struct GroupLds {
  int W1s, b1s, W2s, b2s, X, G, H, total;
};

// What one group of heads needs: its heads [hbase, hbase + nheads), their
// first-layer units and second-layer rows counted from the group's start, and
// the start of each (head, component) run of 16 k upstream gradients in G.
struct GroupDesc {
  int hbase, nheads, nunits, nrows, gtot;
  int lrow0[kHeads];
  int gbase[kHeads];
  GroupLds L;
};

struct GroupPair {
  GroupDesc g[2];
};

struct HeadCtx {
  int h, m, rows, lrow0, lunit0, gbase;
};

// Output row of lane column fl in row tile t0 + i, as (Gaussian of the
// anchor, component), fixed for all tiles.
struct RowMap {
  int gi[4], gc[4];
};

struct Views {
  float* W1s;
  float* b1s;
  float* W2s;
  float* b2s;
  float (*X)[kXS];
  float* G;
  float (*H)[16][kHS];
};

ASGS_DEV Views carve(float* smem, const GroupLds& L) {
  Views S;
  S.W1s = smem + L.W1s;
  S.b1s = smem + L.b1s;
  S.W2s = smem + L.W2s;
  S.b2s = smem + L.b2s;
  S.X = reinterpret_cast<float (*)[kXS]>(smem + L.X);
  S.G = smem + L.G;
  S.H = reinterpret_cast<float (*)[16][kHS]>(smem + L.H);
  return S;
}

// First layer of head c for the tile: H (rows = anchors) into the wave's rows.
ASGS_DEV void head_forward(const Views& S, float (*Hw)[kHS], const HeadCtx& c, int fl, int fg) {
  f4v z0 = {0.f, 0.f, 0.f, 0.f}, z1 = z0;
#pragma unroll
  for (int ks = 0; ks < 9; ++ks) {
    const int kk = 4 * ks + fg;
    const float av = S.X[fl][kk];
    z0 = mfma(av, S.W1s[(c.lunit0 + fl) * kW1S + kk], z0);
    z1 = mfma(av, S.W1s[(c.lunit0 + 16 + fl) * kW1S + kk], z1);
  }
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int u = 16 * half + fl;
    const float b = S.b1s[c.lunit0 + u];
    const f4v z = half ? z1 : z0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float zz = z[r] + b;
      Hw[4 * fg + r][u] = c.h == 4 ? fsoftplus(zz) : fmaxf(zz, 0.f);
    }
  }
}

// One 16-unit half of the first layer of head c (the feature head's units
// are split over two waves that write one shared H).
ASGS_DEV void head_forward_half(const Views& S, float (*Hw)[kHS], const HeadCtx& c, int half, int fl, int fg) {
  f4v z = {0.f, 0.f, 0.f, 0.f};
  const int u = 16 * half + fl;
#pragma unroll
  for (int ks = 0; ks < 9; ++ks) {
    const int kk = 4 * ks + fg;
    z = mfma(S.X[fl][kk], S.W1s[(c.lunit0 + u) * kW1S + kk], z);
  }
  const float b = S.b1s[c.lunit0 + u];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float zz = z[r] + b;
    Hw[4 * fg + r][u] = c.h == 4 ? fsoftplus(zz) : fmaxf(zz, 0.f);
  }
}

// The head and second-layer row tiles [t0, t0 + nt) of wave wv: group 0 one
// head per wave; group 1 the feature head's row tiles over the four waves,
// the first ones taking one more.
ASGS_DEV void assign_rows(const GroupDesc& gd, const HeadTable& ht, int grp, int wv, int k, int fl, HeadCtx& hc,
                          RowMap& rm, int& t0, int& nt) {
  hc.h = grp == 0 ? wv : 4;
  hc.m = ht.m[hc.h];
  hc.rows = k * hc.m;
  hc.lrow0 = gd.lrow0[hc.h];
  hc.lunit0 = 32 * (hc.h - gd.hbase);
  hc.gbase = gd.gbase[hc.h];
  const int T = (hc.rows + 15) / 16;
  if (grp == 0) {
    t0 = 0;
    nt = T;
  } else {
    const int base = T / kWaves, extra = T - base * kWaves;
    nt = base + (wv < extra ? 1 : 0);
    t0 = wv * base + (wv < extra ? wv : extra);
  }
#pragma unroll
  for (int i = 0; i < kAcc; ++i) {
    const int orow = 16 * (t0 + i) + fl;
    rm.gi[i] = orow / hc.m;
    rm.gc[i] = orow - rm.gi[i] * hc.m;
  }
}

// The group's weights into LDS: first-layer rows padded to kW1S, second-layer
// rows to kW2S. Head h's packed parameters start at ht.off[h]: W1 [32][35],
// b1 [32], W2 [rows][32], b2 [rows]; its extra input columns [32][nx] sit at
// ht.xoff[h]. The distance weight (or zero) fills pad column 35, matching the
// distance in column 35 of the anchor rows; the temporal weights are folded
// into the bias with the view's embedding lt (the time input is the same for
// every anchor of a view), the last pad column stays zero. Every load is
// issued before the first store. The index arithmetic is branch-free: the
// head of an element is chosen by comparisons with the group's (uniform) head
// boundaries, a lane past the end loads the last element and stores it into
// the never-read pad column of the first second-layer row.
ASGS_DEV void stage_weights(const Views& S, const GroupDesc& gd, const HeadTable& ht, const float* params, int t,
                            float lt0, float lt1) {
  constexpr int kW1 = kHid * kIn;                          // first-layer weights per head
  constexpr int kQ1 = (4 * kW1 + kNT - 1) / kNT;           // first-layer elements per thread
  constexpr int kQ2 = 16 * ASGS_MAX_K * kHid / kNT;        // second-layer elements per thread
  static_assert(4 * kW1 <= 4480, "the unit index below divides by 35 with a multiply and shift");
  // per head j of the group: source base of its first-layer elements (indexed
  // by the group's element e = j * kW1 + u * kIn + c), of its second-layer
  // elements (e = 32 * local row + c), of b1 (by unit) and b2 (by local row);
  // absent heads repeat the last one and start past the end
  int o1[4], o2[4], ob1[4], ob2[4], r0[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int jj = j < gd.nheads ? j : gd.nheads - 1;
    const int h = gd.hbase + jj;
    const int rows = (jj + 1 < gd.nheads ? gd.lrow0[h + 1] : gd.nrows) - gd.lrow0[h];
    r0[j] = j < gd.nheads ? gd.lrow0[h] : gd.nrows;
    o1[j] = ht.off[h] - jj * kW1;
    o2[j] = ht.off[h] + kW1 + kHid - kHid * gd.lrow0[h];
    ob1[j] = ht.off[h] + kW1 - kHid * jj;
    ob2[j] = ht.off[h] + kW1 + kHid + kHid * rows - gd.lrow0[h];
  }
  const int n1 = gd.nunits * kIn, n2 = gd.nrows * kHid;
  float* const trash = S.W2s + kHid;  // column 32 of second-layer row 0: never read
  float v1[kQ1], v2[kQ2];
  int d1[kQ1], d2[kQ2];
#pragma unroll
  for (int q = 0; q < kQ1; ++q) {
    const int e = t + q * kNT;
    const int ec = e < n1 ? e : n1 - 1;
    int base = o1[0];
    base = ec >= kW1 ? o1[1] : base;
    base = ec >= 2 * kW1 ? o1[2] : base;
    base = ec >= 3 * kW1 ? o1[3] : base;
    v1[q] = params[(unsigned)(base + ec)];
    const int u = (ec * 3745) >> 17;  // ec / 35, exact for ec < 4480
    d1[q] = e < n1 ? ec + (kW1S - kIn) * u : -1;  // row u * kW1S, column ec - kIn * u
  }
#pragma unroll
  for (int q = 0; q < kQ2; ++q) {
    const int e = t + q * kNT;
    const int ec = e < n2 ? e : n2 - 1;
    const int lr = ec >> 5;
    int base = o2[0];
    base = lr >= r0[1] ? o2[1] : base;
    base = lr >= r0[2] ? o2[2] : base;
    base = lr >= r0[3] ? o2[3] : base;
    v2[q] = params[(unsigned)(base + ec)];
    d2[q] = e < n2 ? ec + (kW2S - kHid) * lr : -1;  // row lr * kW2S, column ec & 31
  }
  const int tb1 = t < gd.nunits ? t : gd.nunits - 1;
  int bb1 = ob1[0];
  bb1 = tb1 >= 32 ? ob1[1] : bb1;
  bb1 = tb1 >= 64 ? ob1[2] : bb1;
  bb1 = tb1 >= 96 ? ob1[3] : bb1;
  const float vb1 = params[(unsigned)(bb1 + tb1)];
  const int tb2 = t < gd.nrows ? t : gd.nrows - 1;
  int bb2 = ob2[0];
  bb2 = tb2 >= r0[1] ? ob2[1] : bb2;
  bb2 = tb2 >= r0[2] ? ob2[2] : bb2;
  bb2 = tb2 >= r0[3] ? ob2[3] : bb2;
  const float vb2 = params[(unsigned)(bb2 + tb2)];
#pragma unroll
  for (int q = 0; q < kQ1; ++q) *(d1[q] >= 0 ? S.W1s + d1[q] : trash) = v1[q];
#pragma unroll
  for (int q = 0; q < kQ2; ++q) *(d2[q] >= 0 ? S.W2s + d2[q] : trash) = v2[q];
  // the extra columns after the stores (one more round trip, only for the
  // scene-variant inputs; loading them with the rest costs registers)
  float vxd = 0.f, vxs = 0.f, vxc = 0.f;
  if (ht.nx > 0) {
    const int xsrc = ht.xoff[gd.hbase + (tb1 >> 5)] + (tb1 & 31) * ht.nx;
    vxd = params[(unsigned)xsrc];
    if (ht.nx == 3) {
      vxs = params[(unsigned)(xsrc + 1)];
      vxc = params[(unsigned)(xsrc + 2)];
    }
  }
  if (t < gd.nunits) {
    S.W1s[t * kW1S + kIn] = vxd;
    S.W1s[t * kW1S + kIn + 1] = 0.f;
    S.b1s[t] = vb1 + (vxs * lt0 + vxc * lt1);
  }
  if (t < gd.nrows) S.b2s[t] = vb2;
}

// Forward on the matrix cores, per (view, head group): the first layer and
// output rows as in the backward's recomputation, then the output
// activations; outputs are staged per (head, component) plane in LDS and
// written as the tile's contiguous runs of 16 k values. Group 0 of view 0
// also writes the Gaussian means x_v + l_o O_i (shared by the views).
__global__ void __launch_bounds__(kNT, 3) k_dec_fwd_heads(DecodeConst dc, HeadTable ht, DecodeViews dv,
                                                          const float* __restrict__ xyz,
                                                          const float* __restrict__ feat,
                                                          const float* __restrict__ off,
                                                          const float* __restrict__ params, asgs_gaussians out,
                                                          GroupPair gp, int ngroups) {
  extern __shared__ __attribute__((aligned(16))) float smem[];
  const int grp = blockIdx.y % ngroups;
  const int view = blockIdx.y / ngroups;
  const GroupDesc& gd = gp.g[grp];
  const Views S = carve(smem, gd.L);
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int fl = lane & 15, fg = lane >> 4;
  const int A = (int)dc.A;
  const int k = dc.k;
  const int n = A * k;
  HeadCtx hc;
  RowMap rm;
  int t0, nt;
  assign_rows(gd, ht, grp, wv, k, fl, hc, rm, t0, nt);
  // group 1 (one head over four waves): one H for the workgroup, its two
  // unit halves formed by waves 0 and 1
  float (*Hw)[kHS] = grp == 1 ? S.H[0] : S.H[wv];
  const int run = 16 * k;
  const int nplanes = gd.gtot / run;
  const int ngrid = (A + 15) / 16;
  const int tk = t / k;  // anchor within the tile of the thread's output element
  const bool means = grp == 0 && view == 0;  // this group also writes the Gaussian means
  float xpre[2], ppre[3], mxp[3] = {0.f, 0.f, 0.f}, mop[3] = {0.f, 0.f, 0.f};
  auto fetch = [&](int tile) {
    const int a0 = tile * 16;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = t + q * kNT;
      const int a = e >> 5, c = e & 31;
      xpre[q] = a0 + a < A ? feat[(size_t)(a0 + a) * 32 + c] : 0.f;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) ppre[c] = (t < 16 && a0 + t < A) ? xyz[(size_t)c * A + a0 + t] : 0.f;
    const size_t gidx = (size_t)a0 * k + t;
    if (means && t < run && gidx < (size_t)n) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        mxp[c] = xyz[(size_t)c * A + a0 + tk];
        mop[c] = off[(size_t)c * n + gidx];
      }
    }
  };
  // the first tile's inputs are requested before the weights, so that the
  // two latencies overlap
  if ((int)blockIdx.x < ngrid) fetch(blockIdx.x);
  stage_weights(S, gd, ht, params, t, dv.lt[view][0], dv.lt[view][1]);
  for (int tile = blockIdx.x; tile < ngrid; tile += gridDim.x) {
    const int a0 = tile * 16;
    __syncthreads();  // weights staged / the previous tile's outputs are written
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = t + q * kNT;
      S.X[e >> 5][e & 31] = xpre[q];
    }
    if (t < 16) {
      float D[3] = {0.f, 0.f, 0.f}, dist = 1.f;
      if (a0 + t < A) {
        for (int c = 0; c < 3; ++c) D[c] = ppre[c] - dv.c[view][c];
        dist = sqrtf(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
        for (int c = 0; c < 3; ++c) D[c] /= dist;
      }
      for (int c = 0; c < 3; ++c) S.X[t][32 + c] = D[c];
      S.X[t][35] = ht.nx > 0 && a0 + t < A ? dist : 0.f;  // distance input (weight column 35)
      S.X[t][36] = 0.f;
    }
    const float mx[3] = {mxp[0], mxp[1], mxp[2]}, mo[3] = {mop[0], mop[1], mop[2]};
    __syncthreads();
    if (tile + (int)gridDim.x < ngrid) fetch(tile + gridDim.x);
    if (grp == 1) {
      if (wv < 2) head_forward_half(S, Hw, hc, wv, fl, fg);
      __syncthreads();  // the shared H is complete
    } else {
      head_forward(S, Hw, hc, fl, fg);
      wave_sync();
    }
#pragma unroll
    for (int i = 0; i < kAcc; ++i) {
      if (i >= nt) break;
      const int r0 = 16 * (t0 + i);
      const int orow = r0 + fl;
      const bool rok = orow < hc.rows;
      const int wrow = hc.lrow0 + (rok ? orow : 0);
      f4v y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        const int kk = 4 * ks + fg;
        y = mfma(Hw[fl][kk], S.W2s[wrow * kW2S + kk], y);
      }
      const float bias = S.b2s[wrow];
      const int gi = rm.gi[i], gc = rm.gc[i];
      if (rok) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = 4 * fg + r;
          S.G[hc.gbase + gc * run + a * k + gi] = fout_act(hc.h, y[r] + bias, dc.l_s);
        }
      }
    }
    __syncthreads();
    const size_t gidx = (size_t)a0 * k + t;
    if (t < run && gidx < (size_t)n) {
      for (int pl = 0; pl < nplanes; ++pl) {
        int h = 4, comp = pl;
        if (grp == 0) {
          h = pl < 1 ? 0 : pl < 4 ? 1 : pl < 7 ? 2 : 3;
          comp = pl - (h == 0 ? 0 : h == 1 ? 1 : h == 2 ? 4 : 7);
        }
        out_plane(out, view, h, comp, n)[gidx] = S.G[pl * run + t];
      }
      if (means) {
#pragma unroll
        for (int c = 0; c < 3; ++c) out.mean[(size_t)c * n + gidx] = mx[c] + dc.l_o * mo[c];
      }
    }
  }
}

// LDS of one group.
GroupDesc group_desc(const HeadTable& ht, int k, int hbase, int nheads) {
  GroupDesc g{};
  g.hbase = hbase;
  g.nheads = nheads;
  g.nunits = 32 * nheads;
  int rows = 0, gb = 0;
  for (int h = hbase; h < hbase + nheads; ++h) {
    g.lrow0[h] = rows;
    g.gbase[h] = gb;
    rows += k * ht.m[h];
    gb += ht.m[h] * 16 * k;
  }
  g.nrows = rows;
  g.gtot = gb;
  int o = 0;
  auto take = [&](int floats) {
    const int at = o;
    o += (floats + 3) & ~3;  // 16-byte aligned arrays
    return at;
  };
  g.L.W1s = take(g.nunits * kW1S);
  g.L.b1s = take(g.nunits);
  g.L.W2s = take(rows * kW2S);
  g.L.b2s = take(rows);
  g.L.X = take(16 * kXS);
  g.L.G = take(gb);
  g.L.H = take(kWaves * 16 * kHS);
  g.L.total = o;
  return g;
}

}  // namespace

void launch_dec_fwd_heads(const DecodeConst& dc, const HeadTable& ht, const DecodeViews& dv, const float* xyz,
                          const float* feat, const float* off, const float* params, const asgs_gaussians& out,
                          hipStream_t s) {
  const GroupDesc g0 = group_desc(ht, dc.k, 0, 4);
  const bool has_feat = ht.m[4] > 0;
  const GroupDesc g1 = has_feat ? group_desc(ht, dc.k, 4, 1) : g0;
  const int ng = has_feat ? 2 : 1;
  const int lds = (g0.L.total > g1.L.total ? g0.L.total : g1.L.total) * (int)sizeof(float);
  static bool attr_set = false;  // allow more than 64 KiB of dynamic LDS (at most ~77 KiB for k = 16)
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_dec_fwd_heads),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    attr_set = true;
  }
  // up to three workgroups per compute unit (the forward's LDS allows it)
  const int64_t tiles = (dc.A + 15) / 16;
  const unsigned nblk = (unsigned)(tiles < kMaxFwdWG ? tiles : kMaxFwdWG);
  hipLaunchKernelGGL(k_dec_fwd_heads, dim3(nblk, (unsigned)(ng * dc.n_views)),
                     dim3(kNT), lds, s, dc, ht, dv, xyz, feat, off, params, out, GroupPair{{g0, g1}}, ng);
}

}  // namespace asgs
