// Feature lift F_m and cosine distillation (UP-SLAM Sec. 3.3, Eq. 11, Eq. 12).
//
// Per pixel p: x = F~_p (16), h = relu(W1 x + b1) (128), F^_p = W2 h + b2 (N_h),
// F_p = bilinear upsampling of the DINO patch grid, cos_p = F.F^ / |F||F^|.
// F^ (N_h wide per pixel) is never formed. With the patch vectors G_c:
//   F.F^   = sum_c w_c (Q_c . h + beta_c),   Q_c = W2^T G_c,  beta_c = b2 . G_c
//   |F^|^2 = h^T M h + 2 m . h + mu,         M = W2^T W2,     m = W2^T b2, mu = b2 . b2
//   |F|^2  = sum_{c,c'} w_c w_c' G_c . G_c'
// over the four bilinear corners c of the pixel. Q_c, beta_c and the dot
// products of neighbouring patches are prepared once per patch, M once per
// call; per pixel the work is the 16 -> 128 first layer (matrix cores,
// v_mfma_f32_16x16x4f32: FP32 products and sums) and the 128 x 128 product
// M h (v_mfma_f32_16x16x32_bf16, both operands split into high and low
// bfloat16 parts, three products per pair: FP32 sums of products good to
// ~2^-16 relative).
//
// The backward is the same identities differentiated: with g = dL/dcos,
//   s1 = 1 / (|F||F^|),  dq = -g cos / (2 |F^|^2),
//   dL/dh = g s1 sum_c w_c Q_c + 2 dq (M h + m),  dL/dz = dL/dh [h > 0],
//   dL/dx = W1^T dL/dz,  dW1 = sum_p dL/dz x^T,  db1 = sum_p dL/dz,
//   dL/dM = S = sum_p dq h h^T,  dL/dm = sum_p 2 dq h,  dL/dmu = sum_p dq,
//   dL/dQ_c = sum_p g s1 w_c h,  dL/dbeta_c = sum_p g s1 w_c,
//   dW2 = sum_c G_c dQ_c^T + W2 (S + S^T) + b2 dm^T,
//   db2 = sum_c dbeta_c G_c + W2 dm + 2 dmu b2.
// The pixel sums dQ and dW1 are matrix products with K = pixels, taken on
// the matrix cores from per-round LDS tiles of h, the corner weights, x and
// dL/dz; S comes from a second pass whose register layout needs no tiles.
// Every sum has a fixed order (deterministic).
#include "internal.h"

namespace asgs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kFIn = 16;       // rendered feature channels
constexpr int kFHid = 128;     // hidden width of F_m
constexpr int kFT = 16;        // pixel tile side
constexpr int kSlots = 16;     // patches one tile reaches (at most 4 x 4)
constexpr int kCell = 136;     // floats per patch record: Q[128], beta, s, r, d, rd, x, pad
constexpr int kFrag = 8 * 4 * 2 * 64 * 8;  // bf16 of M as A fragments: 8 mb x 4 kb x (hi, lo) x 64 lanes x 8
constexpr int kBwdWG = 256;    // persistent workgroups of the backward (fixed: the sum order)
constexpr int kPart = 16384 + 2048 + 128 + 128 + 1;  // per workgroup: S, dW1^T, db1, dm, dmu
constexpr int kPartStride = 18944;                   // padded to a multiple of 256 floats
constexpr int kDQ = kFHid + 1;                       // per (tile, slot): dQ[128], dbeta

ASGS_DEV f4v mfma_bf(const bf8v& a, const bf8v& b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
ASGS_DEV uint16_t bf_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
ASGS_DEV float bf_val(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }
// v = hi + lo + O(2^-17 |v|)
ASGS_DEV void bf_split(float v, uint16_t& hi, uint16_t& lo) {
  hi = bf_rne(v);
  lo = bf_rne(v - bf_val(hi));
}
ASGS_DEV bf8v as_bf8(const uint16_t* u) {
  bf8v r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = __builtin_bit_cast(__bf16, u[i]);
  return r;
}
// sum over the four lanes of one pixel column (lanes l, l^16, l^32, l^48);
// every lane of the column gets the same bits
ASGS_DEV float col_sum(float v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}
// LDS position of hidden unit k in tables read one unit per lane group at a
// time (units 32 apart land in neighbouring rows)
ASGS_DEV int hpos(int k) { return (k & 31) * 4 + (k >> 5); }

struct FeatArgs {
  int32_t V, W, H, nh, Hp, Wp;
  int32_t tiles_x, tiles_y, tiles;  // tiles per view; tiles * V in all
  float sx, sy;                     // Wp / W, Hp / H
  const float* feat;                // [V][16][H][W]
  const float* params;              // W1 [128][16], b1 [128], W2 [nh][128], b2 [nh]
  const float* dino;                // [V][nh][Hp][Wp]
  const uint16_t* mfrag;            // M as A fragments (hi, lo)
  const float* mvec;                // m [128], mu at [128]
  const float* cells;               // [V][Hp * Wp][kCell]
  float* cosine;                    // [V][H][W]
  float* tile_loss;                 // [V * tiles]: sum of 1 - cos over the tile
  const float* dcos;                // backward: [V][H][W]
  float* dfeat;                     // backward: [V][16][H][W]
  float* part;                      // backward: [kBwdWG][kPartStride]
  float* dqt;                       // backward: [V * tiles][kSlots][kDQ]
  float* dqpix;                     // backward: [V][H][W] dq of each pixel (first pass -> second)
};

// Patch rectangle a tile reaches: rows cy0 .. cy0 + ncy - 1, cols cx0 ..
struct TileCells {
  int cy0, ncy, cx0, ncx;
};
ASGS_DEV TileCells tile_cells(const FeatArgs& a, int tx, int ty) {
  TileCells t;
  int i0, i1;
  float w;
  const int xa = tx * kFT, xe = min(xa + kFT - 1, a.W - 1);
  const int ya = ty * kFT, ye = min(ya + kFT - 1, a.H - 1);
  bilin(xa, a.Wp, a.sx, i0, i1, w);
  t.cx0 = i0;
  bilin(xe, a.Wp, a.sx, i0, i1, w);
  t.ncx = i1 - t.cx0 + 1;
  bilin(ya, a.Hp, a.sy, i0, i1, w);
  t.cy0 = i0;
  bilin(ye, a.Hp, a.sy, i0, i1, w);
  t.ncy = i1 - t.cy0 + 1;
  return t;
}

// Everything one lane knows about its pixel after the forward.
struct LanePix {
  bool valid;
  int64_t p;           // pixel index in the view
  float h[32];         // hidden units 32 g + u of the lane's group g
  float cw[4];         // corner weights
  int cs[4];           // corner slots in the tile's patch table
  float q, a, nF, den, cos;
  bool floored;
};

// Staged per workgroup: M fragments, first-layer weights, m, the tile's patches.
struct FeatShared {
  uint16_t frag[kFrag];
  // first-layer A operands (FP32 16x16x4, K = four features a step): block b,
  // lane l, step s at (64 b + l) 4 + s holds W1[32 (l % 16 / 4) + 4 b + l % 4][4 s + l / 16]
  float w1[8 * 64 * 4];
  float b1[kFHid];         // at hpos(k)
  float m[kFHid];          // at hpos(k)
  float cell[kSlots][kCell];
};

ASGS_DEV void stage_weights(const FeatArgs& a, FeatShared& S) {
  const int t = threadIdx.x, nt = blockDim.x;
  const uint4* src = reinterpret_cast<const uint4*>(a.mfrag);
  uint4* dst = reinterpret_cast<uint4*>(S.frag);
  for (int q = t; q < kFrag / 8; q += nt) dst[q] = src[q];
  for (int q = t; q < kFHid * kFIn; q += nt) {
    const int k = q / kFIn, c = q - k * kFIn;
    S.w1[(((k & 31) >> 2) * 64 + 16 * (c & 3) + 4 * (k >> 5) + (k & 3)) * 4 + (c >> 2)] = a.params[q];
  }
  for (int k = t; k < kFHid; k += nt) {
    S.b1[hpos(k)] = a.params[kFHid * kFIn + k];
    S.m[hpos(k)] = a.mvec[k];
  }
}

ASGS_DEV void stage_cells(const FeatArgs& a, FeatShared& S, int view, const TileCells& tc) {
  const int n = tc.ncy * tc.ncx;
  const float* base = a.cells + (int64_t)view * a.Hp * a.Wp * kCell;
  for (int q = threadIdx.x; q < n * kCell; q += blockDim.x) {
    const int sl = q / kCell, e = q - sl * kCell;
    const int cy = tc.cy0 + sl / tc.ncx, cx = tc.cx0 + sl % tc.ncx;
    S.cell[sl][e] = base[((int64_t)cy * a.Wp + cx) * kCell + e];
  }
}

// G_c . G_c' of two patches of the tile (at most one row and one column
// apart): the record of the upper-left patch of the pair holds it (self,
// right, lower, lower-right, or right-with-lower for the anti-diagonal).
ASGS_DEV float patch_dot(const FeatShared& S, const TileCells& tc, int ya, int xa, int yb, int xb) {
  const int dy = yb - ya, dx = xb - xa;
  const int e = dy == 0 ? (dx == 0 ? 129 : 130) : (dx == 0 ? 131 : (dx == dy ? 132 : 133));
  const int y = min(ya, yb), x = min(xa, xb);
  return S.cell[(y - tc.cy0) * tc.ncx + (x - tc.cx0)][e];
}

// First layer of the lane's pixel on the matrix cores (v_mfma_f32_16x16x4f32,
// FP32 products and sums; K = the 16 features in four steps of four): block b
// gives units 32 g + 4 b + r, r = 0..3, of pixel n (column n = lane & 15,
// group g = lane >> 4), the bias in the accumulator; xq[s] is feature 4 s + g
// of the pixel. h[4 b + r] = relu(z) holds unit 32 g + 4 b + r.
ASGS_DEV void first_layer(const float* w1, const float* b1g, const float (&xq)[4], int lane, float (&h)[32]) {
  const f4v* wl = reinterpret_cast<const f4v*>(w1) + lane;
  f4v z[8];
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) z[b][r] = b1g[4 * (4 * b + r)];
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int b = 0; b < 8; ++b) z[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(wl[64 * b][st], xq[st], z[b], 0, 0, 0);
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) h[4 * b + r] = fmaxf(z[b][r], 0.f);
}

// Forward of one pixel per lane (column n = lane & 15, group g = lane >> 4):
// first layer and M h on the matrix cores, the scalars of the cosine summed
// over the four lanes of the pixel.
ASGS_DEV void lane_forward(const FeatArgs& a, const FeatShared& S, const TileCells& tc, int view, int px, int py,
                           LanePix& L) {
  const int lane = threadIdx.x & 63, g = lane >> 4;
  L.valid = px < a.W && py < a.H;
  const int cpx = min(px, a.W - 1), cpy = min(py, a.H - 1);
  const int64_t HW = (int64_t)a.W * a.H;
  L.p = (int64_t)cpy * a.W + cpx;
  const float* fx = a.feat + (int64_t)view * kFIn * HW + (int64_t)g * HW + L.p;
  float xq[4];
#pragma unroll
  for (int st = 0; st < 4; ++st) xq[st] = L.valid ? fx[4 * st * HW] : 0.f;
  // unit 32 g + u sits at hpos = 4 u + g: per-lane bases with constant offsets
  const float* const b1g = S.b1 + g;
  const float* const mg = S.m + g;
  first_layer(S.w1, b1g, xq, lane, L.h);
  // hidden units 32 g + u, u = 8 kb + i: B operands of M h (K = hidden)
  bf8v bh[4], bl[4];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    uint16_t hi[8], lo[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) bf_split(L.h[8 * kb + i], hi[i], lo[i]);
    bh[kb] = as_bf8(hi);
    bl[kb] = as_bf8(lo);
  }
  __builtin_amdgcn_sched_barrier(0);
  // M h: row block mb holds units 32 g' + 4 mb + j for lane group g', used
  // at once for h^T (M h + 2 m)
  const uint16_t* fr = S.frag + lane * 8;
  float qp = 0.f, ap = 0.f;
#pragma unroll
  for (int mb = 0; mb < 8; ++mb) {
    f4v d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const bf8v ah = *reinterpret_cast<const bf8v*>(fr + ((mb * 4 + kb) * 2 + 0) * 512);
      const bf8v al = *reinterpret_cast<const bf8v*>(fr + ((mb * 4 + kb) * 2 + 1) * 512);
      d = mfma_bf(ah, bh[kb], d);
      d = mfma_bf(ah, bl[kb], d);
      d = mfma_bf(al, bh[kb], d);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int u = 4 * mb + j;
      qp = fmaf(L.h[u], d[j] + 2.f * mg[4 * u], qp);
    }
    // keep the fragment loads of one row block together (hoisting all 64 of
    // them would take every register)
    __builtin_amdgcn_sched_barrier(0);
  }
  // bilinear corners of the pixel in the tile's patch table
  int y0, y1, x0, x1;
  float wy, wx;
  bilin(cpy, a.Hp, a.sy, y0, y1, wy);
  bilin(cpx, a.Wp, a.sx, x0, x1, wx);
  const int ys[4] = {y0, y0, y1, y1}, xs[4] = {x0, x1, x0, x1};
  L.cw[0] = (1.f - wy) * (1.f - wx);
  L.cw[1] = (1.f - wy) * wx;
  L.cw[2] = wy * (1.f - wx);
  L.cw[3] = wy * wx;
#pragma unroll
  for (int c = 0; c < 4; ++c) L.cs[c] = (ys[c] - tc.cy0) * tc.ncx + (xs[c] - tc.cx0);
  {
    const float* cb[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) cb[c] = &S.cell[L.cs[c]][32 * g];
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      float cs = 0.f;
#pragma unroll
      for (int c = 0; c < 4; ++c) cs = fmaf(L.cw[c], cb[c][u], cs);
      ap = fmaf(cs, L.h[u], ap);
      if ((u & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // four units' corner reads at a time
    }
  }
  L.q = fmaxf(col_sum(qp) + a.mvec[kFHid], 0.f);
  float beta = 0.f, nF = 0.f;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    beta = fmaf(L.cw[c], S.cell[L.cs[c]][128], beta);
    nF = fmaf(L.cw[c] * L.cw[c], patch_dot(S, tc, ys[c], xs[c], ys[c], xs[c]), nF);
#pragma unroll
    for (int e = c + 1; e < 4; ++e)
      nF = fmaf(2.f * L.cw[c] * L.cw[e], patch_dot(S, tc, ys[c], xs[c], ys[e], xs[e]), nF);
  }
  L.a = col_sum(ap) + beta;
  L.nF = fmaxf(nF, 0.f);
  const float den = sqrtf(L.nF) * sqrtf(L.q);
  L.floored = !(den >= 1e-12f);
  L.den = L.floored ? 1e-12f : den;
  L.cos = L.a / L.den;
}

// ---------------------------------------------------------------------------
// Preparation: M = W2^T W2 and m = W2^T b2 come from the split-K product
// (colgemm.hip) as gm = [128][129]; here M becomes bfloat16 hi/lo A
// fragments, and mu = b2 . b2 is summed (one workgroup, fixed order). Per
// patch (k_feat_cells, 16 patches per workgroup): Q, beta and the dot
// products with its right, lower and lower-right neighbours and of its right
// and lower neighbours.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_feat_frag(FeatArgs a, const float* __restrict__ gm, uint16_t* mfrag,
                                                   float* mvec) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < kFrag / 2) {
    // fragment (mb, kb), lane, element i: row unit 32 (rr/4) + 4 mb + rr%4 (rr = lane & 15),
    // column unit 32 (lane/16) + 8 kb + i
    const int i = e & 7, lane = (e >> 3) & 63, kb = (e >> 9) & 3, mb = e >> 11;
    const int rr = lane & 15;
    const int ru = 32 * (rr >> 2) + 4 * mb + (rr & 3);
    const int cu = 32 * (lane >> 4) + 8 * kb + i;
    uint16_t hi, lo;
    bf_split(gm[ru * (kFHid + 1) + cu], hi, lo);
    mfrag[((mb * 4 + kb) * 2 + 0) * 512 + lane * 8 + i] = hi;
    mfrag[((mb * 4 + kb) * 2 + 1) * 512 + lane * 8 + i] = lo;
  }
  if (e < kFHid) mvec[e] = gm[e * (kFHid + 1) + kFHid];
  if (blockIdx.x == 0) {
    __shared__ float red[4];
    const float* b2 = a.params + kFHid * kFIn + kFHid + (int64_t)a.nh * kFHid;
    float acc = 0.f;
    for (int c = threadIdx.x; c < a.nh; c += 256) acc = fmaf(b2[c], b2[c], acc);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) mvec[kFHid] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

constexpr int kQC = 16;  // patches per workgroup (the M side of the product)

// Per run of 16 consecutive patches (flat index): Q = W2^T G for all 16 on
// the matrix cores (v_mfma_f32_16x16x4f32, FP32; M = patches, N = units,
// K = channels four at a time; wave w takes the unit blocks 2 (w % 4),
// 2 (w % 4) + 1 over one half of the channels, the halves added in a fixed
// order), so W2 is read once per run; then beta and the neighbour dot
// products, one patch per lane column and the channels split over the 32
// lane groups of the workgroup, summed in a fixed order.
__global__ void __launch_bounds__(512) k_feat_cells(FeatArgs a, float* cells) {
  __shared__ float qh[kQC][kFHid];
  __shared__ float red[8][kQC][6];
  const int c0 = blockIdx.x * kQC, view = blockIdx.y;
  const int plane = a.Hp * a.Wp;
  const float* G = a.dino + (int64_t)view * a.nh * plane;
  const float* W2 = a.params + kFHid * kFIn + kFHid;
  const float* b2 = W2 + (int64_t)a.nh * kFHid;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, g = lane >> 4, f = lane & 15;
  const int ub = wv & 3, kh = wv >> 2;
  const int half = ((a.nh + 63) / 64) * 32;  // channels of the first half (a multiple of 32)
  f4v q0 = {0.f, 0.f, 0.f, 0.f}, q1 = q0;
  {
    // A: channel 4 s + g of patch c0 + f; B: W2 rows 4 s + g, units 32 ub + f (+ 16)
    const float* Ga = G + min(c0 + f, plane - 1);
    const float* Wb = W2 + 32 * ub + f;
    const int cb = kh * half, ce = min(a.nh, cb + half);
    for (int c = cb + g; c < ce + g; c += 32) {
      float av[8], b0[8], b1[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int ch = c + 4 * i;
        const bool ok = ch < ce;
        av[i] = ok ? Ga[(int64_t)ch * plane] : 0.f;
        b0[i] = ok ? Wb[(int64_t)ch * kFHid] : 0.f;
        b1[i] = ok ? Wb[(int64_t)ch * kFHid + 16] : 0.f;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        q0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], b0[i], q0, 0, 0, 0);
        q1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], b1[i], q1, 0, 0, 0);
      }
    }
    if (kh == 1) {
      // rows: patches 4 g + r; columns: units 32 ub + f (+ 16)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        qh[4 * g + r][32 * ub + f] = q0[r];
        qh[4 * g + r][32 * ub + 16 + f] = q1[r];
      }
    }
  }
  // beta, |G|^2 and the neighbour products of patch c0 + i, i = t % 16,
  // channels t / 16 + 32 k, four at a time
  const int i = t & (kQC - 1), cg = t >> 4;
  const int cell = min(c0 + i, plane - 1);
  const int gy = cell / a.Wp, gx = cell - gy * a.Wp;
  const bool rx = gx + 1 < a.Wp, dy = gy + 1 < a.Hp;
  const int i1 = rx ? cell + 1 : cell, i2 = dy ? cell + a.Wp : cell, i3 = rx && dy ? cell + a.Wp + 1 : cell;
  const float f1 = rx ? 1.f : 0.f, f2 = dy ? 1.f : 0.f, f3 = rx && dy ? 1.f : 0.f;
  float p[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int c = cg; c < a.nh; c += 128) {
    float v0[4], v1[4], v2[4], v3[4], vb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int ch = min(c + 32 * k, a.nh - 1);
      const float* Gc = G + (int64_t)ch * plane;
      const float m = c + 32 * k < a.nh ? 1.f : 0.f;
      v0[k] = m * Gc[cell];
      v1[k] = f1 * Gc[i1];
      v2[k] = f2 * Gc[i2];
      v3[k] = f3 * Gc[i3];
      vb[k] = b2[ch];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      p[0] = fmaf(vb[k], v0[k], p[0]);
      p[1] = fmaf(v0[k], v0[k], p[1]);
      p[2] = fmaf(v0[k], v1[k], p[2]);
      p[3] = fmaf(v0[k], v2[k], p[3]);
      p[4] = fmaf(v0[k], v3[k], p[4]);
      p[5] = fmaf(v1[k] * (c + 32 * k < a.nh ? 1.f : 0.f), v2[k], p[5]);
    }
  }
  // lanes i, i + 16, i + 32, i + 48 of the wave, then the eight waves
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    p[k] += __shfl_xor(p[k], 16);
    p[k] += __shfl_xor(p[k], 32);
  }
  if (lane < kQC) {
#pragma unroll
    for (int k = 0; k < 6; ++k) red[wv][i][k] = p[k];
  }
  __syncthreads();
  if (kh == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int cl = c0 + 4 * g + r;
      if (cl < plane) {
        float* out = cells + ((int64_t)view * plane + cl) * kCell + 32 * ub + f;
        out[0] = q0[r] + qh[4 * g + r][32 * ub + f];
        out[16] = q1[r] + qh[4 * g + r][32 * ub + 16 + f];
      }
    }
  }
  if (t < kQC * 6) {
    const int ii = t / 6, k = t - ii * 6;
    if (c0 + ii < plane) {
      float sum = 0.f;
      for (int w = 0; w < 8; ++w) sum += red[w][ii][k];
      cells[((int64_t)view * plane + c0 + ii) * kCell + kFHid + k] = sum;
    }
  }
}

// ---------------------------------------------------------------------------
// Forward: persistent workgroups of kFwdWaves waves over 16x16 pixel tiles;
// each wave takes one row of 16 pixels per round.
// ---------------------------------------------------------------------------
constexpr int kFwdWaves = 8;

__global__ void __launch_bounds__(64 * kFwdWaves) k_feat_fwd(FeatArgs a) {
  __shared__ __attribute__((aligned(16))) FeatShared S;
  __shared__ float tl[kFwdWaves];
  stage_weights(a, S);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, n = lane & 15;
  const int total = a.tiles * a.V;
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int view = t / a.tiles, lt = t - view * a.tiles;
    const int ty = lt / a.tiles_x, tx = lt - ty * a.tiles_x;
    const TileCells tc = tile_cells(a, tx, ty);
    __syncthreads();  // the previous tile's patches are no longer read
    stage_cells(a, S, view, tc);
    __syncthreads();
    float acc = 0.f;
    for (int row = wv; row < kFT; row += kFwdWaves) {
      LanePix L;
      lane_forward(a, S, tc, view, tx * kFT + n, ty * kFT + row, L);
      if (L.valid && g == 0) {
        a.cosine[(int64_t)view * a.W * a.H + L.p] = L.cos;
        acc += 1.f - L.cos;
      }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) tl[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      float s = 0.f;
      for (int w = 0; w < kFwdWaves; ++w) s += tl[w];
      a.tile_loss[t] = s;
    }
  }
}

// mean of 1 - cos per view: fixed-order sum of the view's tile sums
__global__ void __launch_bounds__(256) k_feat_loss(FeatArgs a, float* loss) {
  __shared__ float red[4];
  const int view = blockIdx.x;
  float s = 0.f;
  for (int t = threadIdx.x; t < a.tiles; t += 256) s += a.tile_loss[(int64_t)view * a.tiles + t];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) loss[view] = ((red[0] + red[1]) + (red[2] + red[3])) / ((float)a.W * (float)a.H);
}

// ---------------------------------------------------------------------------
// Backward: persistent workgroups (kBwdWG, a fixed number so that every sum
// keeps its order on any device) of 4 waves over the tiles; a round is 4
// rows of 16 pixels (64 pixels, one row per wave).
// ---------------------------------------------------------------------------
constexpr int kBwdWaves = 4;
constexpr int kRP = 64;  // pixels per round

// [128 units][64 pixels] bfloat16 with the 8-pixel chunks of row k at chunk ^ (k & 7)
ASGS_DEV int rp_index(int k, int pxl) { return k * kRP + ((((pxl >> 3) ^ (k & 7)) << 3) | (pxl & 7)); }

struct BwdShared {
  FeatShared F;
  uint16_t Hhi[kFHid * kRP], Hlo[kFHid * kRP];    // h
  uint16_t Ghi[kFHid * kRP], Glo[kFHid * kRP];    // dL/dz
  float X[kFIn][kRP];                             // x
  float Wc[kSlots][kRP];                          // g s1 w_c at each pixel's corner slots
};

// A or B fragment of a [128][64] bf16 table: row k, pixels 32 kb + 8 (lane / 16) .. + 7
ASGS_DEV bf8v tab_frag(const uint16_t* T, int k, int kb, int lane) {
  const int p0 = 32 * kb + 8 * (lane >> 4);
  return *reinterpret_cast<const bf8v*>(T + rp_index(k, p0));
}
// A fragment of a [rows][64] fp32 table (row r, the same pixels), split on the fly
ASGS_DEV void f32_frag(const float (*T)[kRP], int r, int kb, int lane, bf8v& hi, bf8v& lo) {
  const int p0 = 32 * kb + 8 * (lane >> 4);
  uint16_t h[8], l[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) bf_split(T[r][p0 + i], h[i], l[i]);
  hi = as_bf8(h);
  lo = as_bf8(l);
}

// Backward, first pass (per round of 64 pixels): the forward again, dL/dz and
// dL/dx (written), dq per pixel (for the second pass), and on the matrix
// cores dQ += (g s1 w_c)^T h per patch slot, dW1^T += x^T dL/dz and
// db1 += 1^T dL/dz (a row of ones).
__global__ void __launch_bounds__(64 * kBwdWaves) k_feat_bwd(FeatArgs a) {
  __shared__ __attribute__((aligned(16))) BwdShared S;
  stage_weights(a, S.F);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, n = lane & 15;
  // dW1^T and db1 column blocks 2 wv, 2 wv + 1; dQ column blocks wv, wv + 4 (and 8 = dbeta on wave 0)
  f4v accW[2], accB[2], accQ[3];
#pragma unroll
  for (int i = 0; i < 2; ++i) accW[i] = accB[i] = f4v{0.f, 0.f, 0.f, 0.f};
  const int total = a.tiles * a.V;
  const int64_t HW = (int64_t)a.W * a.H;
  // A operand of the row of ones (row 0 of the block, exact in bfloat16)
  bf8v ones;
  {
    uint16_t o[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = n == 0 ? bf_rne(1.f) : (uint16_t)0;
    ones = as_bf8(o);
  }
  // A operands of dL/dx = W1^T dL/dz: lane (g, n) supplies W1[32 g + 8 kb + i][n]
  bf8v dxh[4], dxl[4];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    uint16_t wh[8], wl[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) bf_split(a.params[(32 * g + 8 * kb + i) * kFIn + n], wh[i], wl[i]);
    dxh[kb] = as_bf8(wh);
    dxl[kb] = as_bf8(wl);
  }
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int view = t / a.tiles, lt = t - view * a.tiles;
    const int ty = lt / a.tiles_x, tx = lt - ty * a.tiles_x;
    const TileCells tc = tile_cells(a, tx, ty);
#pragma unroll
    for (int i = 0; i < 3; ++i) accQ[i] = f4v{0.f, 0.f, 0.f, 0.f};
    __syncthreads();
    stage_cells(a, S.F, view, tc);
    for (int round = 0; round < kFT / kBwdWaves; ++round) {
      __syncthreads();  // patches staged; the previous round's tables are no longer read
      const int row = round * kBwdWaves + wv;
      // The forward of the lane's pixel and its 32 hidden units again (as in
      // lane_forward), then dL/dz; M h + m is kept at the lane's units for
      // dL/dh (after the cosine's scalars are known).
      const int px = tx * kFT + n, py = ty * kFT + row;
      const bool valid = px < a.W && py < a.H;
      const int cpx = min(px, a.W - 1), cpy = min(py, a.H - 1);
      const int64_t p = (int64_t)cpy * a.W + cpx;
      const int pr = wv * 16 + n;  // pixel of the round
      // unit 32 g + u sits at hpos = 4 u + g: per-lane bases with constant offsets
      const float* const b1g = S.F.b1 + g;
      const float* const mg = S.F.m + g;
      float h[32];
      bf8v bh[4], bl[4];
      {
        float xq[4];
        const float* fx = a.feat + (int64_t)view * kFIn * HW + (int64_t)g * HW + p;
#pragma unroll
        for (int st = 0; st < 4; ++st) xq[st] = valid ? fx[4 * st * HW] : 0.f;
#pragma unroll
        for (int st = 0; st < 4; ++st) S.X[4 * st + g][pr] = xq[st];
        first_layer(S.F.w1, b1g, xq, lane, h);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          uint16_t hi[8], lo[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int u = 8 * kb + i, k = 32 * g + u;
            bf_split(h[u], hi[i], lo[i]);
            S.Hhi[rp_index(k, pr)] = hi[i];
            S.Hlo[rp_index(k, pr)] = lo[i];
            if (i & 1) __builtin_amdgcn_sched_barrier(0);
          }
          bh[kb] = as_bf8(hi);
          bl[kb] = as_bf8(lo);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      // bilinear corners of the pixel in the tile's patch table
      LanePix L;  // corners only
      int ys[4], xs[4];
      {
        int y0, y1, x0, x1;
        float wy, wx;
        bilin(cpy, a.Hp, a.sy, y0, y1, wy);
        bilin(cpx, a.Wp, a.sx, x0, x1, wx);
        ys[0] = ys[1] = y0;
        ys[2] = ys[3] = y1;
        xs[0] = xs[2] = x0;
        xs[1] = xs[3] = x1;
        L.cw[0] = (1.f - wy) * (1.f - wx);
        L.cw[1] = (1.f - wy) * wx;
        L.cw[2] = wy * (1.f - wx);
        L.cw[3] = wy * wx;
#pragma unroll
        for (int c = 0; c < 4; ++c) L.cs[c] = (ys[c] - tc.cy0) * tc.ncx + (xs[c] - tc.cx0);
      }
      const uint16_t* fr = S.F.frag + lane * 8;
      // row block mb of M h: units 32 g + 4 mb + j of the lane's pixel
      auto mh_block = [&](int mb) {
        f4v d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          const bf8v ah = *reinterpret_cast<const bf8v*>(fr + ((mb * 4 + kb) * 2 + 0) * 512);
          const bf8v alo = *reinterpret_cast<const bf8v*>(fr + ((mb * 4 + kb) * 2 + 1) * 512);
          d = mfma_bf(ah, bh[kb], d);
          d = mfma_bf(ah, bl[kb], d);
          d = mfma_bf(alo, bh[kb], d);
        }
        return d;
      };
      float qp = 0.f, ap = 0.f;
      float mh[32];  // (M h + m) at the lane's units
#pragma unroll
      for (int mb = 0; mb < 8; ++mb) {
        const f4v d = mh_block(mb);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int u = 4 * mb + j;
          mh[u] = d[j] + mg[4 * u];
          qp = fmaf(h[u], mh[u] + mg[4 * u], qp);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      const float* cb[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) cb[c] = &S.F.cell[L.cs[c]][32 * g];
      auto csum = [&](int u) {
        float r = 0.f;
#pragma unroll
        for (int c = 0; c < 4; ++c) r = fmaf(L.cw[c], cb[c][u], r);
        return r;
      };
#pragma unroll
      for (int u = 0; u < 32; ++u) {
        ap = fmaf(csum(u), h[u], ap);
        if ((u & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // four units' corner reads at a time
      }
      const float q = fmaxf(col_sum(qp) + a.mvec[kFHid], 0.f);
      float beta = 0.f, nF = 0.f;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        beta = fmaf(L.cw[c], S.F.cell[L.cs[c]][128], beta);
        nF = fmaf(L.cw[c] * L.cw[c], patch_dot(S.F, tc, ys[c], xs[c], ys[c], xs[c]), nF);
#pragma unroll
        for (int e = c + 1; e < 4; ++e)
          nF = fmaf(2.f * L.cw[c] * L.cw[e], patch_dot(S.F, tc, ys[c], xs[c], ys[e], xs[e]), nF);
      }
      const float av = col_sum(ap) + beta;
      const float den0 = sqrtf(fmaxf(nF, 0.f)) * sqrtf(q);
      const bool floored = !(den0 >= 1e-12f);
      const float den = floored ? 1e-12f : den0;
      const float cosv = av / den;
      const float gp = valid ? a.dcos[(int64_t)view * HW + p] : 0.f;
      const float al = gp / den;
      const float dq = floored ? 0.f : -0.5f * gp * cosv / q;
      if (g == 0 && valid) a.dqpix[(int64_t)view * HW + p] = dq;
      __builtin_amdgcn_sched_barrier(0);
      // dL/dz at the lane's units: into the table (dW1, db1 below) and, as
      // they are, the B operand of dL/dx
      uint16_t zh[32], zl[32];
#pragma unroll
      for (int mb = 0; mb < 8; ++mb) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int u = 4 * mb + j, k = 32 * g + u;
          const float dh = fmaf(al, csum(u), 2.f * dq * mh[u]);
          const float dz = h[u] > 0.f ? dh : 0.f;
          bf_split(dz, zh[u], zl[u]);
          S.Ghi[rp_index(k, pr)] = zh[u];
          S.Glo[rp_index(k, pr)] = zl[u];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      // dL/dx (channels x the wave's 16 pixels) = W1^T dL/dz, K = the lane
      // group's own units 32 g + 8 kb .. + 7: A = W1^T (channel n, those
      // units), B = dL/dz at pixel n; lane (n, g) receives channels 4 g + j
      // of its own pixel
      {
        f4v dxa = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          const bf8v bh = as_bf8(&zh[8 * kb]), bl = as_bf8(&zl[8 * kb]);
          dxa = mfma_bf(dxh[kb], bh, dxa);
          dxa = mfma_bf(dxh[kb], bl, dxa);
          dxa = mfma_bf(dxl[kb], bh, dxa);
        }
        if (valid) {
          float* dfx = a.dfeat + (int64_t)view * kFIn * HW + p;
#pragma unroll
          for (int j = 0; j < 4; ++j) dfx[(4 * g + j) * HW] = dxa[j];
        }
      }
      if (g == 1) {
        float wc[kSlots];
#pragma unroll
        for (int sl = 0; sl < kSlots; ++sl) wc[sl] = 0.f;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int sl = 0; sl < kSlots; ++sl) wc[sl] += (L.cs[c] == sl) ? al * L.cw[c] : 0.f;
#pragma unroll
        for (int sl = 0; sl < kSlots; ++sl) S.Wc[sl][pr] = wc[sl];
      }
      __syncthreads();
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        // dQ += Wc^T h (rows = slots), and the constant-one column for dbeta
        bf8v wh, wl;
        f32_frag(S.Wc, n, kb, lane, wh, wl);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const int nb = i == 0 ? wv : (i == 1 ? wv + 4 : 8);
          if (nb == 8 && wv != 0) continue;
          bf8v bh, bl;
          if (nb < 8) {
            bh = tab_frag(S.Hhi, 16 * nb + n, kb, lane);
            bl = tab_frag(S.Hlo, 16 * nb + n, kb, lane);
          } else {
            bh = ones;
            uint16_t zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            bl = as_bf8(zero);
          }
          accQ[i] = mfma_bf(wh, bh, accQ[i]);
          accQ[i] = mfma_bf(wh, bl, accQ[i]);
          accQ[i] = mfma_bf(wl, bh, accQ[i]);
        }
        // dW1^T += x^T dL/dz and db1 += 1^T dL/dz: columns 16 nb + n
        bf8v xh, xl;
        f32_frag(S.X, n, kb, lane, xh, xl);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int ck = 16 * (2 * wv + i) + n;
          const bf8v zh = tab_frag(S.Ghi, ck, kb, lane), zl = tab_frag(S.Glo, ck, kb, lane);
          accW[i] = mfma_bf(xh, zh, accW[i]);
          accW[i] = mfma_bf(xh, zl, accW[i]);
          accW[i] = mfma_bf(xl, zh, accW[i]);
          accB[i] = mfma_bf(ones, zh, accB[i]);
          accB[i] = mfma_bf(ones, zl, accB[i]);
        }
      }
    }
    // the tile's patch gradients: rows = slots 4 (lane / 16) + j, column 16 nb + n
    float* dqt = a.dqt + (int64_t)t * kSlots * kDQ;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int nb = i == 0 ? wv : (i == 1 ? wv + 4 : 8);
      if (nb == 8 && (wv != 0 || n != 0)) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) dqt[(4 * g + j) * kDQ + 16 * nb + n] = accQ[i][j];
    }
  }
  // workgroup partials: dW1^T rows 4 g + j, db1 (row 0 of the ones block)
  float* part = a.part + (int64_t)blockIdx.x * kPartStride;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) part[16384 + (4 * g + j) * kFHid + 16 * (2 * wv + i) + n] = accW[i][j];
    if (g == 0) part[16384 + 2048 + 16 * (2 * wv + i) + n] = accB[i][0];
  }
}

// Backward, second pass: S = sum_p dq h h^T, dm = 2 sum_p dq h, dmu = sum_p dq,
// from dq of the first pass. Each wave takes 32 pixels of one view at a time
// and keeps all of S in registers. h^T (pixels x units) comes from the matrix
// cores: A = the 16 features of a pixel as [high | low] bfloat16 parts (K 32),
// B = W1^T high parts over both halves, then W1^T low parts over the high
// half, the bias in the accumulator (products good to ~2^-16 relative, FP32
// sums). A lane then holds eight pixels of one unit, which is its operand in
// S = (dq h) h^T with K = the 32 pixels (rows: units of dq h, columns: units
// of h), so h never goes through LDS. S is symmetric: the 36 blocks of 16 x 16
// on and above the diagonal are formed; the partial holds T with
// T + T^T = S + S^T (off-diagonal blocks doubled, diagonal blocks once, blocks
// below the diagonal zero). The four waves' sums are added in a fixed order.
constexpr int kSPix = 32;  // pixels per wave step
constexpr int kSBlk = 36;  // blocks of S on and above the diagonal

struct SShared {
  uint4 wfrag[8][2][64];                  // first-layer B fragments: unit block, (high, low), lane
  float red[2][kSBlk * 4 * 64];           // cross-wave sums of S
  float dm[kBwdWaves][kFHid];
  float dmu[kBwdWaves];
};

// the lane's 8 values of the first-layer accumulators as high and low bfloat16
// operands (element j: pixel 4 g + j of the first 16, then of the second 16)
ASGS_DEV void split8(const float (&v)[8], bf8v& hi, bf8v& lo) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int j = 0; j < 8; j += 2) {
    const bf2v h = __builtin_convertvector((f2v{v[j], v[j + 1]}), bf2v);
    const uint32_t u = __builtin_bit_cast(uint32_t, h);
    const bf2v l = __builtin_convertvector(
        (f2v{v[j] - __uint_as_float(u << 16), v[j + 1] - __uint_as_float(u & 0xffff0000u)}), bf2v);
    hi[j] = h[0];
    hi[j + 1] = h[1];
    lo[j] = l[0];
    lo[j + 1] = l[1];
  }
}
// max(z, 0) on the bits: negative floats (and -0) are negative integers
ASGS_DEV float relu_bits(float z) { return __int_as_float(max(__float_as_int(z), 0)); }

__global__ void __launch_bounds__(64 * kBwdWaves) k_feat_bwd_s(FeatArgs a) {
  __shared__ __attribute__((aligned(16))) SShared S;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, n = lane & 15;
  // B fragment of unit block b for lane (lg, ln): unit 16 b + ln, features
  // 8 (lg & 1) .. + 7; high parts, or low parts in lane groups 0, 1 and zero in 2, 3
  for (int e = threadIdx.x; e < 8 * 2 * 64; e += blockDim.x) {
    const int b = e >> 7, lo = (e >> 6) & 1, l = e & 63, lg = l >> 4, ln = l & 15;
    const float* w = a.params + (16 * b + ln) * kFIn + 8 * (lg & 1);
    uint16_t o[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint16_t hi = bf_rne(w[j]);
      o[j] = lo == 0 ? hi : lg < 2 ? bf_rne(w[j] - bf_val(hi)) : (uint16_t)0;
    }
    S.wfrag[b][lo][l] = make_uint4(o[0] | (uint32_t)o[1] << 16, o[2] | (uint32_t)o[3] << 16,
                                   o[4] | (uint32_t)o[5] << 16, o[6] | (uint32_t)o[7] << 16);
  }
  float b1r[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) b1r[b] = a.params[kFHid * kFIn + 16 * b + n];
  f4v acc[kSBlk];
#pragma unroll
  for (int i = 0; i < kSBlk; ++i) acc[i] = f4v{0.f, 0.f, 0.f, 0.f};
  float dmacc[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) dmacc[b] = 0.f;
  float dmuacc = 0.f;
  const int HW = a.W * a.H;
  const int cpv = (HW + kSPix - 1) / kSPix;
  const int nchunk = a.V * cpv;
  const int stride = gridDim.x * kBwdWaves;
  // features and dq of one chunk, loads clamped into the view (the pixels
  // past its end are masked where they are used: their dq is zero)
  float xn[2][8], dqn[8];
  int limn = 0;
  auto fetch = [&](int cc) {
    const int v = cc / cpv, base = (cc - v * cpv) * kSPix;
    const float* fv = a.feat + (int64_t)v * kFIn * HW + (int64_t)(8 * (g & 1)) * HW;
    const float* dv = a.dqpix + (int64_t)v * HW;
#pragma unroll
    for (int P = 0; P < 2; ++P) {
      const int px = min(base + 16 * P + n, HW - 1);
#pragma unroll
      for (int j = 0; j < 8; ++j) xn[P][j] = fv[(int64_t)j * HW + px];
#pragma unroll
      for (int r = 0; r < 4; ++r) dqn[4 * P + r] = dv[min(base + 16 * P + 4 * g + r, HW - 1)];
    }
    limn = HW - base;
  };
  int c = blockIdx.x * kBwdWaves + wv;
  if (c < nchunk) fetch(c);
  for (; c < nchunk; c += stride) {
    float x[2][8], dq[8];
#pragma unroll
    for (int P = 0; P < 2; ++P)
#pragma unroll
      for (int j = 0; j < 8; ++j) x[P][j] = xn[P][j];
#pragma unroll
    for (int j = 0; j < 8; ++j) dq[j] = dqn[j];
    const int lim = limn;
    fetch(min(c + stride, nchunk - 1));
    // A: the pixel's features, high parts in lane groups 0, 1 and low parts in 2, 3
    bf8v A[2];
#pragma unroll
    for (int P = 0; P < 2; ++P) {
      bf8v hi, lo;
      split8(x[P], hi, lo);
      A[P] = g < 2 ? hi : lo;
    }
    float sdq = 0.f;
#pragma unroll
    for (int P = 0; P < 2; ++P)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        dq[4 * P + r] = 16 * P + 4 * g + r < lim ? dq[4 * P + r] : 0.f;
        sdq += dq[4 * P + r];
      }
    if (n == 0) dmuacc += sdq;
    bf8v Ghi[8], Glo[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bf8v whi = __builtin_bit_cast(bf8v, S.wfrag[b][0][lane]);
      const bf8v wlo = __builtin_bit_cast(bf8v, S.wfrag[b][1][lane]);
      f4v z0 = f4v{b1r[b], b1r[b], b1r[b], b1r[b]}, z1 = z0;
      z0 = mfma_bf(A[0], whi, z0);
      z1 = mfma_bf(A[1], whi, z1);
      z0 = mfma_bf(A[0], wlo, z0);
      z1 = mfma_bf(A[1], wlo, z1);
      float h[8], gh[8];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        h[r] = relu_bits(z0[r]);
        h[4 + r] = relu_bits(z1[r]);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        gh[j] = dq[j] * h[j];
        dmacc[b] += gh[j];
      }
      bf8v Hhi, Hlo;
      split8(h, Hhi, Hlo);
      split8(gh, Ghi[b], Glo[b]);
      // the blocks of column b: rows bi <= b
#pragma unroll
      for (int bi = 0; bi <= b; ++bi) acc[b * (b + 1) / 2 + bi] = mfma_bf(Ghi[bi], Hhi, acc[b * (b + 1) / 2 + bi]);
#pragma unroll
      for (int bi = 0; bi <= b; ++bi) acc[b * (b + 1) / 2 + bi] = mfma_bf(Ghi[bi], Hlo, acc[b * (b + 1) / 2 + bi]);
#pragma unroll
      for (int bi = 0; bi <= b; ++bi) acc[b * (b + 1) / 2 + bi] = mfma_bf(Glo[bi], Hhi, acc[b * (b + 1) / 2 + bi]);
    }
  }
  // dm per unit 16 b + n (the four lane groups held different pixels); dmu
#pragma unroll
  for (int b = 0; b < 8; ++b) dmacc[b] = col_sum(dmacc[b]);
  for (int o = 32; o > 0; o >>= 1) dmuacc += __shfl_xor(dmuacc, o);
  if (g == 0) {
#pragma unroll
    for (int b = 0; b < 8; ++b) S.dm[wv][16 * b + n] = dmacc[b];
  }
  if (lane == 0) S.dmu[wv] = dmuacc;
  // S over the waves: (w0 + w1) + (w2 + w3)
  if (wv & 1) {
#pragma unroll
    for (int i = 0; i < kSBlk; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) S.red[wv >> 1][(4 * i + j) * 64 + lane] = acc[i][j];
  }
  __syncthreads();
  if (!(wv & 1)) {
#pragma unroll
    for (int i = 0; i < kSBlk; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += S.red[wv >> 1][(4 * i + j) * 64 + lane];
  }
  __syncthreads();
  if (wv == 2) {
#pragma unroll
    for (int i = 0; i < kSBlk; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) S.red[0][(4 * i + j) * 64 + lane] = acc[i][j];
  }
  __syncthreads();
  float* part = a.part + (int64_t)blockIdx.x * kPartStride;
  if (wv == 0) {
    // rows 16 bi + 4 g + j, columns 16 bj + n; zero blocks below the diagonal
#pragma unroll
    for (int bj = 0; bj < 8; ++bj)
#pragma unroll
      for (int bi = 0; bi <= bj; ++bi) {
        const int i = bj * (bj + 1) / 2 + bi;
        const float f = bi == bj ? 1.f : 2.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float s = acc[i][j] + S.red[0][(4 * i + j) * 64 + lane];
          part[(16 * bi + 4 * g + j) * kFHid + 16 * bj + n] = f * s;
          if (bi != bj) part[(16 * bj + 4 * g + j) * kFHid + 16 * bi + n] = 0.f;
        }
      }
  }
  const int t = threadIdx.x;
  if (t < kFHid)
    part[16384 + 2048 + 128 + t] = 2.f * ((S.dm[0][t] + S.dm[1][t]) + (S.dm[2][t] + S.dm[3][t]));
  if (t == 0) part[16384 + 2048 + 256] = (S.dmu[0] + S.dmu[1]) + (S.dmu[2] + S.dmu[3]);
}

// Sums of the workgroup partials: S, dW1^T, db1, dm, dmu (fixed order): 64
// elements per workgroup, four threads per element (workgroups b = q mod 4,
// sixteen loads in flight per round, summed in a fixed tree), combined in LDS.
__global__ void __launch_bounds__(256) k_feat_reduce(const float* __restrict__ part, int nwg, float* out) {
  __shared__ float red[4][64];
  const int el = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + el;
  float acc = 0.f;
  if (e < kPart) {
    for (int b0 = q; b0 < nwg; b0 += 64) {
      float v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int b = b0 + 4 * i;
        v[i] = b < nwg ? part[(int64_t)b * kPartStride + e] : 0.f;
      }
#pragma unroll
      for (int st = 8; st > 0; st >>= 1)
#pragma unroll
        for (int i = 0; i < st; ++i) v[i] += v[i + st];
      acc += v[0];
    }
  }
  red[q][el] = acc;
  __syncthreads();
  if (q == 0 && e < kPart) out[e] = (red[0][el] + red[1][el]) + (red[2][el] + red[3][el]);
}

// Per patch: dQ and dbeta summed over the tiles that reach it (fixed order).
__global__ void __launch_bounds__(kDQ) k_feat_cell_reduce(FeatArgs a, float* dqc) {
  const int cell = blockIdx.x, view = blockIdx.y, k = threadIdx.x;
  const int cy = cell / a.Wp, cx = cell - cy * a.Wp;
  // the tile rows and the tile columns that reach the patch (a tile's patch
  // rows depend on its row only, its patch columns on its column only)
  // (the first wave: one tile row or column per lane, 64 at a time, then a
  // ballot; the bounds reach the other threads through LDS)
  __shared__ int bounds[4];
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int ty0 = a.tiles_y, ty1 = -1, tx0 = a.tiles_x, tx1 = -1;
    for (int base = 0; base < a.tiles_y; base += 64) {
      const int ty = base + lane;
      bool reach = false;
      if (ty < a.tiles_y) {
        const TileCells r = tile_cells(a, 0, ty);
        reach = cy >= r.cy0 && cy < r.cy0 + r.ncy;
      }
      const uint64_t m = __ballot(reach);
      if (m) {
        ty0 = min(ty0, base + __builtin_ctzll(m));
        ty1 = base + 63 - __builtin_clzll(m);
      }
    }
    for (int base = 0; base < a.tiles_x; base += 64) {
      const int tx = base + lane;
      bool reach = false;
      if (tx < a.tiles_x) {
        const TileCells r = tile_cells(a, tx, 0);
        reach = cx >= r.cx0 && cx < r.cx0 + r.ncx;
      }
      const uint64_t m = __ballot(reach);
      if (m) {
        tx0 = min(tx0, base + __builtin_ctzll(m));
        tx1 = base + 63 - __builtin_clzll(m);
      }
    }
    if (lane == 0) {
      bounds[0] = ty0;
      bounds[1] = ty1;
      bounds[2] = tx0;
      bounds[3] = tx1;
    }
  }
  __syncthreads();
  const int ty0 = bounds[0], ty1 = bounds[1], tx0 = bounds[2], tx1 = bounds[3];
  float s = 0.f;
  for (int ty = ty0; ty <= ty1; ++ty) {
    for (int tx = tx0; tx <= tx1; ++tx) {
      const TileCells tc = tile_cells(a, tx, ty);
      const int64_t t = (int64_t)view * a.tiles + ty * a.tiles_x + tx;
      s += a.dqt[(t * kSlots + (cy - tc.cy0) * tc.ncx + (cx - tc.cx0)) * kDQ + k];
    }
  }
  dqc[((int64_t)view * a.Hp * a.Wp + cell) * kDQ + k] = s;
}

// Parameter gradients: one workgroup per output channel ch of W2, thread j:
//   dW2[ch][j] = (sum_c G_c[ch] dQ_c[j]) + sum_u W2[ch][u] (S[u][j] + S[j][u]) + b2[ch] dm[j]
//   db2[ch]    = (sum_c G_c[ch] dbeta_c) + W2[ch] . dm + 2 dmu b2[ch]
// with the patch sums gq = [129][nh] from the split-K product (colgemm.hip);
// the last workgroup writes dW1 and db1.
__global__ void __launch_bounds__(kFHid) k_feat_params(FeatArgs a, const float* __restrict__ red,
                                                      const float* __restrict__ gq, float* d_params) {
  __shared__ float sred[2];
  const int ch = blockIdx.x, j = threadIdx.x;
  const float* W2 = a.params + kFHid * kFIn + kFHid;
  const float* b2 = W2 + (int64_t)a.nh * kFHid;
  const float* S = red;
  const float* dW1t = red + 16384;
  const float* db1 = red + 16384 + 2048;
  const float* dm = db1 + 128;
  const float dmu = dm[128];
  if (ch == a.nh) {
    for (int c = 0; c < kFIn; ++c) d_params[j * kFIn + c] = dW1t[c * kFHid + j];
    d_params[kFHid * kFIn + j] = db1[j];
    return;
  }
  const float* w2 = W2 + (int64_t)ch * kFHid;
  float acc2 = 0.f;
  for (int u = 0; u < kFHid; ++u) acc2 = fmaf(w2[u], S[u * kFHid + j] + S[j * kFHid + u], acc2);
  float* dW2 = d_params + kFHid * kFIn + kFHid;
  dW2[(int64_t)ch * kFHid + j] = fmaf(b2[ch], dm[j], gq[(int64_t)j * a.nh + ch] + acc2);
  float accb = w2[j] * dm[j];
  for (int o = 32; o > 0; o >>= 1) accb += __shfl_xor(accb, o);
  if ((j & 63) == 0) sred[j >> 6] = accb;
  __syncthreads();
  if (j == 0)
    dW2[(int64_t)a.nh * kFHid + ch] = gq[(int64_t)kFHid * a.nh + ch] + (sred[0] + sred[1]) + 2.f * dmu * b2[ch];
}

ColGemm gram_gemm(const FeatArgs& a) {
  ColGemm g{};
  const float* W2 = a.params + kFHid * kFIn + kFHid;
  g.D = W2;
  g.dstride = kFHid;
  g.ncol = kFHid;
  g.F = W2;
  g.fk = 1;
  g.fr = kFHid;
  g.fview = 0;
  g.nk = kFHid;
  g.tail = W2 + (int64_t)a.nh * kFHid;  // b2: the column m = W2^T b2
  g.V = 1;
  g.rows = a.nh;
  g.nsplit = colgemm_splits(a.nh, kFHid, kFHid + 1);
  return g;
}

ColGemm dq_gemm(const FeatArgs& a, const float* dqc) {
  ColGemm g{};
  g.D = dqc;
  g.dstride = kDQ;
  g.ncol = kDQ;
  g.F = a.dino;
  g.fk = (int64_t)a.Hp * a.Wp;
  g.fr = 1;
  g.fview = (int64_t)a.nh * a.Hp * a.Wp;
  g.nk = a.nh;
  g.V = a.V;
  g.rows = a.Hp * a.Wp;
  g.nsplit = colgemm_splits((int64_t)a.V * a.Hp * a.Wp, kDQ, a.nh);
  return g;
}

}  // namespace

FeatLayout feature_layout(int nh, int n_views, int width, int height, int Hp, int Wp) {
  FeatLayout L{};
  const int64_t tiles = (int64_t)((width + kFT - 1) / kFT) * ((height + kFT - 1) / kFT) * n_views;
  const int64_t cells = (int64_t)Hp * Wp * n_views;
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o = (o + b + 255) & ~(size_t)255;
    return at;
  };
  L.mfrag = take((size_t)kFrag * 2);
  L.mvec = take((kFHid + 1) * 4);
  L.cells = take((size_t)cells * kCell * 4);
  L.tile_loss = take((size_t)tiles * 4);
  L.part = take((size_t)kBwdWG * kPartStride * 4);
  L.dqt = take((size_t)tiles * kSlots * kDQ * 4);
  L.red = take((size_t)kPart * 4);
  L.dqc = take((size_t)cells * kDQ * 4);
  L.dqpix = take((size_t)n_views * width * height * 4);
  FeatArgs ga{};
  ga.V = n_views;
  ga.Hp = Hp;
  ga.Wp = Wp;
  ga.nh = nh;
  L.gpart = take(colgemm_part_floats(gram_gemm(ga)) * 4);
  L.gout = take((size_t)kFHid * (kFHid + 1) * 4);
  L.ppart = take(colgemm_part_floats(dq_gemm(ga, nullptr)) * 4);
  L.pout = take((size_t)kDQ * nh * 4);
  L.total = o;
  return L;
}

int feature_max_patch_span(int width, int height, int Hp, int Wp) {
  // a tile's 16 pixels span 15 steps of the source coordinate: at most
  // floor(15 scale) + 1 first corners, plus the last pixel's second corner,
  // plus one for rounding of the single-precision source coordinate
  const double sx = 15.0 * Wp / width, sy = 15.0 * Hp / height;
  const double s = sx > sy ? sx : sy;
  return (int)(s + 1e-3) + 3;  // the margin covers the rounding of the device's float coordinates
}

namespace {
FeatArgs feat_args(const FeatCall& c, const FeatLayout& L, char* work) {
  FeatArgs a{};
  a.V = c.n_views;
  a.W = c.width;
  a.H = c.height;
  a.nh = c.nh;
  a.Hp = c.Hp;
  a.Wp = c.Wp;
  a.tiles_x = (c.width + kFT - 1) / kFT;
  a.tiles_y = (c.height + kFT - 1) / kFT;
  a.tiles = a.tiles_x * a.tiles_y;
  a.sx = (float)c.Wp / (float)c.width;
  a.sy = (float)c.Hp / (float)c.height;
  a.feat = c.feat;
  a.params = c.params;
  a.dino = c.dino;
  a.mfrag = reinterpret_cast<const uint16_t*>(work + L.mfrag);
  a.mvec = reinterpret_cast<const float*>(work + L.mvec);
  a.cells = reinterpret_cast<const float*>(work + L.cells);
  a.cosine = c.cosine;
  a.tile_loss = reinterpret_cast<float*>(work + L.tile_loss);
  a.dcos = c.dcos;
  a.dfeat = c.dfeat;
  a.part = reinterpret_cast<float*>(work + L.part);
  a.dqt = reinterpret_cast<float*>(work + L.dqt);
  a.dqpix = reinterpret_cast<float*>(work + L.dqpix);
  return a;
}

void launch_prep(const FeatArgs& a, const FeatLayout& L, char* work, hipStream_t s) {
  ColGemm g = gram_gemm(a);
  g.part = reinterpret_cast<float*>(work + L.gpart);
  float* gm = reinterpret_cast<float*>(work + L.gout);
  launch_colgemm(g, gm, s);
  hipLaunchKernelGGL(k_feat_frag, dim3((kFrag / 2 + 255) / 256), dim3(256), 0, s, a, (const float*)gm,
                     reinterpret_cast<uint16_t*>(work + L.mfrag), reinterpret_cast<float*>(work + L.mvec));
  hipLaunchKernelGGL(k_feat_cells, dim3((unsigned)((a.Hp * a.Wp + kQC - 1) / kQC), (unsigned)a.V), dim3(512), 0, s, a,
                     reinterpret_cast<float*>(work + L.cells));
}
}  // namespace

void launch_feature_forward(const FeatCall& c, const FeatLayout& L, char* work, hipStream_t s) {
  const FeatArgs a = feat_args(c, L, work);
  launch_prep(a, L, work, s);
  const int total = a.tiles * a.V;
  hipLaunchKernelGGL(k_feat_fwd, dim3((unsigned)(total < 512 ? total : 512)), dim3(64 * kFwdWaves), 0, s, a);
  if (c.loss) hipLaunchKernelGGL(k_feat_loss, dim3((unsigned)a.V), dim3(256), 0, s, a, c.loss);
}

void launch_feature_backward(const FeatCall& c, const FeatLayout& L, char* work, hipStream_t s) {
  const FeatArgs a = feat_args(c, L, work);
  launch_prep(a, L, work, s);
  const int total = a.tiles * a.V;
  const int nwg = total < kBwdWG ? total : kBwdWG;
  hipLaunchKernelGGL(k_feat_bwd, dim3((unsigned)nwg), dim3(64 * kBwdWaves), 0, s, a);
  hipLaunchKernelGGL(k_feat_bwd_s, dim3((unsigned)nwg), dim3(64 * kBwdWaves), 0, s, a);
  float* red = reinterpret_cast<float*>(work + L.red);
  hipLaunchKernelGGL(k_feat_reduce, dim3((kPart + 63) / 64), dim3(256), 0, s, a.part, nwg, red);
  float* dqc = reinterpret_cast<float*>(work + L.dqc);
  hipLaunchKernelGGL(k_feat_cell_reduce, dim3((unsigned)(a.Hp * a.Wp), (unsigned)a.V), dim3(kDQ), 0, s, a, dqc);
  ColGemm g = dq_gemm(a, dqc);
  g.part = reinterpret_cast<float*>(work + L.ppart);
  float* gq = reinterpret_cast<float*>(work + L.pout);
  launch_colgemm(g, gq, s);
  hipLaunchKernelGGL(k_feat_params, dim3((unsigned)(a.nh + 1)), dim3(kFHid), 0, s, a, red, (const float*)gq,
                     c.dparams);
}

}  // namespace asgs
