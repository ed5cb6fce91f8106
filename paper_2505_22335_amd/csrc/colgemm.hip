// Split-K products over rows, for the parameter gradients and Gram matrices of
// the per-pixel MLPs (feature lift and uncertainty MLP):
//   out[col][k] = sum_r D[r][col] F_k(r)
// where r runs over (view, patch) rows, D is a row-major table (one row per
// r) and F_k(r) a strided view of the DINO grid or of a weight matrix, with an
// optional extra row from a vector (tail) and an optional row of ones (so that
// out[col][.] also holds sum_r D[r][col]). The rows are cut into nsplit
// contiguous chunks; each workgroup forms a 64-column x 32-k tile of one
// chunk's partial product from LDS-staged blocks of D and F on the matrix
// cores (FP32), and a second kernel adds the chunks' partials in chunk order
// (deterministic).
#include "internal.h"

namespace asgs {

namespace {

constexpr int kCT = 64;   // columns per workgroup
constexpr int kKT = 32;   // k per workgroup
constexpr int kRB = 32;   // rows per staged block

typedef float f4v __attribute__((ext_vector_type(4)));

ASGS_DEV float fval(const ColGemm& g, int k, int64_t r) {
  const int64_t v = r / g.rows, c = r - v * g.rows;
  if (k < g.nk) return g.F[v * g.fview + (int64_t)k * g.fk + c * g.fr];
  if (g.tail && k == g.nk) return g.tail[c];
  return 1.f;  // the row of ones
}

__global__ void __launch_bounds__(256) k_colgemm_part(ColGemm g) {
  __shared__ float ds[kRB][kCT + 1];
  __shared__ float fs[kKT][kRB + 1];
  const int t = threadIdx.x;
  const int c0 = blockIdx.x * kCT, k0 = blockIdx.y * kKT, s = blockIdx.z;
  const int lane = t & 63, wv = t >> 6, gq = lane >> 4, f = lane & 15;
  const int nkt = g.nk + (g.tail ? 1 : 0) + (g.ones ? 1 : 0);
  const int64_t R = (int64_t)g.V * g.rows;
  const int64_t r0 = R * s / g.nsplit, r1 = R * (s + 1) / g.nsplit;
  // wave w: columns 16 w .. + 15 of the tile against both 16-wide k blocks,
  // on v_mfma_f32_16x16x4f32 (M = columns, N = k, K = four rows a step)
  f4v acc[2] = {f4v{0.f, 0.f, 0.f, 0.f}, f4v{0.f, 0.f, 0.f, 0.f}};
  // the next block's values are requested before the current block is used
  constexpr int kDP = kRB * kCT / 256, kFP = kKT * kRB / 256;
  float dn[kDP], fn[kFP];
  auto fetch = [&](int64_t rb) {
#pragma unroll
    for (int i = 0; i < kDP; ++i) {
      const int q = t + 256 * i, rr = q / kCT, cc = q - rr * kCT;
      const int64_t r = rb + rr;
      dn[i] = r < r1 && c0 + cc < g.ncol ? g.D[r * g.dstride + c0 + cc] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < kFP; ++i) {
      const int q = t + 256 * i, kk = q / kRB, rr = q - kk * kRB;
      const int64_t r = rb + rr;
      fn[i] = r < r1 && k0 + kk < nkt ? fval(g, k0 + kk, r) : 0.f;
    }
  };
  fetch(r0);
  for (int64_t rb = r0; rb < r1; rb += kRB) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kDP; ++i) {
      const int q = t + 256 * i;
      ds[q / kCT][q % kCT] = dn[i];
    }
#pragma unroll
    for (int i = 0; i < kFP; ++i) {
      const int q = t + 256 * i;
      fs[q / kRB][q % kRB] = fn[i];
    }
    __syncthreads();
    fetch(rb + kRB);  // rows past the chunk read as zero
#pragma unroll
    for (int st = 0; st < kRB / 4; ++st) {
      const float a = ds[4 * st + gq][16 * wv + f];
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
        acc[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, fs[16 * kb + f][4 * st + gq], acc[kb], 0, 0, 0);
    }
  }
  // rows: columns c0 + 16 w + 4 (l / 16) + j; columns: k0 + 16 kb + l % 16
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) {
    const int k = k0 + 16 * kb + f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = c0 + 16 * wv + 4 * gq + j;
      if (col < g.ncol && k < nkt) g.part[((int64_t)s * g.ncol + col) * nkt + k] = acc[kb][j];
    }
  }
}

__global__ void __launch_bounds__(256) k_colgemm_reduce(ColGemm g, float* out) {
  const int nkt = g.nk + (g.tail ? 1 : 0) + (g.ones ? 1 : 0);
  const int64_t n = (int64_t)g.ncol * nkt;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  // chunk order, sixteen loads in flight
  float s = 0.f;
  for (int b0 = 0; b0 < g.nsplit; b0 += 16) {
    float v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = b0 + i < g.nsplit ? g.part[(int64_t)(b0 + i) * n + e] : 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (b0 + i < g.nsplit) s += v[i];
  }
  out[e] = s;
}

}  // namespace

// One chunk per 48 rows (at most 64); products with few tiles take chunks
// down to 24 rows, up to about 256 workgroups (measured: the Gram matrix
// gains from the extra chunks, the patch products lose from them).
int colgemm_splits(int64_t rows, int ncol, int nkt) {
  const int64_t tiles = (int64_t)((ncol + kCT - 1) / kCT) * ((nkt + kKT - 1) / kKT);
  int64_t s = rows / 48;
  if (tiles * s < 256) {
    const int64_t more = min(rows / 24, 256 / tiles);
    if (more > s) s = more;
  }
  return (int)(s < 1 ? 1 : (s > 64 ? 64 : s));
}

size_t colgemm_part_floats(const ColGemm& g) {
  const int nkt = g.nk + (g.tail ? 1 : 0) + (g.ones ? 1 : 0);
  return (size_t)g.nsplit * g.ncol * nkt;
}

void launch_colgemm(const ColGemm& g, float* out, hipStream_t s) {
  const int nkt = g.nk + (g.tail ? 1 : 0) + (g.ones ? 1 : 0);
  hipLaunchKernelGGL(k_colgemm_part, dim3((unsigned)((g.ncol + kCT - 1) / kCT), (unsigned)((nkt + kKT - 1) / kKT),
                                          (unsigned)g.nsplit),
                     dim3(256), 0, s, g);
  const int64_t n = (int64_t)g.ncol * nkt;
  hipLaunchKernelGGL(k_colgemm_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, out);
}

}  // namespace asgs
