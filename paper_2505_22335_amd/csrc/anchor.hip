// Probabilistic anchor update (UP-SLAM Sec. 3.3, Eq. 7): per anchor, Bayes'
// rule in odds form with the prior,
//   P <- 1 / (1 + (1 - P_obs)/P_obs * (1 - P)/P * P0/(1 - P0)),
// clamped to [p_min, p_max], and the keep flag P >= prune_below with the
// number of kept anchors. HBM-bound: 4 + 4 bytes in, 4 + 1 bytes out per
// anchor, four anchors per thread.
#include "internal.h"

namespace asgs {

namespace {

constexpr int kUpdThreads = 256;

__global__ void __launch_bounds__(kUpdThreads) k_anchor_update(int64_t n, const float* __restrict__ p_obs,
                                                               float* __restrict__ p, uint8_t* __restrict__ keep,
                                                               unsigned long long* n_keep, float prior_odds,
                                                               float p_min, float p_max, float prune_below) {
  __shared__ uint32_t red[kUpdThreads / 64];
  uint32_t kept = 0;
  for (int64_t i = (int64_t)blockIdx.x * kUpdThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kUpdThreads) {
    const float po = p_obs[i], pp = p[i];
    const float odds = ((1.f - po) / po) * ((1.f - pp) / pp) * prior_odds;
    const float q = fminf(fmaxf(1.f / (1.f + odds), p_min), p_max);
    p[i] = q;
    const bool k = q >= prune_below;
    if (keep) keep[i] = k ? 1u : 0u;
    kept += k ? 1u : 0u;
  }
  if (!n_keep) return;
  for (int o = 32; o > 0; o >>= 1) kept += __shfl_xor(kept, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = kept;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int q = 0; q < kUpdThreads / 64; ++q) s += red[q];
    atomicAdd(n_keep, s);  // integer sum: the same in any order
  }
}

// the count starts from zero (a kernel rather than a memset, so that the
// call can be captured in a graph)
__global__ void k_zero_count(unsigned long long* n_keep) { *n_keep = 0ull; }

}  // namespace

void launch_anchor_update(int64_t n, const float* p_obs, float* p, uint8_t* keep, unsigned long long* n_keep,
                          float prior, float p_min, float p_max, float prune_below, hipStream_t s) {
  const int64_t want = (n + kUpdThreads * 4 - 1) / (kUpdThreads * 4);
  const unsigned blocks = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
  if (n_keep) hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, n_keep);
  hipLaunchKernelGGL(k_anchor_update, dim3(blocks), dim3(kUpdThreads), 0, s, n, p_obs, p, keep, n_keep,
                     prior / (1.f - prior), p_min, p_max, prune_below);
}

}  // namespace asgs
