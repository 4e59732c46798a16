// Device bodies of small steps shared by the single-run kernels (misc.hip,
// update_afp.hip) and the batched kernels (batched.hip).
#pragma once

#include "lbg_internal.h"

namespace lbg {
namespace misc {

constexpr int kThreads = 256;

// Codebook Splitting of one value: child "+" and child "-", formed in FP64
// and rounded once to FP32.
__device__ __forceinline__ void split_pair(float cv, int mode, double eps, double delta,
                                           float* up, float* dn) {
  const double c = (double)cv;
  double u, d;
  if (mode == LBG_SPLIT_ADD) {
    u = c + delta;
    d = c - delta;
  } else {
    u = c * (1.0 + eps);
    d = c * (1.0 - eps);
  }
  *up = (float)u;
  *dn = (float)d;
}

// Per-block column sums of a row range, FP64, fixed order: thread (q, d)
// adds rows q, q + R, q + 2R, ... of block ``blk``'s range (R = 256 / L rows
// in flight, L <= 256), then the R partial sums of each column are added in
// q order.
__device__ __forceinline__ void colsum_body(const float* __restrict__ X, int64_t M, int L,
                                            int64_t rows_per_block, double* __restrict__ part,
                                            int64_t blk) {
  __shared__ double s[kThreads];
  const int R = kThreads / L;
  const int t = threadIdx.x;
  const int q = t / L, d = t % L;
  const int64_t r0 = blk * rows_per_block;
  const int64_t r1 = min(M, r0 + rows_per_block);
  double acc = 0.0;
  if (q < R)
    for (int64_t r = r0 + q; r < r1; r += R) acc += (double)X[r * L + d];
  s[t] = acc;
  __syncthreads();
  if (t < L) {
    double v = 0.0;
    for (int qi = 0; qi < R; ++qi) v += s[qi * L + t];
    part[blk * L + t] = v;
  }
}

// Column d of the centroid: thread t adds the block partials t, t+256, ... in
// order, then a fixed tree adds the 256 thread sums.
__device__ __forceinline__ void colsum_final_body(const double* __restrict__ part,
                                                  int64_t nparts, int L, int64_t M,
                                                  float* __restrict__ c0, int d) {
  __shared__ double s[kThreads];
  double acc = 0.0;
  for (int64_t p = threadIdx.x; p < nparts; p += kThreads) acc += part[p * L + d];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) c0[d] = (float)(s[0] / (double)M);
}

}  // namespace misc
}  // namespace lbg
