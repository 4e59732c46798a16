// Small kernels around the Lloyd iteration: Codebook Splitting, the initial
// centroid, the distortion of a given allocation, the fixed-order reduction
// of per-workgroup partial sums and the gradient with respect to X.
#include <algorithm>

#include "afp_common.h"
#include "control.h"
#include "lbg_internal.h"
#include "misc_common.h"

namespace lbg {
namespace {

constexpr int kThreads = 256;

// Codebook Splitting: child 2i = "+" and child 2i+1 = "-" of codevector i,
// formed in FP64 and rounded once to FP32.
__global__ __launch_bounds__(kThreads) void split_kernel(const float* __restrict__ C,
                                                         int64_t n, int L, int mode,
                                                         double eps, double delta,
                                                         float* __restrict__ C2,
                                                         const DevState* __restrict__ st,
                                                         CbPair cbp) {
  if (st) {
    if (st->done || st->action != kActSplit) return;
    n = st->n_src;
    C = cbp.c[st->src];
    C2 = cbp.c[st->dst];
  }
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= n * L) return;
  const int64_t i = e / L;
  const int d = (int)(e % L);
  misc::split_pair(C[e], mode, eps, delta, &C2[(2 * i) * L + d], &C2[(2 * i + 1) * L + d]);
}

__global__ __launch_bounds__(kThreads) void colsum_kernel(const float* __restrict__ X,
                                                          int64_t M, int L,
                                                          int64_t rows_per_block,
                                                          double* __restrict__ part) {
  misc::colsum_body(X, M, L, rows_per_block, part, blockIdx.x);
}

// One block per column.
__global__ __launch_bounds__(kThreads) void colsum_final_kernel(
    const double* __restrict__ part, int64_t nparts, int L, int64_t M,
    float* __restrict__ c0) {
  misc::colsum_final_body(part, nparts, L, M, c0, blockIdx.x);
}

// Fixed-order sum of FP64 partials: thread t adds parts t, t+256, ... in
// that order (loads issued kRB at a time, additions in sequence); the 256
// results are added by a fixed tree.
constexpr int kRB = 32;

__global__ __launch_bounds__(kThreads) void reduce_parts_kernel(
    const double* __restrict__ parts, int64_t nparts, double denom,
    double* __restrict__ out) {
  __shared__ double s[kThreads];
  double acc = 0.0;
  int64_t p = threadIdx.x;
  for (; p + (int64_t)(kRB - 1) * kThreads < nparts; p += (int64_t)kRB * kThreads) {
    double v[kRB];
#pragma unroll
    for (int b = 0; b < kRB; ++b) v[b] = parts[p + (int64_t)b * kThreads];
#pragma unroll
    for (int b = 0; b < kRB; ++b) acc += v[b];
  }
  for (; p < nparts; p += kThreads) acc += parts[p];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0] / denom;
}

// Distance of every row to its allocated codevector (FP64 direct form, in
// dimension order), block partial sums in a fixed tree.  The workgroup's 256
// rows pass through LDS kDC dimensions at a time, copied with consecutive
// threads on consecutive words so that the loads of X coalesce; thread t then
// adds row t's dimensions in order.  V4: L % kDC == 0 and X, C 16-byte
// aligned (16-byte loads).
constexpr int kDC = 16;

template <bool V4>
__global__ __launch_bounds__(kThreads) void rowdist_kernel(
    const float* __restrict__ X, int64_t M, int L, const float* __restrict__ C,
    int n, const int32_t* __restrict__ idx, double* __restrict__ part) {
  __shared__ float sx[kThreads * (kDC + 1)];
  __shared__ double s[kThreads];
  const int t = threadIdx.x;
  const int64_t m0 = (int64_t)blockIdx.x * kThreads;
  const int rows = (int)min<int64_t>(kThreads, M - m0);
  const int k = t < rows ? idx[m0 + t] : -1;
  const bool ok = t < rows && (unsigned)k < (unsigned)n;
  const float* c = C + (int64_t)(ok ? k : 0) * L;
  const float* xb = X + m0 * L;
  double d = 0.0;
  for (int c0 = 0; c0 < L; c0 += kDC) {
    const int w = min(kDC, L - c0);
    __syncthreads();  // the previous chunk has been read
    if constexpr (V4) {
      for (int e = t; e < rows * (kDC / 4); e += kThreads) {
        const int r = e / (kDC / 4), q = e % (kDC / 4);
        const float4 v = *reinterpret_cast<const float4*>(xb + (int64_t)r * L + c0 + 4 * q);
        float* dst = sx + r * (kDC + 1) + 4 * q;
        dst[0] = v.x;
        dst[1] = v.y;
        dst[2] = v.z;
        dst[3] = v.w;
      }
    } else {
      for (int e = t; e < rows * kDC; e += kThreads) {
        const int r = e / kDC, j = e % kDC;
        if (j < w) sx[r * (kDC + 1) + j] = xb[(int64_t)r * L + c0 + j];
      }
    }
    __syncthreads();
    if (ok) {
      const float* xr = sx + t * (kDC + 1);
      if constexpr (V4) {
#pragma unroll
        for (int q = 0; q < kDC / 4; ++q) {
          const float4 cv = *reinterpret_cast<const float4*>(c + c0 + 4 * q);
          const double u0 = (double)xr[4 * q] - (double)cv.x;
          d = d + u0 * u0;
          const double u1 = (double)xr[4 * q + 1] - (double)cv.y;
          d = d + u1 * u1;
          const double u2 = (double)xr[4 * q + 2] - (double)cv.z;
          d = d + u2 * u2;
          const double u3 = (double)xr[4 * q + 3] - (double)cv.w;
          d = d + u3 * u3;
        }
      } else {
        for (int j = 0; j < w; ++j) {
          const double u = (double)xr[j] - (double)c[c0 + j];
          d = d + u * u;
        }
      }
    }
  }
  s[t] = d;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (t < off) s[t] += s[t + off];
    __syncthreads();
  }
  if (t == 0) part[blockIdx.x] = s[0];
}

// dD/dX: G lanes per row (a power of two, at least the row's words; VEC:
// words are float4), kThreads / G rows per pass, kGU rows per thread in
// flight.  Rows with an index outside [0, n) get zeros.
constexpr int kGU = 4;

template <int G, bool VEC>
__global__ __launch_bounds__(kThreads) void grad_x_kernel(
    const float* __restrict__ X, int64_t M, int L, const float* __restrict__ C,
    int n, const int32_t* __restrict__ idx, double g2, float* __restrict__ gX) {
  constexpr int RB = kThreads / G;
  const int q = threadIdx.x % G, r = threadIdx.x / G;
  const int W = VEC ? L / 4 : L;  // words per row
  if (q >= W) return;             // (no barrier below)
  const int64_t step = (int64_t)gridDim.x * RB * kGU;
  for (int64_t base = (int64_t)blockIdx.x * RB * kGU; base < M; base += step) {
    int k[kGU];
#pragma unroll
    for (int u = 0; u < kGU; ++u) {
      const int64_t m = base + u * RB + r;
      k[u] = m < M ? idx[m] : -1;
    }
#pragma unroll
    for (int u = 0; u < kGU; ++u) {
      const int64_t m = base + u * RB + r;
      if (m >= M) continue;
      const bool ok = (unsigned)k[u] < (unsigned)n;
      const int64_t crow = (int64_t)(ok ? k[u] : 0) * W;
      if constexpr (VEC) {
        const float4 x = reinterpret_cast<const float4*>(X)[m * W + q];
        const float4 c = reinterpret_cast<const float4*>(C)[crow + q];
        float4 o;
        o.x = ok ? (float)(g2 * ((double)x.x - (double)c.x)) : 0.0f;
        o.y = ok ? (float)(g2 * ((double)x.y - (double)c.y)) : 0.0f;
        o.z = ok ? (float)(g2 * ((double)x.z - (double)c.z)) : 0.0f;
        o.w = ok ? (float)(g2 * ((double)x.w - (double)c.w)) : 0.0f;
        reinterpret_cast<float4*>(gX)[m * W + q] = o;  // (non-temporal: measured slower)
      } else {
        const float x = X[m * W + q];
        const float c = C[crow + q];
        gX[m * W + q] = ok ? (float)(g2 * ((double)x - (double)c)) : 0.0f;
      }
    }
  }
}

// Statistics of a finished run.  cell_count_kernel: sizes of the cells of
// the allocation (privatised per block in LDS when the codebook is small).
constexpr int kHistLds = 16384;  // cells counted in LDS

__global__ __launch_bounds__(1024) void cell_count_kernel(const int32_t* __restrict__ idx,
                                                          int64_t M, int n,
                                                          int32_t* __restrict__ cnt) {
  __shared__ int32_t h[kHistLds];
  const bool lds = n <= kHistLds;
  if (lds) {
    for (int k = threadIdx.x; k < n; k += blockDim.x) h[k] = 0;
    __syncthreads();
  }
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < M;
       m += (int64_t)gridDim.x * blockDim.x) {
    const int k = idx[m];
    if ((unsigned)k < (unsigned)n) {
      if (lds)
        atomicAdd(&h[k], 1);
      else
        atomicAdd(&cnt[k], 1);
    }
  }
  if (lds) {
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x)
      if (h[k]) atomicAdd(&cnt[k], h[k]);
  }
}

// out[0] += number of empty cells among the n.
__global__ __launch_bounds__(256) void empty_count_kernel(const int32_t* __restrict__ cnt, int n,
                                                          unsigned long long* __restrict__ out) {
  int e = 0;
  for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) e += cnt[k] == 0;
  e += __shfl_xor(e, 1);
  e += __shfl_xor(e, 2);
  e += __shfl_xor(e, 4);
  e += __shfl_xor(e, 8);
  e += __shfl_xor(e, 16);
  e += __shfl_xor(e, 32);
  if ((threadIdx.x & 63) == 0 && e) atomicAdd(out, (unsigned long long)e);
}

// out[1] += rows whose two nearest codevectors (FP64 direct form, every
// codevector scored) are within 1e-6 |x|^2 of each other: one thread per row.
__global__ __launch_bounds__(256) void tie_count_kernel(const float* __restrict__ X, int64_t M,
                                                        int L, const float* __restrict__ C,
                                                        int n, unsigned long long* __restrict__ out) {
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int tie = 0;
  if (m < M && n >= 2) {
    const float* x = X + m * (int64_t)L;
    double d1 = INFINITY, d2 = INFINITY, xx = 0.0;
    for (int l = 0; l < L; ++l) xx += (double)x[l] * (double)x[l];
    for (int k = 0; k < n; ++k) {
      const float* c = C + (int64_t)k * L;
      double d = 0.0;
      for (int l = 0; l < L; ++l) {
        const double t = (double)x[l] - (double)c[l];
        d = d + t * t;
      }
      if (d < d1) {
        d2 = d1;
        d1 = d;
      } else if (d < d2) {
        d2 = d;
      }
    }
    tie = (d2 - d1) < 1e-6 * xx;
  }
  const unsigned long long b = __ballot(tie);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(out + 1, (unsigned long long)__popcll(b));
}

}  // namespace

int launch_run_stats(const float* X, int64_t M, int64_t L, const float* C, int64_t n,
                     const int32_t* idx, bool ties, int32_t* cnt, unsigned long long* out,
                     hipStream_t s) {
  LBG_TRY_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)n, s));
  LBG_TRY_HIP(hipMemsetAsync(out, 0, 2 * sizeof(unsigned long long), s));
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(512, (M + 1023) / 1024));
  hipLaunchKernelGGL(cell_count_kernel, dim3(grid), dim3(1024), 0, s, idx, M, (int)n, cnt);
  LBG_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(empty_count_kernel, dim3((unsigned)std::min<int64_t>(64, (n + 255) / 256)),
                     dim3(256), 0, s, cnt, (int)n, out);
  LBG_TRY_HIP(hipGetLastError());
  if (ties) {
    hipLaunchKernelGGL(tie_count_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, X,
                       M, (int)L, C, (int)n, out);
    LBG_TRY_HIP(hipGetLastError());
  }
  return LBG_OK;
}

int launch_split(const float* C, int64_t n, int64_t L, int mode, double eps,
                 double delta, float* C2, hipStream_t s, const DevState* st, CbPair cbp) {
  const int64_t grid = (n * L + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(split_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, C, n,
                     (int)L, mode, eps, delta, C2, st, cbp);
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

// Set-up of a training run in two launches.  setup_pass_kernel: the column
// sums of colsum_kernel (same blocks, same order) and, from the same loads,
// each block's largest finite |x|, largest fine bits and the OR of the low 16
// bits (as absmax_kernel forms them; none depends on the order); the blocks
// also clear the update's second-word array lo (nlo words).
__global__ __launch_bounds__(kThreads) void setup_pass_kernel(const float* __restrict__ X,
                                                              int64_t M, int L,
                                                              int64_t rows_per_block,
                                                              double* __restrict__ part,
                                                              uint32_t* __restrict__ amax,
                                                              unsigned long long* __restrict__ lo,
                                                              int64_t nlo) {
  afp::setup_pass_body(X, M, L, rows_per_block, part, amax, gridDim.x, blockIdx.x, lo, nlo);
}

// setup_final_kernel, one block per dimension d: c0[d] as colsum_final_kernel
// forms it, its split into C2 (children 0 "+" and 1 "-", as split_kernel),
// and in block 0 the fixed-point shift (as shift_kernel), the initial run
// state and the cleared fallback counter.
__global__ __launch_bounds__(kThreads) void setup_final_kernel(
    const double* __restrict__ part, int64_t nparts, int L, int64_t M, float* __restrict__ c0,
    float* __restrict__ C2, int mode, double eps, double delta,
    const uint32_t* __restrict__ amax, int namax, int* __restrict__ shift, DevState init,
    DevState* __restrict__ st, unsigned long long* __restrict__ nfb) {
  const int d = blockIdx.x;
  __shared__ double s[kThreads];
  double acc = 0.0;
  for (int64_t p = threadIdx.x; p < nparts; p += kThreads) acc += part[p * L + d];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float c = (float)(s[0] / (double)M);
    c0[d] = c;
    misc::split_pair(c, mode, eps, delta, &C2[d], &C2[L + d]);
  }
  if (d == 0) {
    afp::shift_body(amax, namax, M, shift);
    if (threadIdx.x == 0) {
      *st = init;
      *nfb = 0ull;
    }
  }
}

__global__ __launch_bounds__(kThreads) void decide_kernel(const double* __restrict__ parts,
                                                          int64_t nparts, DevState* st,
                                                          double* __restrict__ Dtrace,
                                                          int32_t* __restrict__ Atrace) {
  __shared__ double red[kThreads];
  if (st->done) return;
  decide_block(parts, nparts, st, Dtrace, Atrace, red);
}

int launch_decide(const double* dpart, int64_t nparts, DevState* st, double* Dtrace,
                  int32_t* Atrace, hipStream_t s) {
  hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(kThreads), 0, s, dpart, nparts, st, Dtrace,
                     Atrace);
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

void plan_centroid(Carver& c, int64_t M, int64_t L, CentroidWs* ws) {
  ws->nwg = std::min<int64_t>(1024, std::max<int64_t>(1, (M + 255) / 256));
  ws->part = c.take<double>((size_t)(ws->nwg * L));
  ws->amax = c.take<uint32_t>((size_t)(3 * ws->nwg));
}

int launch_setup(const float* X, int64_t M, int64_t L, float* c0, float* C2, int mode,
                 double eps, double delta, const CentroidWs& ws, int* shift,
                 unsigned long long* lo, int64_t nlo, const DevState& init, DevState* st,
                 unsigned long long* nfb, hipStream_t s) {
  const int64_t rpb = (M + ws.nwg - 1) / ws.nwg;
  hipLaunchKernelGGL(setup_pass_kernel, dim3((unsigned)ws.nwg), dim3(kThreads), 0, s, X, M,
                     (int)L, rpb, ws.part, ws.amax, lo, nlo);
  LBG_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(setup_final_kernel, dim3((unsigned)L), dim3(kThreads), 0, s, ws.part,
                     ws.nwg, (int)L, M, c0, C2, mode, eps, delta, ws.amax, (int)ws.nwg, shift,
                     init, st, nfb);
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

int launch_centroid(const float* X, int64_t M, int64_t L, float* c0,
                    const CentroidWs& ws, hipStream_t s) {
  const int64_t rpb = (M + ws.nwg - 1) / ws.nwg;
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)ws.nwg), dim3(kThreads), 0, s, X, M,
                     (int)L, rpb, ws.part);
  LBG_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(colsum_final_kernel, dim3((unsigned)L), dim3(kThreads), 0, s, ws.part,
                     ws.nwg, (int)L, M, c0);
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

int launch_reduce_parts(const double* parts, int64_t nparts, double denom,
                        double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(1), dim3(kThreads), 0, s, parts, nparts,
                     denom, out);
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

void plan_distortion(Carver& c, int64_t M, DistWs* ws) {
  ws->nparts = std::max<int64_t>(1, (M + kThreads - 1) / kThreads);
  ws->part = c.take<double>((size_t)ws->nparts);
}

int launch_distortion(const float* X, int64_t M, int64_t L, const float* C,
                      int64_t N, const int32_t* idx, double* D,
                      const DistWs& ws, hipStream_t s) {
  const bool v4 = (L % kDC == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0) &&
                  ((reinterpret_cast<uintptr_t>(C) & 15) == 0);
  if (v4)
    hipLaunchKernelGGL(rowdist_kernel<true>, dim3((unsigned)ws.nparts), dim3(kThreads), 0, s,
                       X, M, (int)L, C, (int)N, idx, ws.part);
  else
    hipLaunchKernelGGL(rowdist_kernel<false>, dim3((unsigned)ws.nparts), dim3(kThreads), 0, s,
                       X, M, (int)L, C, (int)N, idx, ws.part);
  LBG_TRY_HIP(hipGetLastError());
  return launch_reduce_parts(ws.part, ws.nparts, (double)M, D, s);
}

int launch_grad_x(const float* X, int64_t M, int64_t L, const float* C,
                  int64_t N, const int32_t* idx, double g2, float* gX,
                  hipStream_t s) {
  const bool vec = (L % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(C) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(gX) & 15) == 0);
  const int words = (int)(vec ? L / 4 : L);
  int G = 1;
  while (G < words && G < kThreads) G <<= 1;
  const int64_t per_block = (int64_t)(kThreads / G) * kGU;
  const unsigned grid =
      (unsigned)std::max<int64_t>(1, std::min<int64_t>(2048, (M + per_block - 1) / per_block));
  const int l = (int)L, n = (int)N;
#define LBG_GX(GG, VV)                                                                       \
  if (G == GG && vec == VV) {                                                                \
    hipLaunchKernelGGL((grad_x_kernel<GG, VV>), dim3(grid), dim3(kThreads), 0, s, X, M, l, C, \
                       n, idx, g2, gX);                                                      \
  } else
  LBG_GX(1, true) LBG_GX(2, true) LBG_GX(4, true) LBG_GX(8, true) LBG_GX(16, true)
  LBG_GX(32, true) LBG_GX(64, true)
  LBG_GX(1, false) LBG_GX(2, false) LBG_GX(4, false) LBG_GX(8, false) LBG_GX(16, false)
  LBG_GX(32, false) LBG_GX(64, false) LBG_GX(128, false) LBG_GX(256, false) {
    set_error("internal: no gradient kernel for %d lanes per row", G);
    return LBG_EINVAL;
  }
#undef LBG_GX
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

}  // namespace lbg
