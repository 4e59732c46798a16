// Cell Allocation (Algorithm 1, "Cell Allocation"): the nearest codevector of
// every training vector under the squared Euclidean distance, lowest index
// on ties, plus per-row-tile FP64 sums of the winning distances (the
// per-processor distortion that the master integrates).  This file holds the
// FP32 screen (exact result), the dispatch, and an exhaustive FP64 kernel for
// dimensions above the matrix-core kernels' limit.
#include "assign_common.h"

namespace lbg {
namespace {

using namespace assign_detail;

// Exhaustive FP64 search, one thread per row.
__global__ __launch_bounds__(256) void assign_exact_kernel(
    const float* __restrict__ X, int64_t M, int L, const float* __restrict__ C,
    int n, int32_t* __restrict__ idx, float* __restrict__ mind,
    double* __restrict__ dpart) {
  __shared__ double sD[256];
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double best = 0.0;
  if (m < M) {
    const float* x = X + m * (int64_t)L;
    // the first strictly smaller distance from +inf: a row with no finite
    // distance (a non-finite coordinate) gets index 0 and +inf
    int bi = 0;
    best = INFINITY;
    for (int k = 0; k < n; ++k) {
      const double d = d64(x, C + (int64_t)k * L, L);
      if (d < best) {
        best = d;
        bi = k;
      }
    }
    idx[m] = bi;
    if (mind) mind[m] = (float)best;
  }
  sD[threadIdx.x] = best;
  __syncthreads();
  tile_partial<256>(sD, dpart, blockIdx.x);
}

template <int LP>
size_t prep_size(int64_t N, int precision) {
  const int64_t n_pad = (N + 31) & ~(int64_t)31;
  if (precision == LBG_BF16_RESCORE) {
    constexpr int LB = LP < 16 ? 16 : LP;
    return (size_t)n_pad * Bf16Screen<LB>::S * 2;
  }
  if (LP >= 16 && LP <= 64) return (size_t)n_pad * Bf16x3Screen<LP < 16 ? 16 : LP>::S * 2;
  return (size_t)n_pad * Fp32Screen<LP>::S * 4;
}

}  // namespace

int padded_dim(int64_t L) {
  if (L <= 8) return 8;
  if (L <= 16) return 16;
  if (L <= 32) return 32;
  if (L <= 64) return 64;
  if (L <= 128) return 128;
  return 0;  // exhaustive kernel
}

int tile_bits_for(int64_t n) { return tile_bits_of(n); }

size_t prep_bytes(int64_t L, int64_t N, int precision) {
  switch (padded_dim(L)) {
    case 8: return prep_size<8>(N, precision);
    case 16: return prep_size<16>(N, precision);
    case 32: return prep_size<32>(N, precision);
    case 64: return prep_size<64>(N, precision);
    case 128: return prep_size<128>(N, precision);
    default: return 0;
  }
}

// Matrix-core kernels: one partial of the distortion per 32 vectors;
// exhaustive kernel: one per block of 256 rows.
int64_t assign_num_parts(int64_t M, int64_t L, int64_t N, int precision) {
  (void)N;
  (void)precision;
  if (padded_dim(L) == 0) return (M + 255) / 256;
  return (M + 31) / 32;
}

void plan_assign(Carver& c, int64_t M, int64_t L, int64_t N, int precision, AssignWs* ws) {
  ws->dpart = c.take<double>((size_t)assign_num_parts(M, L, N, precision));
  ws->nfb = c.take<unsigned long long>(1);
  ws->prep = c.take<unsigned char>(prep_bytes(L, N, precision));
}

int launch_assign(const float* X, int64_t M, int64_t L, const float* C, int64_t N,
                  int32_t* idx, float* mind, int precision, double* dpart,
                  unsigned long long* nfb, void* prep, hipStream_t s, Ctl ctl, CbPair cbp) {
  const int LP = padded_dim(L);
  const int Li = (int)L, n = (int)N;
  if (LP == 0) {
    if (ctl.st) {
      set_error("internal: device-side control needs L <= 128");
      return LBG_EINVAL;
    }
    const int64_t grid = (M + 255) / 256;
    hipLaunchKernelGGL(assign_exact_kernel, dim3((unsigned)grid), dim3(256), 0, s, X, M, Li, C,
                       n, idx, mind, dpart);
    LBG_TRY_HIP(hipGetLastError());
    return LBG_OK;
  }
  if (precision == LBG_BF16_RESCORE)
    return launch_assign_bf16(X, M, Li, C, n, idx, mind, dpart, LP, prep, s, ctl, cbp);
  switch (LP) {
    case 8: return launch_screen<Fp32Screen<8>>(X, M, Li, C, n, idx, mind, dpart, nfb, prep, s, ctl, cbp);
    case 16: return launch_screen<Bf16x3Screen<16>>(X, M, Li, C, n, idx, mind, dpart, nfb, prep, s, ctl, cbp);
    case 32: return launch_screen<Bf16x3Screen<32>>(X, M, Li, C, n, idx, mind, dpart, nfb, prep, s, ctl, cbp);
    case 64: return launch_screen<Bf16x3Screen<64>>(X, M, Li, C, n, idx, mind, dpart, nfb, prep, s, ctl, cbp);
    default: return launch_screen<Fp32Screen<128>>(X, M, Li, C, n, idx, mind, dpart, nfb, prep, s, ctl, cbp);
  }
}

}  // namespace lbg
