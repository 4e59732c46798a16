// Encoder and decoder of a trained quantizer (Introduction: the encoder
// replaces a vector by the index of its nearest codevector, the decoder puts
// that codevector back; the rate is log2(N)/L bits per sample).  Encoding is
// the Cell Allocation itself; the kernels here only move data:
//
//   decode        Y[m] = C[idx[m]]; an index outside [0, N) gives a row of
//                 quiet NaNs
//   decode_image  the same written straight into pictures cut into b x b
//                 blocks: pixel (p, y, x) is dimension (y mod b) b + (x mod b)
//                 of the codevector of its block
//   image_blocks  pictures to training vectors: one vector per block, blocks
//                 in raster order, pixels row-major inside a block
//
// Every byte of the output is written once and every byte of the input read
// once; the codebook (at most LBG_MAX_N x L floats) is re-read from cache.
// The kernels are therefore bound by HBM bandwidth.  Vectors: lanes take
// consecutive 16-byte words of a row when L % 4 == 0, each thread keeping kU
// rows in flight.  Pictures with b = 4 or 8: one thread per block, so that
// both sides move in contiguous runs (block_rows_kernel); b = 16 and blocks
// off the 16-byte grid: one thread per word of a picture row.
#include <math.h>

#include "lbg_internal.h"

namespace lbg {
namespace {

constexpr int kT = 256;        // threads per workgroup
constexpr int kU = 4;          // rows per thread in flight
constexpr int kMaxGrid = 2048; // eight workgroups per CU

// Decoder outputs are written once and not read again by the kernel: stores
// marked non-temporal where a wave's store covers whole cache lines
// (consecutive lanes on consecutive 16-byte words).  Where each lane writes
// its own run (pictures -> blocks), non-temporal partial-line writes
// measured three times slower than plain stores, which L2 combines; that
// direction stages through LDS when the layout allows (STAGE below) and
// stores plainly otherwise.
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_nt(float4* p, float4 v) {
  const f4v x = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(x, reinterpret_cast<f4v*>(p));
}

__device__ __forceinline__ float4 nan4() {
  const float q = __builtin_nanf("");
  return make_float4(q, q, q, q);
}

// G lanes per row (a power of two, at least the row's words), kT / G rows
// per pass of the workgroup.  VEC: words are float4.
template <int G, bool VEC>
__global__ __launch_bounds__(kT) void decode_kernel(const int32_t* __restrict__ idx, int64_t M,
                                                    const float* __restrict__ C, int N, int L,
                                                    float* __restrict__ Y) {
  constexpr int RB = kT / G;
  const int q = threadIdx.x % G, r = threadIdx.x / G;
  const int W = VEC ? L / 4 : L;  // words per row
  const bool lane_on = q < W;
  const int64_t step = (int64_t)gridDim.x * RB * kU;
  for (int64_t base = (int64_t)blockIdx.x * RB * kU; base < M; base += step) {
    int k[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t m = base + u * RB + r;
      k[u] = m < M ? idx[m] : -1;
    }
    if constexpr (VEC) {
      const float4* C4 = reinterpret_cast<const float4*>(C);
      float4* Y4 = reinterpret_cast<float4*>(Y);
      float4 v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u)
        v[u] = (lane_on && (unsigned)k[u] < (unsigned)N) ? C4[(int64_t)k[u] * W + q] : nan4();
      // (every load above and below is guarded: an index outside [0, N)
      // never forms an address)
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int64_t m = base + u * RB + r;
        if (lane_on && m < M) st_nt(&Y4[m * W + q], v[u]);
      }
    } else {
      float v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u)
        v[u] = (lane_on && (unsigned)k[u] < (unsigned)N) ? C[(int64_t)k[u] * W + q]
                                                          : __builtin_nanf("");
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int64_t m = base + u * RB + r;
        if (lane_on && m < M) Y[m * W + q] = v[u];
      }
    }
  }
}

// Picture geometry shared by the two picture kernels.  Rows of all pictures
// are numbered r = p H + y (p the picture); a thread takes kU consecutive
// rows, so that one division by H serves kU rows.
struct Geo {
  int H, W;        // picture size (multiples of b)
  int b;           // block side (runtime value for the scalar kernels)
  int nbx;         // blocks per block row, W / b
  int nby;         // block rows per picture, H / b
  int64_t rows;    // nimg * H
};

// Pixel-row position of rows r .. r + kU - 1: picture p and row y of the
// first; later rows step y and wrap to the next picture.
__device__ __forceinline__ void row_pos(int64_t r, int H, int& p, int& y) {
  p = (int)(r / H);
  y = (int)(r - (int64_t)p * H);
}

// BQ = b / 4 float4 words per block row (used for b = 16); TPR lanes per
// picture row.
template <int BQ, int TPR>
__global__ __launch_bounds__(kT) void decode_image_kernel(const int32_t* __restrict__ idx,
                                                          const float* __restrict__ C, int N,
                                                          Geo g, float* __restrict__ img) {
  constexpr int B = 4 * BQ, L = B * B, RB = kT / TPR;
  const int c = threadIdx.x % TPR, rr = threadIdx.x / TPR;
  const int W4 = g.W / 4;
  const float4* C4 = reinterpret_cast<const float4*>(C);
  float4* I4 = reinterpret_cast<float4*>(img);
  const int64_t step = (int64_t)gridDim.x * RB * kU;
  for (int64_t base = ((int64_t)blockIdx.x * RB + rr) * kU; base < g.rows; base += step) {
    int p, y;
    row_pos(base, g.H, p, y);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t r = base + u;
      if (r < g.rows) {
        const int by = y / B, dy = y % B;
        const int32_t* irow = idx + ((int64_t)p * g.nby + by) * g.nbx;
        for (int x4 = c; x4 < W4; x4 += TPR) {
          const int bx = x4 / BQ, dx = x4 % BQ;
          const int k = irow[bx];
          const float4 v = (unsigned)k < (unsigned)N ? C4[((int64_t)k * L + dy * B) / 4 + dx]
                                                     : nan4();
          I4[r * W4 + x4] = v;
        }
      }
      if (++y == g.H) {
        y = 0;
        ++p;
      }
    }
  }
}

// One thread per block for b = 4, 8 (BQ = b / 4): the thread moves the
// whole block, so its vector side is one contiguous run of 4 b^2 bytes (a
// single index read for the decoder) while its picture side stays coalesced
// across lanes (consecutive lanes take consecutive blocks of a block row).
// Block rows R = p (H / b) + by start at picture row R b.  DIR 0: decoder,
// DIR 1: pictures -> vectors.
// STAGE (pictures -> vectors, b = 4, W / b a multiple of 64): a wave's 64
// lanes then hold 64 consecutive blocks of one block row, whose vectors are
// one contiguous run; the wave passes them through LDS so that every store
// instruction writes whole lines (consecutive lanes on consecutive words).
template <int BQ, int TPR, int DIR, bool STAGE = false>
__global__ __launch_bounds__(kT) void block_rows_kernel(const int32_t* __restrict__ idx,
                                                        const float* __restrict__ C, int N,
                                                        Geo g, const float* __restrict__ in,
                                                        float* __restrict__ out) {
  constexpr int B = 4 * BQ, L4 = B * BQ, RB = kT / TPR;  // L4: float4 words per block
  static_assert(!STAGE || (DIR == 1 && TPR >= 64), "staged stores: whole waves in one row");
  __shared__ float4 stg[STAGE ? kT * L4 : 1];
  const int c = threadIdx.x % TPR, rr = threadIdx.x / TPR;
  const int64_t W4 = g.W / 4;
  const int64_t nrows = g.rows / B;  // block rows of all pictures
  for (int64_t R = (int64_t)blockIdx.x * RB + rr; R < nrows; R += (int64_t)gridDim.x * RB) {
    const int64_t prow = R * B * W4;  // first picture row of the block row, in words
    for (int bx = c; bx < g.nbx; bx += TPR) {
      const int64_t v = R * g.nbx + bx;
      float4 w[L4];
      if constexpr (DIR == 0) {
        const int k = idx[v];
        const bool ok = (unsigned)k < (unsigned)N;
        const float4* src = reinterpret_cast<const float4*>(C) + (int64_t)(ok ? k : 0) * L4;
#pragma unroll
        for (int e = 0; e < L4; ++e) w[e] = ok ? src[e] : nan4();
        float4* dst = reinterpret_cast<float4*>(out) + prow + (int64_t)bx * BQ;
#pragma unroll
        for (int dy = 0; dy < B; ++dy)
#pragma unroll
          for (int q = 0; q < BQ; ++q) st_nt(&dst[dy * W4 + q], w[dy * BQ + q]);
      } else {
        const float4* src = reinterpret_cast<const float4*>(in) + prow + (int64_t)bx * BQ;
#pragma unroll
        for (int dy = 0; dy < B; ++dy)
#pragma unroll
          for (int q = 0; q < BQ; ++q) w[dy * BQ + q] = src[dy * W4 + q];
        if constexpr (STAGE) {
          const int wl = threadIdx.x & 63;
          float4* sw = stg + (threadIdx.x >> 6) * 64 * L4;
#pragma unroll
          for (int e = 0; e < L4; ++e) sw[wl * L4 + e] = w[e];
          __builtin_amdgcn_wave_barrier();
          float4* dst = reinterpret_cast<float4*>(out) + (v - wl) * L4;
#pragma unroll
          for (int e = 0; e < L4; ++e) st_nt(&dst[e * 64 + wl], sw[e * 64 + wl]);
          __builtin_amdgcn_wave_barrier();
        } else {
          float4* dst = reinterpret_cast<float4*>(out) + v * L4;
#pragma unroll
          for (int e = 0; e < L4; ++e) dst[e] = w[e];  // (plain: see st_nt)
        }
      }
    }
  }
}

template <int TPR>
__global__ __launch_bounds__(kT) void decode_image_scalar_kernel(const int32_t* __restrict__ idx,
                                                                 const float* __restrict__ C,
                                                                 int N, Geo g,
                                                                 float* __restrict__ img) {
  constexpr int RB = kT / TPR;
  const int c = threadIdx.x % TPR, rr = threadIdx.x / TPR;
  const int B = g.b, L = B * B;
  const int64_t step = (int64_t)gridDim.x * RB * kU;
  for (int64_t base = ((int64_t)blockIdx.x * RB + rr) * kU; base < g.rows; base += step) {
    int p, y;
    row_pos(base, g.H, p, y);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t r = base + u;
      if (r < g.rows) {
        const int by = y / B, dy = y - by * B;
        const int32_t* irow = idx + ((int64_t)p * g.nby + by) * g.nbx;
        for (int x = c; x < g.W; x += TPR) {
          const int bx = x / B, dx = x - bx * B;
          const int k = irow[bx];
          img[r * g.W + x] =
              (unsigned)k < (unsigned)N ? C[(int64_t)k * L + dy * B + dx] : __builtin_nanf("");
        }
      }
      if (++y == g.H) {
        y = 0;
        ++p;
      }
    }
  }
}

template <int BQ, int TPR>
__global__ __launch_bounds__(kT) void image_blocks_kernel(const float* __restrict__ img, Geo g,
                                                          float* __restrict__ X) {
  constexpr int B = 4 * BQ, L = B * B, RB = kT / TPR;
  const int c = threadIdx.x % TPR, rr = threadIdx.x / TPR;
  const int W4 = g.W / 4;
  const float4* I4 = reinterpret_cast<const float4*>(img);
  float4* X4 = reinterpret_cast<float4*>(X);
  const int64_t step = (int64_t)gridDim.x * RB * kU;
  for (int64_t base = ((int64_t)blockIdx.x * RB + rr) * kU; base < g.rows; base += step) {
    int p, y;
    row_pos(base, g.H, p, y);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t r = base + u;
      if (r < g.rows) {
        const int by = y / B, dy = y % B;
        const int64_t vrow = ((int64_t)p * g.nby + by) * g.nbx;
        for (int x4 = c; x4 < W4; x4 += TPR) {
          const int bx = x4 / BQ, dx = x4 % BQ;
          X4[((vrow + bx) * L + dy * B) / 4 + dx] = I4[r * W4 + x4];
        }
      }
      if (++y == g.H) {
        y = 0;
        ++p;
      }
    }
  }
}

template <int TPR>
__global__ __launch_bounds__(kT) void image_blocks_scalar_kernel(const float* __restrict__ img,
                                                                 Geo g, float* __restrict__ X) {
  constexpr int RB = kT / TPR;
  const int c = threadIdx.x % TPR, rr = threadIdx.x / TPR;
  const int B = g.b, L = B * B;
  const int64_t step = (int64_t)gridDim.x * RB * kU;
  for (int64_t base = ((int64_t)blockIdx.x * RB + rr) * kU; base < g.rows; base += step) {
    int p, y;
    row_pos(base, g.H, p, y);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t r = base + u;
      if (r < g.rows) {
        const int by = y / B, dy = y - by * B;
        const int64_t vrow = ((int64_t)p * g.nby + by) * g.nbx;
        for (int x = c; x < g.W; x += TPR) {
          const int bx = x / B, dx = x - bx * B;
          X[(vrow + bx) * L + dy * B + dx] = img[r * g.W + x];
        }
      }
      if (++y == g.H) {
        y = 0;
        ++p;
      }
    }
  }
}

int pow2_at_least(int v, int cap) {
  int g = 1;
  while (g < v && g < cap) g <<= 1;
  return g;
}

unsigned grid_for(int64_t units, int64_t per_block) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(kMaxGrid, (units + per_block - 1) / per_block));
}

bool a16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

int launch_decode(const int32_t* idx, int64_t M, const float* C, int64_t N, int64_t L, float* Y,
                  hipStream_t s) {
  const bool vec = (L % 4 == 0) && a16(C) && a16(Y);
  const int words = (int)(vec ? L / 4 : L);
  const int G = pow2_at_least(words, kT);
  const unsigned grid = grid_for(M, (int64_t)(kT / G) * kU);
  const int n = (int)N, l = (int)L;
#define LBG_DEC(GG, VV)                                                                     \
  if (G == GG && vec == VV) {                                                               \
    hipLaunchKernelGGL((decode_kernel<GG, VV>), dim3(grid), dim3(kT), 0, s, idx, M, C, n, l, Y); \
  } else
  LBG_DEC(1, true) LBG_DEC(2, true) LBG_DEC(4, true) LBG_DEC(8, true) LBG_DEC(16, true)
  LBG_DEC(32, true) LBG_DEC(64, true)
  LBG_DEC(1, false) LBG_DEC(2, false) LBG_DEC(4, false) LBG_DEC(8, false) LBG_DEC(16, false)
  LBG_DEC(32, false) LBG_DEC(64, false) LBG_DEC(128, false) LBG_DEC(256, false) {
    set_error("internal: no decode kernel for %d lanes per row", G);
    return LBG_EINVAL;
  }
#undef LBG_DEC
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

// dir 0: indices -> pictures (decode_image); dir 1: pictures -> vectors.
int launch_image(int dir, const int32_t* idx, const float* C, int64_t N, int64_t nimg,
                 int64_t H, int64_t W, int64_t b, const float* img_in, float* out,
                 hipStream_t s) {
  Geo g;
  g.H = (int)H;
  g.W = (int)W;
  g.b = (int)b;
  g.nbx = (int)(W / b);
  g.nby = (int)(H / b);
  g.rows = nimg * H;
  const bool vec = (b == 4 || b == 8 || b == 16) &&
                   (dir == 0 ? a16(C) && a16(out) : a16(img_in) && a16(out));
  if (vec && b <= 8) {
    const int TB = pow2_at_least(g.nbx, kT);
    const bool stage = dir == 1 && b == 4 && g.nbx % 64 == 0;  // then TB >= 64
    const unsigned gb = grid_for(g.rows / b, kT / TB);
    const int n0 = (int)N;
#define LBG_BR(BB, TT)                                                                       \
  if (b == 4 * BB && TB == TT) {                                                             \
    if (dir == 0)                                                                            \
      hipLaunchKernelGGL((block_rows_kernel<BB, TT, 0>), dim3(gb), dim3(kT), 0, s, idx, C, n0, \
                         g, nullptr, out);                                                   \
    else if (stage)                                                                          \
      hipLaunchKernelGGL((block_rows_kernel<BB, (TT < 64 ? 64 : TT), 1, true>), dim3(gb),     \
                         dim3(kT), 0, s, nullptr, nullptr, 0, g, img_in, out);               \
    else                                                                                     \
      hipLaunchKernelGGL((block_rows_kernel<BB, TT, 1>), dim3(gb), dim3(kT), 0, s, nullptr,    \
                         nullptr, 0, g, img_in, out);                                        \
  } else
    LBG_BR(1, 1) LBG_BR(1, 2) LBG_BR(1, 4) LBG_BR(1, 8) LBG_BR(1, 16) LBG_BR(1, 32)
    LBG_BR(1, 64) LBG_BR(1, 128) LBG_BR(1, 256)
    LBG_BR(2, 1) LBG_BR(2, 2) LBG_BR(2, 4) LBG_BR(2, 8) LBG_BR(2, 16) LBG_BR(2, 32)
    LBG_BR(2, 64) LBG_BR(2, 128) LBG_BR(2, 256) {
      set_error("internal: no block kernel for b=%lld, %d lanes", (long long)b, TB);
      return LBG_EINVAL;
    }
#undef LBG_BR
    LBG_TRY_HIP(hipGetLastError());
    return LBG_OK;
  }
  const int words = (int)(vec ? W / 4 : W);
  const int TPR = pow2_at_least(words, kT);
  const unsigned grid = grid_for(g.rows, (int64_t)(kT / TPR) * kU);
  const int n = (int)N;
  const int BQ = (int)(b / 4);
#define LBG_IMG(BB, TT)                                                                         \
  if (vec && BQ == BB && TPR == TT) {                                                           \
    if (dir == 0)                                                                               \
      hipLaunchKernelGGL((decode_image_kernel<BB, TT>), dim3(grid), dim3(kT), 0, s, idx, C, n, g, \
                         out);                                                                  \
    else                                                                                        \
      hipLaunchKernelGGL((image_blocks_kernel<BB, TT>), dim3(grid), dim3(kT), 0, s, img_in, g,   \
                         out);                                                                  \
  } else
#define LBG_IMGS(TT)                                                                         \
  if (!vec && TPR == TT) {                                                                   \
    if (dir == 0)                                                                            \
      hipLaunchKernelGGL((decode_image_scalar_kernel<TT>), dim3(grid), dim3(kT), 0, s, idx, C, \
                         n, g, out);                                                         \
    else                                                                                     \
      hipLaunchKernelGGL((image_blocks_scalar_kernel<TT>), dim3(grid), dim3(kT), 0, s, img_in, \
                         g, out);                                                            \
  } else
  LBG_IMG(4, 4) LBG_IMG(4, 8) LBG_IMG(4, 16) LBG_IMG(4, 32) LBG_IMG(4, 64) LBG_IMG(4, 128)
  LBG_IMG(4, 256)
  LBG_IMGS(1) LBG_IMGS(2) LBG_IMGS(4) LBG_IMGS(8) LBG_IMGS(16) LBG_IMGS(32) LBG_IMGS(64)
  LBG_IMGS(128) LBG_IMGS(256) {
    set_error("internal: no picture kernel for b=%lld, %d lanes per row", (long long)b, TPR);
    return LBG_EINVAL;
  }
#undef LBG_IMG
#undef LBG_IMGS
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

}  // namespace lbg
