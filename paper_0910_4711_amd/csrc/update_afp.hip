// Codebook Updation by exact fixed-point accumulation.
//
// Every coordinate x is mapped to the integer round(x * 2^s), where the
// shift s is chosen from the largest |x| of the training set so that a sum of
// M such integers cannot overflow 62 bits: s = 61 - e - b with |x| < 2^e and
// M < 2^b.  Cell sums are then formed with 64-bit integer additions, which
// are exact and associative, so the order in which rows arrive (and the
// atomics that LDS accumulation uses) cannot change the result: the update
// is deterministic.  For data whose coordinates are multiples of 2^-s (for
// instance integer pixels) the sums are the exact sums and the centroid is
// the exact mean rounded once to FP64 and once to FP32.  Otherwise each
// coordinate is rounded to a multiple of 2^-s first (relative error below
// 2^-(61-b) of the largest |x|).
//
//   absmax    per block: largest |x| (as float bits; max is order-free)
//   shift     one block: s from the block maxima
//   acc       one block per (row chunk, cell slice): LDS int64 sums and
//             counts for the cells of its slice over the rows of its chunk;
//             dense partials per chunk
//   fin       one block per cell: partials of all chunks added (integers),
//             centroid = sum * 2^-s / count (FP64, rounded to FP32); an empty
//             cell keeps its codevector.  For the gradient, (count * c_k - sum)
//             is formed in integers before the single rounding.
#include <algorithm>

#include "control.h"
#include "lbg_internal.h"

namespace lbg {
namespace {

constexpr int kT = 256;
constexpr int kLdsBytes = 61440;
constexpr int kUnroll = 8;  // rows in flight per group

__global__ __launch_bounds__(kT) void absmax_kernel(const float* __restrict__ X, int64_t n,
                                                     uint32_t* __restrict__ part) {
  __shared__ uint32_t s[kT];
  uint32_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const uint32_t b = __float_as_uint(X[i]) & 0x7fffffffu;
    m = (b > m && b < 0x7f800000u) ? b : m;  // ignore Inf / NaN
  }
  s[threadIdx.x] = m;
  __syncthreads();
  for (int off = kT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] = max(s[threadIdx.x], s[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kT) void shift_kernel(const uint32_t* __restrict__ part, int nparts,
                                                    int64_t M, int* __restrict__ shift) {
  __shared__ uint32_t s[kT];
  uint32_t m = 0;
  for (int i = threadIdx.x; i < nparts; i += kT) m = max(m, part[i]);
  s[threadIdx.x] = m;
  __syncthreads();
  for (int off = kT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] = max(s[threadIdx.x], s[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int b = 0;
    while (b < 63 && ((int64_t)1 << b) <= M) ++b;  // M < 2^b
    const float mx = __uint_as_float(s[0]);
    int e = 0;
    if (mx > 0.0f) frexpf(mx, &e);  // mx < 2^e
    *shift = (s[0] == 0) ? 0 : (61 - e - b);
  }
}

__device__ __forceinline__ unsigned long long fixed(float v, int s) {
  return (unsigned long long)llrint(ldexp((double)v, s));
}

// Row layout of the accumulation: a row is handled by G lanes; lane gl
// covers dimensions (gl + q*G)*VW + v for v < VW (VW = 4: float4 loads) and
// q < DPL.
template <int VW>
struct VLoad;
template <>
struct VLoad<4> {
  static __device__ __forceinline__ void get(const float* p, float* v) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  }
};
template <>
struct VLoad<1> {
  static __device__ __forceinline__ void get(const float* p, float* v) { v[0] = *p; }
};

template <int G, int VW, int DPL>
__device__ __forceinline__ void add_row(unsigned long long* sacc, int32_t* scnt, const float* xrow,
                                        int kk, int L, int gl, int s, const float (&v)[DPL][VW]) {
#pragma unroll
  for (int q = 0; q < DPL; ++q)
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      const int d = (gl + q * G) * VW + e;
      if (d < L) atomicAdd(&sacc[kk * L + d], fixed(v[q][e], s));
    }
  if (gl == 0) atomicAdd(&scnt[kk], 1);
}

template <int G, int VW, int DPL>
__device__ __forceinline__ void load_dims(const float* xrow, int L, int gl, bool on,
                                          float (&v)[DPL][VW]) {
#pragma unroll
  for (int q = 0; q < DPL; ++q) {
    const int d0 = (gl + q * G) * VW;
    if (on && d0 < L) {
      VLoad<VW>::get(xrow + d0, v[q]);
    } else {
#pragma unroll
      for (int e = 0; e < VW; ++e) v[q][e] = 0.0f;
    }
  }
}

// One block per (row chunk, cell slice), slices of one chunk adjacent.  Rows
// stream in batches of kBatch.  With one slice every row is added: a group
// of G lanes walks a contiguous sub-range of the batch, kUnroll rows (cell
// index and coordinates) loaded together.  With several slices the batch's
// cell indices are read first and the rows of this slice are gathered into
// an LDS list (integer sums make the list order immaterial), then added.
constexpr int kBatch = 1024;

template <int G, int VW, int DPL>
__global__ __launch_bounds__(kT) void acc_kernel(
    const float* __restrict__ X, int64_t M, int L, const int32_t* __restrict__ idx, int N,
    int cps, int nslices, int64_t rows_per_chunk, const int* __restrict__ shift_p,
    unsigned long long* __restrict__ part, int32_t* __restrict__ pcnt, Ctl ctl) {
  extern __shared__ unsigned long long sacc[];
  __shared__ int32_t slist[kBatch];
  __shared__ int32_t snsel;
  if (ctl.st) {
    // Decision of this iteration from the allocation's partials, the same in
    // every block; block 0 records the next state in ctl.pend.
    __shared__ double red[kT];
    __shared__ int s_act;
    const DevState* st = ctl.st;
    if (st->done) return;
    const double D = block_distortion(ctl.dpart, ctl.nparts, st->M, red);
    if (threadIdx.x == 0) {
      const Step r = step_of(st, D);
      s_act = r.action;
      if (blockIdx.x == 0) {
        *ctl.pend = *st;
        apply_step(st, ctl.pend, D, r, ctl.Dtrace, ctl.Atrace);
      }
    }
    __syncthreads();
    if (s_act != kActUpdate) return;
    N = st->n;
  }
  const int chunk = blockIdx.x / nslices, slice = blockIdx.x % nslices;
  const int k0 = slice * cps, k1 = min(N, k0 + cps), nk = max(0, k1 - k0);
  int32_t* scnt = reinterpret_cast<int32_t*>(sacc + (size_t)cps * L);
  const int t = threadIdx.x;
  for (int e = t; e < nk * L; e += kT) sacc[e] = 0ull;
  for (int e = t; e < nk; e += kT) scnt[e] = 0;
  if (t == 0) snsel = 0;
  __syncthreads();
  const int s = *shift_p;
  constexpr int NG = kT / G;  // rows in parallel
  const int g = t / G, gl = t % G;
  const int64_t r0 = (int64_t)chunk * rows_per_chunk;
  const int64_t r1 = min(M, r0 + rows_per_chunk);
  for (int64_t b0 = r0; b0 < r1; b0 += kBatch) {
    const int nb = (int)min((int64_t)kBatch, r1 - b0);
    if (nslices == 1) {
      constexpr int PER = kBatch / NG;  // rows of one group per batch
      const int64_t gb = b0 + (int64_t)g * PER;
      for (int i0 = 0; i0 < PER; i0 += kUnroll) {
        int k[kUnroll];
        float v[kUnroll][DPL][VW];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int64_t m = gb + i0 + u;
          const bool on = (i0 + u < PER) && (g * PER + i0 + u < nb);
          k[u] = on ? idx[m] : -1;
          load_dims<G, VW, DPL>(X + m * L, L, gl, on, v[u]);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          if (k[u] >= k0 && k[u] < k1)
            add_row<G, VW, DPL>(sacc, scnt, nullptr, k[u] - k0, L, gl, s, v[u]);
      }
    } else {
#pragma unroll
      for (int u = 0; u < kBatch / kT; ++u) {
        const int r = u * kT + t;
        if (r < nb) {
          const int k = idx[b0 + r];
          if (k >= k0 && k < k1) slist[atomicAdd(&snsel, 1)] = r * 8192 + (k - k0);
        }
      }
      __syncthreads();
      const int nsel = snsel;
      for (int e0 = g; e0 < nsel; e0 += NG * kUnroll) {
        int kk[kUnroll];
        float v[kUnroll][DPL][VW];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int e = e0 + u * NG;
          const int packed = (e < nsel) ? slist[e] : -1;
          const int r = packed >= 0 ? packed >> 13 : 0;
          kk[u] = packed >= 0 ? (packed & 8191) : -1;
          load_dims<G, VW, DPL>(X + (b0 + r) * L, L, gl, packed >= 0, v[u]);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          if (kk[u] >= 0) add_row<G, VW, DPL>(sacc, scnt, nullptr, kk[u], L, gl, s, v[u]);
      }
      __syncthreads();
      if (t == 0) snsel = 0;
      __syncthreads();
    }
  }
  __syncthreads();
  unsigned long long* dst = part + ((int64_t)chunk * N + k0) * L;
  for (int e = t; e < nk * L; e += kT) dst[e] = sacc[e];
  int32_t* cdst = pcnt + (int64_t)chunk * N + k0;
  for (int e = t; e < nk; e += kT) cdst[e] = scnt[e];
}

// One block per cell: thread (q, d) adds the partials of chunks q, q+Q, ...
// (integers, so the order is immaterial), then the Q lane sums.
template <int MODE>
__global__ __launch_bounds__(kT) void fin_kernel(
    const unsigned long long* __restrict__ part, const int32_t* __restrict__ pcnt, int nchunks,
    int N, int L, const int* __restrict__ shift_p, const float* __restrict__ C_old,
    float* __restrict__ out, int32_t* __restrict__ counts, double g2, Ctl ctl, CbPair cbp) {
  __shared__ unsigned long long red[kT];
  __shared__ long long scount;
  const int k = blockIdx.x;
  if (ctl.st) {
    // act on the pending state; block 0 commits it for the next allocation
    if (ctl.st->done) return;
    const DevState* st = ctl.pend;
    if (k == 0 && threadIdx.x == 0) *ctl.st = *st;
    if (st->action == kActSplit) {
      // Codebook Splitting of codevector k (the split kernel's arithmetic):
      // children 2k ("+") and 2k+1 ("-"), formed in FP64, rounded once.
      if (k >= st->n_src) return;
      const float* Cs = cbp.c[st->src];
      float* Cd = cbp.c[st->dst];
      for (int d = threadIdx.x; d < L; d += kT) {
        const double c = (double)Cs[(int64_t)k * L + d];
        double up, dn;
        if (st->split_mode == LBG_SPLIT_ADD) {
          up = c + st->delta;
          dn = c - st->delta;
        } else {
          up = c * (1.0 + st->eps);
          dn = c * (1.0 - st->eps);
        }
        Cd[(int64_t)(2 * k) * L + d] = (float)up;
        Cd[(int64_t)(2 * k + 1) * L + d] = (float)dn;
      }
      return;
    }
    if (st->action != kActUpdate) return;
    N = st->n_src;
    C_old = cbp.c[st->src];
    out = cbp.c[st->dst];
    if (k >= N) return;
  }
  const int t = threadIdx.x;
  if (t < 64) {
    long long c = 0;
    for (int ch = t; ch < nchunks; ch += 64) c += pcnt[(int64_t)ch * N + k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    if (t == 0) scount = c;
  }
  int G2 = 1;
  while (G2 < L && G2 < kT) G2 <<= 1;
  const int Q = kT / G2;
  const int s = *shift_p;
  __syncthreads();
  const long long cnt = scount;
  if (counts && t == 0) counts[k] = (int32_t)cnt;
  for (int d0 = 0; d0 < L; d0 += G2) {
    const int q = t / G2, d = d0 + t % G2;
    unsigned long long a0 = 0, a1 = 0;
    if (d < L && cnt > 0) {
      int ch = q;
      for (; ch + Q < nchunks; ch += 2 * Q) {
        a0 += part[((int64_t)ch * N + k) * L + d];
        a1 += part[((int64_t)(ch + Q) * N + k) * L + d];
      }
      if (ch < nchunks) a0 += part[((int64_t)ch * N + k) * L + d];
    }
    red[t] = a0 + a1;
    __syncthreads();
    if (t < G2 && d < L) {
      const int64_t e = (int64_t)k * L + d;
      if (cnt == 0) {
        if (MODE == 0) {
          if (out != C_old) out[e] = C_old[e];
        } else {
          out[e] = 0.0f;
        }
      } else {
        unsigned long long sum = 0;
        for (int qi = 0; qi < Q; ++qi) sum += red[qi * G2 + t];
        const long long S = (long long)sum;
        if (MODE == 0) {
          out[e] = (float)(ldexp((double)S, -s) / (double)cnt);
        } else {
          const long long ck = llrint(ldexp((double)C_old[e], s));
          const long long diff = (long long)((unsigned long long)(cnt * ck) - (unsigned long long)S);
          out[e] = (float)(g2 * ldexp((double)diff, -s));
        }
      }
    }
    __syncthreads();
  }
}

template <int G, int VW, int DPL>
void launch_acc(dim3 grid, size_t lds, hipStream_t st, const float* X, int64_t M, int L,
                const int32_t* idx, int N, int cps, int nslices, int64_t rpc, const int* sp,
                unsigned long long* part, int32_t* pcnt, Ctl ctl) {
  hipLaunchKernelGGL((acc_kernel<G, VW, DPL>), grid, dim3(kT), lds, st, X, M, L, idx, N, cps,
                     nslices, rpc, sp, part, pcnt, ctl);
}

}  // namespace

void plan_afp(Carver& c, int64_t M, int64_t L, int64_t N, AfpWs* w) {
  w->cps = (int)std::min<int64_t>(std::min<int64_t>(N, 8192), kLdsBytes / (8 * L + 4));
  w->nslices = (int)((N + w->cps - 1) / w->cps);
  // Partials at most half of X's bytes, at least one chunk per 256 rows
  // of work, about 512 blocks in all.
  int64_t nch = std::max<int64_t>(1, 512 / w->nslices);
  nch = std::min<int64_t>(nch, std::max<int64_t>(1, M / (4 * N)));
  nch = std::min<int64_t>(nch, std::max<int64_t>(1, (M + 255) / 256));
  w->nchunks = (int)nch;
  w->rows_per_chunk = (M + nch - 1) / nch;
  w->absmax_blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (M * L + 4095) / 4096));
  w->part = c.take<unsigned long long>((size_t)(nch * N * L));
  w->pcnt = c.take<int32_t>((size_t)(nch * N));
  w->amax = c.take<uint32_t>((size_t)w->absmax_blocks);
  w->shift = c.take<int>(1);
}

bool afp_usable(int64_t L, int64_t N) {
  const int cps = (int)std::min<int64_t>(std::min<int64_t>(N, 8192), kLdsBytes / (8 * L + 4));
  return cps >= 1 && (N + cps - 1) / cps <= 32;
}

int launch_afp_shift(const float* X, int64_t M, int64_t L, const AfpWs& w, hipStream_t s) {
  hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)w.absmax_blocks), dim3(kT), 0, s, X, M * L,
                     w.amax);
  LBG_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(shift_kernel, dim3(1), dim3(kT), 0, s, w.amax, w.absmax_blocks, M, w.shift);
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

int launch_afp(const float* X, int64_t M, int64_t L, const int32_t* idx, const float* C_old,
               int64_t N, float* C_out, int32_t* counts, int mode, double g2, const AfpWs& w,
               hipStream_t s, Ctl ctl, CbPair cbp) {
  const bool vec = (L % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  const int VW = vec ? 4 : 1;
  const int lanes = (int)((L + VW - 1) / VW);
  int G = 1;
  while (G < lanes && G < 64) G <<= 1;
  const int DPL = (lanes + G - 1) / G;
  const dim3 grid((unsigned)(w.nchunks * w.nslices));
  const size_t lds = (size_t)w.cps * L * 8 + (size_t)w.cps * 4;
  const int n = (int)N, Li = (int)L;
#define LBG_ACC(GG, VV, DD)                                                                     \
  if (G == GG && VW == VV && DPL == DD) {                                                       \
    launch_acc<GG, VV, DD>(grid, lds, s, X, M, Li, idx, n, w.cps, w.nslices, w.rows_per_chunk, \
                           w.shift, w.part, w.pcnt, ctl);                                       \
  } else
  LBG_ACC(1, 4, 1) LBG_ACC(2, 4, 1) LBG_ACC(4, 4, 1) LBG_ACC(8, 4, 1) LBG_ACC(16, 4, 1)
  LBG_ACC(32, 4, 1) LBG_ACC(64, 4, 1)
  LBG_ACC(1, 1, 1) LBG_ACC(2, 1, 1) LBG_ACC(4, 1, 1) LBG_ACC(8, 1, 1) LBG_ACC(16, 1, 1)
  LBG_ACC(32, 1, 1) LBG_ACC(64, 1, 1) LBG_ACC(64, 1, 2) LBG_ACC(64, 1, 3) LBG_ACC(64, 1, 4) {
    set_error("internal: no accumulation kernel for G=%d VW=%d DPL=%d", G, VW, DPL);
    return LBG_EINVAL;
  }
#undef LBG_ACC
  LBG_TRY_HIP(hipGetLastError());
  if (mode == 0)
    hipLaunchKernelGGL(fin_kernel<0>, dim3((unsigned)N), dim3(kT), 0, s, w.part, w.pcnt,
                       w.nchunks, n, Li, w.shift, C_old, C_out, counts, g2, ctl, cbp);
  else
    hipLaunchKernelGGL(fin_kernel<1>, dim3((unsigned)N), dim3(kT), 0, s, w.part, w.pcnt,
                       w.nchunks, n, Li, w.shift, C_old, C_out, counts, g2, ctl, cbp);
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

}  // namespace lbg
