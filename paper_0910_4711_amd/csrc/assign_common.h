// Cell Allocation on gfx950 matrix cores: the kernel shared by the FP32
// screen (exact result) and the BF16 screen (precision form).
//
//   * prep: the codebook is written once per call in the LDS row layout of
//     the screen: -2c (exact scaling), zero-padded to LP dimensions, with the
//     squared norm stored in the row's padding; rows are padded to a multiple
//     of 32 with a huge norm so that padding never wins.
//   * One workgroup = 4 waves; a wave owns XT tiles of 32 training vectors,
//     a workgroup a "row tile" of 128*XT vectors.  Workgroups loop over row
//     tiles.  The codebook is staged into LDS with 16-byte copies: once per
//     workgroup when it fits (resident), otherwise chunk by chunk per row tile.
//   * Screen: v_mfma_f32_32x32x2_f32 (FP32) or v_mfma_f32_32x32x16_bf16 (BF16)
//     computes |c|^2 + |x|^2 - 2 x.c for a 32 (codevectors) x 32 (vectors)
//     tile; a first K-step with A = [|c|^2, 1], B = [1, |x|^2] adds both norms,
//     so the accumulator starts at zero.  Codevectors are the A operand, so
//     each lane holds 16 distances of ONE vector.
//   * Each lane keeps the two smallest keys of every accumulator slot; a key
//     is the screened distance with its low mantissa bits replaced by the tile
//     number (3 VALU ops per distance: and-or, med3 as min, med3).
//   * FP32: the best candidate is rescored in FP64, direct form, dimension
//     order; a rigorous bound on the screen's rounding decides whether it is
//     provably the unique nearest codevector, otherwise the wave searches the
//     row again exhaustively in FP64.  BF16: the two best candidates are
//     rescored in FP64 and the closer taken (lowest index on ties).
#pragma once

#include <float.h>
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "lbg_internal.h"

namespace lbg {

int padded_dim(int64_t L);
int tile_bits_for(int64_t n);

namespace assign_detail {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr float kBig = 3.0e38f;    // squared norm of padding codevectors
constexpr int kPersistBlocks = 512;  // grid of the allocation kernel (2 per CU)
constexpr int kLdsBudget = 61440;  // bytes of LDS for the staged codebook

// Row of the 32 x 32 matrix-core result held in accumulator register r of
// ``lane``: four groups of four rows, the two half-waves interleaved by four.
__device__ __forceinline__ int out_row(int lane, int r) {
  return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// ---------------------------------------------------------------- policy --
template <int LP_>
struct Fp32Screen {
  static constexpr int LP = LP_;
  static constexpr int S = LP + 4;   // row stride, elements
  static constexpr int ESZ = 4;      // bytes per element
  static constexpr int NS = LP / 2;  // K-steps of the data
  static constexpr int XT = (LP >= 128) ? 1 : 2;
  static constexpr bool EXACT = true;
  typedef float elem;
};

template <int LP_>
struct Bf16Screen {
  static constexpr int LP = LP_;
  static constexpr int S = LP + 8;
  static constexpr int ESZ = 2;
  static constexpr int NS = LP / 16;
  static constexpr int XT = (LP >= 128) ? 1 : 2;
  static constexpr bool EXACT = false;
  typedef __bf16 elem;
};

template <class SC>
constexpr int rows_per_tile() { return 4 * 32 * SC::XT; }

// Rows of codevectors staged per chunk (multiple of 32) for a codebook of
// n_pad rows: all of it when it fits the LDS budget.
template <class SC>
inline int chunk_rows(int n_pad) {
  const int row_bytes = SC::S * SC::ESZ;
  const int cap = (kLdsBudget / row_bytes) & ~31;
  return n_pad <= cap ? n_pad : cap;
}

__device__ __forceinline__ void split3(float v, __bf16& hi, __bf16& mid, __bf16& lo) {
  hi = (__bf16)v;
  const float r = v - (float)hi;
  mid = (__bf16)r;
  lo = (__bf16)(r - (float)mid);
}

// Codebook in the screen's row layout; one block per row.
template <class SC>
__global__ __launch_bounds__(256) void prep_kernel(const float* __restrict__ C, int n,
                                                   int L, typename SC::elem* __restrict__ Cp,
                                                   const DevState* __restrict__ st, CbPair cbp) {
  const int row = blockIdx.x;
  const int t = threadIdx.x;
  if (st) {
    if (st->done) return;
    n = st->n;
    C = cbp.c[st->cb];
    if (row >= ((n + 31) & ~31)) return;
  }
  typedef typename SC::elem E;
  __shared__ double part[256];
  double q = 0.0;
  for (int d = t; d < SC::LP; d += 256) {
    const float v = (row < n && d < L) ? C[(int64_t)row * L + d] : 0.0f;
    const E e = (E)(-2.0f * v);
    Cp[(int64_t)row * SC::S + d] = e;
    const double r = (double)(float)e;  // -2 * (rounded value)
    q += r * r;
  }
  part[t] = q;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) part[t] += part[t + off];
    __syncthreads();
  }
  if (t == 0) {
    const float nrm = (row < n) ? (float)(0.25 * part[0]) : kBig;
    E* pad = Cp + (int64_t)row * SC::S + SC::LP;
    if constexpr (SC::EXACT) {
      pad[0] = nrm;
      pad[1] = 1.0f;
      pad[2] = 0.0f;
      pad[3] = 0.0f;
    } else {
      __bf16 hi, mid, lo;
      split3(nrm, hi, mid, lo);
      const __bf16 one = (__bf16)1.0f, zero = (__bf16)0.0f;
      pad[0] = hi;
      pad[1] = mid;
      pad[2] = lo;
      pad[3] = one;
      pad[4] = one;
      pad[5] = one;
      pad[6] = zero;
      pad[7] = zero;
    }
  }
}

// ----------------------------------------------------------- candidates --
template <int XT>
struct Slots {
  float mn[XT][16];
  float mn2[XT][16];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int xt = 0; xt < XT; ++xt)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        mn[xt][r] = FLT_MAX;
        mn2[xt][r] = FLT_MAX;
      }
  }
  // key = distance with its low mantissa bits replaced by the tile number;
  // min as med3(a, b, -inf) (no NaN canonicalisation), second via med3.
  __device__ __forceinline__ void push(int xt, const f16v& acc, uint32_t vmask,
                                       uint32_t tb, float ninf) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float k = __uint_as_float((__float_as_uint(acc[r]) & vmask) | tb);
      const float a = mn[xt][r];
      mn2[xt][r] = __builtin_amdgcn_fmed3f(a, mn2[xt][r], k);
      mn[xt][r] = __builtin_amdgcn_fmed3f(a, k, ninf);
    }
  }
};

struct Top2 {
  float k1, k2;
  int i1, i2;
  __device__ __forceinline__ void insert(float v, int id) {
    if (v < k1) {
      k2 = k1;
      i2 = i1;
      k1 = v;
      i1 = id;
    } else if (v < k2) {
      k2 = v;
      i2 = id;
    }
  }
};

__device__ __forceinline__ bool before(float a, int ia, float b, int ib) {
  return a < b || (a == b && ia < ib);
}

// Two smallest keys of one training vector over all slots of both half-
// waves; both lanes of the pair obtain the same result.
template <int XT>
__device__ __forceinline__ Top2 top2_of(const Slots<XT>& sl, int xt, int lane,
                                        uint32_t lowmask) {
  Top2 t{INFINITY, INFINITY, -1, -1};
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int rr = out_row(lane, r);
    const float a = sl.mn[xt][r], b = sl.mn2[xt][r];
    t.insert(a, (int)((__float_as_uint(a) & lowmask) << 5) + rr);
    t.insert(b, (int)((__float_as_uint(b) & lowmask) << 5) + rr);
  }
  const float b1 = __shfl_xor(t.k1, 32), b2 = __shfl_xor(t.k2, 32);
  const int bi1 = __shfl_xor(t.i1, 32), bi2 = __shfl_xor(t.i2, 32);
  const bool aFirst = before(t.k1, t.i1, b1, bi1);
  Top2 o;
  o.k1 = aFirst ? t.k1 : b1;
  o.i1 = aFirst ? t.i1 : bi1;
  const float c1 = aFirst ? b1 : t.k1;
  const int ci1 = aFirst ? bi1 : t.i1;
  const float c2 = aFirst ? t.k2 : b2;
  const int ci2 = aFirst ? t.i2 : bi2;
  const bool cFirst = before(c1, ci1, c2, ci2);
  o.k2 = cFirst ? c1 : c2;
  o.i2 = cFirst ? ci1 : ci2;
  return o;
}

// Row of L floats into registers (LP slots, zero beyond L), loads issued
// together.
template <int LP, bool VEC>
__device__ __forceinline__ void load_row(const float* __restrict__ p, int L, float (&v)[LP]) {
  if (VEC) {
#pragma unroll
    for (int s = 0; s < LP; s += 4) {
      const float4 q = *reinterpret_cast<const float4*>(p + s);
      v[s] = q.x;
      v[s + 1] = q.y;
      v[s + 2] = q.z;
      v[s + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int s = 0; s < LP; ++s) v[s] = (s < L) ? p[s] : 0.0f;
  }
}

// Squared distance, FP64, direct form, dimensions in order, one rounding per
// operation (the library is built without FMA contraction).
template <int LP>
__device__ __forceinline__ double d64_regs(const float (&x)[LP], const float (&c)[LP], int L) {
  double s = 0.0;
#pragma unroll
  for (int l = 0; l < LP; ++l) {
    if (l < L) {
      const double t = (double)x[l] - (double)c[l];
      s = s + t * t;
    }
  }
  return s;
}

__device__ __forceinline__ double d64(const float* x, const float* c, int L) {
  double s = 0.0;
  for (int l = 0; l < L; ++l) {
    const double t = (double)x[l] - (double)c[l];
    s = s + t * t;
  }
  return s;
}

// Rescore, decide, fall back and store for the vectors of this wave.  Lane
// (j, h) handles vector j of tile xt = 2p + h.
//   EXACT (FP32 screen): accept the best candidate w only if
//     d(w) * (1 + 4 (L+2) 2^-53) < K2 / (1 + 2^(tile_bits-23)) - E,
//     E = 2 * gamma_{L+4} * (1 + 2^-24) * (2 |x| + sqrt(d(w)))^2 + 1e-30,
//   gamma_k = k u / (1 - k u), u = 2^-24.  E bounds the FP32 screen's
//   rounding error for every codevector c with d(c) <= d(w) (such a c has
//   |c| <= |x| + sqrt(d(w))); the division undoes the key's replaced mantissa
//   bits; K2 is the second-smallest key.  So every other codevector is
//   strictly farther, in exact arithmetic and in FP64.  Rows that fail are
//   searched exhaustively in FP64 by the whole wave (lowest index on ties).
//   Otherwise (BF16 screen): both candidates are rescored in FP64 and the
//   closer one is taken, the lower index on equal distances.
// Exhaustive FP64 search of one row by the whole wave (FP32 screen only):
// lane l scores codevectors l, l+64, ... in increasing order (strict <), then
// the wave takes the smallest distance, lowest index on equal distances.
// Codevectors come from the LDS-resident screen copy (-2c, exact) when the
// whole codebook is staged, otherwise from C with vector loads.
template <class SC, bool VEC>
__device__ __forceinline__ void search_row(const float* __restrict__ xrow, int L,
                                           const float* __restrict__ C, int n,
                                           const float* resident, int lane, double* best_d,
                                           int* best_i) {
  constexpr int LP = SC::LP;
  float xr[LP];
  load_row<LP, VEC>(xrow, L, xr);
  double best = INFINITY;
  int bi = 0x7fffffff;
  if (resident) {
    for (int k = lane; k < n; k += 64) {
      const float* r = resident + (int64_t)k * SC::S;
      float cr[LP];
#pragma unroll
      for (int s4 = 0; s4 < LP; s4 += 4) {
        const float4 q = *reinterpret_cast<const float4*>(r + s4);
        cr[s4] = -0.5f * q.x;
        cr[s4 + 1] = -0.5f * q.y;
        cr[s4 + 2] = -0.5f * q.z;
        cr[s4 + 3] = -0.5f * q.w;
      }
      const double dk = d64_regs<LP>(xr, cr, L);
      if (dk < best) {
        best = dk;
        bi = k;
      }
    }
  } else {
    int k = lane;
    for (; k + 64 < n; k += 128) {
      float c0[LP], c1[LP];
      load_row<LP, VEC>(C + (int64_t)k * L, L, c0);
      load_row<LP, VEC>(C + (int64_t)(k + 64) * L, L, c1);
      const double d0 = d64_regs<LP>(xr, c0, L);
      const double d1 = d64_regs<LP>(xr, c1, L);
      if (d0 < best) {
        best = d0;
        bi = k;
      }
      if (d1 < best) {
        best = d1;
        bi = k + 64;
      }
    }
    if (k < n) {
      float c0[LP];
      load_row<LP, VEC>(C + (int64_t)k * L, L, c0);
      const double d0 = d64_regs<LP>(xr, c0, L);
      if (d0 < best) {
        best = d0;
        bi = k;
      }
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ob = __shfl_xor(best, off);
    const int oi = __shfl_xor(bi, off);
    if (ob < best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  *best_d = best;
  *best_i = bi;
}

// Returns the sum of the winning distances of the rows this lane handled.
template <class SC, bool VEC, class BF>
__device__ __forceinline__ double finish_rows(const Slots<SC::XT>& sl,
                                              const float* __restrict__ X, int64_t M, int L,
                                              const float* __restrict__ C, int n,
                                              int32_t* __restrict__ idx,
                                              float* __restrict__ mind, int64_t row0,
                                              int tile_bits, unsigned long long* nfb,
                                              const typename SC::elem* resident,
                                              const BF (&xf)[SC::XT][SC::NS]) {
  constexpr int XT = SC::XT;
  constexpr int LP = SC::LP;
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int j = lane & 31;
  const uint32_t lowmask = (1u << tile_bits) - 1u;
  double dsum = 0.0;

  Top2 tp[XT];
#pragma unroll
  for (int xt = 0; xt < XT; ++xt) tp[xt] = top2_of<XT>(sl, xt, lane, lowmask);

  const double gam = (double)(L + 4) * 0x1p-24 / (1.0 - (double)(L + 4) * 0x1p-24);
  const double keyslack = 1.0 + ldexp(1.0, tile_bits - 23);
  const double dslack = 1.0 + 4.0 * (double)(L + 2) * 0x1p-53;

#pragma unroll
  for (int p = 0; p < (XT + 1) / 2; ++p) {
    const int xt = 2 * p + h;
    const bool have = xt < XT;
    Top2 t = tp[0];
#pragma unroll
    for (int q = 1; q < XT; ++q)
      if (xt == q) t = tp[q];
    const int64_t m = row0 + xt * 32 + j;
    const bool live = have && m < M;
    bool flag = false;
    double d = 0.0;
    int win = 0;
    float xr[LP];
    if constexpr (SC::EXACT) {
      // the row from the two half-waves' fragments: this lane's half, and the
      // other half from lane (j, 1-h), which sends its half of the row this
      // lane handles (xt = 2p + h)
      const int sx = 2 * p + (1 - h);
#pragma unroll
      for (int s2 = 0; s2 < LP / 2; ++s2) {
        float own = 0.0f, send = 0.0f;
#pragma unroll
        for (int q = 0; q < XT; ++q) {
          if (q == xt) own = xf[q][s2];
          if (q == sx) send = xf[q][s2];
        }
        const float recv = __shfl_xor(send, 32);
        xr[s2] = h ? recv : own;
        xr[LP / 2 + s2] = h ? own : recv;
      }
    }
    if (live) {
      win = t.i1;
      const bool bad = (unsigned)win >= (unsigned)n;  // non-finite input
      if (bad) win = 0;
      float cr[LP];
      if constexpr (SC::EXACT) {
        if (resident) {
          const float* r = reinterpret_cast<const float*>(resident) + (int64_t)win * SC::S;
#pragma unroll
          for (int s4 = 0; s4 < LP; s4 += 4) {
            const float4 q4 = *reinterpret_cast<const float4*>(r + s4);
            cr[s4] = -0.5f * q4.x;
            cr[s4 + 1] = -0.5f * q4.y;
            cr[s4 + 2] = -0.5f * q4.z;
            cr[s4 + 3] = -0.5f * q4.w;
          }
        } else {
          load_row<LP, VEC>(C + (int64_t)win * L, L, cr);
        }
      } else {
        load_row<LP, VEC>(X + m * (int64_t)L, L, xr);
        load_row<LP, VEC>(C + (int64_t)win * L, L, cr);
      }
      d = d64_regs<LP>(xr, cr, L);
      if constexpr (SC::EXACT) {
        double xx = 0.0;
#pragma unroll
        for (int l = 0; l < LP; ++l) xx += (double)xr[l] * (double)xr[l];
        const double r = 2.0 * sqrt(xx) + sqrt(d * dslack);
        const double E = 2.0 * gam * (1.0 + 0x1p-24) * r * r + 1e-30;
        const double lim = (double)t.k2 / keyslack - E;
        flag = bad || !(d * dslack < lim);
      } else {
        const int i2 = t.i2;
        if (i2 >= 0 && i2 < n && i2 != win) {
          load_row<LP, VEC>(C + (int64_t)i2 * L, L, cr);
          const double d2 = d64_regs<LP>(xr, cr, L);
          if (d2 < d || (d2 == d && i2 < win)) {
            d = d2;
            win = i2;
          }
        }
      }
    }
    if constexpr (SC::EXACT) {
      unsigned long long fl = __ballot(flag);
      if (nfb && lane == 0 && fl) atomicAdd(nfb, (unsigned long long)__popcll(fl));
      while (fl) {
        const int src = __ffsll((long long)fl) - 1;
        fl &= fl - 1;
        const int64_t mf = __shfl(m, src);
        double best;
        int bi;
        search_row<SC, VEC>(X + mf * (int64_t)L, L, C, n, resident, lane, &best, &bi);
        if (lane == src) {
          d = best;
          win = bi;
        }
      }
    }
    if (live) {
      idx[m] = win;
      if (mind) mind[m] = (float)d;
    }
    if (live) dsum += d;
  }
  return dsum;
}

// Fixed-order sum of the tile's ROWS distances into dpart[tile].
template <int ROWS>
__device__ __forceinline__ void tile_partial(const double* sD, double* dpart, int64_t tile) {
  if (dpart == nullptr) return;
  if (threadIdx.x < 64) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < ROWS / 64; ++q) s += sD[threadIdx.x + 64 * q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (threadIdx.x == 0) dpart[tile] = s;
  }
}

// Copy ``bytes`` (multiple of 16) from global to LDS, eight 16-byte loads in
// flight per thread before their stores.
__device__ __forceinline__ void stage(const void* __restrict__ src, void* dst, int bytes) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(dst);
  const int nv = bytes >> 4;
  for (int base = 0; base < nv; base += 8 * kAssignThreads) {
    uint4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + u * kAssignThreads + threadIdx.x;
      if (e < nv) v[u] = s[e];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + u * kAssignThreads + threadIdx.x;
      if (e < nv) d[e] = v[u];
    }
  }
}

// Resident codebook staged straight from C: -2c (exact) zero-padded to LP
// dimensions and n_pad rows, then each row's squared norm (FP64, rounded to
// FP32) in its padding, as prep_kernel writes it.  Loads are issued four at a
// time per thread before their stores.
template <class SC, bool VEC>
__device__ __forceinline__ void stage_from_C(const float* __restrict__ C, int n, int L,
                                             int n_pad, typename SC::elem* sA) {
  constexpr int LP = SC::LP;
  constexpr int S = SC::S;
  typedef typename SC::elem E;
  if (VEC) {
    constexpr int Q = LP / 4;
    const int nv = n_pad * Q;
    for (int base = 0; base < nv; base += 4 * kAssignThreads) {
      float4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = base + u * kAssignThreads + threadIdx.x;
        const int r = e / Q;
        v[u] = (e < nv && r < n) ? *reinterpret_cast<const float4*>(C + (int64_t)e * 4)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = base + u * kAssignThreads + threadIdx.x;
        if (e < nv) {
          E* dst = sA + (e / Q) * S + (e % Q) * 4;
          dst[0] = (E)(-2.0f * v[u].x);
          dst[1] = (E)(-2.0f * v[u].y);
          dst[2] = (E)(-2.0f * v[u].z);
          dst[3] = (E)(-2.0f * v[u].w);
        }
      }
    }
  } else {
    for (int e = threadIdx.x; e < n_pad * LP; e += kAssignThreads) {
      const int r = e / LP, d = e % LP;
      const float v = (r < n && d < L) ? C[(int64_t)r * L + d] : 0.0f;
      sA[r * S + d] = (E)(-2.0f * v);
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < n_pad; r += kAssignThreads) {
    double q = 0.0;
#pragma unroll 8
    for (int d = 0; d < LP; ++d) {
      const double v = (double)(float)sA[r * S + d];
      q += v * v;
    }
    const float nrm = (r < n) ? (float)(0.25 * q) : kBig;
    E* pad = sA + r * S + LP;
    if constexpr (SC::EXACT) {
      pad[0] = nrm;
      pad[1] = 1.0f;
      pad[2] = 0.0f;
      pad[3] = 0.0f;
    } else {
      __bf16 hi, mid, lo;
      split3(nrm, hi, mid, lo);
      const __bf16 one = (__bf16)1.0f, zero = (__bf16)0.0f;
      pad[0] = hi;
      pad[1] = mid;
      pad[2] = lo;
      pad[3] = one;
      pad[4] = one;
      pad[5] = one;
      pad[6] = zero;
      pad[7] = zero;
    }
  }
  __syncthreads();
}

// -------------------------------------------------------------- kernel --
template <class SC, bool VEC>
__global__ __launch_bounds__(kAssignThreads, 2) void assign_kernel(
    const float* __restrict__ X, int64_t M, int L, const float* __restrict__ C, int n,
    const typename SC::elem* __restrict__ Cp, int n_pad, int CR, int32_t* __restrict__ idx,
    float* __restrict__ mind, double* __restrict__ dpart, unsigned long long* __restrict__ nfb,
    int tile_bits, Ctl ctl, CbPair cbp) {
  const DevState* st = ctl.st;
  if (st) {
    if (st->done) return;
    n = st->n;
    C = cbp.c[st->cb];
    n_pad = (n + 31) & ~31;
    tile_bits = tile_bits_of(n);
  }
  constexpr int XT = SC::XT;
  constexpr int LP = SC::LP;
  constexpr int S = SC::S;
  constexpr int NS = SC::NS;
  constexpr int ROWS = rows_per_tile<SC>();
  typedef typename SC::elem E;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  E* sA = reinterpret_cast<E*>(smem);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int h = lane >> 5;
  const int j = lane & 31;
  const int64_t ntiles_rows = (M + ROWS - 1) / ROWS;
  const bool resident = CR >= n_pad;
  // key mask in a VGPR, so that the and-or reads a single SGPR (tile bits)
  uint32_t vmask = ~((1u << tile_bits) - 1u);
  asm volatile("v_mov_b32 %0, %1" : "=v"(vmask) : "v"(vmask));
  const float ninf = -INFINITY;

  if (resident) stage_from_C<SC, VEC>(C, n, L, n_pad, sA);

  double wsum = 0.0;
  for (int64_t rt = blockIdx.x; rt < ntiles_rows; rt += gridDim.x) {
    const int64_t row0 = rt * ROWS + (int64_t)wave * 32 * XT;

    // Training-vector fragments: lane (j, h) keeps dims [h*LP/2, (h+1)*LP/2)
    // of vector j of each of its tiles, as the B operand of the K-steps.
    typedef typename std::conditional<SC::EXACT, float, bf16x8>::type BF;
    BF xf[XT][NS];
    BF xn[XT];
#pragma unroll
    for (int xt = 0; xt < XT; ++xt) {
      const int64_t m = row0 + xt * 32 + j;
      float v[LP / 2];
      if (m < M) {
        const float* xr = X + m * (int64_t)L + h * (LP / 2);
        if (VEC) {
#pragma unroll
          for (int s = 0; s < LP / 2; s += 4) {
            const float4 q = *reinterpret_cast<const float4*>(xr + s);
            v[s] = q.x;
            v[s + 1] = q.y;
            v[s + 2] = q.z;
            v[s + 3] = q.w;
          }
        } else {
#pragma unroll
          for (int s = 0; s < LP / 2; ++s) v[s] = (h * (LP / 2) + s < L) ? xr[s] : 0.0f;
        }
      } else {
#pragma unroll
        for (int s = 0; s < LP / 2; ++s) v[s] = 0.0f;
      }
      double ss = 0.0;
      if constexpr (SC::EXACT) {
#pragma unroll
        for (int s = 0; s < LP / 2; ++s) {
          xf[xt][s] = v[s];
          ss += (double)v[s] * (double)v[s];
        }
        ss += __shfl_xor(ss, 32);
        xn[xt] = h ? (float)ss : 1.0f;
      } else {
#pragma unroll
        for (int s = 0; s < LP / 2; ++s) {
          const __bf16 b = (__bf16)v[s];
          xf[xt][s >> 3][s & 7] = b;
          const double r = (double)(float)b;
          ss += r * r;
        }
        ss += __shfl_xor(ss, 32);
        __bf16 hi, mid, lo;
        split3((float)ss, hi, mid, lo);
        const __bf16 one = (__bf16)1.0f, zero = (__bf16)0.0f;
        const bf16x8 nv = {one, one, one, hi, mid, lo, zero, zero};
        const bf16x8 zv = {zero, zero, zero, zero, zero, zero, zero, zero};
        xn[xt] = h ? zv : nv;
      }
    }

    Slots<XT> sl;
    sl.init();
    for (int c0 = 0; c0 < n_pad; c0 += CR) {
      const int cr = min(CR, n_pad - c0);
      if (!resident) {
        __syncthreads();
        stage(Cp + (int64_t)c0 * S, sA, cr * S * SC::ESZ);
        __syncthreads();
      }
      const E* base = resident ? sA + (int64_t)c0 * S : sA;
      const int nt = cr >> 5;
      for (int t = 0; t < nt; ++t) {
        const E* ar = base + (t * 32 + j) * S;
        f16v acc[XT];
        if constexpr (SC::EXACT) {
          const float an = h ? 1.0f : ar[LP];
#pragma unroll
          for (int xt = 0; xt < XT; ++xt)
            acc[xt] = __builtin_amdgcn_mfma_f32_32x32x2f32(an, xn[xt], f16v{}, 0, 0, 0);
          const float* a = ar + h * (LP / 2);
#pragma unroll
          for (int s = 0; s < NS; s += 4) {
            const float4 a4 = *reinterpret_cast<const float4*>(a + s);
#pragma unroll
            for (int xt = 0; xt < XT; ++xt) {
              acc[xt] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, xf[xt][s], acc[xt], 0, 0, 0);
              acc[xt] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, xf[xt][s + 1], acc[xt], 0, 0, 0);
              acc[xt] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, xf[xt][s + 2], acc[xt], 0, 0, 0);
              acc[xt] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, xf[xt][s + 3], acc[xt], 0, 0, 0);
            }
          }
        } else {
          const __bf16 zero = (__bf16)0.0f;
          const bf16x8 zv = {zero, zero, zero, zero, zero, zero, zero, zero};
          const bf16x8 an = h ? zv : *reinterpret_cast<const bf16x8*>(ar + LP);
#pragma unroll
          for (int xt = 0; xt < XT; ++xt)
            acc[xt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(an, xn[xt], f16v{}, 0, 0, 0);
          const __bf16* a = ar + h * (LP / 2);
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const bf16x8 a8 = *reinterpret_cast<const bf16x8*>(a + 8 * s);
#pragma unroll
            for (int xt = 0; xt < XT; ++xt)
              acc[xt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, xf[xt][s], acc[xt], 0, 0, 0);
          }
        }
        const uint32_t tb = (uint32_t)((c0 >> 5) + t);
#pragma unroll
        for (int xt = 0; xt < XT; ++xt) sl.push(xt, acc[xt], vmask, tb, ninf);
      }
    }

    wsum += finish_rows<SC, VEC, BF>(sl, X, M, L, C, n, idx, mind, row0, tile_bits, nfb,
                                     resident ? sA : nullptr, xf);
  }
  // per-wave partial of the distortion over the block's row tiles (in order),
  // lanes added by a fixed butterfly
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) wsum += __shfl_xor(wsum, off);
  if (dpart && lane == 0) dpart[blockIdx.x * 4 + wave] = wsum;
}

// Host side: prepare the codebook and launch.
// With a device state, n is the largest codebook size (LDS and grids are
// sized for it); the kernels take the current size from the state.
template <class SC>
int launch_screen(const float* X, int64_t M, int L, const float* C, int n, int32_t* idx,
                  float* mind, double* dpart, unsigned long long* nfb, void* prep,
                  hipStream_t s, Ctl ctl, CbPair cbp) {
  const DevState* st = ctl.st;
  typedef typename SC::elem E;
  const int n_pad = (n + 31) & ~31;
  E* Cp = reinterpret_cast<E*>(prep);
  const int CR = chunk_rows<SC>(n_pad);
  if (CR < n_pad) {  // chunked: stage from the prepared copy
    hipLaunchKernelGGL((prep_kernel<SC>), dim3((unsigned)n_pad), dim3(256), 0, s, C, n, L, Cp,
                       st, cbp);
    LBG_TRY_HIP(hipGetLastError());
  }
  constexpr int ROWS = rows_per_tile<SC>();
  const int64_t tiles = (M + ROWS - 1) / ROWS;
  // Persistent grid of two workgroups per CU: a resident codebook is staged
  // once per workgroup, a chunked one per row tile.
  const int64_t grid = std::min<int64_t>(tiles, kPersistBlocks);
  const size_t lds = (size_t)CR * SC::S * SC::ESZ;
  const int tb = tile_bits_for(n);
  bool vec = (L == SC::LP) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  if (st)
    vec = vec && ((reinterpret_cast<uintptr_t>(cbp.c[0]) & 15) == 0) &&
          ((reinterpret_cast<uintptr_t>(cbp.c[1]) & 15) == 0);
  else
    vec = vec && ((reinterpret_cast<uintptr_t>(C) & 15) == 0);
  if (vec)
    hipLaunchKernelGGL((assign_kernel<SC, true>), dim3((unsigned)grid), dim3(kAssignThreads), lds,
                       s, X, M, L, C, n, Cp, n_pad, CR, idx, mind, dpart, nfb, tb, ctl, cbp);
  else
    hipLaunchKernelGGL((assign_kernel<SC, false>), dim3((unsigned)grid), dim3(kAssignThreads),
                       lds, s, X, M, L, C, n, Cp, n_pad, CR, idx, mind, dpart, nfb, tb, ctl, cbp);
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

}  // namespace assign_detail

// Workspace bytes for the prepared codebook of either screen.
size_t prep_bytes(int64_t L, int64_t N, int precision);
int launch_assign_bf16(const float* X, int64_t M, int L, const float* C, int n, int32_t* idx,
                       float* mind, double* dpart, int LP, void* prep, hipStream_t s,
                       Ctl ctl, CbPair cbp);

}  // namespace lbg
