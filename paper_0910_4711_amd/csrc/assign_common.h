// Cell Allocation on gfx950 matrix cores: the kernel shared by the exact
// screens (FP32-accurate: split BF16 parts, or FP32) and the BF16 screen
// (precision form).
//
//   * The codebook is staged into LDS in the screen's row layout: -2c (exact
//     scaling; three BF16 parts for the split screen), zero-padded to LP
//     dimensions, with the squared norm in the row's padding; rows are
//     padded to a multiple of 32 with a huge norm so that padding never
//     wins.  A codebook that fits is staged once per workgroup (resident);
//     otherwise a prepared copy is staged chunk by chunk for every row tile.
//   * One workgroup = 4 waves (8 for a codebook resident only in a whole
//     CU's LDS); a wave owns a tile of 32 training vectors.  Workgroups loop
//     over row tiles; the grid is sized so that 2 to 4 waves share each SIMD
//     (by register use).
//   * Screen: MFMAs compute |c|^2 + |x|^2 - 2 x.c for a 32 (codevectors) x
//     32 (vectors) tile, the norms entering through one K-step.  Codevectors
//     are the A operand, so each lane holds 16 distances of ONE vector; the
//     two lanes (j, 0) and (j, 1) hold the 32 codevectors of a tile for
//     vector j between them.
//   * Each lane keeps the two smallest keys of every accumulator slot; a key
//     is the screened distance with its low mantissa bits replaced by the tile
//     number (3 VALU ops per distance: and-or, med3 as min, med3).  The tile
//     loop is software-pipelined: the products of tile t+1 are issued before
//     the key updates of tile t.
//   * Exact screens: the best candidate is rescored in FP64, direct form,
//     dimension order (lane (j, 0) sums the first half of the dimensions,
//     lane (j, 1) continues); a rigorous bound on the screen's rounding
//     decides whether it is provably the unique nearest codevector; failing
//     that, the two best are rescored and the closer one is tested the same
//     way against a bound on all others; otherwise the wave searches the row
//     again exhaustively in FP64.  Codebooks of at most kDirectN codevectors
//     are searched directly in FP64 instead.  BF16: the two best candidates
//     are rescored in FP64 and the closer taken (lowest index on ties).
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
constexpr int kRowsPerTile = 128;  // training vectors per four-wave row tile
constexpr int kWideLds = 163840;   // LDS of a CU: one eight-wave workgroup

// ---------------------------------------------------------------- policy --
// OCC: waves per SIMD the kernel is built for (2 .. 4, by register use); the
// persistent grid holds 256 * OCC workgroups and each may stage up to
// LDS bytes of codebook.
template <int LP_>
struct Fp32Screen {
  static constexpr int LP = LP_;
  static constexpr int S = LP + 4;   // row stride, elements
  static constexpr int PAD = LP;     // first element of the norm padding
  static constexpr int ESZ = 4;      // bytes per element
  static constexpr int NS = LP / 2;  // data K-steps per tile (half per lane half)
  static constexpr int OCC = LP <= 16 ? 3 : 2;
  static constexpr bool EXACT = true;
  static constexpr bool SPLIT = false;
  static constexpr bool PF = LP <= 32;  // registers for the next tile's vectors
  typedef float elem;
};

// FP32-accurate screen from BF16 parts (exact result): -2c and x are each
// split exactly into hi + mid + lo (BF16, eight significant bits each, RNE),
// and v_mfma_f32_32x32x16_bf16 sums the six products hi.hi, hi.mid, mid.hi,
// hi.lo, lo.hi, mid.mid (the three dropped ones are below 2^-24 |x||c|)
// with the norm parts in FP32.  Row layout: hi, mid, lo (LP each), then the
// norm padding [hi, mid, lo, 1, 1, 1, 0, 0] of |c|^2.
template <int LP_>
struct Bf16x3Screen {
  static constexpr int LP = LP_;
  static constexpr int S = 3 * LP + 8;
  static constexpr int PAD = 3 * LP;
  static constexpr int ESZ = 2;
  static constexpr int NS = LP / 16;  // K-blocks of 16 dimensions per part
  static constexpr int OCC = LP <= 16 ? 3 : 2;
  static constexpr bool EXACT = true;
  static constexpr bool SPLIT = true;
  static constexpr bool PF = LP <= 32;
  typedef __bf16 elem;
};

template <int LP_>
struct Bf16Screen {
  static constexpr int LP = LP_;
  static constexpr int S = LP + 8;
  static constexpr int PAD = LP;
  static constexpr int ESZ = 2;
  static constexpr int NS = LP / 16;
  static constexpr int OCC = LP <= 16 ? 4 : (LP <= 32 ? 3 : 2);
  static constexpr bool EXACT = false;
  static constexpr bool SPLIT = false;
  static constexpr bool PF = LP <= 64;
  typedef __bf16 elem;
};

template <class SC>
constexpr int persist_blocks() { return 256 * SC::OCC; }

template <class SC>
constexpr int lds_budget() { return SC::OCC >= 4 ? 40960 : (SC::OCC == 3 ? 53248 : 81920); }

// Rows of codevectors staged per chunk (multiple of 32) for a codebook of
// n_pad rows: all of it when it fits the LDS budget.
template <class SC>
inline int chunk_rows(int n_pad) {
  const int row_bytes = SC::S * SC::ESZ;
  const int cap = (lds_budget<SC>() / row_bytes) & ~31;
  return n_pad <= cap ? n_pad : cap;
}

// v = hi + mid + lo exactly (for v within the normal BF16 range): each
// residual is exact in FP32 and the last has at most eight significant bits.
__device__ __forceinline__ void split3(float v, __bf16& hi, __bf16& mid, __bf16& lo) {
  hi = (__bf16)v;
  const float r = v - (float)hi;
  mid = (__bf16)r;
  lo = (__bf16)(r - (float)mid);
}

// The FP32 value of three parts (exact: (hi + mid) + lo needs no rounding).
__device__ __forceinline__ float join3(__bf16 hi, __bf16 mid, __bf16 lo) {
  return ((float)hi + (float)mid) + (float)lo;
}

// Norm padding of a screen row (|c|^2 already clamped to kBig).
template <class SC>
__device__ __forceinline__ void write_pad(typename SC::elem* pad, float nrm) {
  if constexpr (SC::ESZ == 4) {
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

// Element d of a screen row: -2c stored (exact), split into parts when SPLIT.
template <class SC>
__device__ __forceinline__ void put_elem(typename SC::elem* row, int d, float c) {
  const float v = -2.0f * c;
  if constexpr (SC::SPLIT) {
    __bf16 hi, mid, lo;
    split3(v, hi, mid, lo);
    row[d] = hi;
    row[SC::LP + d] = mid;
    row[2 * SC::LP + d] = lo;
  } else {
    row[d] = (typename SC::elem)v;
  }
}

// The value the screen uses for element d (-2c, or its BF16 rounding).
template <class SC>
__device__ __forceinline__ float get_elem(const typename SC::elem* row, int d) {
  if constexpr (SC::SPLIT)
    return join3(row[d], row[SC::LP + d], row[2 * SC::LP + d]);
  else
    return (float)row[d];
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
  __shared__ double part[256];
  double q = 0.0;
  typename SC::elem* out = Cp + (int64_t)row * SC::S;
  for (int d = t; d < SC::LP; d += 256) {
    const float v = (row < n && d < L) ? C[(int64_t)row * L + d] : 0.0f;
    put_elem<SC>(out, d, v);
    const double r = (double)get_elem<SC>(out, d);  // -2 * (value the screen uses)
    q += r * r;
  }
  part[t] = q;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) part[t] += part[t + off];
    __syncthreads();
  }
  if (t == 0) {
    // at most kBig, so that the BF16 padding stays finite
    const float nrm = (row < n) ? fminf((float)(0.25 * part[0]), kBig) : kBig;
    write_pad<SC>(out + SC::PAD, nrm);
  }
}

// ----------------------------------------------------------- candidates --
struct Slots {
  float mn[16];
  float mn2[16];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      mn[r] = FLT_MAX;
      mn2[r] = FLT_MAX;
    }
  }
  // key = distance with its low mantissa bits replaced by the tile number;
  // min as med3(a, b, -inf) (ninf must be opaque to the compiler, or the
  // med3 becomes a canonicalising min), second via med3.
  __device__ __forceinline__ void push(const f16v& acc, uint32_t vmask, uint32_t tb,
                                       float ninf) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float k = __uint_as_float((__float_as_uint(acc[r]) & vmask) | tb);
      const float a = mn[r];
      mn2[r] = __builtin_amdgcn_fmed3f(a, mn2[r], k);
      mn[r] = __builtin_amdgcn_fmed3f(a, k, ninf);
    }
  }
};

// Every lane receives the value of lane (j, 0) in lo and of lane (j, 1) in
// hi (one v_permlane32_swap of v with itself).
__device__ __forceinline__ void pair_values(float v, float& lo, float& hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v),
                                                  false, false);
  lo = __uint_as_float(r[0]);
  hi = __uint_as_float(r[1]);
}

__device__ __forceinline__ void pair_values(int v, int& lo, int& hi) {
  float a, b;
  pair_values(__int_as_float(v), a, b);
  lo = __float_as_int(a);
  hi = __float_as_int(b);
}

// Partner of lane l at distance OFF (a power of two below 64) in a pairwise
// reduction over the wave, by VALU instructions only (no LDS round trip):
//   OFF 1, 2:   DPP quad permutation, exactly lane l ^ OFF;
//   OFF 4:      DPP row_half_mirror, lane l ^ 7 within eight lanes; this is
//               the value of lane l ^ 4 when every aligned group of four
//               lanes holds one value (as after the steps 1 and 2 of a
//               reduction);
//   OFF 8:      DPP row_ror:8, exactly lane l ^ 8 within a row of 16;
//   OFF 16, 32: v_permlane16_swap / v_permlane32_swap, exactly lane l ^ OFF.
template <int OFF>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
  if constexpr (OFF == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (threadIdx.x & 32) ? r[0] : r[1];
  } else if constexpr (OFF == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (threadIdx.x & 16) ? r[0] : r[1];
  } else {
    constexpr int ctrl = OFF == 1 ? 0xb1 : OFF == 2 ? 0x4e : OFF == 4 ? 0x141 : 0x128;
    static_assert(OFF == 1 || OFF == 2 || OFF == 4 || OFF == 8, "lane distance");
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, ctrl, 0xf, 0xf, false);
  }
}

template <int OFF>
__device__ __forceinline__ double xor_lane(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint64_t lo = xor_lane<OFF>((uint32_t)b), hi = xor_lane<OFF>((uint32_t)(b >> 32));
  return __longlong_as_double((long long)((hi << 32) | lo));
}

template <int OFF>
__device__ __forceinline__ int xor_lane(int v) {
  return (int)xor_lane<OFF>((uint32_t)v);
}

// Smallest distance over the wave, lowest index on equal distances (a total
// order, so the order of the steps does not matter); steps of increasing
// distance, as xor_lane<4> requires.
template <int OFF>
__device__ __forceinline__ void argmin_step(double& best, int& bi) {
  const double ob = xor_lane<OFF>(best);
  const int oi = xor_lane<OFF>(bi);
  if (ob < best || (ob == best && oi < bi)) {
    best = ob;
    bi = oi;
  }
}

// Sum over the wave by a fixed pairwise tree, partners at distances 1, 2,
// 4, ..., 32 (the same result in every lane).
__device__ __forceinline__ double wave_sum(double v) {
  v += xor_lane<1>(v);
  v += xor_lane<2>(v);
  v += xor_lane<4>(v);
  v += xor_lane<8>(v);
  v += xor_lane<16>(v);
  v += xor_lane<32>(v);
  return v;
}

// Smallest key k1 of the vector (codevector i1, lowest index among equal
// keys), the smallest key k2 of all other codevectors, and for the BF16
// screen a codevector i2 with key k2.  Keys of one tile differ in their rows
// only; equal keys of two tiles cannot occur (the tile number is part of the
// key).  Each lane reduces its 16 slots (slot r holds row 8 (r >> 2) + 4 h +
// (r & 3) of every tile), then the pair (j, 0), (j, 1) merges; both lanes of
// the pair obtain the same result.
struct Cand {
  float k1, k2;
  int i1, i2;
};

// The lane's own reduction, kept for the second acceptance test: its two
// smallest first keys m1 <= m2, the slot r1 of m1 and that slot's second s2.
struct LaneBest {
  float m1, m2, s2;
  int r1;
};

template <bool SECOND>
__device__ __forceinline__ Cand best_of(const Slots& sl, uint32_t lowmask, float ninf, int h,
                                        LaneBest* lb = nullptr) {
  float m1 = INFINITY, m2 = INFINITY;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    m2 = __builtin_amdgcn_fmed3f(m1, m2, sl.mn[r]);
    m1 = __builtin_amdgcn_fmed3f(m1, sl.mn[r], ninf);
  }
  float s2 = INFINITY;
  int r1 = 0;
#pragma unroll
  for (int r = 15; r >= 0; --r) {
    const bool e = sl.mn[r] == m1;
    s2 = e ? sl.mn2[r] : s2;
    r1 = e ? r : r1;
  }
  if (lb) *lb = LaneBest{m1, m2, s2, r1};
  const int row1 = 8 * (r1 >> 2) + 4 * h + (r1 & 3);
  const float k2l = __builtin_amdgcn_fmed3f(m2, s2, ninf);
  const int i1l = (int)((__float_as_uint(m1) & lowmask) << 5) + row1;
  int i2l = -1;
  if constexpr (SECOND) {
    int r2 = 0;
#pragma unroll
    for (int r = 15; r >= 0; --r) {
      const bool e = sl.mn[r] == m2 && r != r1;
      r2 = e ? r : r2;
    }
    const int row2 = 8 * (r2 >> 2) + 4 * h + (r2 & 3);
    i2l = s2 <= m2 ? (int)((__float_as_uint(s2) & lowmask) << 5) + row1
                   : (int)((__float_as_uint(m2) & lowmask) << 5) + row2;
  }
  float a1, b1, a2, b2;
  int ai, bi;
  pair_values(m1, a1, b1);
  pair_values(k2l, a2, b2);
  pair_values(i1l, ai, bi);
  const bool aw = a1 < b1 || (a1 == b1 && ai < bi);
  Cand c;
  c.k1 = aw ? a1 : b1;
  c.i1 = aw ? ai : bi;
  c.k2 = aw ? __builtin_amdgcn_fmed3f(a2, b1, ninf) : __builtin_amdgcn_fmed3f(b2, a1, ninf);
  c.i2 = -1;
  if constexpr (SECOND) {
    int ai2, bi2;
    pair_values(i2l, ai2, bi2);
    c.i2 = aw ? (a2 < b1 ? ai2 : bi) : (b2 < a1 ? bi2 : ai);
  }
  return c;
}

// The two smallest keys of the vector (codevectors i1, i2) and a lower bound
// k3 on the key of every other codevector, for the second acceptance test
// of the FP32 screen.  A lane tracks the two smallest keys of each of its
// slots, and a key it does not track is at least its slot's second; so
// when the lane's two best lie in different slots r1, r2, every other key
// of the lane is at least min(second of r1, second of r2, third smallest
// first), and when both lie in slot r1, at least min(second smallest first,
// second of r1).  The pair (j, 0), (j, 1) then merges its two sorted
// triples.  Both lanes of the pair obtain the same result.
struct Cand3 {
  float k3;
  int i1, i2;
};

__device__ __forceinline__ Cand3 best3_of(const Slots& sl, uint32_t lowmask, int h,
                                          const LaneBest& lb) {
  // m1, m2, r1 and s2 come from the first test's reduction; r2 is the lowest
  // other slot whose first key is m2, t2 its second, m3 the smallest first
  // key of the other slots (the third smallest of the lane)
  const float m1 = lb.m1, m2 = lb.m2, s2 = lb.s2;
  const int r1 = lb.r1;
  int r2 = r1 == 0 ? 1 : 0;
#pragma unroll
  for (int r = 15; r >= 0; --r) r2 = (sl.mn[r] == m2 && r != r1) ? r : r2;
  float t2 = INFINITY, m3 = INFINITY;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    t2 = r == r2 ? sl.mn2[r] : t2;
    m3 = (r != r1 && r != r2) ? fminf(m3, sl.mn[r]) : m3;
  }
  const int row1 = 8 * (r1 >> 2) + 4 * h + (r1 & 3);
  const int row2 = 8 * (r2 >> 2) + 4 * h + (r2 & 3);
  const bool same = s2 <= m2;  // the lane's second best is slot r1's second
  const float a1 = m1, a2 = same ? s2 : m2;
  const float a3 = same ? s2 : fminf(fminf(s2, t2), m3);
  const int ai1 = (int)((__float_as_uint(m1) & lowmask) << 5) + row1;
  const int ai2 = same ? (int)((__float_as_uint(s2) & lowmask) << 5) + row1
                       : (int)((__float_as_uint(m2) & lowmask) << 5) + row2;
  float x1, y1, x2, y2, x3, y3;
  int xi1, yi1, xi2, yi2;
  pair_values(a1, x1, y1);
  pair_values(a2, x2, y2);
  pair_values(a3, x3, y3);
  pair_values(ai1, xi1, yi1);
  pair_values(ai2, xi2, yi2);
  // merge (x1 <= x2 <= x3...) and (y1 <= y2 <= y3...)
  const bool xw = x1 < y1 || (x1 == y1 && xi1 < yi1);
  Cand3 c;
  if (xw) {
    c.i1 = xi1;
    const bool x2w = x2 < y1 || (x2 == y1 && xi2 < yi1);
    c.i2 = x2w ? xi2 : yi1;
    c.k3 = x2w ? fminf(x3, y1) : fminf(x2, y2);
  } else {
    c.i1 = yi1;
    const bool y2w = y2 < x1 || (y2 == x1 && yi2 < xi1);
    c.i2 = y2w ? yi2 : xi1;
    c.k3 = y2w ? fminf(y3, x1) : fminf(y2, x2);
  }
  return c;
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
__device__ __forceinline__ double d64(const float* x, const float* c, int L) {
  double s = 0.0;
  for (int l = 0; l < L; ++l) {
    const double t = (double)x[l] - (double)c[l];
    s = s + t * t;
  }
  return s;
}

// Rescore, decide, fall back and store for the vectors of this wave; lane
// (j, 1) finishes vector j.
//   EXACT (FP32 screen): accept the best candidate w only if
//     d(w) * (1 + 4 (L+2) 2^-53) < K2 / (1 + 2^(tile_bits-23)) - E,
//     E = 2 * gamma_{L+4} * (1 + 2^-24) * (2 |x| + sqrt(d(w)))^2 + 1e-30,
//   gamma_k = k u / (1 - k u), u = 2^-24.  E bounds the FP32 screen's
//   rounding error for every codevector c with d(c) <= d(w) (such a c has
//   |c| <= |x| + sqrt(d(w))); the division undoes the key's replaced mantissa
//   bits; K2 is the second-smallest key.  So every other codevector is
//   strictly farther, in exact arithmetic and in FP64.  E is evaluated in
//   FP32 with its factor raised by 2^-12, which covers the rounding of that
//   evaluation; the right-hand side is lowered by 2^-48 of itself for the
//   FP64 rounding of K2 / (1 + ...) - E.  Rows that fail are searched
//   exhaustively in FP64 by the whole wave (lowest index on ties).
//   Otherwise (BF16 screen): both candidates are rescored in FP64 and the
//   closer one is taken, the lower index on equal distances.
// Exhaustive FP64 search of one row by the whole wave (FP32 screen only):
// lane l scores codevectors l, l+64, ... in increasing order (strict <), then
// the wave takes the smallest distance, lowest index on equal distances.
// Codevectors come from the LDS-resident screen copy (-2c, exact) when the
// whole codebook is staged, otherwise from C with vector loads.  With LP <=
// 32 the row is taken from the registers of the pair that holds it (xv of
// lanes jr and jr + 32, read into every lane) rather than from memory;
// beyond that it is streamed from xrow with the codevectors.
template <class SC, bool VEC>
__device__ __forceinline__ void search_row(const float* __restrict__ xrow, int L,
                                           const float* __restrict__ C, int n,
                                           const float* resident, int lane,
                                           const float (&xv)[SC::LP / 2], int jr,
                                           double* best_d, int* best_i) {
  constexpr int LP = SC::LP;
  constexpr int W = LP < 16 ? LP : 16;
  constexpr bool XREG = LP <= 32;  // the row in registers; else streamed with c
  float xr[XREG ? LP : 1];
  if constexpr (XREG) {
#pragma unroll
    for (int s = 0; s < LP / 2; ++s) {
      xr[s] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xv[s]), jr));
      xr[LP / 2 + s] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xv[s]), jr + 32));
    }
  }
  double best = INFINITY;
  int bi = 0x7fffffff;
  for (int k = lane; k < n; k += 64) {
    double dk = 0.0;
#pragma unroll
    for (int l0 = 0; l0 < LP; l0 += W) {
      float cr[W], xc[W];
      if (resident) {
        const float* r = resident + (int64_t)k * SC::S + l0;
#pragma unroll
        for (int q = 0; q < W; q += 4) {
          const float4 v = *reinterpret_cast<const float4*>(r + q);
          cr[q] = -0.5f * v.x;
          cr[q + 1] = -0.5f * v.y;
          cr[q + 2] = -0.5f * v.z;
          cr[q + 3] = -0.5f * v.w;
        }
      } else {
        const float* r = C + (int64_t)k * L;
        if (VEC) {
#pragma unroll
          for (int q = 0; q < W; q += 4) {
            const float4 v = *reinterpret_cast<const float4*>(r + l0 + q);
            cr[q] = v.x;
            cr[q + 1] = v.y;
            cr[q + 2] = v.z;
            cr[q + 3] = v.w;
          }
        } else {
#pragma unroll
          for (int q = 0; q < W; ++q) cr[q] = (l0 + q < L) ? r[l0 + q] : 0.0f;
        }
      }
      if constexpr (XREG) {
#pragma unroll
        for (int q = 0; q < W; ++q) xc[q] = xr[l0 + q];
      } else if (VEC) {
#pragma unroll
        for (int q = 0; q < W; q += 4) {
          const float4 v = *reinterpret_cast<const float4*>(xrow + l0 + q);
          xc[q] = v.x;
          xc[q + 1] = v.y;
          xc[q + 2] = v.z;
          xc[q + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < W; ++q) xc[q] = (l0 + q < L) ? xrow[l0 + q] : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < W; ++q) {
        if (l0 + q < L) {
          const double t = (double)xc[q] - (double)cr[q];
          dk = dk + t * t;
        }
      }
    }
    if (dk < best) {
      best = dk;
      bi = k;
    }
  }
  argmin_step<1>(best, bi);
  argmin_step<2>(best, bi);
  argmin_step<4>(best, bi);
  argmin_step<8>(best, bi);
  argmin_step<16>(best, bi);
  argmin_step<32>(best, bi);
  *best_d = best;
  *best_i = bi;
}

// Constants of the acceptance test of the exact screens.  E bounds the
// screen's error for a codevector c with |c| <= |x| + sqrt(d(w)) as
// cE rf^2 + eabs (1 + rf) + 1e-30, rf = 2 |x| + sqrt(d(w)) >= |x| + |c|:
//   FP32 screen: cE = 2 gamma_{L+4} (1 + 2^-24);
//   split screen: an FP32 sum of exact products and norm parts (absolute
//     sum at most (1 + 2^-5) (|x| + |c|)^2), each addition taken with a
//     relative error of 2u whatever the order and rounding inside the matrix
//     core, gamma'_k = 2 k u / (1 - 2 k u).  The chain adds the five small
//     products per dimension first, from zero: its n1 = 80 NS additions
//     act on sums of at most 2^-7.9 (|x| + |c|)^2 of them; then the L
//     products hi.hi and the six norm parts, n2 = L + 6 additions, act on
//     the whole (|error| <= gamma'_n2 (1 + gamma'_n1) sum|terms| +
//     gamma'_n1 sum|small terms|).  The dropped products and the norms'
//     rounding to FP32 add below 2^-22 (|x| + |c|)^2; parts, products or
//     sums below the normal range add at most T 2^-124 (1 + |x| + |c|),
//     T = 6 (L + 1).
// cE is raised by 2^-12 for its own FP32 evaluation.
struct Bound {
  float cE;
  double eabs;
  double invks;  // (1 - 2^-48) / (1 + 2^(tile_bits - 23))
  double dslack; // 1 + 4 (L + 2) 2^-53
};

template <class SC>
__device__ __forceinline__ Bound bound_of(int L, int tile_bits) {
  Bound b;
  if constexpr (SC::SPLIT) {
    const double u2 = 0x1p-23;  // 2u
    const double n1 = 80.0 * SC::NS, n2 = (double)L + 6.0;
    const double g1 = n1 * u2 / (1.0 - n1 * u2), g2 = n2 * u2 / (1.0 - n2 * u2);
    b.cE = (float)((g2 * (1.0 + g1) * (1.0 + 0x1p-5) + g1 * 0x1.2p-8 + 0x1p-22) *
                   (1.0 + 0x1p-12));
    b.eabs = 6.0 * (double)(L + 1) * 0x1p-124;
  } else {
    const double k = (double)(L + 4) * 0x1p-24;
    b.cE = (float)(2.0 * (k / (1.0 - k)) * (1.0 + 0x1p-24) * (1.0 + 0x1p-12));
    b.eabs = 0.0;
  }
  b.invks = (1.0 - 0x1p-48) / (1.0 + ldexp(1.0, tile_bits - 23));
  b.dslack = 1.0 + 4.0 * (double)(L + 2) * 0x1p-53;
  return b;
}

// Half of the codevector row that lane half h scores in the chained FP64
// distance: dimensions [h LP/2, (h+1) LP/2), from the resident FP32 screen
// copy (-2c, exact: times -1/2) or from C.  The split screen's resident rows
// hold BF16 parts; its candidates are read from C (a cache hit), which
// measured faster than rebuilding the FP32 values from the parts.
template <class SC, bool VEC>
__device__ __forceinline__ void c_half(const float* __restrict__ C, int L,
                                       const typename SC::elem* resident, int w, int h,
                                       float (&cr)[SC::LP / 2]) {
  constexpr int H = SC::LP / 2;
  if (resident && !SC::SPLIT) {
    const float* r = reinterpret_cast<const float*>(resident) + (int64_t)w * SC::S + h * H;
#pragma unroll
    for (int q = 0; q < H; q += 4) {
      const float4 v = *reinterpret_cast<const float4*>(r + q);
      cr[q] = -0.5f * v.x;
      cr[q + 1] = -0.5f * v.y;
      cr[q + 2] = -0.5f * v.z;
      cr[q + 3] = -0.5f * v.w;
    }
  } else {
    const float* r = C + (int64_t)w * L + h * H;
    if (VEC) {
#pragma unroll
      for (int q = 0; q < H; q += 4) {
        const float4 v = *reinterpret_cast<const float4*>(r + q);
        cr[q] = v.x;
        cr[q + 1] = v.y;
        cr[q + 2] = v.z;
        cr[q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < H; ++q) cr[q] = (h * H + q < L) ? r[q] : 0.0f;
    }
  }
}

// FP64 squared distance of vector j to the codevector whose half-rows the
// pair (j, 0), (j, 1) holds in cr, summed over the dimensions in order: lane
// (j, 0) sums the first half, lane (j, 1) continues from that partial sum
// (the result is valid in lane (j, 1)).
template <int LP>
__device__ __forceinline__ double pair_dist(const float (&xv)[LP / 2], const float (&cr)[LP / 2],
                                            int L) {
  if constexpr (LP <= 32) {
    // the lane's squared differences once; lane (j, 0) adds them as the
    // first half, lane (j, 1) as the second (same operations, same order)
    double t[LP / 2];
#pragma unroll
    for (int q = 0; q < LP / 2; ++q) {
      const double u = (double)xv[q] - (double)cr[q];
      t[q] = u * u;
    }
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < LP / 2; ++q)
      if (q < L) a = a + t[q];
    const uint64_t ab = (uint64_t)__double_as_longlong(a);
    float la, ha, lb, hb;
    pair_values(__uint_as_float((uint32_t)ab), la, ha);
    pair_values(__uint_as_float((uint32_t)(ab >> 32)), lb, hb);
    double c = __longlong_as_double(
        (long long)(((uint64_t)__float_as_uint(lb) << 32) | __float_as_uint(la)));
#pragma unroll
    for (int q = 0; q < LP / 2; ++q)
      if (LP / 2 + q < L) c = c + t[q];
    return c;
  }
  double s0 = 0.0;
#pragma unroll
  for (int q = 0; q < LP / 2; ++q) {
    if (q < L) {
      const double u = (double)xv[q] - (double)cr[q];
      s0 = s0 + u * u;
    }
  }
  const uint64_t b0 = (uint64_t)__double_as_longlong(s0);
  float lo_a, hi_a, lo_b, hi_b;
  pair_values(__uint_as_float((uint32_t)b0), lo_a, hi_a);
  pair_values(__uint_as_float((uint32_t)(b0 >> 32)), lo_b, hi_b);
  double s1 = __longlong_as_double(
      (long long)(((uint64_t)__float_as_uint(lo_b) << 32) | __float_as_uint(lo_a)));
#pragma unroll
  for (int q = 0; q < LP / 2; ++q) {
    if (LP / 2 + q < L) {
      const double u = (double)xv[q] - (double)cr[q];
      s1 = s1 + u * u;
    }
  }
  return s1;
}

// The same for two codevectors at once (half-rows ca, cb).
template <int LP>
__device__ __forceinline__ void pair_dist2(const float (&xv)[LP / 2], const float (&ca)[LP / 2],
                                           const float (&cb)[LP / 2], int L, double& da,
                                           double& db) {
  double s0 = 0.0, t0 = 0.0;
#pragma unroll
  for (int q = 0; q < LP / 2; ++q) {
    if (q < L) {
      const double x = (double)xv[q];
      const double u = x - (double)ca[q], v = x - (double)cb[q];
      s0 = s0 + u * u;
      t0 = t0 + v * v;
    }
  }
  const uint64_t b0 = (uint64_t)__double_as_longlong(s0), c0 = (uint64_t)__double_as_longlong(t0);
  float a_lo, a_hi, b_lo, b_hi, c_lo, c_hi, d_lo, d_hi;
  pair_values(__uint_as_float((uint32_t)b0), a_lo, a_hi);
  pair_values(__uint_as_float((uint32_t)(b0 >> 32)), b_lo, b_hi);
  pair_values(__uint_as_float((uint32_t)c0), c_lo, c_hi);
  pair_values(__uint_as_float((uint32_t)(c0 >> 32)), d_lo, d_hi);
  double s1 = __longlong_as_double(
      (long long)(((uint64_t)__float_as_uint(b_lo) << 32) | __float_as_uint(a_lo)));
  double t1 = __longlong_as_double(
      (long long)(((uint64_t)__float_as_uint(d_lo) << 32) | __float_as_uint(c_lo)));
#pragma unroll
  for (int q = 0; q < LP / 2; ++q) {
    if (LP / 2 + q < L) {
      const double x = (double)xv[q];
      const double u = x - (double)ca[q], v = x - (double)cb[q];
      s1 = s1 + u * u;
      t1 = t1 + v * v;
    }
  }
  da = s1;
  db = t1;
}

// Returns the winning distance of the vector this lane finished (0 for the
// other lanes).  xv: lane (j, h) holds dimensions [h LP/2, (h+1) LP/2) of
// vector j (FP32); xsq: the vector's squared norm (FP32).  Lane (j, 0) sums
// the FP64 distance over the first half of the dimensions, lane (j, 1)
// continues it over the second half and finishes the vector.
template <class SC, bool VEC>
__device__ __forceinline__ double finish_rows(const Slots& sl, const float* __restrict__ X,
                                              int64_t M, int L, const float* __restrict__ C,
                                              int n, int32_t* __restrict__ idx,
                                              float* __restrict__ mind, int64_t row0,
                                              int tile_bits, unsigned long long* nfb,
                                              const typename SC::elem* resident,
                                              const float (&xv)[SC::LP / 2], float xsq,
                                              const Bound& bd, float ninf) {
  constexpr int LP = SC::LP;
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int j = lane & 31;
  const uint32_t lowmask = (1u << tile_bits) - 1u;

  LaneBest lb;
  const Cand t = best_of<!SC::EXACT>(sl, lowmask, ninf, h, SC::EXACT ? &lb : nullptr);
  const int64_t m = row0 + j;
  const bool live = h == 1 && m < M;
  bool flag = false;
  double d = 0.0;
  int win = t.i1;
  const bool bad = (unsigned)win >= (unsigned)n;  // non-finite input
  if (bad) win = 0;
  if constexpr (SC::EXACT) {
    float cr[LP / 2];
    c_half<SC, VEC>(C, L, resident, win, h, cr);
    d = pair_dist<LP>(xv, cr, L);
    if (live) {
      const float rf = 2.0f * __builtin_sqrtf(xsq) + __builtin_sqrtf((float)d);
      const double E = (double)(bd.cE * rf * rf) + bd.eabs * (1.0 + (double)rf) + 1e-30;
      const double lim = (double)t.k2 * bd.invks - E;
      flag = bad || !(d * bd.dslack < lim);
    }
  } else {
    // both candidates' half-rows loaded together, then the two distances
    // (the pair holds the same candidates)
    int i2 = t.i2;
    const bool two = i2 >= 0 && i2 < n && i2 != win;
    if (!two) i2 = win;
    float ca[LP / 2], cb[LP / 2];
    c_half<SC, VEC>(C, L, nullptr, win, h, ca);
    c_half<SC, VEC>(C, L, nullptr, i2, h, cb);
    double da, db;
    pair_dist2<LP>(xv, ca, cb, L, da, db);
    d = da;
    if (two && (db < da || (db == da && i2 < win))) {
      d = db;
      win = i2;
    }
  }
  if constexpr (SC::EXACT) {
    unsigned long long fl = __ballot(flag);
    if (fl) {
      // Second test for the rows that failed: the best two candidates
      // rescored in FP64 (the closer taken, the lower index on equal
      // distances), every other codevector bounded below by k3 through the
      // same inequality.  This settles a near tie of two codevectors, such
      // as the children of one split, without a search.  The best candidate
      // is the first test's (the same keys and rule), so its distance d is
      // reused.
      const Cand3 t3 = best3_of(sl, lowmask, h, lb);
      const bool ok = t3.i1 == win && !bad && (unsigned)t3.i2 < (unsigned)n && t3.i2 != win;
      float cb[LP / 2];
      c_half<SC, VEC>(C, L, resident, ok ? t3.i2 : 0, h, cb);
      const double db = pair_dist<LP>(xv, cb, L);
      if (flag && ok) {
        const double da = d;
        const bool second = db < da || (db == da && t3.i2 < t3.i1);
        const double dw = second ? db : da;
        const float rf = 2.0f * __builtin_sqrtf(xsq) + __builtin_sqrtf((float)dw);
        const double E = (double)(bd.cE * rf * rf) + bd.eabs * (1.0 + (double)rf) + 1e-30;
        const double lim = (double)t3.k3 * bd.invks - E;
        if (dw * bd.dslack < lim) {
          flag = false;
          d = dw;
          win = second ? t3.i2 : t3.i1;
        }
      }
      fl = __ballot(flag);
    }
    if (nfb && lane == 0 && fl) atomicAdd(nfb, (unsigned long long)__popcll(fl));
    while (fl) {
      const int src = __ffsll((long long)fl) - 1;
      fl &= fl - 1;
      const int64_t mf = row0 + (src & 31);
      double best;
      int bi;
      // (the split layout is not read back here: codevectors come from C)
      search_row<SC, VEC>(X + mf * (int64_t)L, L, C, n,
                          SC::SPLIT ? nullptr : reinterpret_cast<const float*>(resident), lane,
                          xv, src & 31, &best, &bi);
      if (lane == src) {
        d = best;
        win = bi;
      }
    }
  }
  // A row whose distances are all NaN or infinite (a non-finite coordinate)
  // has no nearest codevector: index 0 and distance +inf, which is what a
  // search keeping the first strictly smaller distance returns.
  if (!(d < INFINITY)) {
    win = 0;
    d = INFINITY;
  }
  if (live) {
    idx[m] = win;
    if (mind) mind[m] = (float)d;
  }
  return live ? d : 0.0;
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

// Copy ``bytes`` (multiple of 16) from global to LDS with the NT threads of
// the workgroup, eight 16-byte loads in flight per thread before their stores.
template <int NT = kAssignThreads>
__device__ __forceinline__ void stage(const void* __restrict__ src, void* dst, int bytes) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const u32x4* s = reinterpret_cast<const u32x4*>(src);
  u32x4* d = reinterpret_cast<u32x4*>(dst);
  const int nv = bytes >> 4;
  for (int base = 0; base < nv; base += 8 * NT) {
    u32x4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + u * NT + threadIdx.x;
      v[u] = s[e < nv ? e : 0];
    }
    // the loads are used here unconditionally, so the compiler cannot sink
    // them into the stores' branches (one wait for all eight, not eight)
    asm volatile("" ::"v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]),
                 "v"(v[6]), "v"(v[7]));
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + u * NT + threadIdx.x;
      if (e < nv) d[e] = v[u];
    }
  }
}

// Resident codebook staged straight from C: -2c (exact) zero-padded to LP
// dimensions and n_pad rows, then each row's squared norm (FP64, rounded to
// FP32) in its padding, as prep_kernel writes it.  Loads are issued four at a
// time per thread before their stores.
template <class SC, bool VEC, int NT = kAssignThreads>
__device__ __forceinline__ void stage_from_C(const float* __restrict__ C, int n, int L,
                                             int n_pad, typename SC::elem* sA) {
  constexpr int LP = SC::LP;
  constexpr int S = SC::S;
  typedef typename SC::elem E;
  if (VEC) {
    constexpr int Q = LP / 4;
    const int nv = n_pad * Q;
    for (int base = 0; base < nv; base += 4 * NT) {
      float4 v[4];
      bool on[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = base + u * NT + threadIdx.x;
        on[u] = e < nv && e / Q < n;
        v[u] = *reinterpret_cast<const float4*>(C + (int64_t)(on[u] ? e : 0) * 4);
      }
      // used unconditionally: the four loads stay in flight together instead
      // of being sunk into (and waited for in) the branches below
      asm volatile("" ::"v"(v[0].x), "v"(v[1].x), "v"(v[2].x), "v"(v[3].x));
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (!on[u]) v[u] = make_float4(0.f, 0.f, 0.f, 0.f);  // padding rows
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = base + u * NT + threadIdx.x;
        if (e < nv) {
          E* row = sA + (e / Q) * S;
          const int d = (e % Q) * 4;
          put_elem<SC>(row, d, v[u].x);
          put_elem<SC>(row, d + 1, v[u].y);
          put_elem<SC>(row, d + 2, v[u].z);
          put_elem<SC>(row, d + 3, v[u].w);
        }
      }
    }
  } else {
    for (int e = threadIdx.x; e < n_pad * LP; e += NT) {
      const int r = e / LP, d = e % LP;
      const float v = (r < n && d < L) ? C[(int64_t)r * L + d] : 0.0f;
      put_elem<SC>(sA + r * S, d, v);
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < n_pad; r += NT) {
    double q = 0.0;
#pragma unroll 8
    for (int d = 0; d < LP; ++d) {
      const double v = (double)get_elem<SC>(sA + r * S, d);
      q += v * v;
    }
    const float nrm = (r < n) ? fminf((float)(0.25 * q), kBig) : kBig;
    write_pad<SC>(sA + r * S + SC::PAD, nrm);
  }
  __syncthreads();
}

// -------------------------------------------------------------- kernel --
// A-operand fragments of one tile of 32 codevectors for lane (j, h): the
// K-step of the norms and the data K-steps.
template <class SC>
struct Frag;

template <int LP>
struct Frag<Fp32Screen<LP>> {
  float an;
  float a[LP / 2];
  // row layout [-2c (LP), |c|^2, 1, 0, 0]: half h supplies K index h of the
  // norm step ([|c|^2, 1] against [1, |x|^2]) and dimensions [h LP/2, ...)
  __device__ __forceinline__ void load(const float* ar, int h) {
    an = ar[LP + h];
    const float* p = ar + h * (LP / 2);
#pragma unroll
    for (int s = 0; s < LP / 2; s += 4) {
      const float4 q = *reinterpret_cast<const float4*>(p + s);
      a[s] = q.x;
      a[s + 1] = q.y;
      a[s + 2] = q.z;
      a[s + 3] = q.w;
    }
  }
  __device__ __forceinline__ void mma(const float (&xf)[LP / 2], float xn, f16v& acc) const {
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(an, xn, f16v{}, 0, 0, 0);
#pragma unroll
    for (int s = 0; s < LP / 2; ++s)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], xf[s], acc, 0, 0, 0);
  }
};

template <int LP>
struct Frag<Bf16Screen<LP>> {
  static constexpr int NS = LP / 16;
  bf16x8 an;
  bf16x8 a[NS];
  // row layout [bf16(-2c) (LP), hi, mid, lo, 1, 1, 1, 0, 0]: both halves
  // load the padding for the norm step (finite: the norm is clamped), which
  // half 1's zero B operand cancels; dimensions [h LP/2, ...) in steps of 8
  __device__ __forceinline__ void load(const __bf16* ar, int h) {
    an = *reinterpret_cast<const bf16x8*>(ar + LP);
    const __bf16* p = ar + h * (LP / 2);
#pragma unroll
    for (int s = 0; s < NS; ++s) a[s] = *reinterpret_cast<const bf16x8*>(p + 8 * s);
  }
  __device__ __forceinline__ void mma(const bf16x8 (&xf)[NS], const bf16x8& xn,
                                      f16v& acc) const {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(an, xn, f16v{}, 0, 0, 0);
#pragma unroll
    for (int s = 0; s < NS; ++s)
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[s], xf[s], acc, 0, 0, 0);
  }
};

// B operand of the split screen: lane (j, h) holds the parts of dimensions
// [h LP/2, (h+1) LP/2) of vector j, eight per K-block.
template <int NS>
struct XSplit {
  bf16x8 h[NS], m[NS], l[NS];
};

template <int LP>
struct Frag<Bf16x3Screen<LP>> {
  static constexpr int NS = LP / 16;
  bf16x8 an;
  bf16x8 hi[NS], mid[NS], lo[NS];
  // the same K mapping per part as the BF16 screen (dimensions [h LP/2, ...)
  // in steps of 8); both halves load the norm padding, which half 1's zero
  // B operand cancels
  __device__ __forceinline__ void load(const __bf16* ar, int h) {
    an = *reinterpret_cast<const bf16x8*>(ar + 3 * LP);
    const __bf16* p = ar + h * (LP / 2);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      hi[s] = *reinterpret_cast<const bf16x8*>(p + 8 * s);
      mid[s] = *reinterpret_cast<const bf16x8*>(p + LP + 8 * s);
      lo[s] = *reinterpret_cast<const bf16x8*>(p + 2 * LP + 8 * s);
    }
  }
  // small products first, then hi.hi, then the norms.  HIONLY: every
  // vector of the tile is exact in BF16 (its mid and lo parts are zero, as
  // for 8-bit pixels), so the products with them vanish and are skipped:
  // the same sum in the same order without its zero terms.
  template <bool HIONLY = false>
  __device__ __forceinline__ void mma(const XSplit<NS>& x, const bf16x8& xn, f16v& acc) const {
    if constexpr (HIONLY) {
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo[0], x.h[0], f16v{}, 0, 0, 0);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (s > 0) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo[s], x.h[s], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(mid[s], x.h[s], acc, 0, 0, 0);
      }
    } else {
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(mid[0], x.m[0], f16v{}, 0, 0, 0);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (s > 0) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(mid[s], x.m[s], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo[s], x.h[s], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi[s], x.l[s], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(mid[s], x.h[s], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi[s], x.m[s], acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi[s], x.h[s], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(an, xn, acc, 0, 0, 0);
  }
};

// The products of one tile (the vanishing-part chain only for the split
// screen).
template <bool HIONLY, class F, class XF, class XN>
__device__ __forceinline__ void frag_mma(const F& f, const XF& xf, const XN& xn, f16v& acc) {
  if constexpr (HIONLY)
    f.template mma<true>(xf, xn, acc);
  else
    f.mma(xf, xn, acc);
}

// Screens nt tiles of 32 codevectors (row j of tile 0 at ar) against the
// wave's vectors.  Software-pipelined: the matrix-core products of tile t+1
// are issued before the key updates of tile t, so that the two overlap;
// with small dimensions the A fragments are also loaded one tile ahead.
template <class SC, bool HIONLY = false, class XF, class XN>
__device__ __forceinline__ void screen_tiles(const typename SC::elem* ar, int nt, uint32_t tb0,
                                             int h, const XF& xf, const XN& xn, Slots& sl,
                                             uint32_t vmask, float ninf) {
  constexpr int TS = 32 * SC::S;  // elements per tile
  constexpr bool DB = SC::LP <= 32 && !SC::SPLIT;
  if constexpr (SC::LP >= 128) {  // long K: the products dominate, no pipelining
    for (int t = 0; t < nt; ++t) {
      Frag<SC> f;
      f.load(ar + t * TS, h);
      f16v c;
      frag_mma<HIONLY>(f, xf, xn, c);
      sl.push(c, vmask, tb0 + t, ninf);
    }
    return;
  }
  Frag<SC> fa, fb;
  f16v ca, cb;
  fa.load(ar, h);
  frag_mma<HIONLY>(fa, xf, xn, ca);
  if (DB && nt > 1) fb.load(ar + TS, h);
  int t = 0;
  for (; t + 2 < nt; t += 2) {
    // ca: products of tile t; fb: fragments of tile t+1 (DB).  The two
    // phases stay apart, so that each tile's key updates run beside the
    // other tile's products instead of after both.
    if (!DB) fb.load(ar + (t + 1) * TS, h);
    frag_mma<HIONLY>(fb, xf, xn, cb);
    fa.load(ar + (t + 2) * TS, h);
    sl.push(ca, vmask, tb0 + t, ninf);
    __builtin_amdgcn_sched_barrier(0);
    frag_mma<HIONLY>(fa, xf, xn, ca);
    if (DB) fb.load(ar + min(t + 3, nt - 1) * TS, h);
    sl.push(cb, vmask, tb0 + t + 1, ninf);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (t + 1 < nt) {
    if (!DB) fb.load(ar + (t + 1) * TS, h);
    frag_mma<HIONLY>(fb, xf, xn, cb);
    sl.push(ca, vmask, tb0 + t, ninf);
    sl.push(cb, vmask, tb0 + t + 1, ninf);
  } else {
    sl.push(ca, vmask, tb0 + t, ninf);
  }
}

// Half-row of the wave's training vector: lane (j, h) loads dimensions
// [h LP/2, (h+1) LP/2) of vector row0 + j (zero beyond L or M).
template <int LP, bool VEC>
__device__ __forceinline__ void load_x(const float* __restrict__ X, int64_t M, int L,
                                       int64_t row0, int h, int j, float (&v)[LP / 2]) {
  const int64_t m = row0 + j;
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
}

// Per-wave constants of the allocation.  The key mask and -inf live in VGPRs
// the compiler cannot see through (so that the and-or reads one SGPR and
// the med3 stays a med3).
struct WaveCtx {
  int h, j, tile_bits;
  uint32_t vmask;
  float ninf;
  Bound bd;
};

template <class SC>
__device__ __forceinline__ WaveCtx wave_ctx(int L, int tile_bits) {
  WaveCtx w;
  const int lane = threadIdx.x & 63;
  w.h = lane >> 5;
  w.j = lane & 31;
  w.tile_bits = tile_bits;
  uint32_t vmask = ~((1u << tile_bits) - 1u);
  asm volatile("v_mov_b32 %0, %1" : "=v"(vmask) : "v"(vmask));
  float ninf = -INFINITY;
  asm volatile("v_mov_b32 %0, %1" : "=v"(ninf) : "v"(ninf));
  w.vmask = vmask;
  w.ninf = ninf;
  w.bd = bound_of<SC>(L, tile_bits);
  return w;
}

// The calling wave's tile of 32 training vectors (rows row0 .. row0+31):
// screen against the codebook (resident in sA, or staged chunk by chunk from
// Cp by the whole workgroup), then rescore, decide, fall back and store.
// xv holds this lane's half-row on entry; with PF it receives the half-row
// of the tile at next_row0 (when >= 0), loaded while the screen runs.
// Returns this lane's winning distance (0 for lanes that finish no vector).
// HIONLY (split screen): every vector of the tile is exact in BF16, so the
// products with its vanishing mid and lo parts are skipped.
template <class SC, bool VEC, bool PF, int NT = kAssignThreads, bool HIONLY = false>
__device__ __forceinline__ double process_rows(
    float (&xv)[SC::LP / 2], const float* __restrict__ X, int64_t M, int L, int64_t row0,
    int64_t next_row0, const float* __restrict__ C, int n, int n_pad, int CR, bool resident,
    const typename SC::elem* __restrict__ Cp, typename SC::elem* sA, int32_t* __restrict__ idx,
    float* __restrict__ mind, unsigned long long* nfb, const WaveCtx& w) {
  constexpr int LP = SC::LP;
  constexpr int S = SC::S;
  constexpr int NS = SC::NS;
  typedef typename SC::elem E;
  const int h = w.h, j = w.j;

  // B operand: lane (j, h) keeps dims [h*LP/2, (h+1)*LP/2) of vector j and
  // the norm step's [1, |x|^2] (FP32) or [1, 1, 1, hi, mid, lo, 0, 0] /
  // zeros (BF16).
  typedef typename std::conditional<SC::ESZ == 4, float, bf16x8>::type BF;
  typedef typename std::conditional<SC::SPLIT, XSplit<NS>, BF[NS]>::type XF;
  XF xf;
  BF xn;
  double ss = 0.0;
  if constexpr (SC::SPLIT) {
    // |x|^2 in FP64 from the FP32 vector, rounded once, split like |c|^2
#pragma unroll
    for (int s = 0; s < LP / 2; ++s) {
      __bf16 a, b, c;
      split3(xv[s], a, b, c);
      xf.h[s >> 3][s & 7] = a;
      xf.m[s >> 3][s & 7] = b;
      xf.l[s >> 3][s & 7] = c;
      ss += (double)xv[s] * (double)xv[s];
    }
    ss += xor_lane<32>(ss);
    __bf16 hi, mid, lo;
    split3(fminf((float)ss, kBig), hi, mid, lo);
    const __bf16 one = (__bf16)1.0f, zero = (__bf16)0.0f;
    const bf16x8 nv = {one, one, one, hi, mid, lo, zero, zero};
    const bf16x8 zv = {zero, zero, zero, zero, zero, zero, zero, zero};
    xn = h ? zv : nv;
  } else if constexpr (SC::EXACT) {
#pragma unroll
    for (int s = 0; s < LP / 2; ++s) {
      xf[s] = xv[s];
      ss += (double)xv[s] * (double)xv[s];
    }
    ss += xor_lane<32>(ss);
    xn = h ? (float)ss : 1.0f;
  } else {
    // |x|^2 of the rounded vector, FP32 (it keeps the keys near the
    // distances, non-negative, so that equal keys resolve to the lower tile)
    float sf = 0.0f;
#pragma unroll
    for (int s = 0; s < LP / 2; ++s) {
      const __bf16 b = (__bf16)xv[s];
      xf[s >> 3][s & 7] = b;
      sf = __builtin_fmaf((float)b, (float)b, sf);
    }
    sf += __uint_as_float(xor_lane<32>(__float_as_uint(sf)));
    __bf16 hi, mid, lo;
    split3(sf, hi, mid, lo);
    const __bf16 one = (__bf16)1.0f, zero = (__bf16)0.0f;
    const bf16x8 nv = {one, one, one, hi, mid, lo, zero, zero};
    const bf16x8 zv = {zero, zero, zero, zero, zero, zero, zero, zero};
    xn = h ? zv : nv;
  }
  const float xsq = (float)ss;
  // the rescore needs this tile's vectors after the screen
  float xk[LP / 2];
#pragma unroll
  for (int s = 0; s < LP / 2; ++s) xk[s] = xv[s];
  if (PF && next_row0 >= 0) load_x<LP, VEC>(X, M, L, next_row0, h, j, xv);

  Slots sl;
  sl.init();
  for (int c0 = 0; c0 < n_pad; c0 += CR) {
    const int cr = min(CR, n_pad - c0);
    if (!resident) {
      __syncthreads();
      stage<NT>(Cp + (int64_t)c0 * S, sA, cr * S * SC::ESZ);
      __syncthreads();
    }
    const E* base = resident ? sA + (int64_t)c0 * S : sA;
    screen_tiles<SC, HIONLY>(base + j * S, cr >> 5, (uint32_t)(c0 >> 5), h, xf, xn, sl,
                             w.vmask, w.ninf);
  }
  return finish_rows<SC, VEC>(sl, X, M, L, C, n, idx, mind, row0, w.tile_bits, nfb,
                              resident ? sA : nullptr, xk, xsq, w.bd, w.ninf);
}

// Direct allocation for small codebooks (FP32 screen, n <= kDirectN, LP <=
// 32): one training vector per lane, FP64 distances to the n codevectors
// (staged in LDS as FP64), dimensions in order, the first smallest taken.
// That is what the exhaustive search computes and what the certified screen
// returns, so indices and distances are the same; the partial of each 32
// vectors is the butterfly of wave_sum over lanes that hold the distances
// (its last step adds zeros there), so the partials are the same too.  At
// such n this takes fewer instructions per vector than the screen and its
// finishing work.  Each wave takes 64 consecutive vectors at a time and
// loads the next 64 while it searches.
constexpr int kDirectN = 8;

template <class SC, bool VEC, int W>
__device__ __forceinline__ void direct_rows(const float* __restrict__ X, int64_t M, int L,
                                            const float* __restrict__ C, int n,
                                            int32_t* __restrict__ idx, float* __restrict__ mind,
                                            double* __restrict__ dpart, double* sC) {
  constexpr int LP = SC::LP;
  constexpr int NT = 64 * W;
  for (int e = threadIdx.x; e < n * LP; e += NT) {
    const int k = e / LP, l = e - k * LP;
    sC[e] = l < L ? (double)C[(int64_t)k * L + l] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ngroups = (M + 63) >> 6;
  const int64_t step = (int64_t)gridDim.x * W;
  float xr[LP];
  auto load = [&](int64_t gg) {
    const int64_t m = gg * 64 + lane;
    if (gg < ngroups && m < M) {
      load_row<LP, VEC>(X + m * (int64_t)L, L, xr);
    } else {
#pragma unroll
      for (int s = 0; s < LP; ++s) xr[s] = 0.0f;
    }
  };
  int64_t g = (int64_t)blockIdx.x * W + wave;
  load(g);
  for (; g < ngroups; g += step) {
    const int64_t m = g * 64 + lane;
    double xd[LP];
#pragma unroll
    for (int s = 0; s < LP; ++s) xd[s] = (double)xr[s];
    load(g + step);
    double best = INFINITY;
    int bi = 0x7fffffff;
#pragma unroll 2
    for (int k = 0; k < n; ++k) {
      const double* c = sC + k * LP;
      double dk = 0.0;
#pragma unroll
      for (int l = 0; l < LP; ++l) {
        if (l < L) {
          const double t = xd[l] - c[l];
          dk = dk + t * t;
        }
      }
      if (dk < best) {
        best = dk;
        bi = k;
      }
    }
    if (!(best < INFINITY)) bi = 0;  // no finite distance: index 0, as finish_rows
    const bool live = m < M;
    if (live) {
      idx[m] = bi;
      if (mind) mind[m] = (float)best;
    }
    double v = live ? best : 0.0;
    v += xor_lane<1>(v);
    v += xor_lane<2>(v);
    v += xor_lane<4>(v);
    v += xor_lane<8>(v);
    v += xor_lane<16>(v);
    if (dpart && (lane & 31) == 0 && live) dpart[m >> 5] = v;
  }
}

// The persistent row-tile loop of the allocation kernel (HIONLY: see
// process_rows).
template <class SC, bool VEC, int W, bool HIONLY>
__device__ __forceinline__ void assign_rows(const float* __restrict__ X, int64_t M, int L,
                                            const float* __restrict__ C, int n,
                                            const typename SC::elem* __restrict__ Cp, int n_pad,
                                            int CR, int32_t* __restrict__ idx,
                                            float* __restrict__ mind, double* __restrict__ dpart,
                                            unsigned long long* __restrict__ nfb, int tile_bits,
                                            typename SC::elem* sA) {
  constexpr int LP = SC::LP;
  constexpr bool PF = SC::PF;  // prefetch the next row tile's vectors
  constexpr int NT = 64 * W;
  constexpr int RT = 32 * W;  // training vectors per row tile
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform (SGPR)
  const int64_t ntiles_rows = (M + RT - 1) / RT;
  const bool resident = CR >= n_pad;
  const WaveCtx w = wave_ctx<SC>(L, tile_bits);

  float xv[LP / 2];
  int64_t rt = blockIdx.x;
  if (PF && rt < ntiles_rows)
    load_x<LP, VEC>(X, M, L, rt * RT + (int64_t)wave * 32, w.h, w.j, xv);
  if (resident) stage_from_C<SC, VEC, NT>(C, n, L, n_pad, sA);

  for (; rt < ntiles_rows; rt += gridDim.x) {
    const int64_t row0 = rt * RT + (int64_t)wave * 32;
    if (!PF) load_x<LP, VEC>(X, M, L, row0, w.h, w.j, xv);
    const int64_t next =
        (PF && rt + gridDim.x < ntiles_rows) ? row0 + (int64_t)gridDim.x * RT : -1;
    const double d = process_rows<SC, VEC, PF, NT, HIONLY>(
        xv, X, M, L, row0, next, C, n, n_pad, CR, resident, Cp, sA, idx, mind, nfb, w);
    // partial of the distortion per 32 vectors (lanes added by a fixed
    // butterfly), indexed by the vectors: the same for every launch shape
    const double ws = wave_sum(d);
    if (dpart && lane == 0 && row0 < M) dpart[row0 >> 5] = ws;
  }
}

// W waves per workgroup: 4 (OCC workgroups per CU), or 8 with one workgroup
// per CU holding a codebook of up to kWideLds bytes resident.
template <class SC, bool VEC, int W>
__global__ __launch_bounds__(64 * W, W == 4 ? SC::OCC : 1) void assign_kernel(
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
  constexpr int LP = SC::LP;
  constexpr bool PF = SC::PF;  // prefetch the next row tile's vectors
  if (VEC) L = LP;  // vector loads only for rows of exactly LP floats
  typedef typename SC::elem E;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  E* sA = reinterpret_cast<E*>(smem);
  if constexpr (SC::EXACT && LP <= 32) {
    // the LDS holds at least 32 screen rows, more than n <= kDirectN FP64 rows
    if (n <= kDirectN) {
      direct_rows<SC, VEC, W>(X, M, L, C, n, idx, mind, dpart, reinterpret_cast<double*>(smem));
      return;
    }
  }

  // training sets whose every coordinate is exact in BF16 (flag set by the
  // set-up pass of a training run) skip the products with the vanishing
  // parts; the two bodies are separate so that neither costs registers of
  // the other
  if (SC::SPLIT && ctl.xflags && ctl.xflags[2])
    assign_rows<SC, VEC, W, SC::SPLIT>(X, M, L, C, n, Cp, n_pad, CR, idx, mind, dpart, nfb,
                                       tile_bits, sA);
  else
    assign_rows<SC, VEC, W, false>(X, M, L, C, n, Cp, n_pad, CR, idx, mind, dpart, nfb,
                                   tile_bits, sA);
}

// Launch shape of the allocation for a codebook of n_pad rows: waves per
// workgroup, workgroups, codebook rows per LDS chunk and LDS bytes.  A
// codebook that does not fit the LDS of OCC workgroups per CU but fits one
// workgroup's kWideLds bytes runs resident in eight-wave workgroups.  A
// split-screen codebook larger still is staged in chunks of nearly all of a
// CU's LDS into eight-wave workgroups too: each staged chunk then serves 256
// vectors instead of 128 (at M = 4,194,304, L = 64, N = 1024: 2,096 ->
// 1,875 us per allocation).
struct Shape {
  int waves;
  int64_t grid;
  int cr;
  size_t lds;
};

template <class SC>
inline Shape shape_of(int64_t M, int n_pad) {
  Shape sh;
  const int CR = chunk_rows<SC>(n_pad);
  const size_t full = (size_t)n_pad * SC::S * SC::ESZ;
  if (CR < n_pad && full <= (size_t)kWideLds) {
    sh.waves = 8;
    sh.grid = std::min<int64_t>((M + 255) / 256, 256);
    sh.cr = n_pad;
    sh.lds = full;
  } else if (CR < n_pad && SC::SPLIT) {
    sh.waves = 8;
    sh.grid = std::min<int64_t>((M + 255) / 256, 256);
    sh.cr = (int)(((size_t)(kWideLds - 8192) / ((size_t)SC::S * SC::ESZ)) & ~(size_t)31);
    sh.lds = (size_t)sh.cr * SC::S * SC::ESZ;
  } else {
    sh.waves = 4;
    sh.grid = std::min<int64_t>((M + kRowsPerTile - 1) / kRowsPerTile, persist_blocks<SC>());
    sh.cr = CR;
    sh.lds = (size_t)CR * SC::S * SC::ESZ;
  }
  return sh;
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
  const Shape sh = shape_of<SC>(M, n_pad);
  const int CR = sh.cr;
  if (CR < n_pad) {  // chunked: stage from the prepared copy
    hipLaunchKernelGGL((prep_kernel<SC>), dim3((unsigned)n_pad), dim3(256), 0, s, C, n, L, Cp,
                       st, cbp);
    LBG_TRY_HIP(hipGetLastError());
  }
  // Persistent grid: a resident codebook is staged once per workgroup, a
  // chunked one per row tile.
  const int64_t grid = sh.grid;
  const size_t lds = sh.lds;
  const int tb = tile_bits_for(n);
  bool vec = (L == SC::LP) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  if (st)
    vec = vec && ((reinterpret_cast<uintptr_t>(cbp.c[0]) & 15) == 0) &&
          ((reinterpret_cast<uintptr_t>(cbp.c[1]) & 15) == 0);
  else
    vec = vec && ((reinterpret_cast<uintptr_t>(C) & 15) == 0);
  // workgroups may hold more than 64 KB of LDS on gfx950 only after opting
  // in, once per kernel
  static const hipError_t a1 = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&assign_kernel<SC, true, 4>),
      hipFuncAttributeMaxDynamicSharedMemorySize, lds_budget<SC>());
  static const hipError_t a2 = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&assign_kernel<SC, false, 4>),
      hipFuncAttributeMaxDynamicSharedMemorySize, lds_budget<SC>());
  static const hipError_t a3 = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&assign_kernel<SC, true, 8>),
      hipFuncAttributeMaxDynamicSharedMemorySize, kWideLds);
  static const hipError_t a4 = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&assign_kernel<SC, false, 8>),
      hipFuncAttributeMaxDynamicSharedMemorySize, kWideLds);
  const dim3 g((unsigned)grid);
  if (sh.waves == 8) {
    LBG_TRY_HIP(vec ? a3 : a4);
    if (vec)
      hipLaunchKernelGGL((assign_kernel<SC, true, 8>), g, dim3(512), lds, s, X, M, L, C, n, Cp,
                         n_pad, CR, idx, mind, dpart, nfb, tb, ctl, cbp);
    else
      hipLaunchKernelGGL((assign_kernel<SC, false, 8>), g, dim3(512), lds, s, X, M, L, C, n, Cp,
                         n_pad, CR, idx, mind, dpart, nfb, tb, ctl, cbp);
  } else {
    LBG_TRY_HIP(vec ? a1 : a2);
    if (vec)
      hipLaunchKernelGGL((assign_kernel<SC, true, 4>), g, dim3(kAssignThreads), lds, s, X, M, L,
                         C, n, Cp, n_pad, CR, idx, mind, dpart, nfb, tb, ctl, cbp);
    else
      hipLaunchKernelGGL((assign_kernel<SC, false, 4>), g, dim3(kAssignThreads), lds, s, X, M,
                         L, C, n, Cp, n_pad, CR, idx, mind, dpart, nfb, tb, ctl, cbp);
  }
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
