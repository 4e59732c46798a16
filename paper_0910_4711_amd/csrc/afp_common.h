// Device bodies of the fixed-point Codebook Updation, shared by the
// single-run kernels (update_afp.hip) and the batched kernels (batched.hip).
// See update_afp.hip for the method.
#pragma once

#include <algorithm>

#include "control.h"
#include "lbg_internal.h"
#include "misc_common.h"

namespace lbg {
namespace afp {

constexpr int kT = 256;
constexpr int kLdsBytes = 61440;
constexpr int kUnroll = 16;  // rows in flight per group

// Fine bits of one coordinate (FP32 bits b): -log2 of the spacing of its
// significand's lowest set bit, plus 256 (always positive), or 0 for zero,
// Inf and NaN; a coordinate is a multiple of 2^-s exactly when its fine bits
// are at most s + 256.
__device__ __forceinline__ uint32_t fine_bits(uint32_t b) {
  b &= 0x7fffffffu;
  if (b == 0u || b >= 0x7f800000u) return 0u;
  const uint32_t e = b >> 23;
  const uint32_t sig = e ? ((b & 0x7fffffu) | 0x800000u) : b;
  const int q = (int)(e ? e : 1u) - 150 + __builtin_ctz(sig);  // spacing 2^q
  return (uint32_t)(256 - q);
}

// The set-up pass of a training run, block blk of nblk (256 threads): the
// column sums of misc::colsum_body (the same blocks of rows_per_block rows,
// the same order) into part[blk L ...] and, from the same loads, the block's
// largest finite |x|, largest fine bits and the OR of the low 16 bits into
// amax[blk], amax[nblk + blk] and amax[2 nblk + blk] (as absmax_body forms
// them; none depends on the blocks); the blocks also clear lo (nlo words).
__device__ __forceinline__ void setup_pass_body(const float* __restrict__ X, int64_t M, int L,
                                                int64_t rows_per_block,
                                                double* __restrict__ part,
                                                uint32_t* __restrict__ amax, int64_t nblk,
                                                int64_t blk, unsigned long long* __restrict__ lo,
                                                int64_t nlo) {
  __shared__ double s[kT];
  __shared__ uint32_t sm[kT];
  __shared__ uint32_t sf[kT];
  __shared__ uint32_t sr[kT];
  const int R = kT / L;
  const int t = threadIdx.x;
  const int q = t / L, d = t % L;
  for (int64_t e = blk * kT + t; e < nlo; e += nblk * kT) lo[e] = 0ull;
  const int64_t r0 = blk * rows_per_block;
  const int64_t r1 = min(M, r0 + rows_per_block);
  double acc = 0.0;
  uint32_t m = 0, f = 0, rb = 0;
  if (q < R)
    for (int64_t r = r0 + q; r < r1; r += R) {
      const float v = X[r * L + d];
      acc += (double)v;
      const uint32_t b = __float_as_uint(v) & 0x7fffffffu;
      m = (b > m && b < 0x7f800000u) ? b : m;  // ignore Inf / NaN
      f = max(f, fine_bits(b));
      rb |= __float_as_uint(v) & 0xffffu;
    }
  s[t] = acc;
  sm[t] = m;
  sf[t] = f;
  sr[t] = rb;
  __syncthreads();
  if (t < L) {
    double v = 0.0;
    for (int qi = 0; qi < R; ++qi) v += s[qi * L + t];
    part[blk * L + t] = v;
  }
  for (int off = kT / 2; off > 0; off >>= 1) {
    if (t < off) {
      sm[t] = max(sm[t], sm[t + off]);
      sf[t] = max(sf[t], sf[t + off]);
      sr[t] |= sr[t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    amax[blk] = sm[0];
    amax[nblk + blk] = sf[0];
    amax[2 * nblk + blk] = sr[0];
  }
}

// Block maxima over X (n floats): part[block] = largest finite |x| (as
// float bits), part[nblocks + block] = largest fine bits, part[2 nblocks +
// block] = the OR of the coordinates' low 16 bits (zero: all exact in BF16).
// The blocks also
// clear the nlo words of ``lo`` (the residual sums of the update, see
// fin_body), so that every accumulation starts from zero.
__device__ __forceinline__ void absmax_body(const float* __restrict__ X, int64_t n,
                                            uint32_t* __restrict__ part, int64_t block,
                                            int64_t nblocks, unsigned long long* __restrict__ lo,
                                            int64_t nlo) {
  __shared__ uint32_t s[kT];
  __shared__ uint32_t sf[kT];
  __shared__ uint32_t sr[kT];
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  uint32_t m = 0, f = 0, r = 0;
  auto upd = [&m, &f, &r](uint32_t b) {
    f = max(f, fine_bits(b));
    r |= b & 0xffffu;  // nonzero: not exact in BF16
    b &= 0x7fffffffu;
    m = (b > m && b < 0x7f800000u) ? b : m;  // ignore Inf / NaN
  };
  const int64_t stride = nblocks * kT;
  for (int64_t e = block * kT + threadIdx.x; e < nlo; e += stride) lo[e] = 0ull;
  // 16-byte loads, four per thread in flight: a block reads four adjacent
  // 4 KiB pieces per step, so that the grid sweeps X as one contiguous window
  // (four pieces a grid's width apart measured 17% slower), from the end of
  // X backwards, so that the first allocation, which reads X front to back,
  // starts on rows the memory-side cache still holds; then the one-load tail
  // and the scalar tail
  const int64_t nv = (reinterpret_cast<uintptr_t>(X) & 15) == 0 ? n / 4 : 0;
  const u32x4* X4 = reinterpret_cast<const u32x4*>(X);
  const int64_t full = nv / (4 * stride) * (4 * stride);
  for (int64_t base = full - 4 * stride + block * 4 * kT; base >= 0; base -= 4 * stride) {
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = X4[base + u * kT + threadIdx.x];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      upd(v[u].x);
      upd(v[u].y);
      upd(v[u].z);
      upd(v[u].w);
    }
  }
  int64_t i = full + block * kT + threadIdx.x;
  for (; i < nv; i += stride) {
    const u32x4 v = X4[i];
    upd(v.x);
    upd(v.y);
    upd(v.z);
    upd(v.w);
  }
  for (int64_t e = 4 * nv + block * kT + threadIdx.x; e < n; e += stride)
    upd(__float_as_uint(X[e]));
  s[threadIdx.x] = m;
  sf[threadIdx.x] = f;
  sr[threadIdx.x] = r;
  __syncthreads();
  for (int off = kT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s[threadIdx.x] = max(s[threadIdx.x], s[threadIdx.x + off]);
      sf[threadIdx.x] = max(sf[threadIdx.x], sf[threadIdx.x + off]);
      sr[threadIdx.x] |= sr[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[block] = s[0];
    part[nblocks + block] = sf[0];
    part[2 * nblocks + block] = sr[0];
  }
}

// The fixed-point scales of the update from the block maxima (nparts of
// each kind, laid out as absmax_body writes them): shift[0] = s, with
// |x| < 2^e and M < 2^b, s = min(51, 62 - b) - e, so that every round(x 2^s)
// is below 2^51 and a sum of M of them below 2^62; shift[1] = t = 0 when
// every coordinate is a multiple of 2^-s (the sums are then exact, as for
// integer pixels), else t = min(52, 63 - b): each coordinate's residual
// x 2^s - round(x 2^s), at most 1/2, is then also summed, as round(residual
// 2^t), so coordinates down to 2^-(s+t) count exactly and the update keeps
// about 2^-(s+t) of max|x| (2^-80 of it at M = 2^22) where one word kept
// 2^-s; shift[2] = 1 when every coordinate is exact in BF16 (the
// allocation's split screen then skips the products of vanishing parts);
// shift[3] = 1 when every coordinate is a multiple of 2^-g for some g <= s
// with |x| 2^g M < 2^31 (shift[4] = g, the coarsest such grid): every cell
// sum at scale 2^g is then an integer below 2^31 in magnitude, which 32-bit
// words hold exactly, and times 2^(s-g) it is the sum at scale 2^s (for
// example 8-bit pixels: g = 0, sums below 2^8 M).
__device__ __forceinline__ void shift_body(const uint32_t* __restrict__ part, int nparts,
                                           int64_t M, int* __restrict__ shift) {
  __shared__ uint32_t s[kT];
  __shared__ uint32_t sf[kT];
  __shared__ uint32_t sr[kT];
  uint32_t m = 0, f = 0, r = 0;
  for (int i = threadIdx.x; i < nparts; i += kT) {
    m = max(m, part[i]);
    f = max(f, part[nparts + i]);
    r |= part[2 * nparts + i];
  }
  s[threadIdx.x] = m;
  sf[threadIdx.x] = f;
  sr[threadIdx.x] = r;
  __syncthreads();
  for (int off = kT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s[threadIdx.x] = max(s[threadIdx.x], s[threadIdx.x + off]);
      sf[threadIdx.x] = max(sf[threadIdx.x], sf[threadIdx.x + off]);
      sr[threadIdx.x] |= sr[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int b = 0;
    while (b < 63 && ((int64_t)1 << b) <= M) ++b;  // M < 2^b
    const float mx = __uint_as_float(s[0]);
    int e = 0;
    if (mx > 0.0f) frexpf(mx, &e);  // mx < 2^e
    const int sh = (s[0] == 0) ? 0 : (min(51, 62 - b) - e);
    shift[0] = sh;
    shift[1] = (sf[0] != 0u && (int)sf[0] - 256 > sh) ? min(52, 63 - b) : 0;
    shift[2] = sr[0] == 0u;
    const int g = sf[0] == 0u ? 0 : (int)sf[0] - 256;
    const bool narrow = g <= sh && e + g + b <= 31;
    shift[3] = narrow ? 1 : 0;
    shift[4] = narrow ? g : 0;
  }
}

// round(v * 2^s), nearest with ties to even, as a two's-complement 64-bit
// integer, for |v * 2^s| < 2^51 (the shift guarantees it for the training
// data): fma(v, 2^s, 1.5 * 2^52) is exact up to that one rounding, to an
// integer (the sum lies in [2^52, 2^53), whose spacing is 1; 1.5 * 2^52 is
// even, so ties go to even as rint's do), and the integer is the sum's bit
// pattern minus that of 1.5 * 2^52, whose low word is zero.  p2s = 2^s.
__device__ __forceinline__ unsigned long long fixed_of(double y) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(y);
  const uint32_t hi = (uint32_t)(b >> 32) - 0x43380000u;  // no borrow: the low word is kept
  return ((unsigned long long)hi << 32) | (b & 0xffffffffull);
}

__device__ __forceinline__ unsigned long long fixed(float v, double p2s) {
  return fixed_of(__builtin_fma((double)v, p2s, 0x1.8p52));
}

// The coordinate's second word (see shift_body): round(r 2^t) for its
// residual r = v 2^s - round(v 2^s), |r| <= 1/2.  r is exact in FP64 (v 2^s
// and the integer are exact and within 1/2 of each other), and 2^t <= 2^52
// keeps |r 2^t| within the range of the rounding trick.  p2t = 2^t.
__device__ __forceinline__ unsigned long long fixed_res(float v, double p2s, double p2t) {
  const double n = __builtin_fma((double)v, p2s, 0x1.8p52) - 0x1.8p52;  // round(v 2^s)
  const double r = __builtin_fma((double)v, p2s, -n);
  return fixed_of(__builtin_fma(r, p2t, 0x1.8p52));
}

// cnt c - S 2^-s (FP64) for the gradient of a cell with cnt rows whose
// fixed-point sum is S at shift s.  When c 2^s lies below 2^62 in magnitude
// it is rounded onto the sums' grid (ck) and cnt ck - S is formed exactly in
// two 64-bit limbs of base 2^32 (cnt < 2^31, so no limb overflows) before
// the conversion, so nearly equal cnt c and sum lose nothing to cancellation
// and a codevector far outside the data cannot overflow 64 bits.  Beyond
// 2^62 the codevector is at least 2^(62-s) >= 2^11 max|x| away from every
// coordinate, |S 2^-s| <= cnt max|x| is far below |cnt c|, and FP64 forms
// the difference without cancellation.
__device__ __forceinline__ double grad_diff(float c, long long cnt, long long S, int s) {
  const double cs = ldexp((double)c, s);  // exact
  if (fabs(cs) < 0x1p62) {
    const long long ck = llrint(cs);
    const long long ck_hi = ck >> 32;                        // |ck_hi| < 2^30
    const unsigned long long ck_lo = (unsigned long long)ck & 0xffffffffull;
    const long long a = cnt * ck_hi;                         // |a| < 2^61
    const unsigned long long b = (unsigned long long)cnt * ck_lo;  // < 2^63
    const long long top = a + (long long)(b >> 32) - (S >> 32);  // |top| < 2^62
    const long long low = (long long)(b & 0xffffffffull) - (long long)((unsigned long long)S & 0xffffffffull);
    return ldexp(ldexp((double)top, 32) + (double)low, -s);
  }
  return (double)cnt * (double)c - ldexp((double)S, -s);
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

// row += the row's fixed-point coordinates, *cnt += 1.  The caller passes
// a spare row and count, never read, for a row that is off, so that the
// adds need no branch.  In a full row (L = G VW DPL) dimension
// (gl + q G) VW + e is kept at position e G DPL + q G + gl, so that the G
// lanes of a group add into consecutive words (no LDS bank conflicts among
// them); otherwise at position d.  FINE: the coordinates' nonzero second
// words (fixed_res) are added into lo_row (global, natural dimension
// order; NULL for a row that is off) -- rare for data near their grid.
template <int G, int VW, int DPL, bool FINE = false>
__device__ __forceinline__ void add_row(unsigned long long* row, int32_t* cnt, int L, int gl,
                                        double p2s, const float (&v)[DPL][VW],
                                        unsigned long long* lo_row = nullptr, double p2t = 0.0) {
  if (G * VW * DPL == L) {  // a uniform test, once per row
#pragma unroll
    for (int q = 0; q < DPL; ++q)
#pragma unroll
      for (int e = 0; e < VW; ++e) atomicAdd(&row[e * G * DPL + q * G + gl], fixed(v[q][e], p2s));
  } else {
#pragma unroll
    for (int q = 0; q < DPL; ++q)
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const int d = (gl + q * G) * VW + e;
        if (d < L) atomicAdd(&row[d], fixed(v[q][e], p2s));
      }
  }
  if constexpr (FINE) {
    if (lo_row) {
#pragma unroll
      for (int q = 0; q < DPL; ++q)
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          const int d = (gl + q * G) * VW + e;
          const unsigned long long r = fixed_res(v[q][e], p2s, p2t);
          if (d < L && r != 0ull) atomicAdd(&lo_row[d], r);
        }
    }
  }
  if (gl == 0) atomicAdd(cnt, 1);
}

// LDS position of dimension d in a row (see add_row).
template <int G, int VW, int DPL>
__device__ __forceinline__ int acc_pos(int d, int L) {
  return (G * VW * DPL == L) ? (d % VW) * (G * DPL) + d / VW : d;
}

// Rows of sums are L + 1 words apart (rows of random cells then start on
// different LDS banks).  LDS of an accumulation block: cps rows plus the
// spare row, then cps + 1 counts.
inline size_t acc_lds_bytes(int cps, int64_t L) {
  return (size_t)(cps + 1) * (size_t)((L + 1) * 8 + 4);
}

// Loads are unconditional (no branch, so all rows of a batch are in flight
// together): the caller passes a valid row, and lanes whose dimensions lie
// beyond L read dimension 0 instead (add_row skips them).
template <int G, int VW, int DPL>
__device__ __forceinline__ void load_dims(const float* xrow, int L, int gl,
                                          float (&v)[DPL][VW]) {
#pragma unroll
  for (int q = 0; q < DPL; ++q) {
    const int d0 = (gl + q * G) * VW;
    VLoad<VW>::get(xrow + (d0 < L ? d0 : 0), v[q]);
  }
}

// One block per (row chunk, cell slice), slices of one chunk adjacent.  Rows
// stream in batches of kBatch (one slice) or kSel (several).  With one
// slice every row is added: a group
// of G lanes walks a contiguous sub-range of the batch, kUnroll rows (cell
// index and coordinates) loaded together.  With several slices the batch's
// cell indices are read first and the rows of this slice are gathered into
// an LDS list (integer sums make the list order immaterial), then added.
constexpr int kBatch = 1024;
constexpr int kSel = 4096;  // several slices: about kSel / nslices rows gathered per batch
constexpr int kUnrollSel = 16;  // gathered coordinates-groups per lane and stage

// Decision of this iteration from the allocation's partials (the same in every
// block that calls it); the block with ``lead`` records the next state in
// ctl.pend.  Returns true when this iteration updates; *N receives the
// codebook size.  The run state is read into LDS (a word per thread) beside
// the partials' loads, stepped there by thread 0, and the pending state is
// written back a word per thread, so the decision takes one memory round
// trip.
__device__ __forceinline__ bool acc_decide(const Ctl& ctl, bool lead, int* N) {
  constexpr int NW = (int)(sizeof(DevState) / 4);
  static_assert(sizeof(DevState) % 4 == 0 && NW <= kT, "state words");
  __shared__ double red[kT];
  __shared__ DevState sst, spend;
  __shared__ int s_act;
  const int t = threadIdx.x;
  uint32_t word = 0;
  if (t < NW) word = reinterpret_cast<const uint32_t*>(ctl.st)[t];
  const double S = block_sum0(ctl.dpart, ctl.nparts, red);
  if (t < NW) {
    reinterpret_cast<uint32_t*>(&sst)[t] = word;
    reinterpret_cast<uint32_t*>(&spend)[t] = word;  // the next state starts as a copy
  }
  __syncthreads();
  if (t == 0) {
    s_act = kActNone;
    if (!sst.done) {
      const double D = S / (double)sst.M;
      const Step r = step_of(&sst, D);
      s_act = r.action;
      if (lead) apply_step(&sst, &spend, D, r, ctl.Dtrace, ctl.Atrace);
    }
  }
  __syncthreads();
  if (lead && !sst.done && t < NW)
    reinterpret_cast<uint32_t*>(ctl.pend)[t] = reinterpret_cast<const uint32_t*>(&spend)[t];
  *N = sst.n;
  return s_act == kActUpdate;
}

// Accumulation of block ``blk`` = (row chunk, cell slice) of the update;
// slist (kSel entries when SEL) and snsel are the caller's LDS.  SEL: the
// block's slice is one of several (nslices > 1); US: coordinate groups per
// lane and stage of its gathers (registers: two stages of US float4s).  N:
// cells of this update; ns: cells per chunk in the partials' layout (the
// planned codebook size, so that the finishing kernel can address them
// before it knows N).
template <int G, int VW, int DPL, bool SEL, int US = kUnrollSel, int NT = kT, bool FINE = false>
__device__ __forceinline__ void acc_body(const float* __restrict__ X, int64_t M, int L,
                                         const int32_t* __restrict__ idx, int N, int ns,
                                         int cps, int nslices, int64_t rows_per_chunk, int s,
                                         unsigned long long* __restrict__ part,
                                         int32_t* __restrict__ pcnt, int64_t blk,
                                         unsigned long long* sacc, int32_t* slist,
                                         int32_t& snsel, unsigned long long* lo = nullptr,
                                         int tfine = 0) {
  const int chunk = (int)(blk / nslices), slice = (int)(blk % nslices);
  const double p2s = ldexp(1.0, s);
  const double p2t = ldexp(1.0, tfine);
  const int k0 = slice * cps, k1 = min(N, k0 + cps), nk = max(0, k1 - k0);
  constexpr int NG = NT / G;  // rows in parallel
  // With a single slice and few cells, R private copies of the table (row
  // group g adds into copy g % R) keep rows of one cell from meeting in the
  // same LDS atomic; the copies are added (integers) at the end.
  int R = 1;
  if (nslices == 1 && nk > 0)
    while (R < 16 && 2 * R <= NG && 2 * R * nk <= cps) R *= 2;
  const int LS = L + 1;    // row stride
  const int TL = nk * LS;  // entries of one copy
  unsigned long long* spare = sacc + (size_t)cps * LS;  // R * nk <= cps rows are in use
  int32_t* scnt = reinterpret_cast<int32_t*>(sacc + (size_t)(cps + 1) * LS);
  int32_t* cspare = scnt + cps;
  const int t = threadIdx.x;
  for (int e = t; e < R * TL; e += NT) sacc[e] = 0ull;
  for (int e = t; e < R * nk; e += NT) scnt[e] = 0;
  if (t == 0) snsel = 0;
  __syncthreads();
  const int g = t / G, gl = t % G;
  unsigned long long* my_acc = sacc + (g % R) * TL;
  int32_t* my_cnt = scnt + (g % R) * nk;
  const int64_t r0 = (int64_t)chunk * rows_per_chunk;
  const int64_t r1 = min(M, r0 + rows_per_chunk);
  if constexpr (!SEL) {
    // rows b0 + g + NG i of the batch go to group g: a wave's groups load
    // consecutive rows
    constexpr int PER = kBatch / NG;  // rows of one group per batch
    constexpr int KU1 = PER < kUnroll ? PER : kUnroll;
    for (int64_t b0 = r0; b0 < r1; b0 += kBatch) {
      const int nb = (int)min((int64_t)kBatch, r1 - b0);
      for (int i0 = 0; i0 < PER; i0 += KU1) {
        int k[KU1];
        float v[KU1][DPL][VW];
#pragma unroll
        for (int u = 0; u < KU1; ++u) {
          const int r = g + NG * (i0 + u);
          const bool on = r < nb;
          const int64_t m = b0 + (on ? r : 0);  // b0: a row of this batch
          const int kv = idx[m];
          k[u] = on ? kv : -1;
          load_dims<G, VW, DPL>(X + m * L, L, gl, v[u]);
        }
#pragma unroll
        for (int u = 0; u < KU1; ++u) {
          const bool on = k[u] >= k0 && k[u] < k1;
          const int kl = k[u] - k0;
          add_row<G, VW, DPL, FINE>(on ? my_acc + __umul24(kl, LS) : spare,
                                    on ? my_cnt + kl : cspare, L, gl, p2s, v[u],
                                    (FINE && on) ? lo + (int64_t)k[u] * L : nullptr, p2t);
        }
      }
    }
  } else {
    // Several slices: batches of kSel cell indices; the next batch's indices
    // are loaded while this batch's rows of the slice are gathered, KU
    // rows per group in flight.
    constexpr int KR = kSel / NT;
    constexpr int KU = US / DPL > 1 ? US / DPL : 1;  // rows per group and stage
    int kr[KR];
    auto load_idx = [&](int64_t b0, int (&dst)[KR]) {
      const int nb = (int)min((int64_t)kSel, r1 - b0);
#pragma unroll
      for (int u = 0; u < KR; ++u) {
        const int r = u * NT + t;
        dst[u] = idx[b0 + (r < nb ? r : 0)];
      }
    };
    if (r0 < r1) load_idx(r0, kr);
    for (int64_t b0 = r0; b0 < r1; b0 += kSel) {
      const int nb = (int)min((int64_t)kSel, r1 - b0);
#pragma unroll
      for (int u = 0; u < KR; ++u) {
        const int r = u * NT + t;
        const int k = kr[u];
        if (r < nb && k >= k0 && k < k1) slist[atomicAdd(&snsel, 1)] = r * 8192 + (k - k0);
      }
      int kn[KR];
      const int64_t b1 = b0 + kSel;
      load_idx(b1 < r1 ? b1 : b0, kn);  // the last batch reads its own indices again
      __syncthreads();
      const int nsel = snsel;
      // two stages of KU rows per group: the next stage's rows load
      // while this stage's are added
      auto load_stage = [&](int e0, int (&kk)[KU], float (&v)[KU][DPL][VW]) {
#pragma unroll
        for (int u = 0; u < KU; ++u) {
          const int e = e0 + u * NG;
          const int packed = (e < nsel) ? slist[e] : -1;
          const int r = packed >= 0 ? packed >> 13 : 0;
          kk[u] = packed >= 0 ? (packed & 8191) : -1;
          load_dims<G, VW, DPL>(X + (b0 + r) * L, L, gl, v[u]);
        }
      };
      int kka[KU], kkb[KU];
      float va[KU][DPL][VW], vb[KU][DPL][VW];
      if (g < nsel) load_stage(g, kka, va);
      for (int e0 = g; e0 < nsel; e0 += 2 * NG * KU) {
        const int e1 = e0 + NG * KU, e2 = e1 + NG * KU;
        if (e1 < nsel) load_stage(e1, kkb, vb);
#pragma unroll
        for (int u = 0; u < KU; ++u) {
          const bool on = kka[u] >= 0;
          add_row<G, VW, DPL, FINE>(on ? sacc + __umul24(kka[u], LS) : spare,
                                    on ? scnt + kka[u] : cspare, L, gl, p2s, va[u],
                                    (FINE && on) ? lo + (int64_t)(k0 + kka[u]) * L : nullptr,
                                    p2t);
        }
        if (e1 >= nsel) break;
        if (e2 < nsel) load_stage(e2, kka, va);
#pragma unroll
        for (int u = 0; u < KU; ++u) {
          const bool on = kkb[u] >= 0;
          add_row<G, VW, DPL, FINE>(on ? sacc + __umul24(kkb[u], LS) : spare,
                                    on ? scnt + kkb[u] : cspare, L, gl, p2s, vb[u],
                                    (FINE && on) ? lo + (int64_t)(k0 + kkb[u]) * L : nullptr,
                                    p2t);
        }
      }
      __syncthreads();
      if (t == 0) snsel = 0;
      __syncthreads();
#pragma unroll
      for (int u = 0; u < KR; ++u) kr[u] = kn[u];
    }
  }
  __syncthreads();
  unsigned long long* dst = part + ((int64_t)chunk * ns + k0) * L;
  for (int e = t; e < nk * L; e += NT) {
    const int k = e / L, d = e - k * L;
    const int src = k * LS + acc_pos<G, VW, DPL>(d, L);
    unsigned long long a = sacc[src];
    for (int r = 1; r < R; ++r) a += sacc[r * TL + src];
    dst[e] = a;
  }
  int32_t* cdst = pcnt + (int64_t)chunk * ns + k0;
  for (int e = t; e < nk; e += NT) {
    int32_t c = scnt[e];
    for (int r = 1; r < R; ++r) c += scnt[r * nk + e];
    cdst[e] = c;
  }
}

// Accumulation by dimension slices: block (chunk, q) adds dimensions
// [16 q, 16 q + 16) of every row of its chunk into LDS sums of all cells (rows
// of 17 words), so no block filters rows by cell (the cell-slice blocks each
// walk their chunk's whole index stream and gather their rows).  For
// codebooks whose N x 17 words fit one CU's LDS and L a multiple of 16; the
// partials keep the [chunk][cell][L] layout (fin_body reads them as before),
// the counts come from the q = 0 blocks.  1024 threads: 256 groups of four
// lanes, a lane taking one 16-byte word of a row, kDsRows rows per group in
// flight (16-byte loads when X is 16-byte aligned).  The blocks of one chunk
// sit on one XCD (blocks are dealt to the eight XCDs in turn), so the lines
// they share meet in one L2.
constexpr int kDs = 16;      // dimensions per slice
constexpr int kDsRows = 4;   // rows per lane group in flight (8 measured 2% slower)
constexpr int kDsThreads = 1024;

// Dynamic LDS the dimension-slice kernel may take: a CU's 160 KiB less a
// reserve for its static LDS (the reduction buffer and run-state copies of
// the device-side stop decision, about 3 KiB).
constexpr int kAccdLdsMax = 163840 - 8192;

// Dynamic LDS of the batched form's 16-dimension slices (see plan_afp).
constexpr int kBdsLdsMax = 40960;

inline size_t accd_lds_bytes(int64_t N) {
  return (size_t)(N + 1) * (kDs + 1) * 8 + (size_t)(N + 1) * 4;
}

// chunk and slice of block ``blk`` of nch x nds blocks
__device__ __forceinline__ void accd_block(int blk, int nch, int nds, int* chunk, int* q) {
  const int nb = nch * nds;
  if ((nch & 7) == 0 && (nb & 7) == 0) {
    const int x = blk & 7, i = blk >> 3;
    *chunk = (i / nds) * 8 + x;
    *q = i % nds;
  } else {
    *chunk = blk / nds;
    *q = blk % nds;
  }
}

// SPANS (nch chunks): rows dealt in spans of NG kDsRows rows, walked from the
// end of X backwards, as accn_body does (measured on a real-valued mixture
// at M = 4,194,304, L = 64, N = 1024: update 234 -> 210 us per iteration);
// otherwise chunk c holds rows [c rows_per_chunk, (c + 1) rows_per_chunk)
// (the batched form's instances, whose chunks are few: spans measured 0.6%
// slower there).
template <bool FINE, bool VEC, int NT = kDsThreads, bool SPANS = false>
__device__ __forceinline__ void accd_body(const float* __restrict__ X, int64_t M, int L,
                                          const int32_t* __restrict__ idx, int N, int ns,
                                          int64_t rows_per_chunk, int chunk, int q, int s,
                                          unsigned long long* __restrict__ part,
                                          int32_t* __restrict__ pcnt,
                                          unsigned long long* sacc,
                                          unsigned long long* __restrict__ lo, int tfine,
                                          int nch = 0) {
  constexpr int LS = kDs + 1;
  constexpr int NG = NT / 4;
  const double p2s = ldexp(1.0, s);
  const double p2t = ldexp(1.0, tfine);
  int32_t* scnt = reinterpret_cast<int32_t*>(sacc + (size_t)(N + 1) * LS);
  const int t = threadIdx.x;
  for (int e = t; e < (N + 1) * LS; e += NT) sacc[e] = 0ull;
  if (q == 0)
    for (int e = t; e <= N; e += NT) scnt[e] = 0;
  __syncthreads();
  const int g = t >> 2, gl = t & 3;
  const int d0 = kDs * q + 4 * gl;  // this lane's four dimensions
  constexpr int64_t span = (int64_t)NG * kDsRows;
  const int64_t r0 = SPANS ? 0 : (int64_t)chunk * rows_per_chunk;
  const int64_t r1 = SPANS ? M : min(M, r0 + rows_per_chunk);
  int64_t p = 0;  // SPANS: the span, from the chunk's last backwards (-1: none)
  if constexpr (SPANS) {
    const int64_t nsp = (M + span - 1) / span;
    p = chunk < nsp ? chunk + (nsp - 1 - chunk) / nch * nch : -1;
  }
  for (int64_t b = SPANS ? p * span + g : r0 + g; SPANS ? p >= 0 : b < r1;) {
    int k[kDsRows];
    float v[kDsRows][4];
#pragma unroll
    for (int u = 0; u < kDsRows; ++u) {
      const int64_t m = b + (int64_t)u * NG;
      const bool on = m < r1;
      const int64_t mm = on ? m : r0;  // a row of this chunk (SPANS: of X)
      const int kv = idx[mm];
      k[u] = (on && (unsigned)kv < (unsigned)N) ? kv : N;  // N: the spare row
      if constexpr (VEC) {
        const float4 x = *reinterpret_cast<const float4*>(X + mm * L + d0);
        v[u][0] = x.x;
        v[u][1] = x.y;
        v[u][2] = x.z;
        v[u][3] = x.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[u][e] = X[mm * L + d0 + e];
      }
    }
#pragma unroll
    for (int u = 0; u < kDsRows; ++u) {
      unsigned long long* row = sacc + __umul24(k[u], LS) + 4 * gl;
#pragma unroll
      for (int e = 0; e < 4; ++e) atomicAdd(&row[e], fixed(v[u][e], p2s));
      if constexpr (FINE) {
        if (k[u] < N) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const unsigned long long r = fixed_res(v[u][e], p2s, p2t);
            if (r != 0ull) atomicAdd(&lo[(int64_t)k[u] * L + d0 + e], r);
          }
        }
      }
      if (q == 0 && gl == 0) atomicAdd(&scnt[k[u]], 1);
    }
    if constexpr (SPANS) {
      p -= nch;
      b = p * span + g;
    } else {
      b += span;
    }
  }
  __syncthreads();
  unsigned long long* dst = part + (int64_t)chunk * ns * L + kDs * q;
  for (int e = t; e < N * kDs; e += NT) {
    const int kk = e / kDs, d = e - kk * kDs;
    dst[(int64_t)kk * L + d] = sacc[kk * LS + d];
  }
  if (q == 0) {
    int32_t* cdst = pcnt + (int64_t)chunk * ns;
    for (int e = t; e < N; e += NT) cdst[e] = scnt[e];
  }
}

// The 32-bit form of the dimension slices, for data whose cell sums fit 32
// bits at the scale 2^g (shift[3], see shift_body): a slice is 32 dimensions,
// one 128-byte line of a row of 64 floats, so no two blocks read the same
// line (16-dimension slices of 8-byte sums share each line between two
// blocks, which fetch it twice when they drift apart).  A group of eight
// lanes takes one row's slice, a 16-byte word per lane; x 2^g is an integer
// below 2^31 in magnitude, so it converts exactly to int32 and the LDS sums
// add in 32-bit two's complement without overflow.  Lane gl's dimension
// 4 gl + e goes to word 8 e + gl of its cell's row, so that the eight lanes
// of a group add into consecutive words; rows of sums are 33 words apart.
// The partials are int32 [chunk][cell][L].
constexpr int kDn = 32;     // dimensions per 32-bit slice
constexpr int kDnRows = 4;  // rows per lane group in flight (8 measured slower: 218 vs 209 us)

inline size_t accn_lds_bytes(int64_t N) {
  return (size_t)(N + 1) * (kDn + 1) * 4 + (size_t)(N + 1) * 4;
}

// Rows are dealt to the nch chunks in spans of 128 kDnRows rows (span p to
// chunk p mod nch), and every block walks its spans from the end of X
// backwards: the allocation before the update reads X front to back, so
// the update starts on the rows it read last, which the memory-side cache
// still holds, and ends on the rows the next allocation reads first
// (measured: update 212 -> 207 us and allocation 693 -> 659 us per
// iteration at M = 4,194,304, L = 64, N = 1024, against contiguous chunks
// walked forwards).  The chunks' sums do not depend on which rows they hold.
template <bool VEC>
__device__ __forceinline__ void accn_body(const float* __restrict__ X, int64_t M, int L,
                                          const int32_t* __restrict__ idx, int N, int ns,
                                          int nch, int chunk, int q, int g,
                                          int32_t* __restrict__ part, int32_t* __restrict__ pcnt,
                                          uint32_t* sacc) {
  constexpr int LS = kDn + 1;
  constexpr int NG = kDsThreads / 8;
  int32_t* scnt = reinterpret_cast<int32_t*>(sacc + (size_t)(N + 1) * LS);
  const int t = threadIdx.x;
  for (int e = t; e < (N + 1) * LS; e += kDsThreads) sacc[e] = 0u;
  if (q == 0)
    for (int e = t; e <= N; e += kDsThreads) scnt[e] = 0;
  __syncthreads();
  const int gr = t >> 3, gl = t & 7;
  const int d0 = kDn * q + 4 * gl;  // this lane's four dimensions
  constexpr int64_t span = (int64_t)NG * kDnRows;
  const int64_t nsp = (M + span - 1) / span;
  const int64_t last = chunk < nsp ? chunk + (nsp - 1 - chunk) / nch * nch : -1;
  for (int64_t p = last; p >= 0; p -= nch) {
    const int64_t b = p * span + gr;
    int k[kDnRows];
    float v[kDnRows][4];
#pragma unroll
    for (int u = 0; u < kDnRows; ++u) {
      const int64_t m = b + (int64_t)u * NG;
      const bool on = m < M;
      const int64_t mm = on ? m : 0;  // a row of X
      const int kv = idx[mm];
      k[u] = (on && (unsigned)kv < (unsigned)N) ? kv : N;  // N: the spare row
      if constexpr (VEC) {
        const float4 x = *reinterpret_cast<const float4*>(X + mm * L + d0);
        v[u][0] = x.x;
        v[u][1] = x.y;
        v[u][2] = x.z;
        v[u][3] = x.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[u][e] = X[mm * L + d0 + e];
      }
    }
#pragma unroll
    for (int u = 0; u < kDnRows; ++u) {
      uint32_t* row = sacc + __umul24(k[u], LS) + gl;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        atomicAdd(&row[8 * e], (uint32_t)(int32_t)__builtin_amdgcn_ldexpf(v[u][e], g));
      if (q == 0 && gl == 0) atomicAdd(&scnt[k[u]], 1);
    }
  }
  __syncthreads();
  int32_t* dst = part + (int64_t)chunk * ns * L + kDn * q;
  for (int e = t; e < N * kDn; e += kDsThreads) {
    const int kk = e / kDn, d = e - kk * kDn;
    dst[(int64_t)kk * L + d] = (int32_t)sacc[kk * LS + 8 * (d & 3) + (d >> 2)];
  }
  if (q == 0) {
    int32_t* cdst = pcnt + (int64_t)chunk * ns;
    for (int e = t; e < N; e += kDsThreads) cdst[e] = scnt[e];
  }
}

// Under device control: acts on the pending state for cell ``k`` (a split
// of codevector k, or nothing); the block with ``lead`` commits the state.
// Returns true when cell k is to be updated, with N, C_old and out set.
// ``ndone`` (nullable) counts runs that finish with this commit.  The fields
// it needs are loaded together (pend is valid whenever st is not done).
__device__ __forceinline__ bool fin_state(const Ctl& ctl, const CbPair& cbp, int64_t k, bool lead,
                                          int L, int* N, const float** C_old, float** out,
                                          unsigned* ndone = nullptr) {
  constexpr int NW = (int)(sizeof(DevState) / 4);
  static_assert(sizeof(DevState) % 4 == 0 && NW <= kT, "state words");
  const DevState* st = ctl.pend;
  const int t = threadIdx.x;
  // the commit copies the pending state a word per thread; its loads are
  // issued with the others
  uint32_t word = 0;
  if (lead && t < NW) word = reinterpret_cast<const uint32_t*>(st)[t];
  const int done = ctl.st->done;
  const int action = st->action, n_src = st->n_src, src = st->src, dst = st->dst;
  if (done) return false;
  if (lead) {
    if (t < NW) reinterpret_cast<uint32_t*>(ctl.st)[t] = word;
    if (ndone && t == 0 && st->done) atomicAdd(ndone, 1u);
  }
  if (action == kActSplit) {
    // Codebook Splitting of codevector k (the split kernel's arithmetic):
    // children 2k ("+") and 2k+1 ("-"), formed in FP64, rounded once.
    if (k >= n_src) return false;
    const float* Cs = cbp.c[src];
    float* Cd = cbp.c[dst];
    for (int d = threadIdx.x; d < L; d += kT)
      misc::split_pair(Cs[k * L + d], st->split_mode, st->eps, st->delta, &Cd[(2 * k) * L + d],
                       &Cd[(2 * k + 1) * L + d]);
    return false;
  }
  if (action != kActUpdate) return false;
  *N = n_src;
  *C_old = cbp.c[src];
  *out = cbp.c[dst];
  return k < *N;
}

// Centroid (MODE 0) or gradient (MODE 1) of cell k from the chunk partials
// (ns cells per chunk).  The first partials and the counts are loaded
// before ``gate(&C_old, &out)`` runs, so that its reads of the run's state
// overlap them; gate returns false (the same in every thread) when cell k
// is not to be updated.  Thread (q, d) adds the partials of chunks q, q+Q,
// ... (integers, so the order is immaterial), then the Q lane sums.
//   With second words (tfine > 0, see shift_body) cell k's residual sums
// lo[k L + d] are read and cleared before ``gate`` (whatever the decision,
// so the next accumulation starts from zero) and enter as lo 2^-(s+tfine).
//   P32: the partials are the int32 sums of the 32-bit slices at scale
// 2^(s-up) (see accn_body); their 64-bit total times 2^up is the sum at 2^s.
template <int MODE, bool P32 = false, class Gate>
__device__ __forceinline__ void fin_body(const unsigned long long* __restrict__ part,
                                         const int32_t* __restrict__ pcnt, int nchunks, int ns,
                                         int L, int s, int32_t* __restrict__ counts, double g2,
                                         int k, Gate&& gate, unsigned long long* lo = nullptr,
                                         int tfine = 0, int up = 0) {
  constexpr int U = 16;  // 8-byte partial words in flight per thread
  // dimensions per word: the 32-bit partials (L even) are read in pairs
  constexpr int W = P32 ? 2 : 1;
  constexpr int UC = 8;  // counts in flight per thread
  __shared__ unsigned long long red[W][kT];
  __shared__ long long scount;
  __shared__ long long slo[kT];
  const int t = threadIdx.x;
  const bool fine = lo != nullptr && tfine > 0;
  if (fine && t < L) {
    unsigned long long* p = lo + (int64_t)k * L + t;
    slo[t] = (long long)*p;
    *p = 0ull;
  }
  const int LW = L / W;  // words per cell row
  int G2 = 1;
  while (G2 < LW && G2 < kT) G2 <<= 1;
  const int Q = kT / G2;
  const int q = t / G2;
  auto load_u = [&](int dw, int chs, unsigned long long (&v)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ch = chs + q + Q * u;
      v[u] = (dw < LW && ch < nchunks) ? part[((int64_t)ch * ns + k) * LW + dw] : 0ull;
    }
  };
  auto load_c = [&](int chs, int (&v)[UC]) {
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int ch = chs + t + 64 * u;
      v[u] = ch < nchunks ? pcnt[(int64_t)ch * ns + k] : 0;
    }
  };
  int cv[UC];
  if (t < 64) load_c(0, cv);
  unsigned long long a[U];
  load_u(t % G2, 0, a);
  const float* C_old = nullptr;
  float* out = nullptr;
  if (!gate(&C_old, &out)) return;
  if (t < 64) {
    long long c = 0;
    for (int chs = 64 * UC;; chs += 64 * UC) {
#pragma unroll
      for (int u = 0; u < UC; ++u) c += cv[u];
      if (chs >= nchunks) break;
      load_c(chs, cv);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    if (t == 0) scount = c;
  }
  for (int dw0 = 0; dw0 < LW; dw0 += G2) {
    const int dw = dw0 + t % G2;
    if (dw0 > 0) load_u(dw, 0, a);
    unsigned long long acc[W] = {};
    for (int chs = Q * U;; chs += Q * U) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if constexpr (P32) {  // two int32 sums, sign-extended (little-endian: dim 2 dw first)
          acc[0] += (unsigned long long)(long long)(int32_t)(uint32_t)a[u];
          acc[W - 1] += (unsigned long long)(long long)(int32_t)(uint32_t)(a[u] >> 32);
        } else {
          acc[0] += a[u];
        }
      }
      if (chs >= nchunks) break;
      load_u(dw, chs, a);
    }
#pragma unroll
    for (int w = 0; w < W; ++w) red[w][t] = acc[w];
    __syncthreads();
    const long long cnt = scount;
    if (dw0 == 0 && counts && t == 0) counts[k] = (int32_t)cnt;
    if (t < G2 && dw < LW) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const int d = dw * W + w;
        const int64_t e = (int64_t)k * L + d;
        if (cnt == 0) {
          if (MODE == 0) {
            if (out != C_old) out[e] = C_old[e];
          } else {
            out[e] = 0.0f;
          }
        } else {
          unsigned long long sum = 0;
          for (int qi = 0; qi < Q; ++qi) sum += red[w][qi * G2 + t];
          if constexpr (P32) sum <<= up;
          const long long S = (long long)sum;
          const double low = fine ? ldexp((double)slo[d], -(s + tfine)) : 0.0;
          if (MODE == 0) {
            out[e] = (float)((ldexp((double)S, -s) + low) / (double)cnt);
          } else {
            out[e] = (float)(g2 * (grad_diff(C_old[e], cnt, S, s) - low));
          }
        }
      }
    }
    __syncthreads();
  }
}


}  // namespace afp
}  // namespace lbg
