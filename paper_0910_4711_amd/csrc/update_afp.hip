// Codebook Updation by exact fixed-point accumulation.
//
// Every coordinate x is mapped to the integer round(x * 2^s) (nearest, ties
// to even), where the shift s is chosen from the largest |x| of the training
// set: s = min(51, 62 - b) - e with |x| < 2^e and M < 2^b, so that every
// such integer is below 2^51 in magnitude (three operations convert it, see
// fixed()) and a sum of M of them cannot overflow 63 bits.  Cell sums are
// then formed with 64-bit integer additions, which are exact and
// associative, so the order in which rows arrive (and the atomics that LDS
// accumulation uses) cannot change the result: the update is deterministic.
// For data whose coordinates are multiples of 2^-s (for instance integer
// pixels) the sums are the exact sums and the centroid is the exact mean
// rounded once to FP64 and once to FP32.  Otherwise every coordinate also
// contributes a second word, the rounding residual x 2^s - round(x 2^s)
// scaled by 2^t (t = min(52, 63 - b)) and rounded, added (when nonzero) by
// 64-bit integer atomics into an N x L array in global memory; the sums are
// then exact for coordinates down to 2^-(s+t), about 2^-80 of the largest
// |x| at M = 2^22, so a cell of values far below the largest coordinate
// keeps its precision.
//
//   absmax    per block: largest |x| (as float bits; max is order-free) and
//             the largest fine bits (the finest binary digit any coordinate
//             needs); the blocks also clear the second-word array
//   shift     one block: s and t from the block maxima (and whether the
//             sums fit 32 bits at a coarser grid 2^-g, see shift_body)
//   acc       one block per (row chunk, cell slice): LDS int64 sums and
//             counts for the cells of its slice over the rows of its chunk;
//             dense partials per chunk.  accd: one block per (row chunk,
//             16-dimension slice) with every cell in LDS; accn: the same
//             with 32-dimension slices of int32 sums at scale 2^g, whose
//             totals fin shifts to scale 2^s
//   fin       one block per cell: partials of all chunks added (integers),
//             centroid = sum * 2^-s / count (FP64, rounded to FP32); an empty
//             cell keeps its codevector.  For the gradient, (count * c_k - sum)
//             is formed in integers before the single rounding.  The cell's
//             second words join in FP64 and are cleared for the next update.

#include "afp_common.h"

namespace lbg {
namespace {

using namespace afp;

__global__ __launch_bounds__(kT) void absmax_kernel(const float* __restrict__ X, int64_t n,
                                                     uint32_t* __restrict__ part,
                                                     unsigned long long* __restrict__ lo,
                                                     int64_t nlo) {
  absmax_body(X, n, part, blockIdx.x, gridDim.x, lo, nlo);
}

__global__ __launch_bounds__(kT) void shift_kernel(const uint32_t* __restrict__ part, int nparts,
                                                    int64_t M, int* __restrict__ shift) {
  shift_body(part, nparts, M, shift);
}

// One workgroup per (row chunk, cell slice): 1024 threads with a single
// slice (one workgroup per CU keeps 16 waves busy on the chunk), 256 with
// several (the gathers' registers allow no more).
// GENERIC: the second-word decision is read on the device (both bodies in one
// kernel); otherwise the caller knows the data lie on the 2^-s grid and the
// kernel holds the one-word body alone (smaller code: measured 248 against
// 344 us per update at M = 4,194,304, L = 64, N = 1024).
template <int G, int VW, int DPL, bool SEL, bool GENERIC>
__global__ __launch_bounds__(SEL ? kT : 1024) void acc_kernel(
    const float* __restrict__ X, int64_t M, int L, const int32_t* __restrict__ idx, int N,
    int cps, int nslices, int64_t rows_per_chunk, const int* __restrict__ shift_p,
    unsigned long long* __restrict__ part, int32_t* __restrict__ pcnt,
    unsigned long long* __restrict__ lo, Ctl ctl) {
  extern __shared__ unsigned long long sacc[];
  __shared__ int32_t slist[SEL ? kSel : 1];
  __shared__ int32_t snsel;
  const int ns = N;  // cells per chunk in the partials (the planned size)
  if (ctl.st) {
    // the decision (block 0 writes it for the update's last kernel) does not
    // change what is accumulated, so the other blocks do not wait for it
    if (ctl.st->done) return;
    if (blockIdx.x == 0) (void)acc_decide(ctl, true, &N);
    if (forced_stop(ctl.st)) return;  // the level ends here: no update follows
    N = ctl.st->n;
  }
  const int s = shift_p[0], tf = shift_p[1];
  if (GENERIC && tf > 0)  // data off the 2^-s grid: second words
    acc_body<G, VW, DPL, SEL, kUnrollSel, SEL ? kT : 1024, true>(
        X, M, L, idx, N, ns, cps, nslices, rows_per_chunk, s, part, pcnt, blockIdx.x, sacc,
        slist, snsel, lo, tf);
  else
    acc_body<G, VW, DPL, SEL, kUnrollSel, SEL ? kT : 1024>(X, M, L, idx, N, ns, cps, nslices,
                                                           rows_per_chunk, s, part, pcnt,
                                                           blockIdx.x, sacc, slist, snsel);
}

// Dimension slices (see accd_body): one 1024-thread block per (chunk, slice).
template <bool GENERIC, bool VEC>
__global__ __launch_bounds__(kDsThreads) void accd_kernel(
    const float* __restrict__ X, int64_t M, int L, const int32_t* __restrict__ idx, int N,
    int nch, int nds, int64_t rows_per_chunk, const int* __restrict__ shift_p,
    unsigned long long* __restrict__ part, int32_t* __restrict__ pcnt,
    unsigned long long* __restrict__ lo, Ctl ctl) {
  extern __shared__ unsigned long long sacc[];
  const int ns = N;
  if (ctl.st) {
    if (ctl.st->done) return;
    if (blockIdx.x == 0) (void)acc_decide(ctl, true, &N);
    if (forced_stop(ctl.st)) return;  // the level ends here: no update follows
    N = ctl.st->n;
  }
  int chunk, q;
  accd_block(blockIdx.x, nch, nds, &chunk, &q);
  const int s = shift_p[0], tf = shift_p[1];
  if (GENERIC && tf > 0)
    accd_body<true, VEC, kDsThreads, true>(X, M, L, idx, N, ns, rows_per_chunk, chunk, q, s,
                                           part, pcnt, sacc, lo, tf, nch);
  else
    accd_body<false, VEC, kDsThreads, true>(X, M, L, idx, N, ns, rows_per_chunk, chunk, q, s,
                                            part, pcnt, sacc, lo, 0, nch);
}

// The 32-bit dimension slices (see accn_body): one 1024-thread block per
// (chunk, slice), for data whose sums fit 32 bits at scale 2^shift[4].
template <bool VEC>
__global__ __launch_bounds__(kDsThreads) void accn_kernel(
    const float* __restrict__ X, int64_t M, int L, const int32_t* __restrict__ idx, int N,
    int nch, int nds, const int* __restrict__ shift_p, int32_t* __restrict__ part,
    int32_t* __restrict__ pcnt, Ctl ctl) {
  extern __shared__ uint32_t saccn[];
  const int ns = N;
  if (ctl.st) {
    if (ctl.st->done) return;
    if (blockIdx.x == 0) (void)acc_decide(ctl, true, &N);
    if (forced_stop(ctl.st)) return;  // the level ends here: no update follows
    N = ctl.st->n;
  }
  int chunk, q;
  accd_block(blockIdx.x, nch, nds, &chunk, &q);
  accn_body<VEC>(X, M, L, idx, N, ns, nch, chunk, q, shift_p[4], part, pcnt, saccn);
}

// One block per cell.
template <int MODE, bool P32>
__global__ __launch_bounds__(kT) void fin_kernel(
    const unsigned long long* __restrict__ part, const int32_t* __restrict__ pcnt, int nchunks,
    int N, int L, const int* __restrict__ shift_p, const float* __restrict__ C_old,
    float* __restrict__ out, int32_t* __restrict__ counts, double g2,
    unsigned long long* __restrict__ lo, Ctl ctl, CbPair cbp) {
  const int k = blockIdx.x;
  const int s = shift_p[0];
  fin_body<MODE, P32>(
      part, pcnt, nchunks, N, L, s, counts, g2, k,
      [&](const float** c_old, float** dst) {
        *c_old = C_old;
        *dst = out;
        return !ctl.st || fin_state(ctl, cbp, k, k == 0, L, &N, c_old, dst);
      },
      lo, shift_p[1], P32 ? s - shift_p[4] : 0);
}

template <int G, int VW, int DPL>
void launch_acc(dim3 grid, size_t lds, hipStream_t st, const float* X, int64_t M, int L,
                const int32_t* idx, int N, int cps, int nslices, int64_t rpc, const int* sp,
                unsigned long long* part, int32_t* pcnt, unsigned long long* lo, Ctl ctl,
                bool generic) {
  if (nslices > 1) {
    if (generic)
      hipLaunchKernelGGL((acc_kernel<G, VW, DPL, true, true>), grid, dim3(kT), lds, st, X, M, L,
                         idx, N, cps, nslices, rpc, sp, part, pcnt, lo, ctl);
    else
      hipLaunchKernelGGL((acc_kernel<G, VW, DPL, true, false>), grid, dim3(kT), lds, st, X, M,
                         L, idx, N, cps, nslices, rpc, sp, part, pcnt, lo, ctl);
  } else {
    if (generic)
      hipLaunchKernelGGL((acc_kernel<G, VW, DPL, false, true>), grid, dim3(1024), lds, st, X, M,
                         L, idx, N, cps, nslices, rpc, sp, part, pcnt, lo, ctl);
    else
      hipLaunchKernelGGL((acc_kernel<G, VW, DPL, false, false>), grid, dim3(1024), lds, st, X,
                         M, L, idx, N, cps, nslices, rpc, sp, part, pcnt, lo, ctl);
  }
}

}  // namespace

void plan_afp(Carver& c, int64_t M, int64_t L, int64_t N, AfpWs* w, bool dslices, bool many,
              bool bds_ok) {
  w->cps = (int)std::min<int64_t>(std::min<int64_t>(N, 8192), kLdsBytes / (8 * (L + 1) + 4) - 1);
  w->nslices = (int)((N + w->cps - 1) / w->cps);
  // Dimension slices instead of several cell slices when all cells fit one
  // CU's LDS: one block per CU, 256 in all
  w->dslices = 0;
  if (dslices && w->nslices > 1 && L % kDs == 0 && accd_lds_bytes(N) <= (size_t)kAccdLdsMax) {
    w->dslices = (int)(L / kDs);
    w->nslices = 1;
    w->cps = (int)N;
  }
  // Partials at most half of X's bytes, at least one chunk per 256 rows
  // of work; one 1024-thread block per CU with a single slice (one wave of
  // blocks), about 512 blocks in all with several.
  int64_t nch = w->dslices ? std::max<int64_t>(8, 256 / w->dslices)
                           : (w->nslices == 1 ? 256 : std::max<int64_t>(1, 512 / w->nslices));
  nch = std::min<int64_t>(nch, std::max<int64_t>(1, M / (4 * N)));
  nch = std::min<int64_t>(nch, std::max<int64_t>(1, (M + 255) / 256));
  if (many) {
    // one of many instances updated together: the others fill the GPU, so
    // chunks of at least 2048 rows and partials at most 1/16 of X's bytes
    nch = std::min<int64_t>(nch, std::max<int64_t>(1, M / (32 * N)));
    nch = std::min<int64_t>(nch, std::max<int64_t>(1, M / 2048));
  }
  w->nchunks = (int)nch;
  w->rows_per_chunk = (M + nch - 1) / nch;
  // batched form: 16-dimension slices with every cell in at most 40 KiB of
  // LDS, so that four 256-thread workgroups share a CU
  w->bds = (many && bds_ok && L % kDs == 0 && accd_lds_bytes(N) <= (size_t)kBdsLdsMax)
               ? (int)(L / kDs)
               : 0;
  // the 32-bit slices: half as many slices of twice the width, twice the
  // chunks (the same blocks), their int32 partials in the same bytes
  w->nds_n = 0;
  w->nch_n = 0;
  if (w->dslices && L % kDn == 0 && accn_lds_bytes(N) <= (size_t)kAccdLdsMax) {
    w->nds_n = (int)(L / kDn);
    w->nch_n = (int)(nch * w->dslices / w->nds_n);
  }
  w->absmax_blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (M * L + 4095) / 4096));
  w->part = c.take<unsigned long long>((size_t)(nch * N * L));
  w->pcnt = c.take<int32_t>((size_t)(std::max<int64_t>(nch, w->nch_n) * N));
  w->amax = c.take<uint32_t>((size_t)(3 * w->absmax_blocks));
  w->shift = c.take<int>(5);
  w->lo = c.take<unsigned long long>((size_t)(N * L));
  w->nlo = N * L;
}

bool afp_usable(int64_t L, int64_t N) {
  const int cps = (int)std::min<int64_t>(std::min<int64_t>(N, 8192), kLdsBytes / (8 * (L + 1) + 4) - 1);
  return cps >= 1 && (N + cps - 1) / cps <= 32;
}

int launch_afp_shift(const float* X, int64_t M, int64_t L, const AfpWs& w, hipStream_t s) {
  hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)w.absmax_blocks), dim3(kT), 0, s, X, M * L,
                     w.amax, w.lo, w.nlo);
  LBG_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(shift_kernel, dim3(1), dim3(kT), 0, s, w.amax, w.absmax_blocks, M, w.shift);
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

int launch_afp(const float* X, int64_t M, int64_t L, const int32_t* idx, const float* C_old,
               int64_t N, float* C_out, int32_t* counts, int mode, double g2, const AfpWs& w,
               hipStream_t s, Ctl ctl, CbPair cbp, int on_grid) {
  const bool vec = (L % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  if (w.dslices && w.nds_n && on_grid == 2) {
    const dim3 grid((unsigned)(w.nch_n * w.nds_n));
    const size_t lds = accn_lds_bytes(N);
    int32_t* part32 = reinterpret_cast<int32_t*>(w.part);
#define LBG_ACCN(VV)                                                                            \
    {                                                                                           \
      static const hipError_t a = hipFuncSetAttribute(                                          \
          reinterpret_cast<const void*>(&accn_kernel<VV>),                                      \
          hipFuncAttributeMaxDynamicSharedMemorySize, kAccdLdsMax);                              \
      LBG_TRY_HIP(a);                                                                           \
      hipLaunchKernelGGL((accn_kernel<VV>), grid, dim3(kDsThreads), lds, s, X, M, (int)L, idx,  \
                         (int)N, w.nch_n, w.nds_n, w.shift, part32, w.pcnt, ctl);               \
    }
    if (vec) LBG_ACCN(true) else LBG_ACCN(false)
#undef LBG_ACCN
    LBG_TRY_HIP(hipGetLastError());
    return launch_fin(X, M, L, C_old, N, C_out, counts, mode, g2, w, s, ctl, cbp, true);
  }
  if (w.dslices) {
    const dim3 grid((unsigned)(w.nchunks * w.dslices));
    const size_t lds = accd_lds_bytes(N);
#define LBG_ACCD(GEN, VV)                                                                       \
    {                                                                                           \
      static const hipError_t a = hipFuncSetAttribute(                                          \
          reinterpret_cast<const void*>(&accd_kernel<GEN, VV>),                                 \
          hipFuncAttributeMaxDynamicSharedMemorySize, kAccdLdsMax);                              \
      LBG_TRY_HIP(a);                                                                           \
      hipLaunchKernelGGL((accd_kernel<GEN, VV>), grid, dim3(kDsThreads), lds, s, X, M, (int)L,  \
                         idx, (int)N, w.nchunks, w.dslices, w.rows_per_chunk, w.shift, w.part,  \
                         w.pcnt, w.lo, ctl);                                                    \
    }
    if (on_grid == 0) {
      if (vec) LBG_ACCD(true, true) else LBG_ACCD(true, false)
    } else {
      if (vec) LBG_ACCD(false, true) else LBG_ACCD(false, false)
    }
#undef LBG_ACCD
    LBG_TRY_HIP(hipGetLastError());
    return launch_fin(X, M, L, C_old, N, C_out, counts, mode, g2, w, s, ctl, cbp);
  }
  const int VW = vec ? 4 : 1;
  const int lanes = (int)((L + VW - 1) / VW);
  int G = 1;
  while (G < lanes && G < 64) G <<= 1;
  // several slices, 16-byte rows: four vectors per lane, so that a row's
  // bookkeeping is shared by sixteen coordinates
  if (w.nslices > 1 && vec && lanes >= 4 && lanes % 4 == 0) {
    G = 1;
    while (4 * G < lanes) G <<= 1;
  }
  const int DPL = (lanes + G - 1) / G;
  const dim3 grid((unsigned)(w.nchunks * w.nslices));
  const size_t lds = acc_lds_bytes(w.cps, L);
  const int n = (int)N, Li = (int)L;
#define LBG_ACC(GG, VV, DD)                                                                     \
  if (G == GG && VW == VV && DPL == DD) {                                                       \
    launch_acc<GG, VV, DD>(grid, lds, s, X, M, Li, idx, n, w.cps, w.nslices, w.rows_per_chunk, \
                           w.shift, w.part, w.pcnt, w.lo, ctl, on_grid == 0);                   \
  } else
  LBG_ACC(1, 4, 1) LBG_ACC(2, 4, 1) LBG_ACC(4, 4, 1) LBG_ACC(8, 4, 1) LBG_ACC(16, 4, 1)
  LBG_ACC(32, 4, 1) LBG_ACC(64, 4, 1)
  LBG_ACC(1, 4, 4) LBG_ACC(2, 4, 4) LBG_ACC(4, 4, 4) LBG_ACC(8, 4, 4) LBG_ACC(16, 4, 4)
  LBG_ACC(1, 1, 1) LBG_ACC(2, 1, 1) LBG_ACC(4, 1, 1) LBG_ACC(8, 1, 1) LBG_ACC(16, 1, 1)
  LBG_ACC(32, 1, 1) LBG_ACC(64, 1, 1) LBG_ACC(64, 1, 2) LBG_ACC(64, 1, 3) LBG_ACC(64, 1, 4) {
    set_error("internal: no accumulation kernel for G=%d VW=%d DPL=%d", G, VW, DPL);
    return LBG_EINVAL;
  }
#undef LBG_ACC
  LBG_TRY_HIP(hipGetLastError());
  return launch_fin(X, M, L, C_old, N, C_out, counts, mode, g2, w, s, ctl, cbp);
}

int launch_fin(const float* X, int64_t M, int64_t L, const float* C_old, int64_t N,
               float* C_out, int32_t* counts, int mode, double g2, const AfpWs& w,
               hipStream_t s, Ctl ctl, CbPair cbp, bool p32) {
  (void)X;
  (void)M;
  const int n = (int)N, Li = (int)L;
  const int nch = p32 ? w.nch_n : w.nchunks;
#define LBG_FIN(MM, PP)                                                                         \
  hipLaunchKernelGGL((fin_kernel<MM, PP>), dim3((unsigned)N), dim3(kT), 0, s, w.part, w.pcnt,  \
                     nch, n, Li, w.shift, C_old, C_out, counts, g2, w.lo, ctl, cbp)
  if (mode == 0) {
    if (p32) LBG_FIN(0, true); else LBG_FIN(0, false);
  } else {
    if (p32) LBG_FIN(1, true); else LBG_FIN(1, false);
  }
#undef LBG_FIN
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

}  // namespace lbg
