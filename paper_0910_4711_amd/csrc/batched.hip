// Batched LBG: many independent training runs (instances of uneven M, L and
// N), advanced together one Lloyd iteration per round (Algorithm 1 for every
// instance).  A round is three launches for all instances:
//
//   b_assign  persistent: workgroups take chunks of up to `grab` slots of
//             one instance from a queue (slot b = the tiles b, b + G, b + 2G,
//             ... of the single-run kernel's workgroup b), stage that
//             instance's codebook into LDS and run the allocation of those
//             tiles exactly as the single-run kernel does (same tiles, same
//             per-wave partial sums, so the same distortion), each wave
//             loading its next tile's rows while screening the current one.
//   b_acc     one workgroup per (instance, row chunk, cell slice): every
//             instance's decision from its own partials, then the fixed-point
//             cell sums (integers: exact, order-free).
//   b_fin     one workgroup per (instance, cell): centroid, or split, or
//             nothing; the instance's first workgroup commits its state.
//
// Each instance keeps its own device state, so instances stop and split
// independently; finished instances cost one state read per launch.  Results
// are bit-identical to lbg_train run on each instance alone.  The rounds are
// replayed from a hipGraph (or launched directly), and the host reads a
// finished-instance counter every few rounds.  The allocation's queue
// granularity and grid are chosen by timing candidates on the instances'
// final codebook sizes (autotuner, cached per workload signature).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "afp_common.h"
#include "assign_common.h"
#include "misc_common.h"

namespace lbg {
namespace {

using namespace assign_detail;

constexpr int kT = 256;
constexpr int kBatchTrace = 1024;      // distortion trace entries per instance
constexpr int kBatchLds = 81920;       // allocation LDS per workgroup (2 per CU)
constexpr int kRoundsPerGraph = 8;

// Device descriptor of one instance.
struct BInst {
  const float* X;
  int64_t M;
  int32_t L, LP, vec, N;
  float* Cb[2];
  float* C_out;
  int32_t* idx;
  DevState* st;
  DevState* pend;
  double* dpart;   // distortion partial per 32 vectors
  int64_t ntiles;  // row tiles of kRowsPerTile
  int32_t G;       // allocation slots: the single-run kernel's grid
  int32_t cps, nslices, nchunks, absmax_blocks, cnwg;
  int32_t bds;  // > 0: the update runs this many 16-dimension slices (b_accd_kernel)
  int64_t rows_per_chunk, crpb;
  unsigned long long* part;
  int32_t* pcnt;
  uint32_t* amax;
  int* shift;
  unsigned long long* lo;  // second-word sums of the update (N x L)
  double* cpart;
  double* Dtrace;
  int32_t* Atrace;
  unsigned long long* nfb;
  int32_t* counts;  // batched single steps: cell counts out (nullable)
  double* Dout;     // batched single steps: mean distortion out (nullable)
};

// Exclusive prefix sums of each launch's blocks (or items) over instances;
// for every family but the allocation items also a block -> instance table
// (offset tab_off[family] into one int32 array), so that a block finds its
// instance with one load.
enum { kPreItem, kPreAcc, kPreFin, kPreCol, kPreColFin, kPreAmax, kPreAccD, kNumPre };

struct Tabs {
  const int32_t* b2i;         // block -> instance, all families
  int64_t off[kNumPre];       // start of each family in b2i
};


// ------------------------------------------------------------- allocation --
// Slots [b0, b0 + cnt) of instance B: for each slot b the tiles b, b + G, ...
// and partials of the single-run kernel's workgroup b.  Each wave walks its
// rows of those tiles in order, loading the next tile's rows while the
// current one is screened.  The codebook is staged unless this workgroup
// staged the same one last.
template <class SC, bool VEC>
__device__ __forceinline__ void alloc_chunk(const BInst& B, const DevState* st, int b0, int cnt,
                                            int i, int* staged, unsigned char* smem) {
  constexpr int LP = SC::LP;
  constexpr bool PF = LP <= 32;
  typedef typename SC::elem E;
  E* sA = reinterpret_cast<E*>(smem);
  const int n = st->n, cb = st->cb;
  const float* C = B.Cb[cb];
  const int n_pad = (n + 31) & ~31;
  const int L = VEC ? LP : B.L;
  const int key = (((i << 1) | cb) << 1) | (SC::SPLIT ? 1 : 0);
  if (*staged != key) {
    __syncthreads();  // the previous chunk's waves are done with the LDS copy
    stage_from_C<SC, VEC>(C, n, L, n_pad, sA);
    *staged = key;
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const WaveCtx w = wave_ctx<SC>(L, tile_bits_of(n));
  const int G = B.G;
  const int64_t nt = B.ntiles;
  float xv[LP / 2];
  int b = b0;
  int64_t rt = b;
  if (PF) load_x<LP, VEC>(B.X, B.M, L, rt * kRowsPerTile + (int64_t)wave * 32, w.h, w.j, xv);
  for (;;) {
    // the tile after (b, rt): the slot's next tile, else the next slot's first
    int nb = b;
    int64_t nrt = rt + G;
    if (nrt >= nt) {
      nb = b + 1;
      nrt = nb;
    }
    const bool more = nb < b0 + cnt;
    const int64_t row0 = rt * kRowsPerTile + (int64_t)wave * 32;
    if (!PF) load_x<LP, VEC>(B.X, B.M, L, row0, w.h, w.j, xv);
    const int64_t next = (PF && more) ? nrt * kRowsPerTile + (int64_t)wave * 32 : -1;
    const double d = process_rows<SC, VEC, PF>(xv, B.X, B.M, L, row0, next, C, n, n_pad,
                                               n_pad, true, nullptr, sA, B.idx, nullptr,
                                               B.nfb, w);
    // the single-run kernel's partial of these 32 vectors
    const double ws = wave_sum(d);
    if (lane == 0 && row0 < B.M) B.dpart[row0 >> 5] = ws;
    if (!more) break;
    b = nb;
    rt = nrt;
  }
}

// Slots [b0, b0 + cnt) of instance B by direct FP64 search, for codebooks of
// at most kDirectN codevectors: per vector the FP64 squared distances in
// dimension order, the first smallest kept, and the partial of each 32
// vectors by the 32-lane butterfly of the single-run kernel's direct path.
// These are the screened path's numbers bit for bit (its FP64 rescore chains
// the same operations in the same order), so the choice changes no result.
// The two halves of a wave take consecutive tiles of the chunk's sequence
// (slot b's tiles b, b + G, ..., then slot b + 1's), 32 vectors each.  XD:
// the row is converted to FP64 once (registers) rather than per codevector.
template <int LP, bool VEC, bool XD>
__device__ __forceinline__ void direct_chunk(const BInst& B, const DevState* st, int b0, int cnt,
                                             int i, int* staged, unsigned char* smem) {
  const int n = st->n, cb = st->cb;
  const float* C = B.Cb[cb];
  const int L = VEC ? LP : B.L;
  double* sC = reinterpret_cast<double*>(smem);
  // the FP64 layout: never a screen layout's key (>= 0) nor "nothing staged" (-1)
  const int key = -2 - ((i << 1) | cb);
  if (*staged != key) {
    __syncthreads();  // the previous chunk's waves are done with the LDS copy
    for (int e = threadIdx.x; e < n * LP; e += kT) {
      const int k = e / LP, l = e - k * LP;
      sC[e] = l < L ? (double)C[(int64_t)k * L + l] : 0.0;
    }
    __syncthreads();
    *staged = key;
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int half = lane >> 5, j = lane & 31;
  const int G = B.G;
  const int64_t nt = B.ntiles;
  const int bend = b0 + cnt;
  int b = b0;
  int64_t rt = b0;
  auto advance = [&]() {
    rt += G;
    if (rt >= nt) {
      ++b;
      rt = b;
    }
  };
  if (half) advance();
  for (;;) {
    const bool valid = b < bend;
    const int64_t row0 = rt * kRowsPerTile + (int64_t)wave * 32;
    const int64_t m = row0 + j;
    const bool live = valid && m < B.M;
    float xr[LP];
    if (live) {
      load_row<LP, VEC>(B.X + m * (int64_t)L, L, xr);
    } else {
#pragma unroll
      for (int q = 0; q < LP; ++q) xr[q] = 0.0f;
    }
    double xd[XD ? LP : 1];
    if constexpr (XD) {
#pragma unroll
      for (int q = 0; q < LP; ++q) xd[q] = (double)xr[q];
    }
    double best = INFINITY;
    int bi = 0x7fffffff;
    for (int k = 0; k < n; ++k) {
      const double* c = sC + k * LP;
      double dk = 0.0;
#pragma unroll
      for (int l = 0; l < LP; ++l) {
        if (l < L) {
          const double t = (XD ? xd[l] : (double)xr[l]) - c[l];
          dk = dk + t * t;
        }
      }
      if (dk < best) {
        best = dk;
        bi = k;
      }
    }
    if (!(best < INFINITY)) bi = 0;  // no finite distance: index 0
    if (live) B.idx[m] = bi;
    double v = live ? best : 0.0;
    v += xor_lane<1>(v);
    v += xor_lane<2>(v);
    v += xor_lane<4>(v);
    v += xor_lane<8>(v);
    v += xor_lane<16>(v);
    if (j == 0 && valid && row0 < B.M) B.dpart[row0 >> 5] = v;
    advance();
    advance();
    // half 0 holds the earlier tile: the wave is done when it has none
    if (__builtin_amdgcn_readfirstlane(b) >= bend) break;
  }
}

// Split screen for the current codebook: chosen (split != 0) and its row
// layout fits the workgroup's LDS.
template <int LP>
__device__ __forceinline__ bool split_fits(int n) {
  const int n_pad = (n + 31) & ~31;
  return n_pad * Bf16x3Screen<LP>::S * Bf16x3Screen<LP>::ESZ <= kBatchLds;
}

// Persistent: workgroups take chunks (instance, first slot, slot count) from
// the queue until none is left.  Two builds, each with its own queue:
//   SPLIT = false: codebooks of at most kDirectN codevectors (direct search)
//     and, unless ``split``, every other codebook with the FP32 screen;
//   SPLIT = true (launched only when ``split``): the instances with rows of
//     exactly 64 aligned floats whose split BF16 screen layout fits the
//     workgroup's LDS (others keep the FP32 screen: shorter rows' tiles are
//     cheap either way, and a build for several row forms spills registers).
// With ``split`` each build skips the other's chunks, so every chunk is
// allocated once per round.  The split screen is FP32-accurate with the same
// exact certificate as the FP32 screen: the allocation and partials are the
// same whichever build takes a chunk.  (One kernel holding both screens spills
// registers; two keep each at the single-run kernel's register use.)
template <bool SPLIT>
__global__ __launch_bounds__(kT, 2) void b_assign_kernel(const BInst* __restrict__ inst,
                                                         const int32_t* __restrict__ chunks,
                                                         int nchunks, unsigned* __restrict__ qctr,
                                                         int split) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int s_c;
  int staged = -1;
  for (;;) {
    __syncthreads();  // s_c of the previous access has been read
    if (threadIdx.x == 0) s_c = (int)atomicAdd(qctr, 1u);
    __syncthreads();
    const int c = s_c;
    if (c >= nchunks) break;
    const int i = chunks[3 * c], b0 = chunks[3 * c + 1], cnt = chunks[3 * c + 2];
    const BInst& B = inst[i];
    const DevState* st = B.st;
    if (st->done) continue;
    const int n = st->n;
    const bool direct = n <= kDirectN;
    const bool sp = split && !direct && B.LP == 64 && B.vec && split_fits<64>(n);
    if (sp != SPLIT) continue;  // the other build's chunk
    if constexpr (SPLIT) {
      alloc_chunk<Bf16x3Screen<64>, true>(B, st, b0, cnt, i, &staged, smem);
    } else if (direct) {
      if (B.LP == 16) {
        if (B.vec)
          direct_chunk<16, true, true>(B, st, b0, cnt, i, &staged, smem);
        else
          direct_chunk<16, false, true>(B, st, b0, cnt, i, &staged, smem);
      } else {
        if (B.vec)
          direct_chunk<64, true, false>(B, st, b0, cnt, i, &staged, smem);
        else
          direct_chunk<64, false, false>(B, st, b0, cnt, i, &staged, smem);
      }
    } else {
      if (B.LP == 16) {
        if (B.vec)
          alloc_chunk<Fp32Screen<16>, true>(B, st, b0, cnt, i, &staged, smem);
        else
          alloc_chunk<Fp32Screen<16>, false>(B, st, b0, cnt, i, &staged, smem);
      } else {
        if (B.vec)
          alloc_chunk<Fp32Screen<64>, true>(B, st, b0, cnt, i, &staged, smem);
        else
          alloc_chunk<Fp32Screen<64>, false>(B, st, b0, cnt, i, &staged, smem);
      }
    }
  }
}

// ----------------------------------------------------------------- update --
// The round's finish work list: the cells of every instance still running
// (st[i].done clear) below the pending state's n_src, at least cell 0 (which
// commits the state), compacted; b_fin walks it.  One workgroup of 1024
// threads, run after the decisions (b_acc) are made.  st, pend: the
// instances' states, contiguous.  list[item] = instance, first[i] = its first
// item, *total = the number of items.
__global__ __launch_bounds__(1024) void b_list_kernel(const DevState* __restrict__ st,
                                                     const DevState* __restrict__ pend,
                                                     const BInst* __restrict__ inst, int n_inst,
                                                     int32_t* __restrict__ list,
                                                     int32_t* __restrict__ first,
                                                     int32_t* __restrict__ total) {
  __shared__ int32_t ssum[1024];
  __shared__ int32_t sbase;
  const int t = threadIdx.x;
  if (t == 0) sbase = 0;
  for (int i0 = 0; i0 < n_inst; i0 += 1024) {
    const int i = i0 + t;
    int c = 0;
    if (i < n_inst) {
      const int done = st[i].done, n_src = pend[i].n_src, N = inst[i].N;
      if (!done) c = max(1, min(N, n_src));
    }
    ssum[t] = c;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan
      const int v = t >= off ? ssum[t - off] : 0;
      __syncthreads();
      ssum[t] += v;
      __syncthreads();
    }
    const int f = sbase + ssum[t] - c;
    if (i < n_inst) first[i] = f;
    // the batch's items spread over the threads: item v belongs to the
    // first instance whose inclusive count exceeds v (one instance's cells
    // written by one thread had left the list bound by its longest run)
    const int base = sbase, Q = ssum[1023];
    for (int v = t; v < Q; v += 1024) {
      int lo = 0, hi = 1023;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ssum[mid] > v)
          hi = mid;
        else
          lo = mid + 1;
      }
      list[base + v] = i0 + lo;
    }
    __syncthreads();  // every thread has read sbase and ssum
    if (t == 1023) sbase = f + c;
    __syncthreads();
  }
  if (t == 0) *total = sbase;
}

// The fixed-point cell sums of instance B's row chunk x cell slice
// ``local`` for a codebook of N cells.
__device__ __forceinline__ void acc_cells(const BInst& B, int N, int64_t local,
                                          unsigned long long* sacc, int32_t* slist,
                                          int32_t& snsel) {
  // Slices of cps cells the current codebook needs (the launch has the final
  // codebook's): the workgroups of the others have nothing to add, and one
  // slice streams the rows instead of gathering them per slice.  The
  // partials keep the planned layout (cells of slice q from q cps).
  const int nsl = max(1, (N + B.cps - 1) / B.cps);
  const int64_t chunk = local / B.nslices;
  const int slice = (int)(local % B.nslices);
  if (slice >= nsl) return;
  const int64_t blk = chunk * nsl + slice;
  const int s = B.shift[0], tf = B.shift[1];
  const int L = B.L;
#define LBG_BACC1(GG, VV, FF)                                                                 \
  do {                                                                                     \
    if (nsl > 1)                                                                           \
      afp::acc_body<GG, VV, 1, true, 8, kT, FF>(B.X, B.M, L, B.idx, N, B.N, B.cps, nsl,     \
                                                B.rows_per_chunk, s, B.part, B.pcnt, blk,  \
                                                sacc, slist, snsel, B.lo, tf);             \
    else                                                                                   \
      afp::acc_body<GG, VV, 1, false, afp::kUnrollSel, kT, FF>(                            \
          B.X, B.M, L, B.idx, N, B.N, B.cps, 1, B.rows_per_chunk, s, B.part, B.pcnt, blk,   \
          sacc, slist, snsel, B.lo, tf);                                                   \
  } while (0)
#define LBG_BACC(GG, VV)        \
  do {                          \
    if (tf > 0)                 \
      LBG_BACC1(GG, VV, true);  \
    else                        \
      LBG_BACC1(GG, VV, false); \
  } while (0)
  if (B.vec && (L & 3) == 0) {
    const int lanes = L / 4;
    if (lanes <= 1)
      LBG_BACC(1, 4);
    else if (lanes <= 2)
      LBG_BACC(2, 4);
    else if (lanes <= 4)
      LBG_BACC(4, 4);
    else if (lanes <= 8)
      LBG_BACC(8, 4);
    else
      LBG_BACC(16, 4);
  } else {
    if (L <= 1)
      LBG_BACC(1, 1);
    else if (L <= 2)
      LBG_BACC(2, 1);
    else if (L <= 4)
      LBG_BACC(4, 1);
    else if (L <= 8)
      LBG_BACC(8, 1);
    else if (L <= 16)
      LBG_BACC(16, 1);
    else if (L <= 32)
      LBG_BACC(32, 1);
    else
      LBG_BACC(64, 1);
  }
#undef LBG_BACC
#undef LBG_BACC1
}

// One workgroup's share of instance B's update: its decision (local 0),
// then the fixed-point cell sums of row chunk x cell slice ``local``.
__device__ __forceinline__ void acc_item(const BInst& B, int64_t local, unsigned long long* sacc,
                                         int32_t* slist, int32_t& snsel) {
  const Ctl ctl{B.st, B.pend, B.dpart, (B.M + 31) / 32, B.Dtrace, B.Atrace};
  int N = B.N;
  if (B.st->done) return;
  if (local == 0) (void)afp::acc_decide(ctl, true, &N);  // the instance's decision
  if (forced_stop(B.st)) return;  // the level ends here: no update follows
  acc_cells(B, B.st->n, local, sacc, slist, snsel);
}

// One workgroup per (instance, row chunk, cell slice) of every instance; the
// workgroups of finished instances leave at once.  (A persistent form over a
// compacted list of the running instances' workgroups measured slower: the
// list costs a launch and the loop more registers.)
__global__ __launch_bounds__(kT) void b_acc_kernel(const BInst* __restrict__ inst, int n_inst,
                                                   const int64_t* __restrict__ pre, Tabs tb) {
  extern __shared__ unsigned long long sacc[];
  __shared__ int32_t slist[afp::kSel];
  __shared__ int32_t snsel;
  const int64_t* acc_pre = pre + (int64_t)kPreAcc * (n_inst + 1);
  if ((int64_t)blockIdx.x >= acc_pre[n_inst]) return;
  const int i = tb.b2i[tb.off[kPreAcc] + blockIdx.x];
  acc_item(inst[i], (int64_t)blockIdx.x - acc_pre[i], sacc, slist, snsel);
}

// The update of the instances planned with 16-dimension slices (all their
// cells' sums for 16 dimensions in at most 40 KiB of LDS): one workgroup
// per (instance, row chunk, slice), each adding a 64-byte slice of every row
// of its chunk, no filtering by cell; the instance's decision in its
// workgroup 0.  Its own kernel, so that its registers and LDS (four
// workgroups per CU) are not those of the cell-slice path.
__global__ __launch_bounds__(kT) void b_accd_kernel(const BInst* __restrict__ inst, int n_inst,
                                                    const int64_t* __restrict__ pre, Tabs tb) {
  extern __shared__ unsigned long long sacc[];
  const int64_t* p = pre + (int64_t)kPreAccD * (n_inst + 1);
  if ((int64_t)blockIdx.x >= p[n_inst]) return;
  // the last instances first: the allocation before took the instances in
  // order, so their rows are the ones the memory-side cache still holds
  // (and the next allocation starts on the rows read last here)
  const int64_t bx = p[n_inst] - 1 - (int64_t)blockIdx.x;
  const int i = tb.b2i[tb.off[kPreAccD] + bx];
  const BInst& B = inst[i];
  const int64_t local = bx - p[i];
  const Ctl ctl{B.st, B.pend, B.dpart, (B.M + 31) / 32, B.Dtrace, B.Atrace};
  int N = B.N;
  if (B.st->done) return;
  if (local == 0) (void)afp::acc_decide(ctl, true, &N);  // the instance's decision
  if (forced_stop(B.st)) return;  // the level ends here: no update follows
  const int n = B.st->n;
  const int chunk = (int)(local / B.bds), q = (int)(local % B.bds);
  const int s = B.shift[0], tf = B.shift[1];
#define LBG_BACCD(FF, VV)                                                                   \
  afp::accd_body<FF, VV, kT>(B.X, B.M, B.L, B.idx, n, B.N, B.rows_per_chunk, chunk, q, s,  \
                             B.part, B.pcnt, sacc, B.lo, tf)
  if (B.vec) {
    if (tf > 0)
      LBG_BACCD(true, true);
    else
      LBG_BACCD(false, true);
  } else {
    if (tf > 0)
      LBG_BACCD(true, false);
    else
      LBG_BACCD(false, false);
  }
#undef LBG_BACCD
}

// Cell k of instance B by one 64-lane wave: centroid, or split, or nothing;
// cell 0 commits the state.  The same work and results, bit for bit, as
// afp::fin_state with afp::fin_body<0> (one 256-thread workgroup per cell,
// the single run's finish): the pending state's action, the state words
// copied by the commit, the residual sums read and cleared whatever the
// decision, integer sums of the chunk partials (their order immaterial) and
// the same rounding.  A round's cells are many and small here (at most 64
// dimensions, a few chunks each), so each workgroup keeps four cells in
// flight; one cell per workgroup left the finish bound by the round trips
// of 2,048 cells at a time.  (The work list holds only cells below the
// pending n_src of instances still running.)
__device__ __forceinline__ void fin_item_wave(const BInst& B, int k, unsigned* __restrict__ ndone) {
  constexpr int NW = (int)(sizeof(DevState) / 4);
  constexpr int NWL = (NW + 63) / 64;  // state words per lane
  constexpr int U = 16;                // partial words in flight per lane
  static_assert(sizeof(DevState) % 4 == 0, "state words");
  const int lane = threadIdx.x & 63;
  const int L = B.L, ns = B.N, nch = B.nchunks;
  const int s = B.shift[0], tf = B.shift[1];
  const bool fine = B.lo != nullptr && tf > 0;
  const bool lead = k == 0;
  const DevState* pd = B.pend;
  const bool on = lane < L;  // lane d takes dimension d (L <= 64)
  // loads issued together: the commit's words, the residual, the first
  // partials and the counts, then the state
  uint32_t word[NWL];
#pragma unroll
  for (int j = 0; j < NWL; ++j) {
    const int w = lane + 64 * j;
    word[j] = (lead && w < NW) ? reinterpret_cast<const uint32_t*>(pd)[w] : 0u;
  }
  long long slo = 0;
  if (fine && on) {
    unsigned long long* p = B.lo + (int64_t)k * L + lane;
    slo = (long long)*p;
    *p = 0ull;
  }
  unsigned long long a[U];
  auto load_u = [&](int ch0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ch = ch0 + u;
      a[u] = (on && ch < nch) ? B.part[((int64_t)ch * ns + k) * L + lane] : 0ull;
    }
  };
  load_u(0);
  long long c = 0;
  for (int ch = lane; ch < nch; ch += 64) c += B.pcnt[(int64_t)ch * ns + k];
  const int done = B.st->done;
  const int action = pd->action, n_src = pd->n_src, src = pd->src, dst = pd->dst;
  if (done) return;
  if (lead) {
#pragma unroll
    for (int j = 0; j < NWL; ++j) {
      const int w = lane + 64 * j;
      if (w < NW) reinterpret_cast<uint32_t*>(B.st)[w] = word[j];
    }
    if (ndone && lane == 0 && pd->done) atomicAdd(ndone, 1u);
  }
  if (action == kActSplit) {
    // Codebook Splitting of codevector k: children 2k ("+") and 2k+1 ("-")
    if (k >= n_src || !on) return;
    misc::split_pair(B.Cb[src][k * L + lane], pd->split_mode, pd->eps, pd->delta,
                     &B.Cb[dst][(2 * k) * L + lane], &B.Cb[dst][(2 * k + 1) * L + lane]);
    return;
  }
  if (action != kActUpdate || k >= n_src) return;
  const float* C_old = B.Cb[src];
  float* out = B.Cb[dst];
  unsigned long long acc = 0ull;
  for (int ch0 = U;; ch0 += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) acc += a[u];
    if (ch0 >= nch) break;
    load_u(ch0);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
  if (!on) return;
  const int64_t e = (int64_t)k * L + lane;
  if (c == 0) {
    if (out != C_old) out[e] = C_old[e];
  } else {
    const long long S = (long long)acc;
    const double low = fine ? ldexp((double)slo, -(s + tf)) : 0.0;
    out[e] = (float)((ldexp((double)S, -s) + low) / (double)c);
  }
}

// Persistent over the round's finish list (b_list_kernel), a cell per
// wave.  Block 0 also rearms the allocation queues (qctr[0] and qctr[2])
// for the next round (the round's allocation has completed before this
// launch starts).
__global__ __launch_bounds__(kT) void b_fin_kernel(const BInst* __restrict__ inst,
                                                   const int32_t* __restrict__ list,
                                                   const int32_t* __restrict__ first,
                                                   const int32_t* __restrict__ total,
                                                   unsigned* __restrict__ qctr,
                                                   unsigned* __restrict__ ndone) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    qctr[0] = 0u;
    qctr[2] = 0u;
  }
  constexpr int W = kT / 64;
  const int T = *total;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int item = blockIdx.x * W + wave; item < T; item += gridDim.x * W) {
    const int i = list[item];
    fin_item_wave(inst[i], item - first[i], ndone);
  }
}

// ------------------------------------------------------------- set-up, end --
// The set-up pass of every instance (the single run's setup_pass_kernel,
// the same blocks): its column-sum partials and, from the same loads, the
// block maxima that fix its fixed-point shift (b_shift_kernel), the update's
// second-word sums cleared.  One read of X; a column-sum pass and a
// separate maxima pass over X took 775 + 522 us on the 512-instance set.
__global__ __launch_bounds__(kT) void b_setup_kernel(const BInst* __restrict__ inst, int n_inst,
                                                     const int64_t* __restrict__ pre, Tabs tb) {
  const int64_t* p = pre + (int64_t)kPreCol * (n_inst + 1);
  if ((int64_t)blockIdx.x >= p[n_inst]) return;
  const int i = tb.b2i[tb.off[kPreCol] + blockIdx.x];
  const BInst& B = inst[i];
  afp::setup_pass_body(B.X, B.M, B.L, B.crpb, B.cpart, B.amax, B.cnwg,
                       (int64_t)blockIdx.x - p[i], B.lo, (int64_t)B.N * B.L);
}

// Column d of instance i's centroid into Cb[0]; with N > 1 also its split
// into rows 0 ("+") and 1 ("-") of Cb[1] (the split kernel's arithmetic on
// the stored centroid).
__global__ __launch_bounds__(kT) void b_centroid_kernel(const BInst* __restrict__ inst,
                                                        int n_inst,
                                                        const int64_t* __restrict__ pre, Tabs tb,
                                                        int split_mode, double eps,
                                                        double delta) {
  const int64_t* p = pre + (int64_t)kPreColFin * (n_inst + 1);
  if ((int64_t)blockIdx.x >= p[n_inst]) return;
  const int i = tb.b2i[tb.off[kPreColFin] + blockIdx.x];
  const BInst& B = inst[i];
  const int d = (int)((int64_t)blockIdx.x - p[i]);
  misc::colsum_final_body(B.cpart, B.cnwg, B.L, B.M, B.Cb[0], d);
  if (threadIdx.x == 0 && B.N > 1)
    misc::split_pair(B.Cb[0][d], split_mode, eps, delta, &B.Cb[1][d], &B.Cb[1][B.L + d]);
}

__global__ __launch_bounds__(kT) void b_absmax_kernel(const BInst* __restrict__ inst, int n_inst,
                                                      const int64_t* __restrict__ pre, Tabs tb) {
  const int64_t* p = pre + (int64_t)kPreAmax * (n_inst + 1);
  if ((int64_t)blockIdx.x >= p[n_inst]) return;
  const int i = tb.b2i[tb.off[kPreAmax] + blockIdx.x];
  const BInst& B = inst[i];
  afp::absmax_body(B.X, B.M * B.L, B.amax, (int64_t)blockIdx.x - p[i], B.absmax_blocks, B.lo,
                   (int64_t)B.N * B.L);
}

// setup: the maxima come from b_setup_kernel (cnwg blocks), else from
// b_absmax_kernel (absmax_blocks blocks).
__global__ __launch_bounds__(kT) void b_shift_kernel(const BInst* __restrict__ inst, int setup) {
  const BInst& B = inst[blockIdx.x];
  afp::shift_body(B.amax, setup ? B.cnwg : B.absmax_blocks, B.M, B.shift);
}

// Row k of every instance's current codebook into its C_out.
__global__ __launch_bounds__(kT) void b_output_kernel(const BInst* __restrict__ inst, int n_inst,
                                                      const int64_t* __restrict__ pre, Tabs tb) {
  const int64_t* p = pre + (int64_t)kPreFin * (n_inst + 1);
  if ((int64_t)blockIdx.x >= p[n_inst]) return;
  const int i = tb.b2i[tb.off[kPreFin] + blockIdx.x];
  const BInst& B = inst[i];
  const int64_t k = (int64_t)blockIdx.x - p[i];
  const float* src = B.Cb[B.st->cb];
  for (int d = threadIdx.x; d < B.L; d += kT) B.C_out[k * B.L + d] = src[k * B.L + d];
}

// Autotuning set-up: every instance at its final codebook size, codevector k
// = training vector k mod M (allocation only; the states are set again
// before the run).
__global__ __launch_bounds__(kT) void b_tune_setup_kernel(const BInst* __restrict__ inst,
                                                          int n_inst,
                                                          const int64_t* __restrict__ pre, Tabs tb) {
  const int64_t* p = pre + (int64_t)kPreFin * (n_inst + 1);
  if ((int64_t)blockIdx.x >= p[n_inst]) return;
  const int i = tb.b2i[tb.off[kPreFin] + blockIdx.x];
  const BInst& B = inst[i];
  const int64_t k = (int64_t)blockIdx.x - p[i];
  const float* src = B.X + (k % B.M) * B.L;
  for (int d = threadIdx.x; d < B.L; d += kT) B.Cb[0][k * B.L + d] = src[d];
  if (k == 0 && threadIdx.x == 0) {
    B.st->n = B.N;
    B.st->cb = 0;
    B.st->done = 0;
  }
}

// ------------------------------------------------- batched single steps --
// Item i's mean distortion from its allocation partials (one per 32 rows), in
// the order of the single-call reduction (thread t adds partials t, t + 256,
// ... in index order, 32 loads in flight, then a tree over the threads), so
// that it equals lbg_assign_distortion's D bit for bit.  One workgroup per
// item; items without an output pointer are skipped.
__global__ __launch_bounds__(kT) void b_reduce_kernel(const BInst* __restrict__ inst) {
  constexpr int RB = 32;
  __shared__ double sred[kT];
  const BInst& B = inst[blockIdx.x];
  if (!B.Dout) return;
  const int64_t nparts = (B.M + 31) / 32;
  const double* parts = B.dpart;
  double acc = 0.0;
  int64_t p = threadIdx.x;
  for (; p + (int64_t)(RB - 1) * kT < nparts; p += (int64_t)RB * kT) {
    double v[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) v[b] = parts[p + (int64_t)b * kT];
#pragma unroll
    for (int b = 0; b < RB; ++b) acc += v[b];
  }
  for (; p < nparts; p += kT) acc += parts[p];
  sred[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sred[threadIdx.x] += sred[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *B.Dout = sred[0] / (double)B.M;
}

// Codebook Updation of many items without run state: the cell sums of every
// item's chunk x slice workgroups (the item's N cells) ...
__global__ __launch_bounds__(kT) void b_upd_acc_kernel(const BInst* __restrict__ inst, int n_inst,
                                                       const int64_t* __restrict__ pre, Tabs tb) {
  extern __shared__ unsigned long long sacc[];
  __shared__ int32_t slist[afp::kSel];
  __shared__ int32_t snsel;
  const int64_t* acc_pre = pre + (int64_t)kPreAcc * (n_inst + 1);
  if ((int64_t)blockIdx.x >= acc_pre[n_inst]) return;
  const int i = tb.b2i[tb.off[kPreAcc] + blockIdx.x];
  const BInst& B = inst[i];
  acc_cells(B, B.N, (int64_t)blockIdx.x - acc_pre[i], sacc, slist, snsel);
}

// ... or, for the items planned with 16-dimension slices, one workgroup per
// (item, row chunk, slice), as b_accd_kernel without run state.
__global__ __launch_bounds__(kT) void b_upd_accd_kernel(const BInst* __restrict__ inst,
                                                        int n_inst,
                                                        const int64_t* __restrict__ pre,
                                                        Tabs tb) {
  extern __shared__ unsigned long long sacc[];
  const int64_t* p = pre + (int64_t)kPreAccD * (n_inst + 1);
  if ((int64_t)blockIdx.x >= p[n_inst]) return;
  const int i = tb.b2i[tb.off[kPreAccD] + blockIdx.x];
  const BInst& B = inst[i];
  const int64_t local = (int64_t)blockIdx.x - p[i];
  const int chunk = (int)(local / B.bds), q = (int)(local % B.bds);
  const int s = B.shift[0], tf = B.shift[1];
#define LBG_BUACCD(FF, VV)                                                                  \
  afp::accd_body<FF, VV, kT>(B.X, B.M, B.L, B.idx, B.N, B.N, B.rows_per_chunk, chunk, q, s, \
                             B.part, B.pcnt, sacc, B.lo, tf)
  const bool vec = B.vec && (B.L & 3) == 0;
  if (vec) {
    if (tf > 0)
      LBG_BUACCD(true, true);
    else
      LBG_BUACCD(false, true);
  } else {
    if (tf > 0)
      LBG_BUACCD(true, false);
    else
      LBG_BUACCD(false, false);
  }
#undef LBG_BUACCD
}

// ... then every item's centroids (one cell per 64-lane wave; an empty cell
// keeps C_old, Cb[0]) into C_out, with the counts: fin_body<0>'s results
// bit for bit (integer sums of the chunk partials, the same rounding), as
// fin_item_wave forms them in the training rounds.
__global__ __launch_bounds__(kT) void b_upd_fin_kernel(const BInst* __restrict__ inst, int n_inst,
                                                       const int64_t* __restrict__ pre, Tabs tb) {
  constexpr int U = 16;  // partial words in flight per lane
  const int64_t* fin_pre = pre + (int64_t)kPreFin * (n_inst + 1);
  const int64_t g = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
  if (g >= fin_pre[n_inst]) return;
  const int i = tb.b2i[tb.off[kPreFin] + g];
  const BInst& B = inst[i];
  const int k = (int)(g - fin_pre[i]);
  const int lane = threadIdx.x & 63;
  const int L = B.L, ns = B.N, nch = B.nchunks;
  const int s = B.shift[0], tf = B.shift[1];
  const bool fine = B.lo != nullptr && tf > 0;
  const bool on = lane < L;  // lane d takes dimension d (L <= 64)
  long long slo = 0;
  if (fine && on) {
    unsigned long long* p = B.lo + (int64_t)k * L + lane;
    slo = (long long)*p;
    *p = 0ull;
  }
  unsigned long long acc = 0ull;
  for (int ch0 = 0; ch0 < nch; ch0 += U) {
    unsigned long long a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ch = ch0 + u;
      a[u] = (on && ch < nch) ? B.part[((int64_t)ch * ns + k) * L + lane] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += a[u];
  }
  long long c = 0;
  for (int ch = lane; ch < nch; ch += 64) c += B.pcnt[(int64_t)ch * ns + k];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
  if (B.counts && lane == 0) B.counts[k] = (int32_t)c;
  if (!on) return;
  const float* C_old = B.Cb[0];
  float* out = B.C_out;
  const int64_t e = (int64_t)k * L + lane;
  if (c == 0) {
    if (out != C_old) out[e] = C_old[e];
  } else {
    const long long S = (long long)acc;
    const double low = fine ? ldexp((double)slo, -(s + tf)) : 0.0;
    out[e] = (float)((ldexp((double)S, -s) + low) / (double)c);
  }
}

// ---------------------------------------------------------------- planning --
struct InstPlan {
  int LP, vec, G, cnwg;
  int64_t ntiles, crpb;
  AfpWs afp;
  float* Cb[2];
  double* dpart;
  double* cpart;
  double* Dtrace;
  int32_t* Atrace;
};

struct BatchWs {
  BInst* inst;      // device descriptors
  int64_t* pre;     // kNumPre x (n + 1)
  DevState* st;     // n
  DevState* pend;   // n
  unsigned* ctr;    // [0] allocation queue, [1] finished instances, [2] split queue
  unsigned long long* nfb;  // n
  int32_t* b2i;             // block -> instance tables
  int64_t b2i_n;
  int32_t* chunks;          // allocation chunks (instance, first slot, slots)
  int32_t* fin_list;        // the round's finish work list (b_list_kernel)
  int32_t* fin_first;       // n
  int32_t* list_total;      // its item count
  int64_t tot[kNumPre];     // blocks (items) of each family
  std::vector<InstPlan> plans;
};

// Blocks (allocation items) of each launch family for one instance.
void family_counts(const InstPlan& q, int64_t N, int64_t L, int64_t cnt[kNumPre]) {
  cnt[kPreItem] = q.G;
  cnt[kPreAcc] = q.afp.bds ? 0 : (int64_t)q.afp.nchunks * q.afp.nslices;
  cnt[kPreFin] = N;
  cnt[kPreCol] = q.cnwg;
  cnt[kPreColFin] = L;
  cnt[kPreAmax] = q.afp.absmax_blocks;
  cnt[kPreAccD] = q.afp.bds ? (int64_t)q.afp.nchunks * q.afp.bds : 0;
}

int lp_of(int64_t L) { return L <= 16 ? 16 : 64; }

// Slots of the single-run allocation kernel for this instance.
int slots_of(int64_t M, int64_t L) {
  const int64_t tiles = (M + kRowsPerTile - 1) / kRowsPerTile;
  int64_t cap;
  switch (padded_dim(L)) {
    case 8: cap = persist_blocks<Fp32Screen<8>>(); break;
    case 16: cap = persist_blocks<Fp32Screen<16>>(); break;
    case 32: cap = persist_blocks<Fp32Screen<32>>(); break;
    case 64: cap = persist_blocks<Fp32Screen<64>>(); break;
    default: cap = persist_blocks<Fp32Screen<128>>(); break;
  }
  return (int)std::min<int64_t>(tiles, cap);
}

void plan_batch(Carver& c, const lbg_instance* in, int n, BatchWs* w) {
  w->inst = c.take<BInst>((size_t)n);
  w->pre = c.take<int64_t>((size_t)kNumPre * (n + 1));
  w->st = c.take<DevState>((size_t)n);
  w->pend = c.take<DevState>((size_t)n);
  w->ctr = c.take<unsigned>(3);
  w->nfb = c.take<unsigned long long>((size_t)n);
  w->plans.resize((size_t)n);
  for (int i = 0; i < n; ++i) {
    InstPlan& q = w->plans[(size_t)i];
    const int64_t M = in[i].M, L = in[i].L, N = in[i].N;
    q.LP = lp_of(L);
    q.vec = (L == q.LP) && ((reinterpret_cast<uintptr_t>(in[i].X) & 15) == 0);
    q.ntiles = (M + kRowsPerTile - 1) / kRowsPerTile;
    q.G = slots_of(M, L);
    q.cnwg = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (M + 255) / 256));
    q.crpb = (M + q.cnwg - 1) / q.cnwg;
    q.Cb[0] = c.take<float>((size_t)(N * L));
    q.Cb[1] = c.take<float>((size_t)(N * L));
    q.dpart = c.take<double>((size_t)((M + 31) / 32));
    q.cpart = c.take<double>((size_t)(q.cnwg * L));
    q.Dtrace = c.take<double>(kBatchTrace);
    q.Atrace = c.take<int32_t>(kBatchTrace);
    plan_afp(c, M, L, N, &q.afp, false, true, true);
    // the set-up pass writes the maxima of its cnwg blocks there
    if (q.cnwg > q.afp.absmax_blocks) q.afp.amax = c.take<uint32_t>((size_t)(3 * q.cnwg));
  }
  for (int k = 0; k < kNumPre; ++k) w->tot[k] = 0;
  for (int i = 0; i < n; ++i) {
    int64_t cnt[kNumPre];
    family_counts(w->plans[(size_t)i], in[i].N, in[i].L, cnt);
    for (int k = 0; k < kNumPre; ++k) w->tot[k] += cnt[k];
  }
  w->b2i_n = 0;
  for (int k = 0; k < kNumPre; ++k)
    if (k != kPreItem) w->b2i_n += w->tot[k];
  w->b2i = c.take<int32_t>((size_t)w->b2i_n);
  w->chunks = c.take<int32_t>((size_t)(3 * w->tot[kPreItem]));
  w->fin_list = c.take<int32_t>((size_t)w->tot[kPreFin]);
  w->fin_first = c.take<int32_t>((size_t)n);
  w->list_total = c.take<int32_t>(1);
}

// Allocation chunks of at most ``grab`` slots, never spanning two instances,
// in instance order.  Returns their number.
int build_chunks(const std::vector<InstPlan>& plans, int grab, int32_t* out) {
  int nc = 0;
  for (size_t i = 0; i < plans.size(); ++i)
    for (int b0 = 0; b0 < plans[i].G; b0 += grab) {
      out[3 * nc] = (int32_t)i;
      out[3 * nc + 1] = b0;
      out[3 * nc + 2] = std::min(grab, plans[i].G - b0);
      ++nc;
    }
  return nc;
}

// Pinned host staging for the descriptors and states of one call.
unsigned char* pinned_stage(size_t bytes) {
  static thread_local unsigned char* p = nullptr;
  static thread_local size_t have = 0;
  if (have < bytes) {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    have = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(&p), bytes, hipHostMallocDefault) != hipSuccess)
      return nullptr;
    have = bytes;
  }
  return p;
}

struct Launch {
  const BInst* inst;
  int n;
  const int64_t* pre;
  Tabs tb;
  int64_t blocks[kNumPre];  // totals
  unsigned* ctr;
  size_t acc_lds, accd_lds;
  const int32_t* chunks;    // device chunk table for the current grab
  int nchunks;
  const DevState* st;       // the instances' states (contiguous)
  const DevState* pend;
  int32_t* fin_list;        // finish work list (b_list_kernel)
  int32_t* fin_first;
  int32_t* list_total;
};

// Workgroups of the persistent finish launch: enough to fill the GPU several
// times over, never more than the cells a round can have.
constexpr int64_t kFinGrid = 2048;

// ev (nullable): events recorded before the allocation, between it and the
// update, and after the update.
int launch_round(const Launch& l, int grid, int split, hipStream_t s,
                 hipEvent_t* ev = nullptr) {
  if (ev) LBG_TRY_HIP(hipEventRecord(ev[0], s));
  hipLaunchKernelGGL(b_assign_kernel<false>, dim3((unsigned)grid), dim3(kT), kBatchLds, s, l.inst,
                     l.chunks, l.nchunks, l.ctr, split);
  LBG_TRY_HIP(hipGetLastError());
  if (split) {
    hipLaunchKernelGGL(b_assign_kernel<true>, dim3((unsigned)grid), dim3(kT), kBatchLds, s,
                       l.inst, l.chunks, l.nchunks, l.ctr + 2, split);
    LBG_TRY_HIP(hipGetLastError());
  }
  if (ev) LBG_TRY_HIP(hipEventRecord(ev[1], s));
  if (l.blocks[kPreAccD] > 0) {
    hipLaunchKernelGGL(b_accd_kernel, dim3((unsigned)l.blocks[kPreAccD]), dim3(kT), l.accd_lds,
                       s, l.inst, l.n, l.pre, l.tb);
    LBG_TRY_HIP(hipGetLastError());
  }
  if (l.blocks[kPreAcc] > 0) {
    hipLaunchKernelGGL(b_acc_kernel, dim3((unsigned)l.blocks[kPreAcc]), dim3(kT), l.acc_lds, s,
                       l.inst, l.n, l.pre, l.tb);
    LBG_TRY_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(b_list_kernel, dim3(1), dim3(1024), 0, s, l.st, l.pend, l.inst, l.n,
                     l.fin_list, l.fin_first, l.list_total);
  LBG_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(b_fin_kernel, dim3((unsigned)std::min(l.blocks[kPreFin], kFinGrid)), dim3(kT),
                     0, s, l.inst, l.fin_list, l.fin_first, l.list_total, l.ctr, l.ctr + 1);
  LBG_TRY_HIP(hipGetLastError());
  if (ev) LBG_TRY_HIP(hipEventRecord(ev[2], s));
  return LBG_OK;
}

// Event triples of the rounds between two polls (timed runs).
struct RoundEvents {
  std::vector<hipEvent_t> ev;
  ~RoundEvents() {
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  int make(int rounds) {
    ev.assign((size_t)rounds * 3, nullptr);
    for (auto& e : ev) LBG_TRY_HIP(hipEventCreate(&e));
    return LBG_OK;
  }
};

// Autotuner: candidate (screen, grab, grid) triples timed on the allocation at
// every instance's final codebook size; the fastest is cached per workload.
// The screens give the same allocation, so only their speed is compared.
struct TuneKey {
  int n;
  int64_t sumM, work, sumN;
  int screen;  // the screens the caller allowed
  bool operator<(const TuneKey& o) const {
    return std::tie(n, sumM, work, sumN, screen) < std::tie(o.n, o.sumM, o.work, o.sumN, o.screen);
  }
};
std::mutex g_tune_mu;
struct TuneVal {
  int grab, grid, split;
};
std::map<TuneKey, TuneVal> g_tune;

int autotune(Launch l, const std::vector<InstPlan>& plans, int32_t* chunk_host,
             int32_t* chunk_dev, hipStream_t s, int split_req, TuneVal* out, double* ms_out) {
  static const int grabs[] = {1, 2, 4, 8, 16};
  static const int grids[] = {256, 512};
  // split_req: 0 = try both screens, 1 = FP32 screen only, 2 = split only
  const int sp_lo = split_req == 2 ? 1 : 0, sp_hi = split_req == 1 ? 0 : 1;
  hipLaunchKernelGGL(b_tune_setup_kernel, dim3((unsigned)l.blocks[kPreFin]), dim3(kT), 0, s,
                     l.inst, l.n, l.pre, l.tb);
  LBG_TRY_HIP(hipGetLastError());
  hipEvent_t e0, e1;
  LBG_TRY_HIP(hipEventCreate(&e0));
  LBG_TRY_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int bg = 4, bgrid = 512, bsp = sp_lo;
  double total = 0.0;
  int rc = LBG_OK;
  for (int g : grabs) {
    if (rc != LBG_OK) break;
    // the previous candidate's copy has completed (its timing synchronised)
    l.nchunks = build_chunks(plans, g, chunk_host);
    const hipError_t ec = hipMemcpyAsync(chunk_dev, chunk_host, sizeof(int32_t) * 3 * l.nchunks,
                                         hipMemcpyHostToDevice, s);
    if (ec != hipSuccess) {
      rc = hip_fail(ec, "autotune");
      break;
    }
    for (int sp = sp_lo; sp <= sp_hi; ++sp)
    for (int gr : grids) {
      float ms_min = 1e30f;
      for (int rep = 0; rep < 3 && rc == LBG_OK; ++rep) {
        hipError_t e = hipMemsetAsync(l.ctr, 0, 3 * sizeof(unsigned), s);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        if (e == hipSuccess) {
          hipLaunchKernelGGL(b_assign_kernel<false>, dim3((unsigned)gr), dim3(kT), kBatchLds, s,
                             l.inst, l.chunks, l.nchunks, l.ctr, sp);
          e = hipGetLastError();
        }
        if (e == hipSuccess && sp) {
          hipLaunchKernelGGL(b_assign_kernel<true>, dim3((unsigned)gr), dim3(kT), kBatchLds, s,
                             l.inst, l.chunks, l.nchunks, l.ctr + 2, sp);
          e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          rc = hip_fail(e, "autotune");
          break;
        }
        total += ms;
        if (rep > 0) ms_min = std::min(ms_min, ms);  // first run warms up
      }
      if (ms_min < best) {
        best = ms_min;
        bg = g;
        bgrid = gr;
        bsp = sp;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  out->grab = bg;
  out->grid = bgrid;
  out->split = bsp;
  *ms_out = total;
  return rc;
}

// Graph of kRoundsPerGraph rounds, cached per (workspace, stream, config).
struct BGraph {
  bool used = false;
  const void* ws = nullptr;
  hipStream_t stream = nullptr;
  int n = 0, grab = 0, grid = 0, split = 0;
  int64_t blocks[kNumPre] = {};
  size_t acc_lds = 0, accd_lds = 0;
  int nchunks = 0;
  hipGraphExec_t exec = nullptr;
  uint64_t stamp = 0;
};
std::mutex g_bgraph_mu;
BGraph g_bgraph[4];
uint64_t g_bstamp = 0;

int get_graph(const Launch& l, const void* ws, int grab, int grid, int split, hipStream_t s,
              hipGraphExec_t* out) {
  for (auto& e : g_bgraph)
    if (e.used && e.ws == ws && e.stream == s && e.n == l.n && e.grab == grab &&
        e.grid == grid && e.split == split && e.acc_lds == l.acc_lds && e.accd_lds == l.accd_lds &&
        e.nchunks == l.nchunks &&
        memcmp(e.blocks, l.blocks, sizeof(e.blocks)) == 0) {
      e.stamp = ++g_bstamp;
      *out = e.exec;
      return LBG_OK;
    }
  BGraph* slot = &g_bgraph[0];
  for (auto& e : g_bgraph) {
    if (!e.used) {
      slot = &e;
      break;
    }
    if (e.stamp < slot->stamp) slot = &e;
  }
  if (slot->used && slot->exec) (void)hipGraphExecDestroy(slot->exec);
  slot->used = false;
  hipGraph_t g = nullptr;
  LBG_TRY_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = LBG_OK;
  for (int r = 0; r < kRoundsPerGraph && rc == LBG_OK; ++r) rc = launch_round(l, grid, split, s);
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (rc != LBG_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  LBG_TRY_HIP(e);
  hipGraphExec_t ex = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  LBG_TRY_HIP(e2);
  slot->used = true;
  slot->ws = ws;
  slot->stream = s;
  slot->n = l.n;
  slot->grab = grab;
  slot->grid = grid;
  slot->split = split;
  memcpy(slot->blocks, l.blocks, sizeof(slot->blocks));
  slot->acc_lds = l.acc_lds;
  slot->accd_lds = l.accd_lds;
  slot->nchunks = l.nchunks;
  slot->exec = ex;
  slot->stamp = ++g_bstamp;
  *out = ex;
  return LBG_OK;
}

int validate(const lbg_instance* in, int32_t n, const lbg_params* p) {
  if (!in || n < 1) {
    set_error("lbg_train_batched: need at least one instance (n_inst = %d)", (int)n);
    return LBG_EINVAL;
  }
  for (int i = 0; i < n; ++i) {
    const lbg_instance& a = in[i];
    if (!a.X || !a.C_out || !a.idx_out) {
      set_error("lbg_train_batched: instance %d has a NULL pointer", i);
      return LBG_EINVAL;
    }
    if (a.M < 1 || a.M > LBG_MAX_M || a.L < 1 || a.L > 64) {
      set_error("lbg_train_batched: instance %d: M = %lld, L = %lld (need M >= 1, 1 <= L <= 64)",
                i, (long long)a.M, (long long)a.L);
      return LBG_EINVAL;
    }
    if (a.N < 1 || (a.N & (a.N - 1)) != 0) {
      set_error("lbg_train_batched: instance %d: N = %lld is not a power of two", i,
                (long long)a.N);
      return LBG_EINVAL;
    }
    const int64_t npad = (a.N + 31) & ~(int64_t)31;
    if (npad * (lp_of(a.L) + 4) * 4 > kBatchLds) {
      set_error("lbg_train_batched: instance %d: codebook of %lld x %lld does not fit the "
                "allocation's LDS (%d bytes)", i, (long long)a.N, (long long)a.L, kBatchLds);
      return LBG_EINVAL;
    }
    if (!afp_usable(a.L, a.N)) {
      set_error("lbg_train_batched: instance %d: N * L too large for the update", i);
      return LBG_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(a.X) & 3) || (reinterpret_cast<uintptr_t>(a.C_out) & 3) ||
        (reinterpret_cast<uintptr_t>(a.idx_out) & 3)) {
      set_error("lbg_train_batched: instance %d: pointers must be 4-byte aligned", i);
      return LBG_EINVAL;
    }
  }
  if (p) {
    if (!(p->thr >= 0.0) || !std::isfinite(p->thr)) {
      set_error("lbg_train_batched: thr must be finite and >= 0");
      return LBG_EINVAL;
    }
    if (p->split_mode == LBG_SPLIT_MULT && !(p->eps_split > 0.0 && p->eps_split < 1.0)) {
      set_error("lbg_train_batched: eps_split must lie in (0, 1)");
      return LBG_EINVAL;
    }
    if (p->split_mode != LBG_SPLIT_MULT && p->split_mode != LBG_SPLIT_ADD) {
      set_error("lbg_train_batched: unknown split_mode %d", (int)p->split_mode);
      return LBG_EINVAL;
    }
    if (p->precision != LBG_FP32) {
      set_error("lbg_train_batched: only LBG_FP32 is supported");
      return LBG_EINVAL;
    }
    if (p->C_init || p->n_forced > 0) {
      set_error("lbg_train_batched: C_init and forced_iters are not supported");
      return LBG_EINVAL;
    }
    if (p->max_iter < 1) {
      set_error("lbg_train_batched: max_iter must be >= 1");
      return LBG_EINVAL;
    }
  }
  return LBG_OK;
}

}  // namespace
}  // namespace lbg

using namespace lbg;

extern "C" size_t lbg_train_batched_workspace(const lbg_instance* inst, int32_t n_inst) {
  if (!inst || n_inst < 1) return 0;
  Carver c{nullptr, 0};
  BatchWs w;
  plan_batch(c, inst, n_inst, &w);
  return c.off + 256;
}

extern "C" void lbg_batch_config_default(lbg_batch_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->grab = 0;
  cfg->grid = 0;
  cfg->graph = 1;
  cfg->rounds_per_poll = kRoundsPerGraph;
  cfg->screen = 0;
}

extern "C" int lbg_train_batched(const lbg_instance* inst, int32_t n_inst, const lbg_params* p,
                                 const lbg_batch_config* cfg, lbg_batch_result* res,
                                 lbg_batch_stats* stats, void* ws, size_t ws_bytes,
                                 void* stream) {
  clear_error();
  lbg_params def;
  lbg_params_default(&def);
  if (!p) p = &def;
  lbg_batch_config cdef;
  lbg_batch_config_default(&cdef);
  if (!cfg) cfg = &cdef;
  LBG_TRY(validate(inst, n_inst, p));
  if (!ws) {
    set_error("lbg_train_batched: workspace is NULL");
    return LBG_EINVAL;
  }
  if (reinterpret_cast<uintptr_t>(ws) & 255) {
    set_error("lbg_train_batched: workspace must be 256-byte aligned");
    return LBG_EINVAL;
  }
  const size_t need = lbg_train_batched_workspace(inst, n_inst);
  if (ws_bytes < need) {
    set_error("lbg_train_batched: workspace of %zu bytes, %zu needed", ws_bytes, need);
    return LBG_ENOWS;
  }
  if (cfg->grab < 0 || cfg->grid < 0 || cfg->rounds_per_poll < 0) {
    set_error("lbg_train_batched: negative configuration value");
    return LBG_EINVAL;
  }
  if (cfg->screen < 0 || cfg->screen > 2) {
    set_error("lbg_train_batched: screen must be 0 (autotuned), 1 (FP32) or 2 (split BF16)");
    return LBG_EINVAL;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int n = n_inst;

  Carver c{reinterpret_cast<char*>(ws), 0};
  BatchWs w;
  plan_batch(c, inst, n, &w);

  // host images: descriptors, prefix sums, initial states
  const size_t b_inst = sizeof(BInst) * (size_t)n;
  const size_t b_pre = sizeof(int64_t) * (size_t)kNumPre * (n + 1);
  const size_t b_st = sizeof(DevState) * (size_t)n;
  const size_t b_tab = sizeof(int32_t) * (size_t)w.b2i_n;
  const size_t b_chunk = sizeof(int32_t) * 3 * (size_t)w.tot[kPreItem];
  unsigned char* host = pinned_stage(b_inst + b_pre + b_st + 64 + b_tab + b_chunk);
  if (!host) {
    set_error("lbg_train_batched: could not allocate pinned host memory");
    return LBG_EHIP;
  }
  BInst* hi = reinterpret_cast<BInst*>(host);
  int64_t* hp = reinterpret_cast<int64_t*>(host + b_inst);
  DevState* hs = reinterpret_cast<DevState*>(host + b_inst + b_pre);
  int64_t tot[kNumPre];
  for (int k = 0; k < kNumPre; ++k) {
    hp[(int64_t)k * (n + 1)] = 0;
    tot[k] = 0;
  }
  size_t acc_lds = 0, accd_lds = 0;
  int64_t work = 0, sumM = 0, sumN = 0;
  for (int i = 0; i < n; ++i) {
    const lbg_instance& a = inst[i];
    const InstPlan& q = w.plans[(size_t)i];
    BInst& B = hi[i];
    memset(&B, 0, sizeof(B));
    B.X = a.X;
    B.M = a.M;
    B.L = (int32_t)a.L;
    B.LP = q.LP;
    B.vec = q.vec;
    B.N = (int32_t)a.N;
    B.Cb[0] = q.Cb[0];
    B.Cb[1] = q.Cb[1];
    B.C_out = a.C_out;
    B.idx = a.idx_out;
    B.st = w.st + i;
    B.pend = w.pend + i;
    B.dpart = q.dpart;
    B.ntiles = q.ntiles;
    B.G = q.G;
    B.cps = q.afp.cps;
    B.nslices = q.afp.nslices;
    B.bds = q.afp.bds;
    B.nchunks = q.afp.nchunks;
    B.absmax_blocks = q.afp.absmax_blocks;
    B.cnwg = q.cnwg;
    B.rows_per_chunk = q.afp.rows_per_chunk;
    B.crpb = q.crpb;
    B.part = q.afp.part;
    B.pcnt = q.afp.pcnt;
    B.amax = q.afp.amax;
    B.lo = q.afp.lo;
    B.shift = q.afp.shift;
    B.cpart = q.cpart;
    B.Dtrace = q.Dtrace;
    B.Atrace = q.Atrace;
    B.nfb = w.nfb + i;
    int64_t cnt[kNumPre];
    family_counts(q, a.N, a.L, cnt);
    for (int k = 0; k < kNumPre; ++k) {
      tot[k] += cnt[k];
      hp[(int64_t)k * (n + 1) + i + 1] = tot[k];
    }
    if (q.afp.bds)
      accd_lds = std::max(accd_lds, afp::accd_lds_bytes(a.N));
    else
      acc_lds = std::max(acc_lds, afp::acc_lds_bytes(q.afp.cps, a.L));
    work += a.M * a.N * a.L;
    sumM += a.M;
    sumN += a.N;

    DevState& d = hs[i];
    memset(&d, 0, sizeof(d));
    d.N = (int32_t)a.N;
    d.M = a.M;
    d.max_iter = p->max_iter;
    d.fixed_iters = p->fixed_iters;
    d.split_mode = p->split_mode;
    d.thr = p->thr;
    d.eps = p->eps_split;
    d.delta = p->delta;
    d.D_cap = kBatchTrace;
    d.first = 1;
    d.D_prev = INFINITY;
    d.status = LBG_OK;
    if (a.N == 1) {
      d.cb = 0;
      d.n = 1;
      d.n_forced = 1;
      d.forced[0] = 0;
    } else {
      d.cb = 1;
      d.n = 2;
    }
  }
  for (int k = 0; k < kNumPre; ++k)
    if (tot[k] > 0x7fffffff) {
      set_error("lbg_train_batched: too many blocks for one launch");
      return LBG_EINVAL;
    }

  // block -> instance tables
  int32_t* htab = reinterpret_cast<int32_t*>(host + b_inst + b_pre + b_st + 64);
  Tabs tb;
  tb.b2i = w.b2i;
  {
    int64_t off = 0;
    for (int k = 0; k < kNumPre; ++k) {
      tb.off[k] = off;
      if (k == kPreItem) continue;
      for (int i = 0; i < n; ++i)
        for (int64_t b = hp[(int64_t)k * (n + 1) + i]; b < hp[(int64_t)k * (n + 1) + i + 1]; ++b)
          htab[off + b] = i;
      off += tot[k];
    }
  }
  int32_t* hchunk = reinterpret_cast<int32_t*>(host + b_inst + b_pre + b_st + 64 + b_tab);
  Launch l{w.inst, n, w.pre, tb, {}, w.ctr, acc_lds, accd_lds, w.chunks, 0,
           w.st, w.pend, w.fin_list, w.fin_first, w.list_total};
  for (int k = 0; k < kNumPre; ++k) l.blocks[k] = tot[k];

  static const hipError_t lds_ok = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&b_assign_kernel<false>),
      hipFuncAttributeMaxDynamicSharedMemorySize, kBatchLds);
  static const hipError_t lds_ok2 = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&b_assign_kernel<true>),
      hipFuncAttributeMaxDynamicSharedMemorySize, kBatchLds);
  LBG_TRY_HIP(lds_ok);
  LBG_TRY_HIP(lds_ok2);

  LBG_TRY_HIP(hipMemcpyAsync(w.inst, hi, b_inst + 0, hipMemcpyHostToDevice, s));
  LBG_TRY_HIP(hipMemcpyAsync(w.pre, hp, b_pre, hipMemcpyHostToDevice, s));
  LBG_TRY_HIP(hipMemcpyAsync(w.b2i, htab, b_tab, hipMemcpyHostToDevice, s));

  // autotune (before the states are set: it uses them as scratch)
  int grab = cfg->grab, grid = cfg->grid;
  int split = cfg->screen == 2 ? 1 : 0;
  bool tuned = false;
  double ms_tune = 0.0;
  if (grab == 0 || grid == 0 || cfg->screen == 0) {
    const TuneKey key{n, sumM, work, sumN, cfg->screen};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    TuneVal tv;
    if (it != g_tune.end()) {
      tv = it->second;
    } else {
      LBG_TRY_HIP(hipMemsetAsync(w.st, 0, b_st, s));
      LBG_TRY(autotune(l, w.plans, hchunk, w.chunks, s, cfg->screen, &tv, &ms_tune));
      g_tune[key] = tv;
      tuned = true;
    }
    if (grab == 0) grab = tv.grab;
    if (grid == 0) grid = tv.grid;
    if (cfg->screen == 0) split = tv.split;
  }

  // the allocation chunks for the chosen grab
  l.nchunks = build_chunks(w.plans, grab, hchunk);
  LBG_TRY_HIP(hipMemcpyAsync(w.chunks, hchunk, sizeof(int32_t) * 3 * l.nchunks,
                             hipMemcpyHostToDevice, s));

  // set-up: states, counters, centroids and first split, fixed-point shifts
  LBG_TRY_HIP(hipMemcpyAsync(w.st, hs, b_st, hipMemcpyHostToDevice, s));
  LBG_TRY_HIP(hipMemcpyAsync(w.pend, hs, b_st, hipMemcpyHostToDevice, s));
  LBG_TRY_HIP(hipMemsetAsync(w.ctr, 0, 3 * sizeof(unsigned), s));
  LBG_TRY_HIP(hipMemsetAsync(w.nfb, 0, sizeof(unsigned long long) * (size_t)n, s));
  hipLaunchKernelGGL(b_setup_kernel, dim3((unsigned)tot[kPreCol]), dim3(kT), 0, s, w.inst, n,
                     w.pre, tb);
  LBG_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(b_centroid_kernel, dim3((unsigned)tot[kPreColFin]), dim3(kT), 0, s, w.inst,
                     n, w.pre, tb, p->split_mode, p->eps_split, p->delta);
  LBG_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(b_shift_kernel, dim3((unsigned)n), dim3(kT), 0, s, w.inst, 1);
  LBG_TRY_HIP(hipGetLastError());

  // rounds until every instance has finished
  const bool timing = cfg->timing != 0;
  const bool use_graph = cfg->graph != 0 && s != nullptr && !timing;
  const int per_poll = use_graph ? kRoundsPerGraph
                                 : (cfg->rounds_per_poll > 0 ? cfg->rounds_per_poll
                                                             : kRoundsPerGraph);
  unsigned* ndone_host = reinterpret_cast<unsigned*>(host + b_inst + b_pre + b_st);
  int rounds = 0;
  // every instance finishes within (levels) x (max_iter + 1) allocations
  int64_t max_rounds = 0;
  for (int i = 0; i < n; ++i) {
    int lv = 1;
    while ((int64_t)1 << (lv - 1) < inst[i].N) ++lv;
    const int64_t per = p->fixed_iters > 0 ? p->fixed_iters : p->max_iter;
    max_rounds = std::max<int64_t>(max_rounds, lv * (per + 2));
  }
  std::unique_lock<std::mutex> glk(g_bgraph_mu, std::defer_lock);
  hipGraphExec_t gexec = nullptr;
  if (use_graph) {
    glk.lock();
    LBG_TRY(get_graph(l, ws, grab, grid, split, s, &gexec));
  }
  RoundEvents rev;
  if (timing) LBG_TRY(rev.make(per_poll));
  double ms_assign = 0.0, ms_update = 0.0;
  for (;;) {
    if (use_graph) {
      LBG_TRY_HIP(hipGraphLaunch(gexec, s));
    } else {
      for (int r = 0; r < per_poll; ++r)
        LBG_TRY(launch_round(l, grid, split, s, timing ? &rev.ev[(size_t)r * 3] : nullptr));
    }
    rounds += per_poll;
    LBG_TRY_HIP(hipMemcpyAsync(ndone_host, w.ctr + 1, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    LBG_TRY_HIP(hipStreamSynchronize(s));
    for (int r = 0; timing && r < per_poll; ++r) {
      float a = 0.0f, u = 0.0f;
      LBG_TRY_HIP(hipEventElapsedTime(&a, rev.ev[(size_t)r * 3], rev.ev[(size_t)r * 3 + 1]));
      LBG_TRY_HIP(hipEventElapsedTime(&u, rev.ev[(size_t)r * 3 + 1], rev.ev[(size_t)r * 3 + 2]));
      ms_assign += a;
      ms_update += u;
    }
    if ((int)*ndone_host >= n) break;
    if (rounds > max_rounds + 2 * kRoundsPerGraph) {
      set_error("lbg_train_batched: %d of %d instances unfinished after %d rounds",
                n - (int)*ndone_host, n, rounds);
      return LBG_EHIP;
    }
  }
  if (glk.owns_lock()) glk.unlock();

  hipLaunchKernelGGL(b_output_kernel, dim3((unsigned)tot[kPreFin]), dim3(kT), 0, s, w.inst, n,
                     w.pre, tb);
  LBG_TRY_HIP(hipGetLastError());
  // states and fallback counters back to the host
  LBG_TRY_HIP(hipMemcpyAsync(hs, w.st, b_st, hipMemcpyDeviceToHost, s));
  std::vector<unsigned long long> nf((size_t)n);
  LBG_TRY_HIP(hipMemcpyAsync(nf.data(), w.nfb, sizeof(unsigned long long) * (size_t)n,
                             hipMemcpyDeviceToHost, s));
  LBG_TRY_HIP(hipStreamSynchronize(s));
  int status = LBG_OK;
  int64_t dist = 0;
  for (int i = 0; i < n; ++i) {
    const DevState& d = hs[i];
    // an instance stopped on non-finite data outranks a capped one
    if (d.status == LBG_EINVAL || (d.status != LBG_OK && status == LBG_OK)) status = d.status;
    dist += d.distances;
    if (res) {
      res[i].D = d.D;
      res[i].status = d.status;
      res[i].n_levels = d.level;
      res[i].n_assign = d.n_assign;
      res[i].n_update = d.n_update;
      res[i].fallback_rows = (int64_t)nf[(size_t)i];
      res[i].distances = d.distances;
    }
  }
  if (status == LBG_EINVAL)
    set_error("lbg_train_batched: the distortion of an instance is not finite (a NaN or "
              "infinite training value); that instance's status is LBG_EINVAL, the others "
              "were trained");
  if (stats) {
    stats->rounds = rounds;
    stats->grab = grab;
    stats->grid = grid;
    stats->graph = use_graph ? 1 : 0;
    stats->tuned = tuned ? 1 : 0;
    stats->total_distances = dist;
    stats->ms_tune = ms_tune;
    stats->ms_assign = ms_assign;
    stats->ms_update = ms_update;
    stats->screen = split ? 2 : 1;
  }
  return status;
}

// ------------------------------------------------- batched single steps --
namespace lbg {
namespace {

struct AsgWs {
  BInst* inst;
  DevState* st;
  unsigned* ctr;
  unsigned long long* nfb;
  int32_t* chunks;
  std::vector<InstPlan> plans;  // G and the partials of each item
};

void plan_asg(Carver& c, const lbg_assign_item* in, int n, AsgWs* w) {
  w->inst = c.take<BInst>((size_t)n);
  w->st = c.take<DevState>((size_t)n);
  w->ctr = c.take<unsigned>(3);
  w->nfb = c.take<unsigned long long>((size_t)n);
  w->plans.assign((size_t)n, InstPlan{});
  int64_t totG = 0;
  for (int i = 0; i < n; ++i) {
    InstPlan& q = w->plans[(size_t)i];
    q.G = slots_of(in[i].M, in[i].L);
    q.ntiles = (in[i].M + kRowsPerTile - 1) / kRowsPerTile;
    q.dpart = c.take<double>((size_t)((in[i].M + 31) / 32));
    totG += q.G;
  }
  w->chunks = c.take<int32_t>((size_t)(3 * totG));
}

int validate_asg(const lbg_assign_item* in, int32_t n) {
  if (!in || n < 1) {
    set_error("lbg_assign_batched: need at least one item (n = %d)", (int)n);
    return LBG_EINVAL;
  }
  for (int i = 0; i < n; ++i) {
    const lbg_assign_item& a = in[i];
    if (!a.X || !a.C || !a.idx) {
      set_error("lbg_assign_batched: item %d has a NULL pointer", i);
      return LBG_EINVAL;
    }
    if (a.M < 1 || a.M > LBG_MAX_M || a.L < 1 || a.L > 64 || a.N < 1 || a.N > LBG_MAX_N) {
      set_error("lbg_assign_batched: item %d: M = %lld, L = %lld, N = %lld (need M >= 1, "
                "1 <= L <= 64, N >= 1)", i, (long long)a.M, (long long)a.L, (long long)a.N);
      return LBG_EINVAL;
    }
    const int64_t npad = (a.N + 31) & ~(int64_t)31;
    if (npad * (lp_of(a.L) + 4) * 4 > kBatchLds) {
      set_error("lbg_assign_batched: item %d: codebook of %lld x %lld does not fit the "
                "allocation's LDS (%d bytes)", i, (long long)a.N, (long long)a.L, kBatchLds);
      return LBG_EINVAL;
    }
    if (((reinterpret_cast<uintptr_t>(a.X) | reinterpret_cast<uintptr_t>(a.C) |
          reinterpret_cast<uintptr_t>(a.idx)) & 3) ||
        (reinterpret_cast<uintptr_t>(a.D) & 7)) {
      set_error("lbg_assign_batched: item %d: misaligned pointer", i);
      return LBG_EINVAL;
    }
  }
  return LBG_OK;
}

struct UpdWs {
  BInst* inst;
  int64_t* pre;
  int32_t* b2i;
  int64_t tot[kNumPre];
  std::vector<AfpWs> afp;
};

// Blocks of the update launches for one item (the other families unused).
void upd_counts(const AfpWs& a, int64_t N, int64_t cnt[kNumPre]) {
  for (int k = 0; k < kNumPre; ++k) cnt[k] = 0;
  cnt[kPreAcc] = a.bds ? 0 : (int64_t)a.nchunks * a.nslices;
  cnt[kPreAccD] = a.bds ? (int64_t)a.nchunks * a.bds : 0;
  cnt[kPreFin] = N;
  cnt[kPreAmax] = a.absmax_blocks;
}

void plan_upd(Carver& c, const lbg_update_item* in, int n, UpdWs* w) {
  w->inst = c.take<BInst>((size_t)n);
  w->pre = c.take<int64_t>((size_t)kNumPre * (n + 1));
  w->afp.assign((size_t)n, AfpWs{});
  for (int k = 0; k < kNumPre; ++k) w->tot[k] = 0;
  for (int i = 0; i < n; ++i) {
    plan_afp(c, in[i].M, in[i].L, in[i].N, &w->afp[(size_t)i], false, true, true);
    int64_t cnt[kNumPre];
    upd_counts(w->afp[(size_t)i], in[i].N, cnt);
    for (int k = 0; k < kNumPre; ++k) w->tot[k] += cnt[k];
  }
  int64_t nb = 0;
  for (int k = 0; k < kNumPre; ++k) nb += w->tot[k];
  w->b2i = c.take<int32_t>((size_t)std::max<int64_t>(1, nb));
}

int validate_upd(const lbg_update_item* in, int32_t n) {
  if (!in || n < 1) {
    set_error("lbg_update_batched: need at least one item (n = %d)", (int)n);
    return LBG_EINVAL;
  }
  for (int i = 0; i < n; ++i) {
    const lbg_update_item& a = in[i];
    if (!a.X || !a.idx || !a.C_old || !a.C_new) {
      set_error("lbg_update_batched: item %d has a NULL pointer", i);
      return LBG_EINVAL;
    }
    if (a.M < 1 || a.M > LBG_MAX_M || a.L < 1 || a.L > 64 || a.N < 1 || a.N > LBG_MAX_N) {
      set_error("lbg_update_batched: item %d: M = %lld, L = %lld, N = %lld (need M >= 1, "
                "1 <= L <= 64, N >= 1)", i, (long long)a.M, (long long)a.L, (long long)a.N);
      return LBG_EINVAL;
    }
    if (!afp_usable(a.L, a.N)) {
      set_error("lbg_update_batched: item %d: N * L too large for the batched update; use "
                "lbg_update", i);
      return LBG_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(a.X) | reinterpret_cast<uintptr_t>(a.idx) |
         reinterpret_cast<uintptr_t>(a.C_old) | reinterpret_cast<uintptr_t>(a.C_new) |
         reinterpret_cast<uintptr_t>(a.counts)) & 3) {
      set_error("lbg_update_batched: item %d: misaligned pointer", i);
      return LBG_EINVAL;
    }
  }
  return LBG_OK;
}

int check_ws(const char* what, void* ws, size_t ws_bytes, size_t need) {
  if (!ws) {
    set_error("%s: workspace is NULL", what);
    return LBG_EINVAL;
  }
  if (reinterpret_cast<uintptr_t>(ws) & 255) {
    set_error("%s: workspace must be 256-byte aligned", what);
    return LBG_EINVAL;
  }
  if (ws_bytes < need) {
    set_error("%s: workspace of %zu bytes, %zu needed", what, ws_bytes, need);
    return LBG_ENOWS;
  }
  return LBG_OK;
}

}  // namespace
}  // namespace lbg

extern "C" size_t lbg_assign_batched_workspace(const lbg_assign_item* items, int32_t n) {
  if (!items || n < 1) return 0;
  Carver c{nullptr, 0};
  AsgWs w;
  plan_asg(c, items, n, &w);
  return c.off + 256;
}

extern "C" int lbg_assign_batched(const lbg_assign_item* items, int32_t n, void* ws,
                                  size_t ws_bytes, void* stream) {
  clear_error();
  LBG_TRY(validate_asg(items, n));
  LBG_TRY(check_ws("lbg_assign_batched", ws, ws_bytes, lbg_assign_batched_workspace(items, n)));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Carver c{reinterpret_cast<char*>(ws), 0};
  AsgWs w;
  plan_asg(c, items, n, &w);
  std::vector<BInst> hi((size_t)n);
  std::vector<DevState> hs((size_t)n);
  for (int i = 0; i < n; ++i) {
    const lbg_assign_item& a = items[i];
    const InstPlan& q = w.plans[(size_t)i];
    BInst& B = hi[(size_t)i];
    memset(&B, 0, sizeof(B));
    B.X = a.X;
    B.M = a.M;
    B.L = (int32_t)a.L;
    B.LP = lp_of(a.L);
    B.vec = (a.L == B.LP) && ((reinterpret_cast<uintptr_t>(a.X) & 15) == 0) &&
            ((reinterpret_cast<uintptr_t>(a.C) & 15) == 0);
    B.N = (int32_t)a.N;
    B.Cb[0] = B.Cb[1] = const_cast<float*>(a.C);  // read only by the allocation
    B.idx = a.idx;
    B.st = w.st + i;
    B.dpart = q.dpart;
    B.ntiles = q.ntiles;
    B.G = q.G;
    B.nfb = w.nfb + i;
    B.Dout = a.D;
    DevState& d = hs[(size_t)i];
    memset(&d, 0, sizeof(d));
    d.n = (int32_t)a.N;
    d.N = (int32_t)a.N;
    d.M = a.M;
  }
  std::vector<int32_t> hchunk;
  int64_t totG = 0;
  for (const auto& q : w.plans) totG += q.G;
  hchunk.resize((size_t)(3 * totG));
  constexpr int kGrab = 16, kGrid = 512;
  const int nchunks = build_chunks(w.plans, kGrab, hchunk.data());
  static const hipError_t lds_ok = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&b_assign_kernel<false>),
      hipFuncAttributeMaxDynamicSharedMemorySize, kBatchLds);
  LBG_TRY_HIP(lds_ok);
  LBG_TRY_HIP(hipMemcpyAsync(w.inst, hi.data(), sizeof(BInst) * (size_t)n,
                             hipMemcpyHostToDevice, s));
  LBG_TRY_HIP(hipMemcpyAsync(w.st, hs.data(), sizeof(DevState) * (size_t)n,
                             hipMemcpyHostToDevice, s));
  LBG_TRY_HIP(hipMemcpyAsync(w.chunks, hchunk.data(), sizeof(int32_t) * 3 * (size_t)nchunks,
                             hipMemcpyHostToDevice, s));
  LBG_TRY_HIP(hipMemsetAsync(w.ctr, 0, 3 * sizeof(unsigned), s));
  // the FP32 screen (and the direct search for small codebooks): the split
  // screen's build measured slower here too (5.3 vs 5.0 ms for the 512
  // instances of the batched workload with codebooks of their final sizes)
  hipLaunchKernelGGL(b_assign_kernel<false>, dim3(kGrid), dim3(kT), kBatchLds, s, w.inst,
                     w.chunks, nchunks, w.ctr, 0);
  LBG_TRY_HIP(hipGetLastError());
  bool anyD = false;
  for (int i = 0; i < n; ++i) anyD = anyD || items[i].D != nullptr;
  if (anyD) {
    hipLaunchKernelGGL(b_reduce_kernel, dim3((unsigned)n), dim3(kT), 0, s, w.inst);
    LBG_TRY_HIP(hipGetLastError());
  }
  // the host images are released on return
  LBG_TRY_HIP(hipStreamSynchronize(s));
  return LBG_OK;
}

extern "C" size_t lbg_update_batched_workspace(const lbg_update_item* items, int32_t n) {
  if (!items || n < 1) return 0;
  Carver c{nullptr, 0};
  UpdWs w;
  plan_upd(c, items, n, &w);
  return c.off + 256;
}

extern "C" int lbg_update_batched(const lbg_update_item* items, int32_t n, void* ws,
                                  size_t ws_bytes, void* stream) {
  clear_error();
  LBG_TRY(validate_upd(items, n));
  LBG_TRY(check_ws("lbg_update_batched", ws, ws_bytes, lbg_update_batched_workspace(items, n)));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Carver c{reinterpret_cast<char*>(ws), 0};
  UpdWs w;
  plan_upd(c, items, n, &w);
  for (int k = 0; k < kNumPre; ++k)
    if (w.tot[k] > 0x7fffffff) {
      set_error("lbg_update_batched: too many blocks for one launch");
      return LBG_EINVAL;
    }
  std::vector<BInst> hi((size_t)n);
  std::vector<int64_t> hp((size_t)kNumPre * (n + 1), 0);
  size_t acc_lds = 0, accd_lds = 0;
  for (int i = 0; i < n; ++i) {
    const lbg_update_item& a = items[i];
    const AfpWs& q = w.afp[(size_t)i];
    BInst& B = hi[(size_t)i];
    memset(&B, 0, sizeof(B));
    B.X = a.X;
    B.M = a.M;
    B.L = (int32_t)a.L;
    B.LP = lp_of(a.L);
    B.vec = (reinterpret_cast<uintptr_t>(a.X) & 15) == 0;
    B.N = (int32_t)a.N;
    B.Cb[0] = B.Cb[1] = const_cast<float*>(a.C_old);  // read only (may equal C_new)
    B.C_out = a.C_new;
    B.idx = const_cast<int32_t*>(a.idx);  // read only by the update
    B.cps = q.cps;
    B.nslices = q.nslices;
    B.bds = q.bds;
    B.nchunks = q.nchunks;
    B.absmax_blocks = q.absmax_blocks;
    B.rows_per_chunk = q.rows_per_chunk;
    B.part = q.part;
    B.pcnt = q.pcnt;
    B.amax = q.amax;
    B.lo = q.lo;
    B.shift = q.shift;
    B.counts = a.counts;
    int64_t cnt[kNumPre];
    upd_counts(q, a.N, cnt);
    for (int k = 0; k < kNumPre; ++k)
      hp[(size_t)k * (n + 1) + i + 1] = hp[(size_t)k * (n + 1) + i] + cnt[k];
    if (q.bds)
      accd_lds = std::max(accd_lds, afp::accd_lds_bytes(a.N));
    else
      acc_lds = std::max(acc_lds, afp::acc_lds_bytes(q.cps, a.L));
  }
  // block -> item tables of the families
  std::vector<int32_t> htab;
  Tabs tb;
  tb.b2i = w.b2i;
  for (int k = 0; k < kNumPre; ++k) {
    tb.off[k] = (int64_t)htab.size();
    for (int i = 0; i < n; ++i)
      for (int64_t b = hp[(size_t)k * (n + 1) + i]; b < hp[(size_t)k * (n + 1) + i + 1]; ++b)
        htab.push_back(i);
  }
  if (htab.empty()) htab.push_back(0);
  LBG_TRY_HIP(hipMemcpyAsync(w.inst, hi.data(), sizeof(BInst) * (size_t)n,
                             hipMemcpyHostToDevice, s));
  LBG_TRY_HIP(hipMemcpyAsync(w.pre, hp.data(), sizeof(int64_t) * hp.size(),
                             hipMemcpyHostToDevice, s));
  LBG_TRY_HIP(hipMemcpyAsync(w.b2i, htab.data(), sizeof(int32_t) * htab.size(),
                             hipMemcpyHostToDevice, s));
  // the fixed-point scales of every item (and its second-word sums cleared)
  hipLaunchKernelGGL(b_absmax_kernel, dim3((unsigned)w.tot[kPreAmax]), dim3(kT), 0, s, w.inst, n,
                     w.pre, tb);
  LBG_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(b_shift_kernel, dim3((unsigned)n), dim3(kT), 0, s, w.inst, 0);
  LBG_TRY_HIP(hipGetLastError());
  if (w.tot[kPreAccD] > 0) {
    hipLaunchKernelGGL(b_upd_accd_kernel, dim3((unsigned)w.tot[kPreAccD]), dim3(kT), accd_lds, s,
                       w.inst, n, w.pre, tb);
    LBG_TRY_HIP(hipGetLastError());
  }
  if (w.tot[kPreAcc] > 0) {
    hipLaunchKernelGGL(b_upd_acc_kernel, dim3((unsigned)w.tot[kPreAcc]), dim3(kT), acc_lds, s,
                       w.inst, n, w.pre, tb);
    LBG_TRY_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(b_upd_fin_kernel, dim3((unsigned)((w.tot[kPreFin] + kT / 64 - 1) / (kT / 64))),
                     dim3(kT), 0, s, w.inst, n, w.pre, tb);
  LBG_TRY_HIP(hipGetLastError());
  // the host images are released on return
  LBG_TRY_HIP(hipStreamSynchronize(s));
  return LBG_OK;
}
