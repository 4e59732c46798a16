// Cell Allocation with a BF16 matrix-core screen (precision form).
//
// Training vectors and codevectors are rounded to BF16 (round to nearest
// even) and the expanded squared distance |c|^2 - 2 x.c of the rounded
// vectors (|x|^2 is the same for every codevector and left out) is
// accumulated in FP32 on v_mfma_f32_32x32x16_bf16; the squared norm of each
// rounded codevector enters one K-step as three BF16 parts whose sum is that
// norm exactly.  The two best candidates per vector are rescored in FP32 in
// the direct form sum_l (x_l - c_l)^2 on the original FP32 data and the
// closer one is taken (lowest index on equal distances).  A vector whose true
// nearest codevector is not among the two candidates is misassigned; the
// error against the FP64 reference is measured, not bounded.
//
// Codebooks that fit one CU's LDS (n_pad (LP + 8) BF16 rows) run in a kernel
// built for this form alone:
//   * a workgroup of 8 waves per CU holds the codebook resident; a wave owns
//     64 training vectors (two B-operand tiles of 32) at a time, so that each
//     codebook fragment read from LDS feeds two products, and the norm
//     product (the same for every vector) is formed once per codebook tile
//     and enters both tiles' chains as their accumulator input: 1 + 2 LP/16
//     MFMAs per 32 codevectors x 64 vectors;
//   * every accumulator slot keeps only its smallest key (the screened value
//     with its low mantissa bits replaced by the tile number): two VALU
//     operations per distance;
//   * the candidates are the smallest key of all 32 slots a vector's two
//     lanes hold and the smallest of the other 31 slots;
//   * the fragments of tile t+2 are read while tile t+1's products run
//     beside tile t's key updates.
// Other codebooks use the general kernel of assign_common.h (Bf16Screen).
#include "assign_common.h"

namespace lbg {

using namespace assign_detail;

namespace {

constexpr int kV2Waves = 8;
constexpr int kV2Threads = 64 * kV2Waves;

// Products of one codebook tile (fragments f) with the wave's two vector
// tiles: the norm step once, then the two chains interleaved.
template <int LP>
__device__ __forceinline__ void mma2(const Frag<Bf16Screen<LP>>& f, const bf16x8 (&xa)[LP / 16],
                                     const bf16x8 (&xb)[LP / 16], const bf16x8& bn, f16v& ca,
                                     f16v& cb) {
  constexpr int NS = LP / 16;
  const f16v cn = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.an, bn, f16v{}, 0, 0, 0);
  ca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[0], xa[0], cn, 0, 0, 0);
  cb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[0], xb[0], cn, 0, 0, 0);
#pragma unroll
  for (int s = 1; s < NS; ++s) {
    ca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[s], xa[s], ca, 0, 0, 0);
    cb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[s], xb[s], cb, 0, 0, 0);
  }
}

// Key of a screened value v for tile number tb: v with its low mantissa bits
// (those the tile number needs) replaced by tb, one v_and_or_b32.  Only the
// tile number is embedded: every further bit would coarsen the keys (at
// n = 1024 five bits already merge values within 2^5 ulps), and the slot is
// known from the register that holds the key.
__device__ __forceinline__ float tile_key(float v, uint32_t vmask, uint32_t tb) {
  return __uint_as_float((__float_as_uint(v) & vmask) | tb);
}

// mn[r] = min(mn[r], key of acc[r]) for tile number tb.
__device__ __forceinline__ void keys1(const f16v& acc, float (&mn)[16], uint32_t vmask,
                                      uint32_t tb, float ninf) {
#pragma unroll
  for (int r = 0; r < 16; ++r)
    mn[r] = __builtin_amdgcn_fmed3f(mn[r], tile_key(acc[r], vmask, tb), ninf);
}

// Keys G0 .. G0+K-1 of the 32 a lane updates per tile (16 slots of vector
// tile a, then 16 of b), each key two VALU operations.
template <int G0, int K>
__device__ __forceinline__ void keys_part(const f16v& ka, const f16v& kb, float (&ma)[16],
                                          float (&mb)[16], uint32_t vmask, uint32_t tb,
                                          float ninf) {
#pragma unroll
  for (int g = G0; g < G0 + K; ++g) {
    const float v = g < 16 ? ka[g & 15] : kb[g & 15];
    const float k = tile_key(v, vmask, tb);
    if (g < 16)
      ma[g & 15] = __builtin_amdgcn_fmed3f(ma[g & 15], k, ninf);
    else
      mb[g & 15] = __builtin_amdgcn_fmed3f(mb[g & 15], k, ninf);
  }
}

// One pipeline phase in a fixed issue order: the products of one codebook
// tile (fragments f) into (ca, cb) -- the norm step, then the two chains
// alternately -- with the key updates of the previous tile (ka, kb, tile
// number tb) spread between them, 32 / (2 LP/16) keys after each product
// but the last, so that the matrix core runs while the keys are updated.
// The scheduling barriers keep that order.
template <int LP>
__device__ __forceinline__ void phase(const Frag<Bf16Screen<LP>>& f, const bf16x8 (&xa)[LP / 16],
                                      const bf16x8 (&xb)[LP / 16], const bf16x8& bn, f16v& ca,
                                      f16v& cb, const f16v& ka, const f16v& kb, float (&ma)[16],
                                      float (&mb)[16], uint32_t vmask, uint32_t tb,
                                      float ninf) {
  constexpr int NS = LP / 16;
  constexpr int KPG = 32 / (2 * NS);  // keys per gap
  const f16v cn = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.an, bn, f16v{}, 0, 0, 0);
  __builtin_amdgcn_sched_barrier(0);
  keys_part<0, KPG>(ka, kb, ma, mb, vmask, tb, ninf);
  __builtin_amdgcn_sched_barrier(0);
  ca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[0], xa[0], cn, 0, 0, 0);
  __builtin_amdgcn_sched_barrier(0);
  keys_part<KPG, KPG>(ka, kb, ma, mb, vmask, tb, ninf);
  __builtin_amdgcn_sched_barrier(0);
  cb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[0], xb[0], cn, 0, 0, 0);
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (NS >= 2) {
    keys_part<2 * KPG, KPG>(ka, kb, ma, mb, vmask, tb, ninf);
    __builtin_amdgcn_sched_barrier(0);
    ca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[1], xa[1], ca, 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    keys_part<3 * KPG, KPG>(ka, kb, ma, mb, vmask, tb, ninf);
    __builtin_amdgcn_sched_barrier(0);
    cb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[1], xb[1], cb, 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
  if constexpr (NS >= 4) {
    keys_part<4 * KPG, KPG>(ka, kb, ma, mb, vmask, tb, ninf);
    __builtin_amdgcn_sched_barrier(0);
    ca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[2], xa[2], ca, 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    keys_part<5 * KPG, KPG>(ka, kb, ma, mb, vmask, tb, ninf);
    __builtin_amdgcn_sched_barrier(0);
    cb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[2], xb[2], cb, 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    keys_part<6 * KPG, KPG>(ka, kb, ma, mb, vmask, tb, ninf);
    __builtin_amdgcn_sched_barrier(0);
    ca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[3], xa[3], ca, 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    keys_part<7 * KPG, KPG>(ka, kb, ma, mb, vmask, tb, ninf);
    __builtin_amdgcn_sched_barrier(0);
    cb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[3], xb[3], cb, 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
  static_assert(NS == 1 || NS == 2 || NS == 4, "phase: LP 16, 32 or 64");
}

// Lane's two smallest slot keys (k1 <= k2; the lower slot first on equal
// keys) and their codevector indices: tile from the key's low bits, slot r
// holding row 8 (r >> 2) + 4 h + (r & 3) of its tile.
__device__ __forceinline__ void lane_top2(const float (&mn)[16], uint32_t lowmask, int h,
                                          float& k1, int& i1, float& k2, int& i2) {
  k1 = INFINITY;
  k2 = INFINITY;
  int r1 = 0, r2 = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const float v = mn[r];
    const bool b1 = v < k1, b2 = v < k2;
    k2 = b1 ? k1 : (b2 ? v : k2);
    r2 = b1 ? r1 : (b2 ? r : r2);
    k1 = b1 ? v : k1;
    r1 = b1 ? r : r1;
  }
  i1 = (int)((__float_as_uint(k1) & lowmask) << 5) + 8 * (r1 >> 2) + 4 * h + (r1 & 3);
  i2 = (int)((__float_as_uint(k2) & lowmask) << 5) + 8 * (r2 >> 2) + 4 * h + (r2 & 3);
}

// Candidates of the 32 vectors of one tile: the smallest and the second
// smallest of the four keys a vector's two lanes hold (lower index first on
// equal keys).  w2 == w1 when there is no second candidate.
struct Cands {
  int w1, w2;
  bool two;
};

__device__ __forceinline__ Cands tile_cands(const float (&mn)[16], uint32_t lowmask, int h,
                                            int n) {
  float k1, k2;
  int i1, i2;
  lane_top2(mn, lowmask, h, k1, i1, k2, i2);
  float a1, b1, a2, b2;
  int ai1, bi1, ai2, bi2;
  pair_values(k1, a1, b1);
  pair_values(k2, a2, b2);
  pair_values(i1, ai1, bi1);
  pair_values(i2, ai2, bi2);
  const bool aw = a1 < b1 || (a1 == b1 && ai1 < bi1);
  Cands c;
  c.w1 = aw ? ai1 : bi1;
  if (aw) {
    const bool s = a2 < b1 || (a2 == b1 && ai2 < bi1);
    c.w2 = s ? ai2 : bi1;
  } else {
    const bool s = b2 < a1 || (b2 == a1 && bi2 < ai1);
    c.w2 = s ? bi2 : ai1;
  }
  if ((unsigned)c.w1 >= (unsigned)n) c.w1 = 0;  // non-finite keys
  c.two = (unsigned)c.w2 < (unsigned)n && c.w2 != c.w1;
  if (!c.two) c.w2 = c.w1;
  return c;
}

// FP32 direct-form distances of one tile's vectors to their two candidates
// (lane (j, 0) sums the first half of the dimensions, lane (j, 1) the
// second; the halves are added), the closer taken and stored for rows
// row0 .. row0+31.  xv: the lane's FP32 half-row (zeros past M and L); ca,
// cb: the candidates' half-rows.  Returns the winning distance in lane
// (j, 1) (0 elsewhere and past M).
template <int LP>
__device__ __forceinline__ float rescore_tile(const float (&xv)[LP / 2], const float (&ca)[LP / 2],
                                              const float (&cb)[LP / 2], Cands c, int64_t M,
                                              int L, int64_t row0, int32_t* __restrict__ idx,
                                              float* __restrict__ mind) {
  constexpr int H = LP / 2;
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5, j = lane & 31;
  float pa = 0.0f, pb = 0.0f;
#pragma unroll
  for (int q = 0; q < H; ++q) {
    if (h * H + q < L) {
      const float u = xv[q] - ca[q], v = xv[q] - cb[q];
      pa = __builtin_fmaf(u, u, pa);
      pb = __builtin_fmaf(v, v, pb);
    }
  }
  float pa0, pa1, pb0, pb1;
  pair_values(pa, pa0, pa1);
  pair_values(pb, pb0, pb1);
  float d = pa0 + pa1;
  const float db = pb0 + pb1;
  int win = c.w1;
  if (c.two && (db < d || (db == d && c.w2 < c.w1))) {
    d = db;
    win = c.w2;
  }
  if (!(d < INFINITY)) {  // no finite distance: index 0, +inf
    win = 0;
    d = INFINITY;
  }
  const int64_t m = row0 + j;
  const bool live = h == 1 && m < M;
  if (live) {
    idx[m] = win;
    if (mind) mind[m] = d;
  }
  return live ? d : 0.0f;
}

template <int LP, bool VEC>
__global__ __launch_bounds__(kV2Threads, 1) void bf16v2_kernel(
    const float* __restrict__ X, int64_t M, int L, const float* __restrict__ C, int n,
    int32_t* __restrict__ idx, float* __restrict__ mind, double* __restrict__ dpart, Ctl ctl,
    CbPair cbp) {
  typedef Bf16Screen<LP> SC;
  constexpr int NS = LP / 16;
  constexpr int S = SC::S;
  constexpr int TS = 32 * S;  // elements per codebook tile
  if (ctl.st) {
    if (ctl.st->done) return;
    n = ctl.st->n;
    C = cbp.c[ctl.st->cb];
  }
  if (VEC) L = LP;
  const int n_pad = (n + 31) & ~31;
  const int nt = n_pad >> 5;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __bf16* sA = reinterpret_cast<__bf16*>(smem);
  stage_from_C<SC, VEC, kV2Threads>(C, n, L, n_pad, sA);

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int h = lane >> 5, j = lane & 31;
  const uint32_t lowmask = (1u << tile_bits_of(n)) - 1u;
  uint32_t vmask = ~lowmask;
  asm volatile("v_mov_b32 %0, %1" : "=v"(vmask) : "v"(vmask));
  float ninf = -INFINITY;
  asm volatile("v_mov_b32 %0, %1" : "=v"(ninf) : "v"(ninf));
  const __bf16 one = (__bf16)1.0f, zero = (__bf16)0.0f;
  const bf16x8 bn = h ? bf16x8{zero, zero, zero, zero, zero, zero, zero, zero}
                      : bf16x8{one, one, one, zero, zero, zero, zero, zero};
  const __bf16* ar = sA + j * S;

  const int64_t ngroups = (M + 63) >> 6;
  const int64_t step = (int64_t)gridDim.x * kV2Waves;
  int64_t g = (int64_t)blockIdx.x * kV2Waves + wave;
  // FP32 half-rows of the group's two vector tiles: loaded while the
  // previous group finishes, converted to BF16 for the screen and (HOLD)
  // kept for the rescore
  constexpr bool HOLD = VEC || LP < 64;
  float pa[LP / 2], pb[LP / 2];
  if (g < ngroups) {
    load_x<LP, VEC>(X, M, L, g * 64, h, j, pa);
    load_x<LP, VEC>(X, M, L, g * 64 + 32, h, j, pb);
  }
  for (; g < ngroups; g += step) {
    const int64_t row0 = g * 64;
    bf16x8 xa[NS], xb[NS];
#pragma unroll
    for (int q = 0; q < LP / 2; ++q) {
      xa[q >> 3][q & 7] = (__bf16)pa[q];
      xb[q >> 3][q & 7] = (__bf16)pb[q];
    }
    float ma[16], mb[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      ma[r] = FLT_MAX;
      mb[r] = FLT_MAX;
    }
    Frag<SC> f0, f1;
    f16v a0, b0, a1, b1;
    f0.load(ar, h);
    mma2<LP>(f0, xa, xb, bn, a0, b0);
    f1.load(ar + min(1, nt - 1) * TS, h);
    int t = 0;
    // (a0, b0): products of tile t; f1: fragments of tile t + 1.  A tile
    // number past the end is clamped to the last tile (loaded, not used).
    for (; t + 2 < nt; t += 2) {
      f0.load(ar + (t + 2) * TS, h);
      phase<LP>(f1, xa, xb, bn, a1, b1, a0, b0, ma, mb, vmask, (uint32_t)t, ninf);
      f1.load(ar + min(t + 3, nt - 1) * TS, h);
      phase<LP>(f0, xa, xb, bn, a0, b0, a1, b1, ma, mb, vmask, (uint32_t)(t + 1), ninf);
    }
    if (t + 1 < nt) {
      phase<LP>(f1, xa, xb, bn, a1, b1, a0, b0, ma, mb, vmask, (uint32_t)t, ninf);
      keys1(a1, ma, vmask, (uint32_t)(t + 1), ninf);
      keys1(b1, mb, vmask, (uint32_t)(t + 1), ninf);
    } else {
      keys1(a0, ma, vmask, (uint32_t)t, ninf);
      keys1(b0, mb, vmask, (uint32_t)t, ninf);
    }
    // rescore from the held rows (the unaligned LP = 64 form reloads them:
    // holding them there would spill)
    if (!HOLD) {
      load_x<LP, VEC>(X, M, L, row0, h, j, pa);
      load_x<LP, VEC>(X, M, L, row0 + 32, h, j, pb);
    }
    // both tiles' candidates first, then all four gathers in one round
    const Cands qa = tile_cands(ma, lowmask, h, n), qb = tile_cands(mb, lowmask, h, n);
    float caa[LP / 2], cab[LP / 2], cba[LP / 2], cbb[LP / 2];
    c_half<SC, VEC>(C, L, nullptr, qa.w1, h, caa);
    c_half<SC, VEC>(C, L, nullptr, qa.w2, h, cab);
    c_half<SC, VEC>(C, L, nullptr, qb.w1, h, cba);
    c_half<SC, VEC>(C, L, nullptr, qb.w2, h, cbb);
    // the next group's rows are loaded into each tile's registers once its
    // rescore is done: issued after the gathers, so that waiting for the
    // gathers (loads complete in order) does not wait for them
    const bool more = g + step < ngroups;
    const float da = rescore_tile<LP>(pa, caa, cab, qa, M, L, row0, idx, mind);
    if (more) load_x<LP, VEC>(X, M, L, (g + step) * 64, h, j, pa);
    const float db = rescore_tile<LP>(pb, cba, cbb, qb, M, L, row0 + 32, idx, mind);
    if (more) load_x<LP, VEC>(X, M, L, (g + step) * 64 + 32, h, j, pb);
    // distortion partials of the two 32-vector groups (FP64, fixed tree)
    if (dpart) {
      const double sa = wave_sum((double)da), sb = wave_sum((double)db);
      if (lane == 0) {
        if (row0 < M) dpart[row0 >> 5] = sa;
        if (row0 + 32 < M) dpart[(row0 >> 5) + 1] = sb;
      }
    }
  }
}

template <int LP>
int launch_v2(const float* X, int64_t M, int L, const float* C, int n, int32_t* idx,
              float* mind, double* dpart, hipStream_t s, Ctl ctl, CbPair cbp) {
  const int n_pad = (n + 31) & ~31;
  const size_t lds = (size_t)n_pad * Bf16Screen<LP>::S * 2;
  bool vec = (L == LP) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  if (ctl.st)
    vec = vec && ((reinterpret_cast<uintptr_t>(cbp.c[0]) & 15) == 0) &&
          ((reinterpret_cast<uintptr_t>(cbp.c[1]) & 15) == 0);
  else
    vec = vec && ((reinterpret_cast<uintptr_t>(C) & 15) == 0);
  static const hipError_t a1 = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&bf16v2_kernel<LP, true>),
      hipFuncAttributeMaxDynamicSharedMemorySize, kWideLds);
  static const hipError_t a2 = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&bf16v2_kernel<LP, false>),
      hipFuncAttributeMaxDynamicSharedMemorySize, kWideLds);
  LBG_TRY_HIP(vec ? a1 : a2);
  const int64_t ngroups = (M + 63) / 64;
  const unsigned grid =
      (unsigned)std::max<int64_t>(1, std::min<int64_t>(256, (ngroups + kV2Waves - 1) / kV2Waves));
  if (vec)
    hipLaunchKernelGGL((bf16v2_kernel<LP, true>), dim3(grid), dim3(kV2Threads), lds, s, X, M, L,
                       C, n, idx, mind, dpart, ctl, cbp);
  else
    hipLaunchKernelGGL((bf16v2_kernel<LP, false>), dim3(grid), dim3(kV2Threads), lds, s, X, M,
                       L, C, n, idx, mind, dpart, ctl, cbp);
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

}  // namespace

bool bf16_v2_fits(int LP, int64_t n) {
  if (LP != 16 && LP != 32 && LP != 64) return false;
  const int64_t n_pad = (n + 31) & ~(int64_t)31;
  return n_pad * (LP + 8) * 2 <= kWideLds;
}

int launch_assign_bf16(const float* X, int64_t M, int L, const float* C, int n, int32_t* idx,
                       float* mind, double* dpart, int LP, void* prep, hipStream_t s,
                       Ctl ctl, CbPair cbp) {
  const int LB = LP < 16 ? 16 : LP;
  if (bf16_v2_fits(LB, n)) {
    switch (LB) {
      case 16: return launch_v2<16>(X, M, L, C, n, idx, mind, dpart, s, ctl, cbp);
      case 32: return launch_v2<32>(X, M, L, C, n, idx, mind, dpart, s, ctl, cbp);
      default: return launch_v2<64>(X, M, L, C, n, idx, mind, dpart, s, ctl, cbp);
    }
  }
  switch (LP) {
    case 8:
    case 16: return launch_screen<Bf16Screen<16>>(X, M, L, C, n, idx, mind, dpart, nullptr, prep, s, ctl, cbp);
    case 32: return launch_screen<Bf16Screen<32>>(X, M, L, C, n, idx, mind, dpart, nullptr, prep, s, ctl, cbp);
    case 64: return launch_screen<Bf16Screen<64>>(X, M, L, C, n, idx, mind, dpart, nullptr, prep, s, ctl, cbp);
    default: return launch_screen<Bf16Screen<128>>(X, M, L, C, n, idx, mind, dpart, nullptr, prep, s, ctl, cbp);
  }
}

}  // namespace lbg
