// Codebook Updation (Algorithm 1, "Codebook Updation"): every codevector
// becomes the centroid of the training vectors whose cell value is its
// index; an empty cell keeps its codevector.  The same machinery sums
// (c_k - x) per cell for the gradient of the distortion.
//
// The paper updates one codevector per processor, each scanning the whole
// cell table (round robin over codevectors).  Here the cell table is sorted
// once by cell (a stable counting sort) and every cell's rows are summed
// from the sorted order, so X is read once per update:
//   1. hist      per tile of T rows: cell counts            ghist[cell][tile]
//   2. scan      per cell: exclusive scan over tiles; cell totals
//   3. offsets   exclusive scan over cells            bin_off[cell], counts
//   4. scatter   per tile, one wave, rows in order: stable position of
//                every row in cell order               perm[pos] = row
//   5. segsum    the sorted order is cut into runs of P positions; a group
//                of lanes (one dimension per lane) walks its run in order,
//                summing rows in FP64; a cell wholly inside the run is
//                finished here, a cell crossing a run boundary leaves one
//                partial per run
//   6. finalize  cells crossing run boundaries: partials added in run order;
//                empty cells keep their codevector
// Every sum has a fixed order (rows ascending within a run, runs ascending),
// so the result is bit-reproducible.  Integer atomics are used only for
// counting, where order does not matter.
#include "lbg_internal.h"

namespace lbg {
namespace {

constexpr int kThreads = 256;
constexpr int kLdsCells = 8192;  // cells counted in LDS (32 KB)

__global__ __launch_bounds__(kThreads) void hist_kernel(
    const int32_t* __restrict__ idx, int64_t M, int N, int64_t T,
    int64_t ntiles, int32_t* __restrict__ ghist) {
  extern __shared__ int32_t sh[];
  const int64_t tile = blockIdx.x;
  for (int b = threadIdx.x; b < N; b += kThreads) sh[b] = 0;
  __syncthreads();
  const int64_t r0 = tile * T, r1 = min(M, r0 + T);
  for (int64_t r = r0 + threadIdx.x; r < r1; r += kThreads) {
    const int k = idx[r];
    if ((unsigned)k < (unsigned)N) atomicAdd(&sh[k], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < N; b += kThreads) ghist[(int64_t)b * ntiles + tile] = sh[b];
}

// Same as hist_kernel for codebooks too large for an LDS histogram: the
// column of this tile is cleared by the tile itself, then counted with
// global integer atomics.
__global__ __launch_bounds__(kThreads) void hist_global_kernel(
    const int32_t* __restrict__ idx, int64_t M, int N, int64_t T,
    int64_t ntiles, int32_t* __restrict__ ghist) {
  const int64_t tile = blockIdx.x;
  for (int b = threadIdx.x; b < N; b += kThreads) ghist[(int64_t)b * ntiles + tile] = 0;
  __threadfence();
  __syncthreads();
  const int64_t r0 = tile * T, r1 = min(M, r0 + T);
  for (int64_t r = r0 + threadIdx.x; r < r1; r += kThreads) {
    const int k = idx[r];
    if ((unsigned)k < (unsigned)N) atomicAdd(&ghist[(int64_t)k * ntiles + tile], 1);
  }
}

// Block-wide exclusive scan of one value per thread; returns the total.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* out,
                                                        int64_t* sbuf) {
  const int t = threadIdx.x;
  sbuf[t] = v;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    int64_t add = (t >= off) ? sbuf[t - off] : 0;
    __syncthreads();
    sbuf[t] += add;
    __syncthreads();
  }
  const int64_t incl = sbuf[t];
  const int64_t total = sbuf[blockDim.x - 1];
  __syncthreads();
  *out = incl - v;
  return total;
}

__global__ __launch_bounds__(kThreads) void scan_tiles_kernel(
    int32_t* __restrict__ ghist, int64_t ntiles, int32_t* __restrict__ cnt) {
  __shared__ int64_t sbuf[kThreads];
  int32_t* row = ghist + (int64_t)blockIdx.x * ntiles;
  const int64_t q = (ntiles + kThreads - 1) / kThreads;
  const int64_t t0 = threadIdx.x * q, t1 = min(ntiles, t0 + q);
  int64_t s = 0;
  for (int64_t t = t0; t < t1; ++t) s += row[t];
  int64_t ex;
  const int64_t total = block_exclusive_scan(s, &ex, sbuf);
  for (int64_t t = t0; t < t1; ++t) {
    const int32_t v = row[t];
    row[t] = (int32_t)ex;
    ex += v;
  }
  if (threadIdx.x == 0) cnt[blockIdx.x] = (int32_t)total;
}

__global__ __launch_bounds__(1024) void scan_bins_kernel(
    const int32_t* __restrict__ cnt, int N, int32_t* __restrict__ bin_off,
    int32_t* __restrict__ counts) {
  __shared__ int64_t sbuf[1024];
  const int q = (N + 1023) / 1024;
  const int b0 = threadIdx.x * q, b1 = min(N, b0 + q);
  int64_t s = 0;
  for (int b = b0; b < b1; ++b) s += cnt[b];
  int64_t ex;
  const int64_t total = block_exclusive_scan(s, &ex, sbuf);
  for (int b = b0; b < b1; ++b) {
    bin_off[b] = (int32_t)ex;
    ex += cnt[b];
    if (counts) counts[b] = cnt[b];
  }
  if (threadIdx.x == 0) bin_off[N] = (int32_t)total;
}

// One wave per tile walks its rows in order, 64 at a time; rows of one step
// that share a cell are ranked by lane order, so positions are stable.  The
// running position of every cell lives in LDS (LDS_RUN) or, for codebooks
// too large for LDS, in this tile's own column of ghist.
template <bool LDS_RUN>
__global__ __launch_bounds__(64) void scatter_kernel(
    const int32_t* __restrict__ idx, int64_t M, int N, int nbits, int64_t T,
    int64_t ntiles, int32_t* __restrict__ ghist,
    const int32_t* __restrict__ bin_off, int32_t* __restrict__ perm) {
  extern __shared__ int32_t run_lds[];
  const int64_t tile = blockIdx.x;
  const int lane = threadIdx.x;
  int32_t* run = run_lds;
  int64_t stride = 1;
  if (LDS_RUN) {
    for (int b = lane; b < N; b += 64) run[b] = bin_off[b] + ghist[(int64_t)b * ntiles + tile];
  } else {
    run = ghist + tile;
    stride = ntiles;
    for (int b = lane; b < N; b += 64) run[b * stride] += bin_off[b];
    __threadfence_block();
  }
  __syncthreads();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t r0 = tile * T, r1 = min(M, r0 + T);
  // the cell indices of kPF steps are loaded together, ahead of the steps
  constexpr int kPF = 16;
  int kq[kPF];
  for (int64_t base = r0; base < r1; base += 64) {
    const int st = (int)(((base - r0) >> 6) % kPF);
    if (st == 0) {
#pragma unroll
      for (int u = 0; u < kPF; ++u) {
        const int64_t ru = base + 64 * u + lane;
        kq[u] = (ru < r1) ? idx[ru] : -1;
      }
    }
    int k = kq[0];
#pragma unroll
    for (int u = 1; u < kPF; ++u) k = (st == u) ? kq[u] : k;
    const int64_t r = base + lane;
    const bool valid = (unsigned)k < (unsigned)N;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = valid && ((k >> b) & 1);
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    int pos = 0;
    if (valid) {
      pos = run[k * stride] + __popcll(peers & below);
      perm[pos] = (int32_t)r;
    }
    __builtin_amdgcn_wave_barrier();
    if (!LDS_RUN) __threadfence_block();
    if (valid && (peers & below) == 0) run[k * stride] += __popcll(peers);
    if (!LDS_RUN) __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
}

// G lanes per run, DPL dimensions per lane (dimension d = lane + q*G).
template <int G, int DPL, int MODE>
__global__ __launch_bounds__(kThreads) void segsum_kernel(
    const float* __restrict__ X, int L, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ bin_off, int N, int64_t P, int64_t nruns,
    const float* __restrict__ C_old, float* __restrict__ out, double g2,
    double* __restrict__ partial) {
  constexpr int LPD = G * DPL;
  constexpr int U = 8;
  const int64_t run = (int64_t)blockIdx.x * (kThreads / G) + threadIdx.x / G;
  const int gl = threadIdx.x % G;
  if (run >= nruns) return;
  const int64_t total = bin_off[N];
  const int64_t s0 = run * P;
  if (s0 >= total) return;
  const int64_t s1 = min(total, s0 + P);
  // cell holding position s0: the largest k with bin_off[k] <= s0
  int lo = 0, hi = N;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bin_off[mid] <= s0) lo = mid; else hi = mid - 1;
  }
  int k = lo;
  int64_t cend = bin_off[k + 1];
  double acc[DPL];
#pragma unroll
  for (int q = 0; q < DPL; ++q) acc[q] = 0.0;
  // MODE 1: the current cell's codevector, held in registers and reloaded
  // when the cell changes (not once per row)
  double cq[DPL];
  auto load_c = [&]() {
#pragma unroll
    for (int q = 0; q < DPL; ++q) {
      const int d = gl + q * G;
      cq[q] = (MODE == 1 && d < L) ? (double)C_old[(int64_t)k * L + d] : 0.0;
    }
  };
  load_c();

  for (int64_t j0 = s0; j0 < s1; j0 += U) {
    int32_t rows[U];
    float xs[U][DPL];
#pragma unroll
    for (int u = 0; u < U; ++u) rows[u] = (j0 + u < s1) ? perm[j0 + u] : 0;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < DPL; ++q) {
        const int d = gl + q * G;
        xs[u][q] = (j0 + u < s1 && d < L) ? X[(int64_t)rows[u] * L + d] : 0.0f;
      }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t jj = j0 + u;
      if (jj >= s1) break;
#pragma unroll
      for (int q = 0; q < DPL; ++q) {
        if (MODE == 0) {
          acc[q] += (double)xs[u][q];
        } else {
          acc[q] += cq[q] - (double)xs[u][q];
        }
      }
      if (jj + 1 == cend || jj + 1 == s1) {
        const int64_t ca = bin_off[k];
        const bool complete = ca >= s0 && cend <= s0 + P;
#pragma unroll
        for (int q = 0; q < DPL; ++q) {
          const int d = gl + q * G;
          if (d >= L) continue;
          if (complete) {
            const double v = (MODE == 0) ? acc[q] / (double)(cend - ca) : g2 * acc[q];
            out[(int64_t)k * L + d] = (float)v;
          } else {
            const int slot = (ca < s0) ? 0 : 1;
            partial[(run * 2 + slot) * LPD + d] = acc[q];
          }
          acc[q] = 0.0;
        }
        if (jj + 1 < s1) {
          do {
            ++k;
          } while (bin_off[k + 1] <= jj + 1);
          cend = bin_off[k + 1];
          load_c();
        }
      }
    }
  }
}

// One block per cell.  A cell that crosses run boundaries is combined from
// its runs' partials in a fixed tree: thread (q, d) adds the "first" partials
// of runs r0+1+q, r0+1+q+Q, ... in order (Q = 256 / G2 run lanes, G2 lanes
// per dimension slice), the Q lane sums are added in q order, and the "last"
// partial of run r0 comes first.  Empty cells keep their codevector (MODE 0)
// or get a zero gradient (MODE 1); cells inside one run were finished by
// segsum.
template <int MODE>
__global__ __launch_bounds__(kThreads) void finalize_kernel(
    const int32_t* __restrict__ bin_off, int N, int L, int LPD, int64_t P,
    const double* __restrict__ partial, const float* __restrict__ C_old,
    float* __restrict__ out, double g2) {
  __shared__ double red[kThreads];
  const int k = blockIdx.x;
  const int64_t ca = bin_off[k], cb = bin_off[k + 1];
  const int64_t cnt = cb - ca;
  const int t = threadIdx.x;
  if (cnt == 0) {
    for (int d = t; d < L; d += kThreads) {
      const int64_t e = (int64_t)k * L + d;
      if (MODE == 0) {
        if (out != C_old) out[e] = C_old[e];
      } else {
        out[e] = 0.0f;
      }
    }
    return;
  }
  const int64_t r0 = ca / P, r1 = (cb - 1) / P;
  if (r0 == r1) return;  // finished by segsum
  int G2 = 1;
  while (G2 < L && G2 < kThreads) G2 <<= 1;
  const int Q = kThreads / G2;
  for (int d0 = 0; d0 < L; d0 += G2) {
    const int q = t / G2, d = d0 + t % G2;
    double s = 0.0;
    if (d < L) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int64_t r = r0 + 1 + q;
      for (; r + 3 * Q <= r1; r += 4 * Q) {
        a0 += partial[(r * 2) * LPD + d];
        a1 += partial[((r + Q) * 2) * LPD + d];
        a2 += partial[((r + 2 * Q) * 2) * LPD + d];
        a3 += partial[((r + 3 * Q) * 2) * LPD + d];
      }
      for (; r <= r1; r += Q) a0 += partial[(r * 2) * LPD + d];
      s = (a0 + a1) + (a2 + a3);
    }
    red[t] = s;
    __syncthreads();
    if (t < G2 && d < L) {
      double v = partial[(r0 * 2 + 1) * LPD + d];
      for (int qi = 0; qi < Q; ++qi) v += red[qi * G2 + t];
      out[(int64_t)k * L + d] = (float)((MODE == 0) ? v / (double)cnt : g2 * v);
    }
    __syncthreads();
  }
}

int group_lanes(int64_t L) {
  int g = 1;
  while (g < L && g < 64) g <<= 1;
  return g;
}

template <int MODE>
int launch_segsum(int G, int DPL, const float* X, int L, const int32_t* perm,
                  const int32_t* bin_off, int N, int64_t P, int64_t nruns,
                  const float* C_old, float* out, double g2, double* partial,
                  hipStream_t s) {
  const int64_t grid = (nruns + (kThreads / G) - 1) / (kThreads / G);
  const dim3 gd((unsigned)grid), bd(kThreads);
#define LBG_SEG(GG, DD)                                                        \
  if (G == GG && DPL == DD) {                                                  \
    hipLaunchKernelGGL((segsum_kernel<GG, DD, MODE>), gd, bd, 0, s, X, L, perm, \
                       bin_off, N, P, nruns, C_old, out, g2, partial);          \
    LBG_TRY_HIP(hipGetLastError());                                            \
    return LBG_OK;                                                             \
  }
  LBG_SEG(1, 1)
  LBG_SEG(2, 1)
  LBG_SEG(4, 1)
  LBG_SEG(8, 1)
  LBG_SEG(16, 1)
  LBG_SEG(32, 1)
  LBG_SEG(64, 1)
  LBG_SEG(64, 2)
  LBG_SEG(64, 3)
  LBG_SEG(64, 4)
#undef LBG_SEG
  set_error("internal: no segmented-sum kernel for G=%d DPL=%d", G, DPL);
  return LBG_EINVAL;
}

}  // namespace

void plan_update(Carver& c, int64_t M, int64_t L, int64_t N, UpdateWs* ws) {
  ws->use_afp = afp_usable(L, N);
  if (ws->use_afp) {
    plan_afp(c, M, L, N, &ws->afp);
    return;
  }
  // Sort tile: enough tiles for parallelism, histogram at most 4M entries.
  const int64_t max_entries = (int64_t)4 << 20;
  int64_t T = 256;
  while (T < 8192 && ((M + T - 1) / T) * N > max_entries) T <<= 1;
  if (((M + T - 1) / T) * N > max_entries) {
    const int64_t nt = max((int64_t)1, max_entries / N);
    T = ((M + nt - 1) / nt + 63) / 64 * 64;
  }
  ws->T = T;
  ws->ntiles = max((int64_t)1, (M + T - 1) / T);
  // Runs of the sorted order: about 8192 groups of lanes.
  ws->P = max((int64_t)16, (M + 8191) / 8192);
  ws->nruns = max((int64_t)1, (M + ws->P - 1) / ws->P);
  const int G = group_lanes(L);
  const int DPL = (int)((L + G - 1) / G);
  ws->LP = (int64_t)G * DPL;
  ws->ghist = c.take<int32_t>((size_t)(N * ws->ntiles));
  ws->bin_off = c.take<int32_t>((size_t)(N + 1));
  ws->perm = c.take<int32_t>((size_t)max((int64_t)1, M));
  ws->partial = c.take<double>((size_t)(ws->nruns * 2 * ws->LP));
  ws->cnt = c.take<int32_t>((size_t)N);
}

int launch_update(const float* X, int64_t M, int64_t L, const int32_t* idx,
                  const float* C_old, int64_t N, float* C_out, int32_t* counts,
                  int mode, double g2, const UpdateWs& ws, bool shift_ready,
                  hipStream_t s, int on_grid) {
  if (ws.use_afp) {
    if (!shift_ready) LBG_TRY(launch_afp_shift(X, M, L, ws.afp, s));
    return launch_afp(X, M, L, idx, C_old, N, C_out, counts, mode, g2, ws.afp, s,
                      Ctl{nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr},
                      CbPair{{nullptr, nullptr}}, shift_ready ? on_grid : 0);
  }
  const int n = (int)N, Li = (int)L;
  int32_t* cnt = ws.cnt;
  const bool lds = N <= kLdsCells;
  if (lds) {
    hipLaunchKernelGGL(hist_kernel, dim3((unsigned)ws.ntiles), dim3(kThreads),
                       (size_t)N * sizeof(int32_t), s, idx, M, n, ws.T, ws.ntiles,
                       ws.ghist);
  } else {
    hipLaunchKernelGGL(hist_global_kernel, dim3((unsigned)ws.ntiles), dim3(kThreads), 0,
                       s, idx, M, n, ws.T, ws.ntiles, ws.ghist);
  }
  LBG_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)N), dim3(kThreads), 0, s,
                     ws.ghist, ws.ntiles, cnt);
  LBG_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(scan_bins_kernel, dim3(1), dim3(1024), 0, s, cnt, n, ws.bin_off,
                     counts);
  LBG_TRY_HIP(hipGetLastError());
  int nbits = 0;
  while ((1 << nbits) < n) ++nbits;
  if (lds)
    hipLaunchKernelGGL(scatter_kernel<true>, dim3((unsigned)ws.ntiles), dim3(64),
                       (size_t)N * sizeof(int32_t), s, idx, M, n, nbits, ws.T, ws.ntiles,
                       ws.ghist, ws.bin_off, ws.perm);
  else
    hipLaunchKernelGGL(scatter_kernel<false>, dim3((unsigned)ws.ntiles), dim3(64), 0, s,
                       idx, M, n, nbits, ws.T, ws.ntiles, ws.ghist, ws.bin_off, ws.perm);
  LBG_TRY_HIP(hipGetLastError());
  const int G = group_lanes(L);
  const int DPL = (int)((L + G - 1) / G);
  if (mode == 0)
    LBG_TRY(launch_segsum<0>(G, DPL, X, Li, ws.perm, ws.bin_off, n, ws.P, ws.nruns,
                             C_old, C_out, g2, ws.partial, s));
  else
    LBG_TRY(launch_segsum<1>(G, DPL, X, Li, ws.perm, ws.bin_off, n, ws.P, ws.nruns,
                             C_old, C_out, g2, ws.partial, s));
  const int64_t grid = N;
  if (mode == 0)
    hipLaunchKernelGGL(finalize_kernel<0>, dim3((unsigned)grid), dim3(kThreads), 0, s,
                       ws.bin_off, n, Li, (int)ws.LP, ws.P, ws.partial, C_old, C_out, g2);
  else
    hipLaunchKernelGGL(finalize_kernel<1>, dim3((unsigned)grid), dim3(kThreads), 0, s,
                       ws.bin_off, n, Li, (int)ws.LP, ws.P, ws.partial, C_old, C_out, g2);
  LBG_TRY_HIP(hipGetLastError());
  return LBG_OK;
}

}  // namespace lbg
