// Device-side control of a training run: the block-wide "decide" step that
// follows every allocation (see DevState in lbg_internal.h).
#pragma once

#include <math.h>

#include "lbg_internal.h"

namespace lbg {

// Outcome of the stop test after one allocation (Algorithm 1 with the
// library's readings):
//   - a forced count for the level (fixed_iters / forced): stop after it;
//   - otherwise stop when not first and (D_prev - D) <= thr * D_prev, or at
//     max_iter updates (status LBG_WMAXITER);
//   - on a stop: done if the codebook has N codevectors, else split;
//   - otherwise update.
//   - a distortion that is not finite (a NaN or infinite coordinate in the
//     training set or the starting codebook) ends the run with LBG_EINVAL.
struct Step {
  int action;
  bool stop, capped, bad;
};

__device__ inline Step step_of(const DevState* st, double D) {
  if (!isfinite(D)) return Step{kActNone, true, false, true};
  int forced = -1;
  if (st->fixed_iters > 0) forced = st->fixed_iters;
  if (st->level < st->n_forced && st->level < 32) forced = st->forced[st->level];
  Step r{kActUpdate, false, false, false};
  if (forced >= 0) {
    r.stop = st->it >= forced;
  } else {
    r.stop = !st->first && (st->D_prev - D) <= st->thr * st->D_prev;
    if (!r.stop && st->it >= st->max_iter) {
      r.stop = true;
      r.capped = true;
    }
  }
  if (r.stop) r.action = (st->n >= st->N) ? kActNone : kActSplit;
  return r;
}

// Whether this allocation ends its level by a forced update count
// (fixed_iters / forced), which does not depend on the distortion: the
// accumulation of such an iteration is never used and can be skipped.
__device__ inline bool forced_stop(const DevState* st) {
  int forced = -1;
  if (st->fixed_iters > 0) forced = st->fixed_iters;
  if (st->level < st->n_forced && st->level < 32) forced = st->forced[st->level];
  return forced >= 0 && st->it >= forced;
}

// The state after the step: names the buffers of this iteration's update /
// split and the codebook of the next allocation.  ``out`` starts as a copy
// of ``in``; one thread.
__device__ inline void apply_step(const DevState* in, DevState* out, double D, Step r,
                                  double* Dtrace, int32_t* Atrace) {
  const int a = in->n_assign;
  out->n_assign = a + 1;
  out->distances = in->distances + in->M * (int64_t)in->n;
  out->D = D;
  if (Dtrace && a < in->D_cap) Dtrace[a] = D;
  if (Atrace && a < in->D_cap) Atrace[a] = r.action;
  if (r.capped) out->status = LBG_WMAXITER;
  if (r.bad) out->status = LBG_EINVAL;
  out->action = r.action;
  if (r.stop) {
    if (in->level < 32) {
      out->level_n[in->level] = in->n;
      out->level_iters[in->level] = in->it;
    }
    out->level = in->level + 1;
    if (r.action == kActNone) {
      out->done = 1;
    } else {
      out->src = in->cb;
      out->dst = in->cb ^ 1;
      out->n_src = in->n;
      out->cb = in->cb ^ 1;
      out->n = 2 * in->n;
      out->D_prev = INFINITY;
      out->first = 1;
      out->it = 0;
    }
  } else {
    out->src = in->cb;
    out->dst = in->cb ^ 1;
    out->n_src = in->n;
    out->cb = in->cb ^ 1;
    out->D_prev = D;
    out->first = 0;
    out->it = in->it + 1;
    out->n_update = in->n_update + 1;
  }
}

// Value of lane l ^ OFF (exactly), by VALU lane operations except for OFF 4.
template <int OFF>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
  if constexpr (OFF == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (threadIdx.x & 32) ? r[0] : r[1];
  } else if constexpr (OFF == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (threadIdx.x & 16) ? r[0] : r[1];
  } else if constexpr (OFF == 8) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x128, 0xf, 0xf, false);  // row_ror:8
  } else if constexpr (OFF == 4) {
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (4 << 10) | 0x1f);
  } else {
    static_assert(OFF == 1 || OFF == 2, "lane distance");
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, OFF == 1 ? 0xb1 : 0x4e, 0xf,
                                                 0xf, false);  // quad_perm
  }
}

template <int OFF>
__device__ __forceinline__ double lane_xor(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint64_t lo = lane_xor<OFF>((uint32_t)b), hi = lane_xor<OFF>((uint32_t)(b >> 32));
  return __longlong_as_double((long long)((hi << 32) | lo));
}

// Block-wide sum(parts) in a fixed order, valid in thread 0: thread t < 256
// adds parts t, t+256, ... in order, then the tree red[t] += red[t + off]
// for off = 128, 64, ..., 1.  Wave 0 forms the levels 128 and 64 from LDS
// (lane l: (red[l] + red[l+128]) + (red[l+64] + red[l+192])) and the rest
// from its registers (lane l < off adds lane l + off = l ^ off), so there is
// one barrier.  ``red`` is 256 doubles of LDS; blockDim.x must be at least 256.
// A thread issues 32 loads before its first addition (up to 8192 partials
// in one memory round trip); positions past the end read as +0, which
// leaves the non-negative sum unchanged.
__device__ inline double block_sum0(const double* __restrict__ parts, int64_t nparts,
                                    double* red) {
  constexpr int U = 32;
  double acc = 0.0;
  if (threadIdx.x < 256) {
    for (int64_t b = threadIdx.x; b < nparts; b += 256 * U) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t p = b + 256 * u;
        v[u] = p < nparts ? parts[p] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc += v[u];
    }
    red[threadIdx.x] = acc;
  }
  __syncthreads();
  double v = 0.0;
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    v = (red[l] + red[l + 128]) + (red[l + 64] + red[l + 192]);
    v = v + lane_xor<32>(v);
    v = v + lane_xor<16>(v);
    v = v + lane_xor<8>(v);
    v = v + lane_xor<4>(v);
    v = v + lane_xor<2>(v);
    v = v + lane_xor<1>(v);
  }
  __syncthreads();  // red may be reused
  return v;
}

// Decide step by one block (the standalone kernel): the state is updated in
// place.
__device__ inline void decide_block(const double* __restrict__ parts, int64_t nparts,
                                    DevState* st, double* __restrict__ Dtrace,
                                    int32_t* __restrict__ Atrace, double* red) {
  const double S = block_sum0(parts, nparts, red);
  if (threadIdx.x != 0) return;
  const double D = S / (double)st->M;
  const Step r = step_of(st, D);
  apply_step(st, st, D, r, Dtrace, Atrace);
}

}  // namespace lbg
