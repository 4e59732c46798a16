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
struct Step {
  int action;
  bool stop, capped;
};

__device__ inline Step step_of(const DevState* st, double D) {
  int forced = -1;
  if (st->fixed_iters > 0) forced = st->fixed_iters;
  if (st->level < st->n_forced && st->level < 32) forced = st->forced[st->level];
  Step r{kActUpdate, false, false};
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

// Block-wide D = sum(parts) / M in a fixed order: thread t adds parts t,
// t+256, ..., then a fixed tree.  Every block that calls it gets the same
// value.  ``red`` is 256 doubles of LDS; blockDim.x must be at least 256
// (threads beyond the first 256 only take part in the barriers).  A thread
// issues 32 loads before its first addition (up to 8192 partials in one
// memory round trip); positions past the end read as +0, which leaves the
// non-negative sum unchanged.
__device__ inline double block_distortion(const double* __restrict__ parts, int64_t nparts,
                                          int64_t M, double* red) {
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
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double D = red[0] / (double)M;
  __syncthreads();
  return D;
}

// Decide step by one block (the standalone kernel): the state is updated in
// place.
__device__ inline void decide_block(const double* __restrict__ parts, int64_t nparts,
                                    DevState* st, double* __restrict__ Dtrace,
                                    int32_t* __restrict__ Atrace, double* red) {
  const double D = block_distortion(parts, nparts, st->M, red);
  if (threadIdx.x != 0) return;
  const Step r = step_of(st, D);
  apply_step(st, st, D, r, Dtrace, Atrace);
}

}  // namespace lbg
