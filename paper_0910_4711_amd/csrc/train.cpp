// LBG with splitting (Algorithm 1) with the iteration / level control on the
// device.  The host enqueues batches of kBatchIters iterations -- allocation,
// decide, update, split -- and reads the device state after each batch; the
// decide kernel makes every later kernel of a finished run a no-op.  On a
// non-default stream a batch is a hipGraph, captured once per set of
// buffers and sizes and kept in a small cache.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "lbg_internal.h"

namespace lbg {
namespace {

constexpr int kBatchIters = 8;
// Iterations per batch once the final level has begun (untimed direct
// launches): a run ends during it, and a shorter batch leaves fewer no-op
// launches queued behind the last iteration.
constexpr int kTailIters = 2;
// Timing events only order the stream on the device: no system-scope fence.
constexpr unsigned kEventFlags = hipEventDisableSystemFence;

struct GraphKey {
  const void* X;
  const void* ws;
  const void* idx;
  int64_t M, L, N;
  int precision, split_mode, timed, on_grid;
  double eps, delta;
  hipStream_t stream;
  bool operator==(const GraphKey& o) const { return memcmp(this, &o, sizeof(*this)) == 0; }
};

struct GraphEntry {
  bool used = false;
  GraphKey key;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  bool timed = false;
  hipEvent_t ev[kBatchIters][3][2];
  uint64_t stamp = 0;
};

constexpr int kCacheSize = 8;
std::mutex g_cache_mu;
GraphEntry g_cache[kCacheSize];
uint64_t g_stamp = 0;

void release(GraphEntry& e) {
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.graph) (void)hipGraphDestroy(e.graph);
  if (e.timed)
    for (int i = 0; i < kBatchIters; ++i)
      for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 2; ++j) (void)hipEventDestroy(e.ev[i][k][j]);
  e = GraphEntry();
}

struct Batch {
  const float* X;
  int64_t M, L, N;
  int precision, split_mode;
  double eps, delta;
  int32_t* idx;
  const TrainWs* w;
  int64_t nparts;
  int on_grid;  // 1: the training set lies on the update's 2^-s grid; 2: its
                // cell sums also fit 32 bits (shift[3])
};

// One iteration is two pieces: the allocation, then the update, whose
// accumulation kernel also takes the decision of the iteration and whose
// last kernel performs a split instead when that is the decision.
constexpr int kPieces = 2;

int enqueue_piece(const Batch& b, int piece, hipStream_t s) {
  const TrainWs& w = *b.w;
  CbPair cbp{{w.Cb[0], w.Cb[1]}};
  const Ctl ctl{w.st, w.pend, w.as.dpart, b.nparts, w.Dtrace, w.Atrace, w.up.afp.shift};
  if (piece == 0)
    return launch_assign(b.X, b.M, b.L, nullptr, b.N, b.idx, nullptr, b.precision, w.as.dpart,
                         w.as.nfb, w.as.prep, s, ctl, cbp);
  return launch_afp(b.X, b.M, b.L, b.idx, nullptr, b.N, nullptr, nullptr, 0, 0.0, w.up.afp, s,
                    ctl, cbp, b.on_grid);
}

// Timing events of iteration i (nullable): ev[i][0][0] before the
// allocation, ev[i][0][1] between the allocation and the update, ev[i][1][1]
// after the update (three records per iteration).
inline hipEvent_t event_before(hipEvent_t (*ev)[3][2], int i, int piece) {
  return piece == 0 ? ev[i][0][0] : nullptr;
}
inline hipEvent_t event_after(hipEvent_t (*ev)[3][2], int i, int piece) {
  return piece == 0 ? ev[i][0][1] : ev[i][1][1];
}

// ``iters`` (at most kBatchIters) iterations launched directly; skip0: the
// first iteration's allocation is already enqueued.
int enqueue_batch(const Batch& b, hipStream_t s, hipEvent_t (*ev)[3][2],
                  int iters = kBatchIters, bool skip0 = false) {
  for (int i = 0; i < iters; ++i)
    for (int piece = (i == 0 && skip0) ? 1 : 0; piece < kPieces; ++piece) {
      if (ev && event_before(ev, i, piece))
        LBG_TRY_HIP(hipEventRecord(event_before(ev, i, piece), s));
      LBG_TRY(enqueue_piece(b, piece, s));
      if (ev) LBG_TRY_HIP(hipEventRecord(event_after(ev, i, piece), s));
    }
  return LBG_OK;
}

// The same iterations as one graph (opt-in: on gfx950 with ROCm 7.2 direct
// launches measured faster): each piece is captured once into a child graph;
// the batch chains kBatchIters copies of the four children, with
// event-record nodes around the timed pieces (events recorded by graph nodes
// added this way can be timed; events recorded during a capture cannot).
int build_batch_graph(const Batch& b, hipStream_t s, hipEvent_t (*ev)[3][2], hipGraph_t* out) {
  hipGraph_t child[kPieces] = {nullptr, nullptr};
  hipGraph_t g = nullptr;
  int rc = LBG_OK;
  auto cleanup = [&]() {
    for (auto& c : child)
      if (c) (void)hipGraphDestroy(c);
  };
  for (int piece = 0; piece < kPieces && rc == LBG_OK; ++piece) {
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      rc = hip_fail(e, "hipStreamBeginCapture");
      break;
    }
    rc = enqueue_piece(b, piece, s);
    e = hipStreamEndCapture(s, &child[piece]);
    if (rc == LBG_OK && e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
  }
  if (rc == LBG_OK) {
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) rc = hip_fail(e, "hipGraphCreate");
  }
  hipGraphNode_t prev = nullptr;
  for (int i = 0; i < kBatchIters && rc == LBG_OK; ++i)
    for (int piece = 0; piece < kPieces && rc == LBG_OK; ++piece) {
      hipGraphNode_t node;
      hipError_t e;
      if (ev && event_before(ev, i, piece)) {
        e = hipGraphAddEventRecordNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0,
                                       event_before(ev, i, piece));
        if (e != hipSuccess) { rc = hip_fail(e, "hipGraphAddEventRecordNode"); break; }
        prev = node;
      }
      e = hipGraphAddChildGraphNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, child[piece]);
      if (e != hipSuccess) { rc = hip_fail(e, "hipGraphAddChildGraphNode"); break; }
      prev = node;
      if (ev) {
        e = hipGraphAddEventRecordNode(&node, g, &prev, 1, event_after(ev, i, piece));
        if (e != hipSuccess) { rc = hip_fail(e, "hipGraphAddEventRecordNode"); break; }
        prev = node;
      }
    }
  cleanup();
  if (rc != LBG_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  *out = g;
  return LBG_OK;
}

double* pinned_block(size_t bytes) {
  static thread_local double* p = nullptr;
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

}  // namespace

bool train_device_ok(int64_t L, const TrainWs& w) { return w.up.use_afp && L <= 128; }

int train_device(const float* X, int64_t M, int64_t L, int64_t N, const lbg_params* p,
                 float* C_out, int32_t* idx_out, double* D_out, lbg_stats* st,
                 const TrainWs& w, hipStream_t s) {
  DevState hs;
  memset(&hs, 0, sizeof(hs));
  hs.N = (int32_t)N;
  hs.M = M;
  hs.max_iter = p->max_iter;
  hs.fixed_iters = p->fixed_iters;
  hs.split_mode = p->split_mode;
  hs.thr = p->thr;
  hs.eps = p->eps_split;
  hs.delta = p->delta;
  hs.D_cap = kTraceCap;
  // a level starts afresh, or resumes from C_init in its middle
  hs.D_prev = p->C_init ? p->D_prev_init : INFINITY;
  hs.first = hs.D_prev == INFINITY;
  hs.it = p->C_init ? p->it_init : 0;
  hs.status = LBG_OK;
  hs.n_forced = std::min(p->n_forced, 32);
  for (int i = 0; i < hs.n_forced; ++i) hs.forced[i] = p->forced_iters[i];

  CbPair cbp{{w.Cb[0], w.Cb[1]}};
  // the common start (centroid, split, shift, state) in two launches
  const bool fused_setup = !p->C_init && N >= 2;
  if (fused_setup) {
    hs.cb = 1;
    hs.n = 2;
  } else if (p->C_init) {
    LBG_TRY_HIP(hipMemcpyAsync(w.Cb[0], p->C_init, (size_t)(p->N_init * L) * sizeof(float),
                               hipMemcpyDeviceToDevice, s));
    hs.cb = 0;
    hs.n = (int32_t)p->N_init;
  } else {
    // N = 1: the centroid is the one-level codebook: one allocation, no update
    LBG_TRY(launch_centroid(X, M, L, w.Cb[0], w.ce, s));
    hs.cb = 0;
    hs.n = 1;
    hs.n_forced = 1;
    hs.forced[0] = 0;
  }
  // pinned host block: action trace, two state copies, the set-up flags,
  // the statistics words, the distortion trace.  Every readback lands in
  // pinned memory, so that the copies stay asynchronous (a copy into
  // pageable memory costs a host round trip of 20-30 us each).
  static_assert(sizeof(DevState) % 8 == 0, "state alignment");
  const size_t off_state = (size_t)kTraceCap * 4;
  const size_t off_flags = off_state + 2 * sizeof(DevState);
  const size_t off_words = off_flags + 8 * sizeof(int);
  const size_t off_trace = off_words + 4 * sizeof(unsigned long long);
  char* pbase = reinterpret_cast<char*>(pinned_block(off_trace + (size_t)kTraceCap * 8));
  if (!pbase) {
    set_error("could not allocate pinned host memory");
    return LBG_EHIP;
  }
  int32_t* acts = reinterpret_cast<int32_t*>(pbase);
  DevState* pins[2] = {reinterpret_cast<DevState*>(pbase + off_state),
                       reinterpret_cast<DevState*>(pbase + off_state) + 1};
  int* flags = reinterpret_cast<int*>(pbase + off_flags);
  unsigned long long* words = reinterpret_cast<unsigned long long*>(pbase + off_words);
  double* dtrace = reinterpret_cast<double*>(pbase + off_trace);
  DevState* pin = pins[0];
  memcpy(pin, &hs, sizeof(hs));
  if (fused_setup) {
    LBG_TRY(launch_setup(X, M, L, w.Cb[0], w.Cb[1], p->split_mode, p->eps_split, p->delta, w.ce,
                         w.up.afp.shift, w.up.afp.lo, w.up.afp.nlo, hs, w.st, w.as.nfb, s));
  } else {
    LBG_TRY_HIP(hipMemcpyAsync(w.st, pin, sizeof(DevState), hipMemcpyHostToDevice, s));
    LBG_TRY_HIP(hipMemsetAsync(w.as.nfb, 0, sizeof(unsigned long long), s));
    LBG_TRY(launch_afp_shift(X, M, L, w.up.afp, s));
  }

  // Whether the training set lies on the update's 2^-s grid (set-up pass):
  // read once, so that the accumulation runs its one-word kernel (the
  // kernel that decides on the device is larger and measured slower).
  // Untimed direct launches: the first allocation (which does not depend on
  // the flags) is enqueued before the host waits for them, so that the
  // device does not idle through that round trip.
  const bool timed = p->timing != 0 && st != nullptr;
  const bool use_graph = s != nullptr && p->graph != 0;
  Batch b{X, M, L, N, p->precision, p->split_mode, p->eps_split, p->delta, idx_out, &w,
          assign_num_parts(M, L, N, p->precision), 0};
  LBG_TRY_HIP(hipMemcpyAsync(flags, w.up.afp.shift, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
  bool skip0 = false;
  if (!timed && !use_graph) {
    hipEvent_t fev = nullptr;
    LBG_TRY_HIP(hipEventCreateWithFlags(&fev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(fev, s);
    int rc0 = e == hipSuccess ? enqueue_piece(b, 0, s) : hip_fail(e, "hipEventRecord");
    if (rc0 == LBG_OK) {
      skip0 = true;
      e = hipEventSynchronize(fev);
      if (e != hipSuccess) rc0 = hip_fail(e, "hipEventSynchronize");
    }
    (void)hipEventDestroy(fev);
    if (rc0 != LBG_OK) return rc0;
  } else {
    LBG_TRY_HIP(hipStreamSynchronize(s));
  }
  b.on_grid = flags[1] != 0 ? 0 : (flags[3] ? 2 : 1);

  GraphEntry* ge = nullptr;
  std::unique_lock<std::mutex> lk(g_cache_mu, std::defer_lock);
  hipEvent_t local_ev[kBatchIters][3][2];
  int local_ev_n = 0;
  auto destroy_local = [&]() {
    hipEvent_t* flat = &local_ev[0][0][0];
    for (int i = 0; i < local_ev_n; ++i) (void)hipEventDestroy(flat[i]);
    local_ev_n = 0;
  };
  if (use_graph) {
    lk.lock();
    GraphKey key;
    memset(&key, 0, sizeof(key));
    key.X = X;
    key.ws = w.Cb[0];
    key.idx = idx_out;
    key.M = M;
    key.L = L;
    key.N = N;
    key.precision = p->precision;
    key.split_mode = p->split_mode;
    key.timed = timed;
    key.on_grid = b.on_grid;
    key.eps = p->eps_split;
    key.delta = p->delta;
    key.stream = s;
    for (auto& e : g_cache)
      if (e.used && e.key == key) ge = &e;
    if (!ge) {
      GraphEntry* slot = &g_cache[0];
      for (auto& e : g_cache) {
        if (!e.used) {
          slot = &e;
          break;
        }
        if (e.stamp < slot->stamp) slot = &e;
      }
      release(*slot);
      slot->key = key;
      slot->timed = timed;
      if (timed)
        for (int i = 0; i < kBatchIters; ++i)
          for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 2; ++j)
              LBG_TRY_HIP(hipEventCreateWithFlags(&slot->ev[i][k][j], kEventFlags));
      hipGraph_t g = nullptr;
      const int rc = build_batch_graph(b, s, timed ? slot->ev : nullptr, &g);
      if (rc < 0) {
        release(*slot);
        return rc;
      }
      slot->graph = g;
      LBG_TRY_HIP(hipGraphInstantiate(&slot->exec, g, nullptr, nullptr, 0));
      slot->used = true;
      ge = slot;
    }
    ge->stamp = ++g_stamp;
  } else if (timed) {
    for (int i = 0; i < kBatchIters; ++i)
      for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 2; ++j) {
          LBG_TRY_HIP(hipEventCreateWithFlags(&local_ev[i][k][j], kEventFlags));
          ++local_ev_n;
        }
  }

  // When every level's update count is forced (fixed_iters, or a forced
  // list covering every level) the run takes exactly sum(count + 1)
  // iterations whatever its distortions (fewer only if one is not finite):
  // the host then enqueues no iteration beyond that, so no launches that
  // return at once trail the run.  -1: no such bound.
  int64_t left = -1;
  {
    int levels = 1;
    for (int64_t n = hs.n; n < N; n *= 2) ++levels;
    int64_t sum = 0;
    int it = hs.it;
    for (int l = 0; l < levels && sum >= 0; ++l) {
      int f = hs.fixed_iters > 0 ? hs.fixed_iters : -1;
      if (l < hs.n_forced && l < 32) f = hs.forced[l];
      sum = f < 0 ? -1 : sum + std::max(f - it, 0) + 1;
      it = 0;
    }
    left = sum;
  }
  double ms[3] = {0.0, 0.0, 0.0};
  int32_t prev_assign = 0;
  int rc = LBG_OK;
  int iters = kBatchIters;  // of the next untimed direct batch
  int64_t enqueued = 0;     // iterations enqueued directly so far
  auto launch_batch = [&]() -> int {
    if (ge) {
      const hipError_t e = hipGraphLaunch(ge->exec, s);
      return e == hipSuccess ? LBG_OK : hip_fail(e, "hipGraphLaunch");
    }
    int k = timed ? kBatchIters : iters;
    if (left >= 0) {
      k = (int)std::min<int64_t>(k, left);
      left -= k;
    }
    enqueued += k;
    if (k == 0) return LBG_OK;
    const bool sk = skip0;
    skip0 = false;
    return timed ? enqueue_batch(b, s, local_ev, k) : enqueue_batch(b, s, nullptr, k, sk);
  };
  if (!timed) {
    // The next batch is enqueued before this batch's state is read back (its
    // kernels return at once when the run has finished in this batch), so
    // the device does not wait for the host between batches.
    hipEvent_t read[2] = {nullptr, nullptr};
    int64_t before_read[2] = {0, 0};  // iterations enqueued ahead of each readback
    for (auto& e : read)
      if (rc == LBG_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        rc = hip_fail(hipGetLastError(), "hipEventCreate");
    if (rc == LBG_OK) rc = launch_batch();
    for (int cur = 0; rc == LBG_OK; cur ^= 1) {
      if (hipMemcpyAsync(pins[cur], w.st, sizeof(DevState), hipMemcpyDeviceToHost, s) !=
              hipSuccess ||
          hipEventRecord(read[cur], s) != hipSuccess) {
        rc = hip_fail(hipGetLastError(), "state readback");
        break;
      }
      before_read[cur] = enqueued;
      rc = launch_batch();
      if (rc < 0) break;
      if (hipEventSynchronize(read[cur]) != hipSuccess) {
        rc = hip_fail(hipGetLastError(), "state readback");
        break;
      }
      if (pins[cur]->done) {
        pin = pins[cur];
        break;
      }
      // not done after every bounded iteration (not expected): go on unbounded
      if (left == 0 && before_read[cur] == enqueued) left = -1;
      if (pins[cur]->n >= N) iters = kTailIters;
    }
    for (auto& e : read)
      if (e) (void)hipEventDestroy(e);
  }
  // timed: one batch at a time, its events read after it
  for (; timed && rc == LBG_OK;) {
    rc = launch_batch();
    if (rc < 0) break;
    if (hipMemcpyAsync(pin, w.st, sizeof(DevState), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(acts, w.Atrace, kTraceCap * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = hip_fail(hipGetLastError(), "state readback");
      break;
    }
    hipEvent_t(*ev)[3][2] = ge ? ge->ev : local_ev;
    for (int i = 0; i < kBatchIters; ++i) {
      const int a = prev_assign + i;
      if (a >= pin->n_assign) break;
      float t = 0.0f;
      if (hipEventElapsedTime(&t, ev[i][0][0], ev[i][0][1]) == hipSuccess) ms[0] += t;
      const int act = a < kTraceCap ? acts[a] : kActNone;
      if (act == kActUpdate && hipEventElapsedTime(&t, ev[i][0][1], ev[i][1][1]) == hipSuccess)
        ms[1] += t;
    }
    prev_assign = pin->n_assign;
    if (pin->done) break;
    if (left == 0) left = -1;  // not done after every bounded iteration (not expected)
  }
  if (lk.owns_lock()) lk.unlock();
  destroy_local();
  if (rc < 0) return rc;

  LBG_TRY_HIP(hipMemcpyAsync(C_out, w.Cb[pin->cb], (size_t)(N * L) * sizeof(float),
                             hipMemcpyDeviceToDevice, s));
  if (st) {
    unsigned long long* rs = words;  // empty cells, near-tie rows
    unsigned long long* nf = words + 2;
    rs[0] = rs[1] = *nf = 0;
    // statistics of the final allocation (before the one synchronisation)
    if (pin->status != LBG_EINVAL) {
      LBG_TRY(launch_run_stats(X, M, L, w.Cb[pin->cb], N, idx_out, p->stats_ties != 0,
                               w.cellcnt, w.runstat, s));
      LBG_TRY_HIP(hipMemcpyAsync(rs, w.runstat, 2 * sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, s));
    }
    LBG_TRY_HIP(hipMemcpyAsync(nf, w.as.nfb, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    const int nD = std::min(pin->n_assign, std::min(st->D_cap, kTraceCap));
    if (st->D_trace && nD > 0)
      LBG_TRY_HIP(hipMemcpyAsync(dtrace, w.Dtrace, (size_t)nD * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
    LBG_TRY_HIP(hipStreamSynchronize(s));
    if (st->D_trace && nD > 0) memcpy(st->D_trace, dtrace, (size_t)nD * sizeof(double));
    st->fallback_rows = (int64_t)*nf;
    st->n_D = pin->n_assign;
    st->total_assigns = pin->n_assign;
    st->total_updates = pin->n_update;
    st->total_distances = pin->distances;
    st->n_levels = pin->level;
    for (int i = 0; i < std::min(pin->level, 32); ++i) {
      st->level_n[i] = pin->level_n[i];
      st->level_iters[i] = pin->level_iters[i];
    }
    st->ms_assign = ms[0];
    st->ms_update = ms[1];
    st->ms_split = ms[2];
    st->empty_cells = (int32_t)rs[0];
    st->near_tie_rows = p->stats_ties && pin->status != LBG_EINVAL ? (int64_t)rs[1] : -1;
  } else {
    LBG_TRY_HIP(hipStreamSynchronize(s));
  }
  *D_out = pin->D;
  if (pin->status == LBG_EINVAL)
    set_error("the distortion is not finite: the training set or the starting codebook holds "
              "a NaN or infinite value");
  return pin->status;
}

}  // namespace lbg
