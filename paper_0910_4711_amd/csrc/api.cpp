// C ABI entry points: argument checks, workspace layout, and the level /
// iteration control of LBG with splitting (Algorithm 1).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "lbg_internal.h"

namespace lbg {

static thread_local char g_err[512];

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = 0; }

int hip_fail(hipError_t e, const char* what) {
  set_error("HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
  return LBG_EHIP;
}

namespace {

bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3) == 0; }
bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int check_dims(int64_t M, int64_t L, int64_t N) {
  if (M < 1 || M > LBG_MAX_M) {
    set_error("M = %lld outside [1, %lld]", (long long)M, (long long)LBG_MAX_M);
    return LBG_EINVAL;
  }
  if (L < 1 || L > LBG_MAX_L) {
    set_error("L = %lld outside [1, %d]", (long long)L, LBG_MAX_L);
    return LBG_EINVAL;
  }
  if (N < 1 || N > LBG_MAX_N) {
    set_error("N = %lld outside [1, %d]", (long long)N, LBG_MAX_N);
    return LBG_EINVAL;
  }
  return LBG_OK;
}

int need(const void* p, const char* name) {
  if (!p) {
    set_error("%s is NULL", name);
    return LBG_EINVAL;
  }
  if (!aligned4(p)) {
    set_error("%s is not 4-byte aligned", name);
    return LBG_EINVAL;
  }
  return LBG_OK;
}

int check_ws(void* ws, size_t have, size_t want) {
  if (have < want) {
    set_error("workspace too small: %zu bytes given, %zu needed", have, want);
    return LBG_ENOWS;
  }
  if (want > 0 && !ws) {
    set_error("workspace is NULL");
    return LBG_EINVAL;
  }
  if (want > 0 && (reinterpret_cast<uintptr_t>(ws) & 255)) {
    set_error("workspace is not 256-byte aligned");
    return LBG_EINVAL;
  }
  return LBG_OK;
}

int check_precision(int precision) {
  if (precision != LBG_FP32 && precision != LBG_BF16_RESCORE) {
    set_error("unknown precision %d", precision);
    return LBG_EINVAL;
  }
  return LBG_OK;
}

}  // namespace

void plan_train(Carver& c, int64_t M, int64_t L, int64_t N, int precision, TrainWs* w) {
  w->Cb[0] = c.take<float>((size_t)(N * L));
  w->Cb[1] = c.take<float>((size_t)(N * L));
  w->D = c.take<double>(1);
  plan_assign(c, M, L, N, precision, &w->as);
  plan_update(c, M, L, N, &w->up);
  plan_centroid(c, M, L, &w->ce);
  w->st = c.take<DevState>(1);
  w->pend = c.take<DevState>(1);
  w->Dtrace = c.take<double>((size_t)kTraceCap);
  w->Atrace = c.take<int32_t>((size_t)kTraceCap);
  w->cellcnt = c.take<int32_t>((size_t)N);
  w->runstat = c.take<unsigned long long>(2);
}

int run_stats(const float* X, int64_t M, int64_t L, int64_t N, const float* C,
              const int32_t* idx, const lbg_params* p, lbg_stats* st, const TrainWs& w,
              hipStream_t s) {
  LBG_TRY(launch_run_stats(X, M, L, C, N, idx, p->stats_ties != 0, w.cellcnt, w.runstat, s));
  unsigned long long h[2] = {0, 0};
  LBG_TRY_HIP(hipMemcpyAsync(h, w.runstat, sizeof(h), hipMemcpyDeviceToHost, s));
  LBG_TRY_HIP(hipStreamSynchronize(s));
  st->empty_cells = (int32_t)h[0];
  st->near_tie_rows = p->stats_ties ? (int64_t)h[1] : -1;
  return LBG_OK;
}

namespace {

double* pinned_scalar() {
  static thread_local double* p = nullptr;
  if (!p) {
    if (hipHostMalloc(reinterpret_cast<void**>(&p), 2 * sizeof(double),
                      hipHostMallocDefault) != hipSuccess)
      p = nullptr;
  }
  return p;
}

int read_scalar(const double* dev, double* host, hipStream_t s) {
  double* pin = pinned_scalar();
  if (!pin) {
    set_error("could not allocate pinned host memory");
    return LBG_EHIP;
  }
  LBG_TRY_HIP(hipMemcpyAsync(pin, dev, sizeof(double), hipMemcpyDeviceToHost, s));
  LBG_TRY_HIP(hipStreamSynchronize(s));
  *host = pin[0];
  return LBG_OK;
}

// Event pairs around kernel groups; durations are summed per kind once the
// stream has passed both events (collect() after a synchronisation).
struct Timer {
  enum { kAssign = 0, kUpdate = 1, kSplit = 2, kKinds = 3, kPairs = 8 };
  bool on;
  hipEvent_t ev[kPairs][2];
  int kind[kPairs];
  int used = 0;
  int created = 0;
  double ms[kKinds] = {0.0, 0.0, 0.0};
  explicit Timer(bool enable) : on(enable) {}
  ~Timer() {
    for (int i = 0; i < created; ++i) {
      (void)hipEventDestroy(ev[i][0]);
      (void)hipEventDestroy(ev[i][1]);
    }
  }
  int init() {
    if (!on) return LBG_OK;
    for (; created < kPairs; ++created) {
      LBG_TRY_HIP(hipEventCreate(&ev[created][0]));
      if (hipEventCreate(&ev[created][1]) != hipSuccess) {
        (void)hipEventDestroy(ev[created][0]);
        set_error("hipEventCreate failed");
        return LBG_EHIP;
      }
    }
    return LBG_OK;
  }
  int begin(int k, hipStream_t s) {
    if (!on) return LBG_OK;
    if (used == kPairs) {  // all pairs pending: wait and harvest them
      LBG_TRY_HIP(hipStreamSynchronize(s));
      LBG_TRY(collect());
    }
    kind[used] = k;
    LBG_TRY_HIP(hipEventRecord(ev[used][0], s));
    return LBG_OK;
  }
  int end(hipStream_t s) {
    if (!on) return LBG_OK;
    LBG_TRY_HIP(hipEventRecord(ev[used][1], s));
    ++used;
    return LBG_OK;
  }
  // Only after the stream has been synchronised past every recorded pair.
  int collect() {
    if (!on) return LBG_OK;
    for (int i = 0; i < used; ++i) {
      float t = 0.0f;
      LBG_TRY_HIP(hipEventElapsedTime(&t, ev[i][0], ev[i][1]));
      ms[kind[i]] += t;
    }
    used = 0;
    return LBG_OK;
  }
};

}  // namespace
}  // namespace lbg

using namespace lbg;

extern "C" {

const char* lbg_last_error(void) { return g_err; }

const char* lbg_version(void) { return "lbg-mi355x 0.1 (gfx950)"; }

void lbg_params_default(lbg_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->thr = 1e-3;
  p->eps_split = 0.01;
  p->delta = 0.0;
  p->split_mode = LBG_SPLIT_MULT;
  p->max_iter = 1000;
  p->precision = LBG_FP32;
  p->fixed_iters = 0;
  p->forced_iters = nullptr;
  p->n_forced = 0;
  p->C_init = nullptr;
  p->N_init = 0;
  p->timing = 0;
  p->graph = 0;
  p->D_prev_init = INFINITY;
  p->it_init = 0;
  p->stats_ties = 0;
}

size_t lbg_workspace_size(int op, int64_t M, int64_t L, int64_t N, int precision) {
  Carver c{nullptr, 0};
  M = std::max<int64_t>(M, 1);
  L = std::max<int64_t>(L, 1);
  N = std::max<int64_t>(N, 1);
  switch (op) {
    case LBG_OP_ASSIGN: {
      AssignWs w;
      plan_assign(c, M, L, N, precision, &w);
      return c.size();
    }
    case LBG_OP_UPDATE:
    case LBG_OP_BACKWARD: {
      UpdateWs w;
      plan_update(c, M, L, N, &w);
      return c.size();
    }
    case LBG_OP_DISTORTION: {
      DistWs w;
      plan_distortion(c, M, &w);
      return c.size();
    }
    case LBG_OP_CENTROID: {
      CentroidWs w;
      plan_centroid(c, M, L, &w);
      return c.size();
    }
    case LBG_OP_TRAIN: {
      TrainWs w;
      plan_train(c, M, L, N, precision, &w);
      return c.size();
    }
    default:
      return 0;
  }
}

int lbg_split(const float* C, int64_t n, int64_t L, double eps, float* C2,
              void* stream) {
  clear_error();
  LBG_TRY(check_dims(1, L, n));
  if (2 * n > LBG_MAX_N) {
    set_error("split would exceed %d codevectors", LBG_MAX_N);
    return LBG_EINVAL;
  }
  LBG_TRY(need(C, "C"));
  LBG_TRY(need(C2, "C2"));
  if (!(eps > 0.0 && eps < 1.0)) {
    set_error("eps = %g outside (0, 1)", eps);
    return LBG_EINVAL;
  }
  const char* a = reinterpret_cast<const char*>(C);
  const char* b = reinterpret_cast<const char*>(C2);
  if (b < a + n * L * 4 && a < b + 2 * n * L * 4) {
    set_error("C2 overlaps C");
    return LBG_EINVAL;
  }
  return launch_split(C, n, L, LBG_SPLIT_MULT, eps, 0.0, C2, (hipStream_t)stream);
}

int lbg_split_add(const float* C, int64_t n, int64_t L, double delta, float* C2,
                  void* stream) {
  clear_error();
  LBG_TRY(check_dims(1, L, n));
  if (2 * n > LBG_MAX_N) {
    set_error("split would exceed %d codevectors", LBG_MAX_N);
    return LBG_EINVAL;
  }
  LBG_TRY(need(C, "C"));
  LBG_TRY(need(C2, "C2"));
  if (!isfinite(delta)) {
    set_error("delta is not finite");
    return LBG_EINVAL;
  }
  const char* a = reinterpret_cast<const char*>(C);
  const char* b = reinterpret_cast<const char*>(C2);
  if (b < a + n * L * 4 && a < b + 2 * n * L * 4) {
    set_error("C2 overlaps C");
    return LBG_EINVAL;
  }
  return launch_split(C, n, L, LBG_SPLIT_ADD, 0.0, delta, C2, (hipStream_t)stream);
}

int lbg_centroid(const float* X, int64_t M, int64_t L, float* c0, void* ws,
                 size_t ws_bytes, void* stream) {
  clear_error();
  LBG_TRY(check_dims(M, L, 1));
  LBG_TRY(need(X, "X"));
  LBG_TRY(need(c0, "c0"));
  Carver c{reinterpret_cast<char*>(ws), 0};
  CentroidWs w;
  plan_centroid(c, M, L, &w);
  LBG_TRY(check_ws(ws, ws_bytes, c.size()));
  return launch_centroid(X, M, L, c0, w, (hipStream_t)stream);
}

int lbg_assign(const float* X, int64_t M, int64_t L, const float* C, int64_t N,
               int32_t* idx, float* mind, int precision, void* ws, size_t ws_bytes,
               void* stream) {
  clear_error();
  LBG_TRY(check_dims(M, L, N));
  LBG_TRY(check_precision(precision));
  LBG_TRY(need(X, "X"));
  LBG_TRY(need(C, "C"));
  LBG_TRY(need(idx, "idx"));
  if (mind && !aligned4(mind)) {
    set_error("mind is not 4-byte aligned");
    return LBG_EINVAL;
  }
  Carver c{reinterpret_cast<char*>(ws), 0};
  AssignWs w;
  plan_assign(c, M, L, N, precision, &w);
  LBG_TRY(check_ws(ws, ws_bytes, c.size()));
  return launch_assign(X, M, L, C, N, idx, mind, precision, nullptr, nullptr, w.prep,
                       (hipStream_t)stream);
}

int lbg_assign_distortion(const float* X, int64_t M, int64_t L, const float* C, int64_t N,
                          int32_t* idx, float* mind, int precision, double* D, void* ws,
                          size_t ws_bytes, void* stream) {
  clear_error();
  LBG_TRY(check_dims(M, L, N));
  LBG_TRY(check_precision(precision));
  LBG_TRY(need(X, "X"));
  LBG_TRY(need(C, "C"));
  LBG_TRY(need(idx, "idx"));
  LBG_TRY(need(D, "D"));
  if (mind && !aligned4(mind)) {
    set_error("mind is not 4-byte aligned");
    return LBG_EINVAL;
  }
  Carver c{reinterpret_cast<char*>(ws), 0};
  AssignWs w;
  plan_assign(c, M, L, N, precision, &w);
  LBG_TRY(check_ws(ws, ws_bytes, c.size()));
  hipStream_t s = (hipStream_t)stream;
  LBG_TRY(launch_assign(X, M, L, C, N, idx, mind, precision, w.dpart, nullptr, w.prep, s));
  return launch_reduce_parts(w.dpart, assign_num_parts(M, L, N, precision), (double)M, D, s);
}

int lbg_update(const float* X, int64_t M, int64_t L, const int32_t* idx,
               const float* C_old, int64_t N, float* C_new, int32_t* counts,
               void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  LBG_TRY(check_dims(M, L, N));
  LBG_TRY(need(X, "X"));
  LBG_TRY(need(idx, "idx"));
  LBG_TRY(need(C_old, "C_old"));
  LBG_TRY(need(C_new, "C_new"));
  if (counts && !aligned4(counts)) {
    set_error("counts is not 4-byte aligned");
    return LBG_EINVAL;
  }
  if (C_new != C_old) {
    const char* a = reinterpret_cast<const char*>(C_old);
    const char* b = reinterpret_cast<const char*>(C_new);
    if (b < a + N * L * 4 && a < b + N * L * 4) {
      set_error("C_new partially overlaps C_old");
      return LBG_EINVAL;
    }
  }
  Carver c{reinterpret_cast<char*>(ws), 0};
  UpdateWs w;
  plan_update(c, M, L, N, &w);
  LBG_TRY(check_ws(ws, ws_bytes, c.size()));
  return launch_update(X, M, L, idx, C_old, N, C_new, counts, 0, 0.0, w, false,
                       (hipStream_t)stream);
}

int lbg_distortion(const float* X, int64_t M, int64_t L, const float* C, int64_t N,
                   const int32_t* idx, double* D, void* ws, size_t ws_bytes,
                   void* stream) {
  clear_error();
  LBG_TRY(check_dims(M, L, N));
  LBG_TRY(need(X, "X"));
  LBG_TRY(need(C, "C"));
  LBG_TRY(need(idx, "idx"));
  LBG_TRY(need(D, "D"));
  Carver c{reinterpret_cast<char*>(ws), 0};
  DistWs w;
  plan_distortion(c, M, &w);
  LBG_TRY(check_ws(ws, ws_bytes, c.size()));
  return launch_distortion(X, M, L, C, N, idx, D, w, (hipStream_t)stream);
}

int lbg_distortion_backward(const float* X, int64_t M, int64_t L, const float* C,
                            int64_t N, const int32_t* idx, double g, float* gX,
                            float* gC, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  LBG_TRY(check_dims(M, L, N));
  LBG_TRY(need(X, "X"));
  LBG_TRY(need(C, "C"));
  LBG_TRY(need(idx, "idx"));
  if ((gX && !aligned4(gX)) || (gC && !aligned4(gC))) {
    set_error("gradient output is not 4-byte aligned");
    return LBG_EINVAL;
  }
  if (!isfinite(g)) {
    set_error("g is not finite");
    return LBG_EINVAL;
  }
  const double g2 = 2.0 * g / (double)M;
  hipStream_t s = (hipStream_t)stream;
  if (gC) {
    Carver c{reinterpret_cast<char*>(ws), 0};
    UpdateWs w;
    plan_update(c, M, L, N, &w);
    LBG_TRY(check_ws(ws, ws_bytes, c.size()));
    LBG_TRY(launch_update(X, M, L, idx, C, N, gC, nullptr, 1, g2, w, false, s));
  }
  if (gX) LBG_TRY(launch_grad_x(X, M, L, C, N, idx, g2, gX, s));
  return LBG_OK;
}

int lbg_train(const float* X, int64_t M, int64_t L, int64_t N, const lbg_params* p,
              float* C_out, int32_t* idx_out, double* D_out, lbg_stats* st, void* ws,
              size_t ws_bytes, void* stream) {
  clear_error();
  LBG_TRY(check_dims(M, L, N));
  if (!is_pow2(N)) {
    set_error("N = %lld is not a power of two", (long long)N);
    return LBG_EINVAL;
  }
  LBG_TRY(need(X, "X"));
  LBG_TRY(need(C_out, "C_out"));
  LBG_TRY(need(idx_out, "idx_out"));
  if (!D_out) {
    set_error("D_out is NULL");
    return LBG_EINVAL;
  }
  lbg_params def;
  lbg_params_default(&def);
  if (!p) p = &def;
  if (!(p->thr >= 0.0) || !isfinite(p->thr)) {
    set_error("thr = %g must be finite and >= 0", p->thr);
    return LBG_EINVAL;
  }
  if (p->split_mode == LBG_SPLIT_MULT) {
    if (!(p->eps_split > 0.0 && p->eps_split < 1.0)) {
      set_error("eps_split = %g outside (0, 1)", p->eps_split);
      return LBG_EINVAL;
    }
  } else if (p->split_mode == LBG_SPLIT_ADD) {
    if (!isfinite(p->delta)) {
      set_error("delta is not finite");
      return LBG_EINVAL;
    }
  } else {
    set_error("unknown split_mode %d", p->split_mode);
    return LBG_EINVAL;
  }
  if (p->max_iter < 0 || p->fixed_iters < 0 || p->n_forced < 0) {
    set_error("negative iteration parameter");
    return LBG_EINVAL;
  }
  if (p->n_forced > 0 && !p->forced_iters) {
    set_error("forced_iters is NULL");
    return LBG_EINVAL;
  }
  LBG_TRY(check_precision(p->precision));
  if (p->C_init) {
    if (!is_pow2(p->N_init) || p->N_init > N) {
      set_error("N_init = %lld must be a power of two <= N", (long long)p->N_init);
      return LBG_EINVAL;
    }
    LBG_TRY(need(p->C_init, "C_init"));
  }
  if (!(p->D_prev_init >= 0.0) || p->it_init < 0) {
    set_error("D_prev_init must be >= 0 or +inf and it_init >= 0");
    return LBG_EINVAL;
  }
  if (!p->C_init && (p->D_prev_init != INFINITY || p->it_init != 0)) {
    set_error("D_prev_init and it_init resume a level from C_init: C_init is NULL");
    return LBG_EINVAL;
  }
  Carver c{reinterpret_cast<char*>(ws), 0};
  TrainWs w;
  plan_train(c, M, L, N, p->precision, &w);
  LBG_TRY(check_ws(ws, ws_bytes, c.size()));
  hipStream_t s = (hipStream_t)stream;

  if (st) {
    double* keep = st->D_trace;
    int32_t cap = st->D_cap;
    memset(st, 0, sizeof(*st));
    st->D_trace = keep;
    st->D_cap = cap;
  }
  if (train_device_ok(L, w))
    return train_device(X, M, L, N, p, C_out, idx_out, D_out, st, w, s);
  LBG_TRY_HIP(hipMemsetAsync(w.as.nfb, 0, sizeof(unsigned long long), s));

  // Optional kernel timing: an event pair around every allocation, update
  // and split; pairs are read once the stream has passed them.
  Timer tm(p->timing != 0 && st != nullptr);
  LBG_TRY(tm.init());

  int cur = 0;
  int64_t n;
  bool need_split;
  if (p->C_init) {
    LBG_TRY_HIP(hipMemcpyAsync(w.Cb[0], p->C_init, (size_t)(p->N_init * L) * sizeof(float),
                               hipMemcpyDeviceToDevice, s));
    n = p->N_init;
    need_split = false;
  } else {
    LBG_TRY(launch_centroid(X, M, L, w.Cb[0], w.ce, s));
    n = 1;
    need_split = N > 1;
  }

  int on_grid = 0;
  if (w.up.use_afp) {
    LBG_TRY(launch_afp_shift(X, M, L, w.up.afp, s));
    int flags[5] = {0, 0, 0, 0, 0};
    LBG_TRY_HIP(hipMemcpyAsync(flags, w.up.afp.shift, sizeof(flags), hipMemcpyDeviceToHost, s));
    LBG_TRY_HIP(hipStreamSynchronize(s));
    on_grid = flags[1] != 0 ? 0 : (flags[3] ? 2 : 1);
  }
  auto assign_and_D = [&](double* Dh) -> int {
    LBG_TRY(tm.begin(Timer::kAssign, s));
    LBG_TRY(launch_assign(X, M, L, w.Cb[cur], n, idx_out, nullptr, p->precision,
                          w.as.dpart, w.as.nfb, w.as.prep, s));
    LBG_TRY(tm.end(s));
    LBG_TRY(launch_reduce_parts(w.as.dpart, assign_num_parts(M, L, n, p->precision), (double)M,
                                w.D, s));
    LBG_TRY(read_scalar(w.D, Dh, s));
    LBG_TRY(tm.collect());
    if (!isfinite(*Dh)) {
      set_error("the distortion is not finite: the training set or the starting codebook "
                "holds a NaN or infinite value");
      return LBG_EINVAL;
    }
    if (st) {
      if (st->D_trace && st->n_D < st->D_cap) st->D_trace[st->n_D] = *Dh;
      st->n_D++;
      st->total_assigns++;
      st->total_distances += M * n;
    }
    return LBG_OK;
  };

  int status = LBG_OK;
  double D = 0.0;
  if (!p->C_init && N == 1) {
    LBG_TRY(assign_and_D(&D));
    if (st) {
      st->n_levels = 1;
      st->level_n[0] = 1;
      st->level_iters[0] = 0;
    }
  } else {
    int level = 0;
    for (;;) {
      if (need_split) {
        LBG_TRY(tm.begin(Timer::kSplit, s));
        LBG_TRY(launch_split(w.Cb[cur], n, L, p->split_mode, p->eps_split, p->delta,
                             w.Cb[cur ^ 1], s));
        LBG_TRY(tm.end(s));
        cur ^= 1;
        n *= 2;
      }
      // (C_init may resume its level in the middle: see lbg_params)
      const bool resume = p->C_init && level == 0;
      double D_prev = resume ? p->D_prev_init : INFINITY;
      bool first = D_prev == INFINITY;
      int32_t it = resume ? p->it_init : 0;
      int32_t forced = -1;
      if (p->fixed_iters > 0) forced = p->fixed_iters;
      if (p->forced_iters && level < p->n_forced) forced = p->forced_iters[level];
      for (;;) {
        LBG_TRY(assign_and_D(&D));
        bool stop;
        if (forced >= 0) {
          stop = it >= forced;
        } else {
          stop = !first && (D_prev - D) <= p->thr * D_prev;
          if (!stop && it >= p->max_iter) {
            stop = true;
            status = LBG_WMAXITER;
          }
        }
        if (stop) break;
        LBG_TRY(tm.begin(Timer::kUpdate, s));
        LBG_TRY(launch_update(X, M, L, idx_out, w.Cb[cur], n, w.Cb[cur ^ 1], nullptr, 0,
                              0.0, w.up, true, s, on_grid));
        LBG_TRY(tm.end(s));
        cur ^= 1;
        D_prev = D;
        first = false;
        ++it;
        if (st) st->total_updates++;
      }
      if (st && level < 32) {
        st->level_n[level] = (int32_t)n;
        st->level_iters[level] = it;
      }
      ++level;
      if (st) st->n_levels = level;
      if (n >= N) break;
      need_split = true;
    }
  }
  LBG_TRY_HIP(hipMemcpyAsync(C_out, w.Cb[cur], (size_t)(N * L) * sizeof(float),
                             hipMemcpyDeviceToDevice, s));
  if (st) {
    unsigned long long nf = 0;
    LBG_TRY_HIP(hipMemcpyAsync(&nf, w.as.nfb, sizeof(nf), hipMemcpyDeviceToHost, s));
    LBG_TRY_HIP(hipStreamSynchronize(s));
    st->fallback_rows = (int64_t)nf;
    LBG_TRY(tm.collect());
    st->ms_assign = tm.ms[Timer::kAssign];
    st->ms_update = tm.ms[Timer::kUpdate];
    st->ms_split = tm.ms[Timer::kSplit];
    LBG_TRY(run_stats(X, M, L, N, C_out, idx_out, p, st, w, s));
  } else {
    LBG_TRY_HIP(hipStreamSynchronize(s));
  }
  *D_out = D;
  return status;
}

int lbg_encode(const float* X, int64_t M, int64_t L, const float* C, int64_t N, int32_t* idx,
               void* ws, size_t ws_bytes, void* stream) {
  return lbg_assign(X, M, L, C, N, idx, nullptr, LBG_FP32, ws, ws_bytes, stream);
}

int lbg_decode(const int32_t* idx, int64_t M, const float* C, int64_t N, int64_t L, float* Y,
               void* stream) {
  clear_error();
  LBG_TRY(check_dims(M, L, N));
  LBG_TRY(need(idx, "idx"));
  LBG_TRY(need(C, "C"));
  LBG_TRY(need(Y, "Y"));
  const char* a = reinterpret_cast<const char*>(C);
  const char* b = reinterpret_cast<const char*>(Y);
  if (b < a + N * L * 4 && a < b + M * L * 4) {
    set_error("Y overlaps C");
    return LBG_EINVAL;
  }
  return launch_decode(idx, M, C, N, L, Y, (hipStream_t)stream);
}

namespace {

int check_pictures(int64_t nimg, int64_t H, int64_t W, int64_t b) {
  if (b < 1 || b * b > LBG_MAX_L) {
    set_error("block side b = %lld outside [1, %d]", (long long)b, (int)sqrt((double)LBG_MAX_L));
    return LBG_EINVAL;
  }
  if (nimg < 1 || H < 1 || W < 1 || H > INT32_MAX || W > INT32_MAX || nimg > INT32_MAX) {
    set_error("bad picture size %lld x %lld x %lld", (long long)nimg, (long long)H,
              (long long)W);
    return LBG_EINVAL;
  }
  if (H % b || W % b) {
    set_error("picture size %lld x %lld is not a multiple of b = %lld", (long long)H,
              (long long)W, (long long)b);
    return LBG_EINVAL;
  }
  if ((H / b) * (W / b) > LBG_MAX_M / nimg) {
    set_error("more than %lld blocks", (long long)LBG_MAX_M);
    return LBG_EINVAL;
  }
  return LBG_OK;
}

bool overlap(const void* p, int64_t pbytes, const void* q, int64_t qbytes) {
  const char* a = reinterpret_cast<const char*>(p);
  const char* b = reinterpret_cast<const char*>(q);
  return b < a + pbytes && a < b + qbytes;
}

}  // namespace

int lbg_image_blocks(const float* img, int64_t nimg, int64_t H, int64_t W, int64_t b, float* X,
                     void* stream) {
  clear_error();
  LBG_TRY(check_pictures(nimg, H, W, b));
  LBG_TRY(need(img, "img"));
  LBG_TRY(need(X, "X"));
  const int64_t bytes = nimg * H * W * 4;
  if (overlap(img, bytes, X, bytes)) {
    set_error("X overlaps img");
    return LBG_EINVAL;
  }
  return launch_image(1, nullptr, nullptr, 0, nimg, H, W, b, img, X, (hipStream_t)stream);
}

int lbg_decode_image(const int32_t* idx, const float* C, int64_t N, int64_t nimg, int64_t H,
                     int64_t W, int64_t b, float* img, void* stream) {
  clear_error();
  LBG_TRY(check_pictures(nimg, H, W, b));
  if (N < 1 || N > LBG_MAX_N) {
    set_error("N = %lld outside [1, %d]", (long long)N, LBG_MAX_N);
    return LBG_EINVAL;
  }
  LBG_TRY(need(idx, "idx"));
  LBG_TRY(need(C, "C"));
  LBG_TRY(need(img, "img"));
  if (overlap(C, N * b * b * 4, img, nimg * H * W * 4)) {
    set_error("img overlaps C");
    return LBG_EINVAL;
  }
  return launch_image(0, idx, C, N, nimg, H, W, b, nullptr, img, (hipStream_t)stream);
}

int lbg_rate(int64_t N, int64_t L, double* out) {
  clear_error();
  if (N < 1 || L < 1 || !out) {
    set_error("lbg_rate needs N >= 1, L >= 1 and an output");
    return LBG_EINVAL;
  }
  *out = log2((double)N) / (double)L;
  return LBG_OK;
}

int lbg_psnr(double D, int64_t L, double peak, double* out) {
  clear_error();
  if (!(D >= 0.0) || !isfinite(D) || L < 1 || !(peak > 0.0) || !isfinite(peak) || !out) {
    set_error("lbg_psnr needs a finite D >= 0, L >= 1, a finite peak > 0 and an output");
    return LBG_EINVAL;
  }
  *out = D == 0.0 ? HUGE_VAL : 10.0 * log10(peak * peak * (double)L / D);
  return LBG_OK;
}


}  // extern "C"
