/*
 * lbg_oracle.c -- plain FP64 CPU reference of LBG codebook design.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * constant with the GPU path.
 *
 * What it computes follows the paper "Parallelization of the LBG Vector
 * Quantization Algorithm for Shared Memory Systems" (Annaji & Rao):
 *
 *   - the LBG algorithm of Linde, Buzo and Gray as restated in Sec. 2.2
 *     ("LBG Algorithm": minimum-distortion partition, average distortion D_m,
 *     relative-change stop test, centroid update);
 *   - Algorithm 1 ("Parallelized Vector Quantization Algorithm") and its
 *     step descriptions in Sec. 3.2: initial codebook = centroid of the
 *     input (Initialization, Table 1), codebook splitting that doubles the
 *     codebook (Codebook Splitting), nearest-codevector allocation with the
 *     summed minimum distances (Cell Allocation), the termination test on
 *     the total distortion, and per-codevector centroids of the cell table
 *     (Codebook Updation).
 *
 * All arithmetic is FP64.  Training vectors arrive as FP32 and are widened
 * exactly.  Codebooks are FP64; with ``store_fp32`` set, every codebook value
 * is rounded to FP32 where it is stored (after a split and after an update),
 * which is the arithmetic of an implementation that keeps its codebook in
 * FP32 while computing distances and means in FP64.
 *
 * Readings taken where the paper is silent or garbled (each is listed in the
 * design notes of the repository):
 *   R1 distance: squared Euclidean distance sum_l (x_l - c_l)^2, summed over
 *      l in index order ("Euclidean distance", Sec. 2.2 terms; D_m of the
 *      LBG restatement).
 *   R2 ties: the lowest codevector index wins (x in S_i if d(x,y_i) <=
 *      d(x,y_l) for all l; the first such i).
 *   R3 distortion: the mean n^-1 sum_j min d(x_j, y) of the LBG restatement,
 *      summed in training-vector index order.
 *   R4 stop test: (D_prev - D) <= thr * D_prev, with D_prev the distortion
 *      of the previous allocation (termination condition of Sec. 3.2); the
 *      first allocation after a split never stops (D_-1 = "very high",
 *      reset at every split so each level performs at least one update).
 *   R5 on convergence the codebook that produced the last allocation is kept
 *      (the test precedes Updation in Algorithm 1); it is the one that is
 *      split or returned.
 *   R6 split: multiplicative c(1+eps), c(1-eps) (default), or the paper's
 *      additive c+delta, c-delta; the "+" child takes index 2i and the "-"
 *      child index 2i+1.
 *   R7 an empty cell keeps its previous codevector (centroid of an empty set
 *      is undefined in Codebook Updation).
 *   R8 iteration cap per level: max_iter updates; reaching it is reported.
 *
 * Threads: the allocation loop over training vectors may run on several
 * OpenMP threads (static chunks, as Algorithm 1 distributes the input).  Each
 * vector's result is computed on its own and every sum is formed afterwards
 * in index order, so results do not depend on the thread count.
 */

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_SPLIT_MULT 0
#define ORACLE_SPLIT_ADD 1

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_WMAXITER 1

typedef struct oracle_params {
  double thr;          /* relative distortion-change threshold, >= 0 */
  double eps_split;    /* multiplicative split factor */
  double delta;        /* additive split offset (split_mode == ADD) */
  int32_t split_mode;  /* ORACLE_SPLIT_MULT or ORACLE_SPLIT_ADD */
  int32_t max_iter;    /* cap on updates per level */
  int32_t store_fp32;  /* round stored codebooks to FP32 */
  int32_t fixed_iters; /* > 0: exactly this many updates per level */
  const int32_t* forced_iters; /* per level (nullable): updates per level */
  int32_t n_forced;            /* entries in forced_iters */
  const double* C_init;        /* nullable: starting codebook (N_init x L) */
  int64_t N_init;              /* rows of C_init */
  int32_t nthreads;            /* OpenMP threads for allocation, 0 = default */
} oracle_params;

/* Per-run record.  ``D`` holds the distortion of every allocation in order,
 * ``level_n`` / ``level_iters`` the codebook size and number of updates of
 * every level, ``level_stop_ratio`` the relative change (D_prev-D)/D_prev
 * that ended each level (NaN when a cap or a forced count ended it). */
typedef struct oracle_trace {
  int64_t cap_D;
  int64_t n_D;
  double* D;
  int64_t cap_levels;
  int64_t n_levels;
  int64_t* level_n;
  int32_t* level_iters;
  double* level_stop_ratio;
} oracle_trace;

static double store(double v, int fp32) { return fp32 ? (double)(float)v : v; }

/* Squared Euclidean distance between a training vector and a codevector,
 * direct form, dimensions in index order (reading R1). */
static double sqdist(const float* x, const double* c, int64_t L) {
  double s = 0.0;
  for (int64_t l = 0; l < L; ++l) {
    double d = (double)x[l] - c[l];
    s += d * d;
  }
  return s;
}

/* Initialization (Table 1): the centroid of all M training vectors,
 * summed in index order and divided by M. */
void lbg_oracle_centroid(const float* X, int64_t M, int64_t L, double* c0) {
  for (int64_t l = 0; l < L; ++l) c0[l] = 0.0;
  for (int64_t m = 0; m < M; ++m)
    for (int64_t l = 0; l < L; ++l) c0[l] += (double)X[m * L + l];
  for (int64_t l = 0; l < L; ++l) c0[l] /= (double)M;
}

/* Codebook Splitting: each codevector c_i yields two children, the "+"
 * child at row 2i and the "-" child at row 2i+1 (reading R6). */
void lbg_oracle_split(const double* C, int64_t n, int64_t L, int32_t mode,
                      double eps, double delta, int32_t store_fp32,
                      double* C2) {
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t l = 0; l < L; ++l) {
      double c = C[i * L + l];
      double up, dn;
      if (mode == ORACLE_SPLIT_ADD) {
        up = c + delta;
        dn = c - delta;
      } else {
        up = c * (1.0 + eps);
        dn = c * (1.0 - eps);
      }
      C2[(2 * i) * L + l] = store(up, store_fp32);
      C2[(2 * i + 1) * L + l] = store(dn, store_fp32);
    }
  }
}

/* Cell Allocation: for every training vector the nearest codevector (lowest
 * index on ties, reading R2), its distance d1 and the second-smallest
 * distance d2 over the other codevectors (+inf when n == 1). */
void lbg_oracle_assign(const float* X, int64_t M, int64_t L, const double* C,
                       int64_t n, int32_t* idx, double* d1, double* d2,
                       int32_t nthreads) {
#ifdef _OPENMP
  int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
#else
  (void)nthreads;
#endif
  for (int64_t m = 0; m < M; ++m) {
    const float* x = X + m * L;
    double best = INFINITY, second = INFINITY;
    int64_t bi = 0;
    for (int64_t k = 0; k < n; ++k) {
      double d = sqdist(x, C + k * L, L);
      if (d < best) {
        second = best;
        best = d;
        bi = k;
      } else if (d < second) {
        second = d;
      }
    }
    idx[m] = (int32_t)bi;
    if (d1) d1[m] = best;
    if (d2) d2[m] = second;
  }
}

/* Average distortion D = M^-1 sum_m ||x_m - c_{idx_m}||^2, summed in
 * training-vector index order (reading R3). */
double lbg_oracle_distortion(const float* X, int64_t M, int64_t L,
                             const double* C, const int32_t* idx) {
  double s = 0.0;
  for (int64_t m = 0; m < M; ++m) s += sqdist(X + m * L, C + (int64_t)idx[m] * L, L);
  return s / (double)M;
}

/* Codebook Updation: every codevector becomes the centroid (mean) of the
 * training vectors whose cell value is its index; sums run in training-
 * vector index order.  An empty cell keeps its codevector (reading R7).
 * ``counts`` (nullable) receives the cell sizes. */
void lbg_oracle_update(const float* X, int64_t M, int64_t L,
                       const int32_t* idx, const double* C_old, int64_t n,
                       int32_t store_fp32, double* C_new, int64_t* counts) {
  double* sum = (double*)calloc((size_t)(n * L), sizeof(double));
  int64_t* cnt = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  for (int64_t m = 0; m < M; ++m) {
    int64_t k = idx[m];
    cnt[k] += 1;
    for (int64_t l = 0; l < L; ++l) sum[k * L + l] += (double)X[m * L + l];
  }
  for (int64_t k = 0; k < n; ++k) {
    for (int64_t l = 0; l < L; ++l) {
      double v = cnt[k] > 0 ? sum[k * L + l] / (double)cnt[k] : C_old[k * L + l];
      C_new[k * L + l] = store(v, store_fp32);
    }
    if (counts) counts[k] = cnt[k];
  }
  free(sum);
  free(cnt);
}

/* Gradient of D(C, X) = M^-1 sum_m min_k ||x_m - c_k||^2 at an allocation
 * ``idx`` (the minimiser, lowest index on ties), scaled by g:
 *   dD/dx_m = g * 2/M * (x_m - c_{idx_m})
 *   dD/dc_k = g * 2/M * sum_{m : idx_m = k} (c_k - x_m)
 * Either output may be NULL. */
void lbg_oracle_grad(const float* X, int64_t M, int64_t L, const double* C,
                     int64_t n, const int32_t* idx, double g, double* gX,
                     double* gC) {
  double s = 2.0 * g / (double)M;
  if (gC)
    for (int64_t i = 0; i < n * L; ++i) gC[i] = 0.0;
  for (int64_t m = 0; m < M; ++m) {
    const double* c = C + (int64_t)idx[m] * L;
    for (int64_t l = 0; l < L; ++l) {
      double diff = (double)X[m * L + l] - c[l];
      if (gX) gX[m * L + l] = s * diff;
      if (gC) gC[(int64_t)idx[m] * L + l] -= s * diff;
    }
  }
}

static void trace_D(oracle_trace* tr, double D) {
  if (!tr) return;
  if (tr->n_D < tr->cap_D) tr->D[tr->n_D] = D;
  tr->n_D++;
}

static void trace_level(oracle_trace* tr, int64_t n, int32_t iters, double ratio) {
  if (!tr) return;
  if (tr->n_levels < tr->cap_levels) {
    tr->level_n[tr->n_levels] = n;
    tr->level_iters[tr->n_levels] = iters;
    tr->level_stop_ratio[tr->n_levels] = ratio;
  }
  tr->n_levels++;
}

static int is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

/* LBG with splitting (Algorithm 1 with readings R1-R8).
 *
 * Returns ORACLE_OK, ORACLE_WMAXITER (some level hit max_iter; results
 * valid) or ORACLE_EINVAL.  On success C_out (N x L) holds the codebook that
 * produced the last allocation, idx_out (M) that allocation and *D_out its
 * distortion. */
int lbg_oracle_train(const float* X, int64_t M, int64_t L, int64_t N,
                     const oracle_params* p, double* C_out, int32_t* idx_out,
                     double* D_out, oracle_trace* tr) {
  if (M < 1 || L < 1 || !is_pow2(N) || !p || p->thr < 0.0) return ORACLE_EINVAL;
  if (p->C_init && (p->N_init < 1 || p->N_init > N || !is_pow2(p->N_init)))
    return ORACLE_EINVAL;
  int status = ORACLE_OK;
  double* C = (double*)malloc(sizeof(double) * (size_t)(N * L));
  double* Cn = (double*)malloc(sizeof(double) * (size_t)(N * L));
  int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
  double* d1 = (double*)malloc(sizeof(double) * (size_t)M);
  int64_t n;
  int need_split;
  if (p->C_init) {
    n = p->N_init;
    for (int64_t i = 0; i < n * L; ++i) C[i] = store(p->C_init[i], p->store_fp32);
    need_split = 0;
  } else {
    lbg_oracle_centroid(X, M, L, C);
    for (int64_t l = 0; l < L; ++l) C[l] = store(C[l], p->store_fp32);
    n = 1;
    need_split = N > 1;
  }
  int32_t level = 0;
  double D = 0.0;
  if (!p->C_init && N == 1) {
    /* The centroid is already the optimal one-level codebook: one
     * allocation gives the cell table and the distortion. */
    lbg_oracle_assign(X, M, L, C, n, idx, d1, NULL, p->nthreads);
    double s = 0.0;
    for (int64_t m = 0; m < M; ++m) s += d1[m];
    D = s / (double)M;
    trace_D(tr, D);
    trace_level(tr, 1, 0, NAN);
    memcpy(C_out, C, sizeof(double) * (size_t)L);
    memcpy(idx_out, idx, sizeof(int32_t) * (size_t)M);
    if (D_out) *D_out = D;
    free(C);
    free(Cn);
    free(idx);
    free(d1);
    return status;
  }
  for (;;) {
    if (need_split) {
      lbg_oracle_split(C, n, L, p->split_mode, p->eps_split, p->delta,
                       p->store_fp32, Cn);
      n *= 2;
      double* t = C;
      C = Cn;
      Cn = t;
    }
    /* Lloyd iterations at this level. */
    double D_prev = INFINITY;
    int first = 1;
    int32_t it = 0;
    int32_t forced = -1;
    if (p->fixed_iters > 0) forced = p->fixed_iters;
    if (p->forced_iters && level < p->n_forced) forced = p->forced_iters[level];
    double ratio = NAN;
    for (;;) {
      lbg_oracle_assign(X, M, L, C, n, idx, d1, NULL, p->nthreads);
      double s = 0.0;
      for (int64_t m = 0; m < M; ++m) s += d1[m];
      D = s / (double)M;
      trace_D(tr, D);
      int stop;
      if (forced >= 0) {
        stop = it >= forced;
      } else {
        stop = !first && (D_prev - D) <= p->thr * D_prev;
        if (stop) ratio = D_prev > 0.0 ? (D_prev - D) / D_prev : 0.0;
        if (!stop && it >= p->max_iter) {
          stop = 1;
          status = ORACLE_WMAXITER;
        }
      }
      if (stop) break;
      lbg_oracle_update(X, M, L, idx, C, n, p->store_fp32, Cn, NULL);
      double* t = C;
      C = Cn;
      Cn = t;
      D_prev = D;
      first = 0;
      it++;
    }
    trace_level(tr, n, it, ratio);
    level++;
    if (n >= N) break;
    need_split = 1;
  }
  memcpy(C_out, C, sizeof(double) * (size_t)(N * L));
  memcpy(idx_out, idx, sizeof(int32_t) * (size_t)M);
  if (D_out) *D_out = D;
  free(C);
  free(Cn);
  free(idx);
  free(d1);
  return status;
}

/* Number of OpenMP threads the allocation loop would use by default. */
int32_t lbg_oracle_max_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}
