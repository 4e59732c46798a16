/*
 * lbg.h -- C ABI of the MI355X (gfx950) LBG codebook-design library.
 *
 * LBG (Linde-Buzo-Gray) vector-quantizer design as parallelised in Annaji &
 * Rao, "Parallelization of the LBG Vector Quantization Algorithm for Shared
 * Memory Systems": a training set of M vectors of dimension L (the paper's
 * "M x k" input, Sec. 3.1 Notations) is turned into a codebook of N
 * codevectors ("N x k" output, Algorithm 1).  The Lloyd iteration of
 * Algorithm 1 -- Cell Allocation (nearest codevector for every training
 * vector), the distortion sum, the termination test and Codebook Updation
 * (cell centroids) -- runs on the GPU; codebooks grow by Codebook Splitting.
 *
 * Conventions for every entry point:
 *   - Arrays are row-major and contiguous.  Unless a parameter says "host",
 *     pointers are DEVICE pointers on the current HIP device.  Float arrays
 *     must be 4-byte aligned; X and C are read with 16-byte vector loads when
 *     16-byte aligned and L % 4 == 0, and with scalar loads otherwise.
 *   - The caller owns every buffer.  The library never frees caller memory
 *     and allocates no caller-visible memory; scratch space is the caller's
 *     workspace ``ws`` of at least lbg_workspace_size(...) bytes (device,
 *     256-byte aligned).  ws may be NULL only when that size is 0.
 *   - ``stream`` is a hipStream_t (NULL = the legacy default stream).  Calls
 *     enqueue work on it and return without waiting, except lbg_train, which
 *     waits on its stream to run the level / iteration control.
 *   - Return codes: LBG_OK, LBG_EINVAL (bad size, NULL required pointer,
 *     misalignment, N not a power of two in lbg_train, bad parameter),
 *     LBG_ENOWS (workspace too small), LBG_EHIP (a HIP runtime error; the
 *     message names it), LBG_WMAXITER (warning from lbg_train: some level hit
 *     its iteration cap; results are valid).  On failure no kernel has been
 *     enqueued and lbg_last_error() returns a message (thread-local).
 *   - Cell indices are int32; codevector index ties go to the lowest index.
 *   - Results are deterministic: the same inputs give bit-identical outputs
 *     on every run (no floating-point atomics anywhere).
 *   - Non-finite values: a training vector with a NaN or infinite coordinate
 *     has no finite distance to any codevector; the allocation gives it
 *     index 0 and distance +inf (the first strictly smaller distance,
 *     starting from +inf, never occurs), so a distortion over it is +inf
 *     (lbg_assign_distortion) or NaN / +inf (lbg_distortion, the direct
 *     distance to codevector 0).  lbg_train and lbg_train_batched stop a run
 *     whose distortion is not finite at that allocation and report
 *     LBG_EINVAL.  Codebooks must be finite; lbg_update and the gradient
 *     assume finite X.
 */
#ifndef LBG_H
#define LBG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBG_OK 0
#define LBG_EINVAL (-1)
#define LBG_ENOWS (-2)
#define LBG_EHIP (-3)
#define LBG_WMAXITER 1

/* Distance arithmetic of the allocation. */
#define LBG_FP32 0         /* FP32 matrix-core distances, exact result (below) */
#define LBG_BF16_RESCORE 1 /* BF16 matrix-core distances, top-2 rescored */

/* Codebook split forms. */
#define LBG_SPLIT_MULT 0 /* c(1+eps), c(1-eps) */
#define LBG_SPLIT_ADD 1  /* c+delta, c-delta (the paper's additive form) */

/* Workspace queries. */
#define LBG_OP_ASSIGN 1
#define LBG_OP_UPDATE 2
#define LBG_OP_DISTORTION 3
#define LBG_OP_TRAIN 4
#define LBG_OP_BACKWARD 5
#define LBG_OP_CENTROID 6

/* Largest supported sizes. */
#define LBG_MAX_M ((((int64_t)1) << 31) - 1) /* rows: int32 cell table */
#define LBG_MAX_L 256                   /* vector dimension */
#define LBG_MAX_N 65536                 /* codevectors */

/*
 * Codebook Splitting (Algorithm 1, "Codebook Splitting"; Sec. 3.2): every
 * codevector c_i of C (n x L) yields two children, written to C2 (2n x L):
 *   C2[2i]   = c_i * (1 + eps)      C2[2i+1] = c_i * (1 - eps)
 * each product formed in FP64 and rounded once to FP32.  C2 must not
 * overlap C.  eps in (0, 1).
 */
int lbg_split(const float* C, int64_t n, int64_t L, double eps, float* C2,
              void* stream);

/* Additive form of the split (the paper's [c + delta], [c - delta]):
 *   C2[2i] = c_i + delta, C2[2i+1] = c_i - delta (FP64, rounded to FP32). */
int lbg_split_add(const float* C, int64_t n, int64_t L, double delta,
                  float* C2, void* stream);

/*
 * Initial codebook (Algorithm 1, Initialization; Table 1): c0 = mean of the M
 * rows of X, summed in FP64 in a fixed order, rounded to FP32.  c0: 1 x L.
 */
int lbg_centroid(const float* X, int64_t M, int64_t L, float* c0, void* ws,
                 size_t ws_bytes, void* stream);

/*
 * Cell Allocation (Algorithm 1, "Cell Allocation"; Sec. 3.2): for every row
 * x_m of X (M x L) the index of the nearest row of C (N x L) under the
 * squared Euclidean distance, lowest index on ties:
 *   idx[m] = min { k : d(x_m, c_k) = min_j d(x_m, c_j) }.
 * mind[m] (nullable) receives d(x_m, c_idx[m]) rounded to FP32 (+inf and
 * index 0 for a row with a non-finite coordinate).
 *
 * precision == LBG_FP32: distances are screened on matrix cores in the
 * expanded form |x|^2 - 2 x.c + |c|^2 with FP32 accuracy (from exact
 * three-part BF16 splits of x and -2c for 8 < L <= 64, in FP32 otherwise);
 * the best candidate is rescored in FP64 in the direct form
 * sum_l (x_l - c_l)^2 and accepted only when a rigorous error bound proves
 * no other codevector can be as close; failing that, the two best are
 * rescored and the closer one accepted under the same bound against all
 * others; otherwise the row is searched again exhaustively in FP64.
 * Codebooks of at most 8 codevectors (L <= 32) are searched directly in
 * FP64.  The result equals the FP64 direct-form argmin exactly.
 * precision == LBG_BF16_RESCORE: the screen runs in BF16 with FP32
 * accumulation; the two best candidates are rescored in the direct form and
 * the closer one (lowest index on ties) is taken: in FP32 for codebooks of
 * up to 64 dimensions whose BF16 copy fits one CU's LDS (N (L + 8) 2 bytes
 * <= 160 KiB, L rounded up to 16, 32 or 64), in FP64 otherwise.
 * Approximate: a row whose true nearest codevector is not among the BF16 top
 * two can be misassigned.
 */
int lbg_assign(const float* X, int64_t M, int64_t L, const float* C, int64_t N,
               int32_t* idx, float* mind, int precision, void* ws,
               size_t ws_bytes, void* stream);

/*
 * Codebook Updation (Algorithm 1, "Codebook Updation"; Sec. 3.2): every
 * codevector becomes the centroid of its cell,
 *   C_new[k] = (1/|S_k|) sum_{m : idx[m] = k} x_m,
 * rounded to FP32.  The sum is formed exactly, in 64-bit integers, from
 * every coordinate taken as round(x 2^s) (s from the largest |x| and M) and,
 * for data off that grid, its residual as a second integer word at 2^-(s+t)
 * (t = min(52, 63 - log2 M)): exact for coordinates down to 2^-(s+t), about
 * 2^-80 of the largest |x| at M = 2^22, so the result does not depend on the
 * order of the rows; it is divided once in FP64.  (Codebooks with more than
 * 32 x 60 KB of sums use fixed-order FP64 segmented sums instead.)  An empty
 * cell keeps C_old[k].  counts[k] (nullable, int32) receives |S_k|.
 * C_new may equal C_old (in place); otherwise they must not overlap.
 * Entries of idx outside [0, N) are ignored (they join no cell).
 */
int lbg_update(const float* X, int64_t M, int64_t L, const int32_t* idx,
               const float* C_old, int64_t N, float* C_new, int32_t* counts,
               void* ws, size_t ws_bytes, void* stream);

/*
 * Average distortion (LBG restatement, Sec. 2.2; the master's
 * IntegrateDistortions of Algorithm 1):
 *   D = (1/M) sum_m d(x_m, c_idx[m])
 * per-row distances in FP64 direct form, summed in FP64 in a fixed order.
 * D is a single DEVICE double.  idx entries must lie in [0, N); rows with an
 * index outside that range contribute 0.
 */
int lbg_distortion(const float* X, int64_t M, int64_t L, const float* C,
                   int64_t N, const int32_t* idx, double* D, void* ws,
                   size_t ws_bytes, void* stream);

/*
 * Cell Allocation and its average distortion in one pass over X (the
 * allocation followed by IntegrateDistortions of Algorithm 1): idx and mind
 * as lbg_assign; D (one DEVICE double) = (1/M) sum_m d(x_m, c_idx[m]), the
 * FP64 direct-form distance of each row's winner (summed over the dimensions
 * in order), added in FP64 in an order fixed by M and L alone (partials of
 * consecutive rows by a fixed pairwise tree, then the partials by a fixed
 * strided sum and tree).  Same per-row values as lbg_distortion on the
 * returned allocation.  ws: lbg_workspace_size(LBG_OP_ASSIGN, M, L, N,
 * precision) bytes.
 */
int lbg_assign_distortion(const float* X, int64_t M, int64_t L, const float* C,
                          int64_t N, int32_t* idx, float* mind, int precision,
                          double* D, void* ws, size_t ws_bytes, void* stream);

/*
 * Gradient of D(C, X) = (1/M) sum_m min_k d(x_m, c_k) at the allocation idx,
 * scaled by g (the upstream gradient of a scalar loss):
 *   gX[m] = g * 2/M * (x_m - c_idx[m])
 *   gC[k] = g * 2/M * sum_{m : idx[m] = k} (c_k - x_m)
 * gC[k] is formed as count * c_k - (the cell sum of lbg_update), the
 * difference taken exactly in integers on the sums' grid (and in FP64 for
 * a codevector beyond 2^62 of that grid, where it cannot cancel) before
 * one rounding.  Either output may be NULL.  At a tie the gradient is the
 * one of the lowest-index minimiser (the allocation passed in).
 */
int lbg_distortion_backward(const float* X, int64_t M, int64_t L,
                            const float* C, int64_t N, const int32_t* idx,
                            double g, float* gX, float* gC, void* ws,
                            size_t ws_bytes, void* stream);

/*
 * Encoder and decoder of the trained quantizer (Introduction: a vector is
 * coded by the index of its nearest codevector, which the decoder maps back;
 * log2(N) bits per vector, log2(N)/L bits per sample).
 *
 * lbg_encode: idx[m] = index of the codevector of C (N x L) nearest to row m
 * of X (M x L), lowest index on ties: lbg_assign with LBG_FP32 and no
 * distances.  ws: lbg_workspace_size(LBG_OP_ASSIGN, M, L, N, LBG_FP32) bytes.
 */
int lbg_encode(const float* X, int64_t M, int64_t L, const float* C, int64_t N,
               int32_t* idx, void* ws, size_t ws_bytes, void* stream);

/*
 * lbg_decode: Y[m] = C[idx[m]] for the M indices idx, Y M x L (device,
 * caller-owned, may not overlap C).  An index outside [0, N) gives a row of
 * quiet NaNs, so that a corrupt code stays visible.  No workspace.
 */
int lbg_decode(const int32_t* idx, int64_t M, const float* C, int64_t N,
               int64_t L, float* Y, void* stream);

/*
 * Pictures cut into b x b blocks (the training vectors of an image coder,
 * L = b * b): nimg pictures of H rows by W columns, row-major, picture after
 * picture (img: nimg x H x W floats); H and W multiples of b.  Vector v =
 * (p * (H / b) + by) * (W / b) + bx holds block (by, bx) of picture p, its
 * pixels row-major: dimension dy * b + dx is pixel (by b + dy, bx b + dx).
 *
 * lbg_image_blocks: img -> X (nimg (H/b)(W/b) x b*b).
 * lbg_decode_image: the decoder written straight into pictures: pixel
 *   (p, y, x) of img is dimension (y mod b) b + (x mod b) of codevector
 *   idx[v] of C (N x b*b), v the block that holds the pixel; an index outside
 *   [0, N) gives NaN pixels.  Equals lbg_decode followed by the inverse of
 *   lbg_image_blocks, in one pass.
 * Limits: 1 <= b, b * b <= LBG_MAX_L; H, W <= 2^31 - 1; nimg (H/b)(W/b) <=
 * LBG_MAX_M.  Output and input must not overlap.  No workspace.
 */
int lbg_image_blocks(const float* img, int64_t nimg, int64_t H, int64_t W,
                     int64_t b, float* X, void* stream);
int lbg_decode_image(const int32_t* idx, const float* C, int64_t N,
                     int64_t nimg, int64_t H, int64_t W, int64_t b,
                     float* img, void* stream);

/*
 * Host-only figures of merit (no GPU work; *out is a HOST double).
 * lbg_rate: log2(N) / L bits per sample (Introduction).  N >= 1, L >= 1.
 * lbg_psnr: peak signal-to-noise ratio of a reconstruction whose average
 *   distortion (lbg_distortion: mean over vectors of the squared error) is
 *   D: the mean squared error per sample is D / L, and
 *   PSNR = 10 log10(peak^2 / (D / L)) dB; +infinity when D == 0.  D >= 0,
 *   L >= 1, peak > 0 (255 for 8-bit pictures).
 */
int lbg_rate(int64_t N, int64_t L, double* out);
int lbg_psnr(double D, int64_t L, double peak, double* out);

/* Parameters of lbg_train.  lbg_params_default() fills the defaults. */
typedef struct lbg_params {
  double thr;        /* relative distortion-change threshold (1e-3), >= 0 */
  double eps_split;  /* multiplicative split factor (0.01), in (0, 1) */
  double delta;      /* additive split offset (split_mode == LBG_SPLIT_ADD) */
  int32_t split_mode;  /* LBG_SPLIT_MULT (default) or LBG_SPLIT_ADD */
  int32_t max_iter;    /* cap on updates per level (1000) */
  int32_t precision;   /* LBG_FP32 (default) or LBG_BF16_RESCORE */
  int32_t fixed_iters; /* > 0: exactly this many updates per level */
  const int32_t* forced_iters; /* HOST, nullable: updates for level i */
  int32_t n_forced;            /* entries of forced_iters */
  const float* C_init;         /* DEVICE, nullable: starting codebook */
  int64_t N_init;              /* rows of C_init (power of two, <= N) */
  int32_t timing;              /* nonzero: time kernels with HIP events */
  int32_t graph;               /* nonzero: replay batches of iterations as
                                  hipGraphs (non-NULL streams only); the
                                  default launches kernels directly */
  /* Resume in the middle of a level (with C_init only): C_init is the
   * codebook after it_init updates at its level and D_prev_init the
   * distortion of the allocation before the last of them, so the first stop
   * test compares against it (a run stopped there and resumed gives the
   * uninterrupted run's results bit for bit).  Defaults +inf and 0: C_init
   * starts a level. */
  double D_prev_init;          /* >= 0 or +inf */
  int32_t it_init;             /* >= 0 */
  int32_t stats_ties;          /* nonzero (with st): count near-tie rows of
                                  the final allocation (one extra FP64 pass) */
} lbg_params;

void lbg_params_default(lbg_params* p);

/* Statistics of one lbg_train run (HOST struct).  D_trace (HOST, nullable)
 * receives the distortion of every allocation, up to D_cap entries. */
typedef struct lbg_stats {
  int32_t n_levels;
  int32_t level_n[32];      /* codebook size of each level */
  int32_t level_iters[32];  /* updates performed at each level */
  int32_t total_updates;
  int32_t total_assigns;
  int64_t total_distances;  /* sum of M * n over all allocations */
  int64_t fallback_rows;    /* rows searched again exhaustively (FP32 mode) */
  double* D_trace;
  int32_t D_cap;
  int32_t n_D;
  /* With p->timing set: summed durations (milliseconds, HIP events on the
   * call's stream) of the allocation kernels and of the update kernels;
   * ms_split is not measured (zero). */
  double ms_assign;
  double ms_update;
  double ms_split;
  /* Codevectors of the returned codebook whose cell is empty in the final
   * allocation (they kept their value through the last update). */
  int32_t empty_cells;
  /* With p->stats_ties: rows of the final allocation whose two nearest
   * codevectors lie within 1e-6 |x|^2 of each other (FP64 direct form: the
   * tie band in which another rounding of the codebook may change the
   * allocation); -1 when not counted. */
  int64_t near_tie_rows;
} lbg_stats;

/*
 * LBG with splitting (Algorithm 1): start from the centroid of X (or from
 * C_init), then alternately split and iterate Cell Allocation / Updation at
 * each level until the relative distortion change (D_prev - D) <= thr *
 * D_prev, where D_prev is the distortion of the previous allocation at the
 * same level (the first allocation after a split never stops), until the
 * codebook has N codevectors (N a power of two, Terms of Sec. 2.2).
 * On return C_out (DEVICE, N x L) holds the codebook that produced the last
 * allocation, idx_out (DEVICE, M) that allocation and *D_out (HOST) its
 * distortion.  st (HOST, nullable) receives statistics.  Synchronises
 * ``stream``.  A distortion that is not finite (a NaN or infinite value in
 * X or C_init) stops the run at that allocation with LBG_EINVAL; C_out,
 * idx_out and *D_out then hold that allocation's state.
 */
int lbg_train(const float* X, int64_t M, int64_t L, int64_t N,
              const lbg_params* p, float* C_out, int32_t* idx_out,
              double* D_out, lbg_stats* st, void* ws, size_t ws_bytes,
              void* stream);

/* ------------------------------------------------------------ batched --
 * Many independent LBG runs (Algorithm 1 on each instance) advanced together:
 * every round performs one Lloyd iteration of every unfinished instance with
 * one persistent allocation launch, one accumulation launch and one update
 * launch for all of them.  Each instance's codebook, allocation, distortion,
 * level and iteration counts are bit-identical to lbg_train on that
 * instance alone with the same parameters.
 */
typedef struct lbg_instance {
  const float* X;    /* DEVICE, M x L FP32 row-major; 16-byte aligned for
                        vector loads (4-byte aligned at least) */
  int64_t M;         /* 1 <= M <= LBG_MAX_M */
  int64_t L;         /* 1 <= L <= 64 */
  int64_t N;         /* power of two; the N x L codebook must fit the
                        allocation's LDS (N <= 1024 at L <= 16, N <= 256 at
                        L <= 64) */
  float* C_out;      /* DEVICE, N x L: the final codebook */
  int32_t* idx_out;  /* DEVICE, M: its allocation */
} lbg_instance;

/* Launch configuration of the batched form.  grab: allocation slots (one
 * slot = one instance's share of one workgroup of the single-run kernel) a
 * workgroup takes per queue access; grid: workgroups of the persistent
 * allocation launch.  0 selects them by the autotuner, which times the
 * candidates on the instances' final codebook sizes once per workload
 * signature (instance count, sum of M, sum of M*N*L, sum of N) and caches
 * the result for the process.  graph != 0 (default) replays rounds from a
 * hipGraph (non-NULL streams), else launches them directly;
 * rounds_per_poll: rounds between host checks of the finished count
 * (direct launches); timing != 0: direct launches with an event pair around
 * every round's allocation and update (their sums in lbg_batch_stats).
 * screen: the allocation's screen for codebooks of more than 8 codevectors
 * (0 = chosen by the autotuner with grab and grid, 1 = FP32 screen, 2 = the
 * split BF16 screen wherever its codebook layout fits the workgroup's LDS,
 * the FP32 screen elsewhere).  Every choice gives the exact FP64 allocation,
 * so results do not depend on it. */
typedef struct lbg_batch_config {
  int32_t grab;
  int32_t grid;
  int32_t graph;
  int32_t rounds_per_poll;
  int32_t timing;
  int32_t screen;
} lbg_batch_config;

void lbg_batch_config_default(lbg_batch_config* cfg);

/* Per-instance outcome (HOST). */
typedef struct lbg_batch_result {
  double D;               /* distortion of the final allocation */
  int32_t status;         /* LBG_OK or LBG_WMAXITER */
  int32_t n_levels;
  int32_t n_assign;       /* allocations performed */
  int32_t n_update;       /* updates performed */
  int64_t fallback_rows;  /* rows searched again exhaustively */
  int64_t distances;      /* sum over its allocations of M * n */
} lbg_batch_result;

typedef struct lbg_batch_stats {
  int32_t rounds;   /* rounds launched (multiple of the poll interval) */
  int32_t grab;     /* configuration used */
  int32_t grid;
  int32_t graph;
  int32_t tuned;    /* 1 if this call ran the autotuner */
  int64_t total_distances;  /* sum over instances of sum M * n */
  double ms_tune;   /* time spent timing candidates */
  double ms_assign; /* with timing: all rounds' allocation launches */
  double ms_update; /* with timing: all rounds' update launches */
  int32_t screen;   /* screen used: 1 FP32, 2 split BF16 (where it fits) */
} lbg_batch_stats;

/* Workspace bytes for lbg_train_batched on these instances (0 on bad
 * arguments). */
size_t lbg_train_batched_workspace(const lbg_instance* inst, int32_t n_inst);

/*
 * Train every instance (HOST array inst[n_inst]) as lbg_train would, with
 * the shared parameters p (precision LBG_FP32; C_init and forced_iters are
 * not supported).  res (HOST, nullable) receives one lbg_batch_result per
 * instance, st (HOST, nullable) the statistics.  Returns LBG_OK,
 * LBG_WMAXITER if any instance hit the cap, LBG_EINVAL if an instance's
 * distortion was not finite (a NaN or infinite training value: that
 * instance's status is LBG_EINVAL, the other instances are trained and
 * their results valid), or another error code (nothing is trained then).
 * Synchronises ``stream``.
 */
int lbg_train_batched(const lbg_instance* inst, int32_t n_inst, const lbg_params* p,
                      const lbg_batch_config* cfg, lbg_batch_result* res,
                      lbg_batch_stats* st, void* ws, size_t ws_bytes, void* stream);

/*
 * Batched single steps: many independent items in a few launches for all of
 * them (the batched form's kernels), each item's result bit-identical to the
 * single call on it.  HOST arrays items[n]; device pointers inside.  The
 * workspace (device, 256-byte aligned) is sized by the *_workspace call on
 * the same items.  Both synchronise ``stream`` (the items' descriptors are
 * uploaded from host memory that is released on return).
 *
 * Cell Allocation (Algorithm 1, "Cell Allocation"; Sec. 3.2) of item i:
 * idx[m] = the nearest row of C (squared Euclidean distance, lowest index
 * on ties) for every row of X, exactly as lbg_assign(X, M, L, C, N, idx,
 * NULL, LBG_FP32, ...); D (nullable) receives (1/M) sum_m d(x_m, c_idx[m])
 * in FP64, lbg_assign_distortion's D bit for bit.  1 <= L <= 64, N >= 1, and
 * the codebook must fit the allocation's LDS as for lbg_instance
 * ((N rounded up to 32) * (16 or 64, L rounded up, + 4) * 4 <= 81920 bytes).
 * A non-finite row gets index 0 and makes D +inf.
 */
typedef struct lbg_assign_item {
  const float* X;  /* DEVICE, M x L FP32 row-major (16-byte aligned rows for
                      vector loads; 4-byte aligned at least) */
  int64_t M;       /* 1 <= M <= LBG_MAX_M */
  int64_t L;       /* 1 <= L <= 64 */
  const float* C;  /* DEVICE, N x L FP32 */
  int64_t N;       /* 1 <= N; see the LDS limit above */
  int32_t* idx;    /* DEVICE, M: the allocation (out) */
  double* D;       /* DEVICE, nullable: the mean distortion (out) */
} lbg_assign_item;

size_t lbg_assign_batched_workspace(const lbg_assign_item* items, int32_t n);
int lbg_assign_batched(const lbg_assign_item* items, int32_t n, void* ws, size_t ws_bytes,
                       void* stream);

/*
 * Codebook Updation (Algorithm 1, "Codebook Updation"; Sec. 3.2) of item i:
 * C_new[k] = the mean of the rows with idx == k (an empty cell keeps
 * C_old[k]; entries of idx outside [0, N) join no cell), from exact
 * fixed-point sums as lbg_update does, so C_new and counts equal
 * lbg_update's bit for bit.  C_new may equal C_old (in place); otherwise
 * they must not overlap.  1 <= L <= 64, and N * L within the fixed-point
 * path's limit (LBG_EINVAL names the item otherwise: use lbg_update).
 */
typedef struct lbg_update_item {
  const float* X;        /* DEVICE, M x L FP32 row-major */
  int64_t M;             /* 1 <= M <= LBG_MAX_M */
  int64_t L;             /* 1 <= L <= 64 */
  const int32_t* idx;    /* DEVICE, M */
  const float* C_old;    /* DEVICE, N x L */
  int64_t N;             /* >= 1 */
  float* C_new;          /* DEVICE, N x L (out) */
  int32_t* counts;       /* DEVICE, N, nullable: the cell sizes (out) */
} lbg_update_item;

size_t lbg_update_batched_workspace(const lbg_update_item* items, int32_t n);
int lbg_update_batched(const lbg_update_item* items, int32_t n, void* ws, size_t ws_bytes,
                       void* stream);

/*
 * lbg_assign_distortion without a workspace, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and error
 * behaviour as lbg_assign_distortion, bit for bit, minus ws / ws_bytes: the
 * scratch space (the distortion partials, the prepared codebook) is a fixed
 * device array inside the library of lbg_noalloc_scratch_bytes() bytes
 * (8 MiB), one per GPU, kept until the process ends.  A problem whose
 * scratch, lbg_workspace_size(LBG_OP_ASSIGN, M, L, N, precision), exceeds
 * it is rejected with LBG_EINVAL (roughly M <= 2^24 rows with a small
 * codebook).  Allocates nothing: no hipMalloc / hipFree, no library
 * allocation.  Every call on one GPU uses the same array: calls that overlap
 * on one GPU (different streams, or threads) race and must be ordered by the
 * caller.  D must be 8-byte aligned.
 */
int lbg_assign_distortion_noalloc(const float* X, int64_t M, int64_t L,
                                  const float* C, int64_t N, int32_t* idx,
                                  float* mind, int precision, double* D,
                                  void* stream);
size_t lbg_noalloc_scratch_bytes(void);

/* Bytes of workspace the operation ``op`` (LBG_OP_*) needs. */
size_t lbg_workspace_size(int op, int64_t M, int64_t L, int64_t N,
                          int precision);

/* Message of the last failed call on this thread ("" if none). */
const char* lbg_last_error(void);

/* Library version string. */
const char* lbg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBG_H */
