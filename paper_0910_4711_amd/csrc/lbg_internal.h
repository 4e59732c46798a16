// Internal declarations shared by the host entry points and the kernel
// launchers of the LBG library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lbg.h"

namespace lbg {

// ---------------------------------------------------------------- errors --
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();
int hip_fail(hipError_t e, const char* what);

#define LBG_TRY_HIP(call)                                  \
  do {                                                     \
    hipError_t e__ = (call);                               \
    if (e__ != hipSuccess) return ::lbg::hip_fail(e__, #call); \
  } while (0)

#define LBG_TRY(call)          \
  do {                         \
    int r__ = (call);          \
    if (r__ < 0) return r__;   \
  } while (0)

// ---------------------------------------------------- device-side control --
// State of a training run kept in device memory, so that the iteration and
// level control of Algorithm 1 runs on the GPU without host round trips.
// The "decide" kernel (one block, after each allocation) applies the stop
// test and sets the action of the iteration; the update and split kernels
// read it and do nothing unless it names them; every kernel of an iteration
// does nothing once the run is done.
enum { kActNone = 0, kActUpdate = 1, kActSplit = 2 };
struct DevState {
  int32_t n, cb;                     // codebook of the next allocation
  int32_t src, dst, n_src, action;   // this iteration's update / split
  int32_t done, status;              // status: LBG_OK or LBG_WMAXITER
  int32_t level, it, first;
  int32_t n_assign, n_update;
  int32_t N, max_iter, fixed_iters, n_forced, split_mode, D_cap;
  int32_t forced[32];
  int32_t level_n[32], level_iters[32];
  int64_t M, distances;
  double D, D_prev, thr, eps, delta;
};
struct CbPair {
  float* c[2];  // the two codebook buffers the state's indices refer to
};
// Launch-time bundle for kernels under device-side control (null st: not).
// The update's accumulation kernel derives the decision of the iteration
// from the allocation's per-wave partials (every block the same way) and its
// block 0 writes the next state into ``pend``; the update's last kernel
// acts on ``pend`` and its block 0 commits it to ``st``.
struct Ctl {
  DevState* st;
  DevState* pend;
  const double* dpart;
  int64_t nparts;
  double* Dtrace;   // distortion of every allocation
  int32_t* Atrace;  // action decided after every allocation
  // (allocation, nullable) the training set's fixed-point scales and
  // properties as the set-up pass writes them; [2] != 0: every coordinate
  // is exact in BF16
  const int* xflags;
};

__host__ __device__ inline int tile_bits_of(int64_t n) {
  const int tiles = (int)((n + 31) / 32);
  int b = 0;
  while ((1 << b) < tiles) ++b;
  return b;
}

// ------------------------------------------------------------- workspace --
// Carves a caller workspace into 256-byte aligned pieces.  With base ==
// nullptr it only counts, so the same plan yields the size query and the
// layout.
struct Carver {
  char* base;
  size_t off;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  size_t size() const { return (off + 255) & ~(size_t)255; }
};

// ----------------------------------------------------------- allocation --
constexpr int kAssignThreads = 256;

struct AssignWs {
  double* dpart;           // distortion partial sums, one per 32 vectors
  unsigned long long* nfb; // rows that fell back to the exhaustive search
  unsigned char* prep;     // codebook in the screen's LDS row layout
};
void plan_assign(Carver& c, int64_t M, int64_t L, int64_t N, int precision,
                 AssignWs* ws);

// Enqueue the allocation.  dpart (nullable) receives FP64 partial sums of
// the winning distances (assign_num_parts of them); nfb (nullable) counts
// fallback rows.
// With ``st`` set, the codebook and its size come from the device state
// (buffer cbp.c[st->cb], st->n rows, N the largest size) and the launch does
// nothing once the run is done.
int launch_assign(const float* X, int64_t M, int64_t L, const float* C,
                  int64_t N, int32_t* idx, float* mind, int precision,
                  double* dpart, unsigned long long* nfb, void* prep, hipStream_t s,
                  Ctl ctl = Ctl{nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr},
                  CbPair cbp = CbPair{{nullptr, nullptr}});
// Partials of the distortion that the allocation writes.
int64_t assign_num_parts(int64_t M, int64_t L, int64_t N, int precision);

// Sum ``nparts`` FP64 partials in a fixed order and divide by ``denom``.
int launch_reduce_parts(const double* parts, int64_t nparts, double denom,
                        double* out, hipStream_t s);

// ------------------------------------------------------------ updation --
// Exact fixed-point accumulation (default for codebooks of moderate size).
struct AfpWs {
  unsigned long long* part;  // [nchunks][N][L] integer partial sums
  int32_t* pcnt;             // [nchunks][N] partial counts
  uint32_t* amax;            // [3 absmax_blocks] block maxima of |x|, fine bits, BF16 rest
  int* shift;                // [5] fixed-point shift s, second-word shift t (0: none),
                             // every coordinate exact in BF16, 32-bit sums possible and
                             // their shift g
  unsigned long long* lo;    // [N][L] second-word sums (kept zero between updates)
  int64_t nlo;
  int cps, nslices, nchunks, absmax_blocks;
  int dslices;  // > 0: accumulation by this many 16-dimension slices (all cells per block)
  int64_t rows_per_chunk;
  // > 0: the 32-bit accumulation by this many 32-dimension slices is
  // possible (when shift[3] says so), in nch_n chunks (rows dealt in spans),
  // its partials int32 [nch_n][N][L] in the bytes of ``part``
  int nds_n, nch_n;
  // > 0: one of many instances whose update runs this many 16-dimension
  // slices with all cells in LDS (batched form)
  int bds;
};
bool afp_usable(int64_t L, int64_t N);
// dslices: the single-run kernels may accumulate by dimension slices
// bds_ok (with many): the batched form may run 16-dimension slices.
void plan_afp(Carver& c, int64_t M, int64_t L, int64_t N, AfpWs* w, bool dslices = true,
              bool many = false, bool bds_ok = false);
int launch_afp_shift(const float* X, int64_t M, int64_t L, const AfpWs& w, hipStream_t s);
// The finishing kernel of the update (centroids or gradient from the partials).
// p32: the partials are those of the 32-bit slices.
int launch_fin(const float* X, int64_t M, int64_t L, const float* C_old, int64_t N,
               float* C_out, int32_t* counts, int mode, double g2, const AfpWs& w,
               hipStream_t s, Ctl ctl, CbPair cbp, bool p32 = false);
// on_grid: 1 when the caller knows every coordinate lies on the 2^-s grid
// (shift[1] == 0: one-word kernels), 2 when shift[3] is also set (the 32-bit
// dimension slices where planned), else 0: the kernels read that on the
// device.
int launch_afp(const float* X, int64_t M, int64_t L, const int32_t* idx, const float* C_old,
               int64_t N, float* C_out, int32_t* counts, int mode, double g2, const AfpWs& w,
               hipStream_t s, Ctl ctl = Ctl{nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr},
               CbPair cbp = CbPair{{nullptr, nullptr}}, int on_grid = 0);

// Sort-based fixed-order segmented sums (codebooks too large for the above).
struct UpdateWs {
  int32_t* ghist;    // [N][ntiles] per-tile cell counts, then offsets
  int32_t* bin_off;  // [N + 1] first sorted position of every cell
  int32_t* perm;     // [M] rows in cell order
  double* partial;   // [nruns][2][LP] run-boundary partial sums
  int32_t* cnt;      // [N] cell sizes
  int64_t T, ntiles, P, nruns, LP;
  bool use_afp;
  AfpWs afp;
};
void plan_update(Carver& c, int64_t M, int64_t L, int64_t N, UpdateWs* ws);

// mode 0: centroids (C_new, counts); mode 1: gC = g2 * sum (c_k - x).
// shift_ready: the fixed-point shift for X is already in the workspace.
int launch_update(const float* X, int64_t M, int64_t L, const int32_t* idx,
                  const float* C_old, int64_t N, float* C_out, int32_t* counts,
                  int mode, double g2, const UpdateWs& ws, bool shift_ready,
                  hipStream_t s, int on_grid = 0);

// ----------------------------------------------------------------- misc --
struct CentroidWs {
  double* part;    // [nwg][L]
  uint32_t* amax;  // [3 nwg] block maxima of |x|, fine bits, BF16 rest (set-up of a run)
  int64_t nwg;
};
void plan_centroid(Carver& c, int64_t M, int64_t L, CentroidWs* ws);
int launch_centroid(const float* X, int64_t M, int64_t L, float* c0,
                    const CentroidWs& ws, hipStream_t s);
// Set-up of a training run from the centroid (two launches): c0, its split
// into C2 (two codevectors), the fixed-point shift of X, the initial device
// state and the cleared fallback counter.  The same values as
// launch_centroid, launch_split, launch_afp_shift and the state copy.
int launch_setup(const float* X, int64_t M, int64_t L, float* c0, float* C2, int mode,
                 double eps, double delta, const CentroidWs& ws, int* shift,
                 unsigned long long* lo, int64_t nlo,
                 const DevState& init, DevState* st, unsigned long long* nfb, hipStream_t s);

int launch_split(const float* C, int64_t n, int64_t L, int mode, double eps,
                 double delta, float* C2, hipStream_t s, const DevState* st = nullptr,
                 CbPair cbp = CbPair{{nullptr, nullptr}});
// One block: D = sum(dpart) / M (fixed order), trace, stop test, action.
int launch_decide(const double* dpart, int64_t nparts, DevState* st, double* Dtrace,
                  int32_t* Atrace, hipStream_t s);

struct DistWs {
  double* part;
  int64_t nparts;
};
void plan_distortion(Carver& c, int64_t M, DistWs* ws);
int launch_distortion(const float* X, int64_t M, int64_t L, const float* C,
                      int64_t N, const int32_t* idx, double* D,
                      const DistWs& ws, hipStream_t s);

// Statistics of a finished run: cell sizes of the allocation idx over n
// codevectors into cnt [n] (workspace), out[0] = empty cells, out[1] (with
// ties) = rows within the tie band (FP64 top two); out is 2 device words.
int launch_run_stats(const float* X, int64_t M, int64_t L, const float* C, int64_t n,
                     const int32_t* idx, bool ties, int32_t* cnt, unsigned long long* out,
                     hipStream_t s);

int launch_grad_x(const float* X, int64_t M, int64_t L, const float* C,
                  int64_t N, const int32_t* idx, double g2, float* gX,
                  hipStream_t s);

// ---------------------------------------------------------------- codec --
int launch_decode(const int32_t* idx, int64_t M, const float* C, int64_t N, int64_t L, float* Y,
                  hipStream_t s);
// dir 0: indices -> pictures; dir 1: pictures -> block vectors.
int launch_image(int dir, const int32_t* idx, const float* C, int64_t N, int64_t nimg,
                 int64_t H, int64_t W, int64_t b, const float* img_in, float* out,
                 hipStream_t s);

// ------------------------------------------------------------- training --
constexpr int kTraceCap = 32768;  // allocations recorded on the device

struct TrainWs {
  float* Cb[2];
  double* D;
  AssignWs as;
  UpdateWs up;
  CentroidWs ce;
  DevState* st;
  DevState* pend;
  double* Dtrace;
  int32_t* Atrace;
  int32_t* cellcnt;              // [N] cell sizes (statistics)
  unsigned long long* runstat;   // [2] empty cells, near-tie rows
};
void plan_train(Carver& c, int64_t M, int64_t L, int64_t N, int precision, TrainWs* w);

// Whether the device-controlled loop can run this problem.
bool train_device_ok(int64_t L, const TrainWs& w);
// LBG with splitting, controlled on the device (see DevState).  Returns
// LBG_OK / LBG_WMAXITER or an error.
int train_device(const float* X, int64_t M, int64_t L, int64_t N, const lbg_params* p,
                 float* C_out, int32_t* idx_out, double* D_out, lbg_stats* st,
                 const TrainWs& w, hipStream_t s);

}  // namespace lbg
