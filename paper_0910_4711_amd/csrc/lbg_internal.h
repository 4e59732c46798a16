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

// Rows handled by one workgroup of the matrix-core allocation kernels.
int assign_rows_per_wg(int64_t L, int precision);

struct AssignWs {
  double* dpart;           // per-row-tile distortion partial sums
  unsigned long long* nfb; // rows that fell back to the exhaustive search
  unsigned char* prep;     // codebook in the screen's LDS row layout
};
void plan_assign(Carver& c, int64_t M, int64_t L, int64_t N, int precision,
                 AssignWs* ws);

// Enqueue the allocation.  dpart (nullable) receives per-workgroup FP64
// partial sums of the winning distances; nfb (nullable) counts fallback rows.
int launch_assign(const float* X, int64_t M, int64_t L, const float* C,
                  int64_t N, int32_t* idx, float* mind, int precision,
                  double* dpart, unsigned long long* nfb, void* prep, hipStream_t s);
int64_t assign_num_parts(int64_t M, int64_t L, int precision);

// Sum ``nparts`` FP64 partials in a fixed order and divide by ``denom``.
int launch_reduce_parts(const double* parts, int64_t nparts, double denom,
                        double* out, hipStream_t s);

// ------------------------------------------------------------ updation --
// Exact fixed-point accumulation (default for codebooks of moderate size).
struct AfpWs {
  unsigned long long* part;  // [nchunks][N][L] integer partial sums
  int32_t* pcnt;             // [nchunks][N] partial counts
  uint32_t* amax;            // [absmax_blocks] block maxima of |x|
  int* shift;                // [1] fixed-point shift s
  int cps, nslices, nchunks, absmax_blocks;
  int64_t rows_per_chunk;
};
bool afp_usable(int64_t L, int64_t N);
void plan_afp(Carver& c, int64_t M, int64_t L, int64_t N, AfpWs* w);
int launch_afp_shift(const float* X, int64_t M, int64_t L, const AfpWs& w, hipStream_t s);
int launch_afp(const float* X, int64_t M, int64_t L, const int32_t* idx, const float* C_old,
               int64_t N, float* C_out, int32_t* counts, int mode, double g2, const AfpWs& w,
               hipStream_t s);

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
                  hipStream_t s);

// ----------------------------------------------------------------- misc --
struct CentroidWs {
  double* part;  // [nwg][L]
  int64_t nwg;
};
void plan_centroid(Carver& c, int64_t M, int64_t L, CentroidWs* ws);
int launch_centroid(const float* X, int64_t M, int64_t L, float* c0,
                    const CentroidWs& ws, hipStream_t s);

int launch_split(const float* C, int64_t n, int64_t L, int mode, double eps,
                 double delta, float* C2, hipStream_t s);

struct DistWs {
  double* part;
  int64_t nparts;
};
void plan_distortion(Carver& c, int64_t M, DistWs* ws);
int launch_distortion(const float* X, int64_t M, int64_t L, const float* C,
                      int64_t N, const int32_t* idx, double* D,
                      const DistWs& ws, hipStream_t s);

int launch_grad_x(const float* X, int64_t M, int64_t L, const float* C,
                  int64_t N, const int32_t* idx, double g2, float* gX,
                  hipStream_t s);

}  // namespace lbg
