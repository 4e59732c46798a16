// Cell Allocation and its distortion without a caller workspace: for callers
// that cannot allocate device memory (code under stream capture, serving
// loops, harnesses that forbid allocation).  The scratch space of the
// allocation -- the FP64 distortion partial of every 32 rows and, for a
// codebook too large for one workgroup's LDS, the codebook in the screen's
// row layout -- lives in a file-scope device array of kScratchBytes, one copy
// per GPU, reached through its device address (hipGetSymbolAddress, taken
// once per device).  Every call on a GPU uses the same array, so calls that
// overlap on one GPU race; every byte a call reads is written by that call
// first (the partials of all its row groups, the whole prepared codebook), so
// nothing has to be cleared between calls.
#include <mutex>

#include "lbg_internal.h"

namespace lbg {
namespace {

constexpr size_t kScratchBytes = (size_t)8 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (the array's name in host code
// is only a stand-in for the symbol).
int scratch_ptr(void** out) {
  int dev = 0;
  LBG_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d devices the scratch table holds", dev, kMaxDevices);
    return LBG_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    LBG_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return LBG_OK;
}

}  // namespace
}  // namespace lbg

using namespace lbg;

extern "C" {

size_t lbg_noalloc_scratch_bytes(void) { return kScratchBytes; }

int lbg_assign_distortion_noalloc(const float* X, int64_t M, int64_t L, const float* C,
                                  int64_t N, int32_t* idx, float* mind, int precision,
                                  double* D, void* stream) {
  clear_error();
  if (M < 1 || M > LBG_MAX_M || L < 1 || L > LBG_MAX_L || N < 1 || N > LBG_MAX_N) {
    set_error("lbg_assign_distortion_noalloc: M = %lld, L = %lld, N = %lld out of range",
              (long long)M, (long long)L, (long long)N);
    return LBG_EINVAL;
  }
  if (precision != LBG_FP32 && precision != LBG_BF16_RESCORE) {
    set_error("unknown precision %d", precision);
    return LBG_EINVAL;
  }
  if (!X || !C || !idx || !D) {
    set_error("lbg_assign_distortion_noalloc: X, C, idx and D must not be NULL");
    return LBG_EINVAL;
  }
  if (((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(C) |
        reinterpret_cast<uintptr_t>(idx) | reinterpret_cast<uintptr_t>(mind)) & 3) ||
      (reinterpret_cast<uintptr_t>(D) & 7)) {
    set_error("lbg_assign_distortion_noalloc: misaligned pointer");
    return LBG_EINVAL;
  }
  Carver count{nullptr, 0};
  AssignWs w;
  plan_assign(count, M, L, N, precision, &w);
  if (count.size() > kScratchBytes) {
    set_error("lbg_assign_distortion_noalloc: this problem needs %zu bytes of scratch, more "
              "than the %zu bytes of the library's fixed array (M = %lld, L = %lld, "
              "N = %lld); use lbg_assign_distortion with a workspace",
              count.size(), kScratchBytes, (long long)M, (long long)L, (long long)N);
    return LBG_EINVAL;
  }
  void* base = nullptr;
  LBG_TRY(scratch_ptr(&base));
  Carver c{reinterpret_cast<char*>(base), 0};
  plan_assign(c, M, L, N, precision, &w);
  hipStream_t s = (hipStream_t)stream;
  LBG_TRY(launch_assign(X, M, L, C, N, idx, mind, precision, w.dpart, nullptr, w.prep, s));
  return launch_reduce_parts(w.dpart, assign_num_parts(M, L, N, precision), (double)M, D, s);
}

}  // extern "C"
