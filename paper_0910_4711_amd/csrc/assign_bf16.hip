// Cell Allocation with a BF16 matrix-core screen (precision form).
//
// Training vectors and codevectors are rounded to BF16 (round to nearest
// even) and the expanded squared distance of the rounded vectors is
// accumulated in FP32 on v_mfma_f32_32x32x16_bf16; each FP32 squared norm
// enters the extra K-step as three BF16 parts whose sum is that norm exactly.
// The two best candidates per vector are rescored in FP64 (direct form, on
// the original FP32 data) and the closer one is taken.  A vector whose true
// nearest codevector is not among the BF16 top two is misassigned; the error
// against the FP64 reference is measured, not bounded.
#include "assign_common.h"

namespace lbg {

using namespace assign_detail;

int launch_assign_bf16(const float* X, int64_t M, int L, const float* C, int n, int32_t* idx,
                       float* mind, double* dpart, int LP, void* prep, hipStream_t s,
                       Ctl ctl, CbPair cbp) {
  switch (LP) {
    case 8:
    case 16: return launch_screen<Bf16Screen<16>>(X, M, L, C, n, idx, mind, dpart, nullptr, prep, s, ctl, cbp);
    case 32: return launch_screen<Bf16Screen<32>>(X, M, L, C, n, idx, mind, dpart, nullptr, prep, s, ctl, cbp);
    case 64: return launch_screen<Bf16Screen<64>>(X, M, L, C, n, idx, mind, dpart, nullptr, prep, s, ctl, cbp);
    default: return launch_screen<Bf16Screen<128>>(X, M, L, C, n, idx, mind, dpart, nullptr, prep, s, ctl, cbp);
  }
}

}  // namespace lbg
