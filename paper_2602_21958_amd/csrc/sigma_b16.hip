// 16-bit operand Sigma GEMM (BF16 / FP16 / split BF16) - placeholder until
// the MFMA operand layouts are confirmed.
#include "rt_internal.h"

namespace rtsn {

void launch_sigma_b16(const Problem&, int, const void*, const float*, float*, const double*,
                      double, hipStream_t) {
  fail(RT_E_INVALID, "16-bit Sigma path not available in this build");
}

}  // namespace rtsn
