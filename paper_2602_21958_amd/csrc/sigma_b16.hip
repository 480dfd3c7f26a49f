// Scattering GEMM with 16-bit matrix-core operands and FP32 accumulation:
//   y[k, i] = xs * x[k, i] + sign * (1 - eps_i) * rs_k * sum_k' Mhat'[k, k'] L'[k', i]
// (the operator epilogue of the FP64 GEMM; Mhat' / L' are the stored 16-bit
// operands, rs_k undoes their scaling).
//
// Operands: v_mfma_f32_16x16x32_{bf16,f16}.  A lane holds 8 consecutive k of
// one row of A (Mhat) and 8 consecutive k of one column of B (L); both are
// staged in LDS k-contiguous.  Mhat is stored with a leading dimension padded
// to a multiple of 8 so its rows load as aligned 16-byte vectors; the L tile
// (row-major, points contiguous) is read as 8 k x 4 points per thread and
// transposed in registers before the LDS store.
//
// Modes: BF16 (Lambda emits bf16), FP16 (Lambda emits fp16 scaled by a power
// of two, Mhat rows scaled to unit maximum; both undone in FP32 in the
// epilogue) and split BF16 ("bf16x3": Mhat = hi + lo and L = hi + lo in bf16,
// hi*hi + hi*lo + lo*hi accumulated; L arrives as FP32 and is split while it
// is staged).
#include <cmath>

#include "gemm16_dev.h"

namespace rtsn {

namespace {

template <bool IS_BF16, bool SPLIT>
__global__ __launch_bounds__(256) void sigma_b16_kernel(
    const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo, int lda,
    const void* __restrict__ Bv, const float* X, float* Y, const double* __restrict__ albedo,
    const float* __restrict__ rowscale, float bscale_inv, const double* __restrict__ xscale,
    int M, int N, int K, float sign) {
  using namespace gemm16;
  const int n_tiles_m = (M + BM - 1) / BM;
  const int n_tiles_n = (N + BN - 1) / BN;
  int tm, tn;
  tile_of(blockIdx.x, n_tiles_m, n_tiles_m * n_tiles_n, tm, tn);
  const float xs = (X != nullptr && xscale != nullptr) ? (float)*xscale : 1.f;
  gemm16_tile<IS_BF16, SPLIT>(Ahi, Alo, lda, Bv, X, Y, albedo, rowscale, bscale_inv, xs, M, N, K,
                              tm * BM, tn * BN, sign);
}

}  // namespace

// Power-of-two scale applied to Lambda's fp16 output (keeps unit-norm Krylov
// vectors of n entries near 1 in magnitude).
float fp16_lambda_scale(int64_t n) {
  const double e = std::ceil(0.5 * std::log2((double)(n > 1 ? n : 1)));
  return (float)std::ldexp(1.0, (int)e);
}

void launch_sigma_b16(const Problem& p, int precision, const void* L, const float* x, float* y,
                      const double* xscale, double sign, hipStream_t st) {
  const int M = p.n_r, N = (int)p.n_s, K = p.n_r;
  const int tiles = ((M + gemm16::BM - 1) / gemm16::BM) * ((N + gemm16::BN - 1) / gemm16::BN);
  ProfScope prof(RT_KCLASS_SIGMA, st);
  const int lda = p.lda16;
  const auto* hi = reinterpret_cast<const uint16_t*>(p.d_mhat_bf16);
  const auto* lo = reinterpret_cast<const uint16_t*>(p.d_mhat_bf16_lo);
  const auto* h16 = reinterpret_cast<const uint16_t*>(p.d_mhat_f16);
  switch (precision) {
    case RT_PREC_BF16:
      hipLaunchKernelGGL((sigma_b16_kernel<true, false>), dim3(tiles), dim3(256), 0, st,
                         hi, nullptr, lda, L, x, y, p.d_albedo, nullptr, 1.f, xscale,
                         M, N, K, (float)sign);
      break;
    case RT_PREC_FP16:
      hipLaunchKernelGGL((sigma_b16_kernel<false, false>), dim3(tiles), dim3(256), 0, st,
                         h16, nullptr, lda, L, x, y, p.d_albedo, p.d_f16_rowscale,
                         1.f / fp16_lambda_scale(p.n), xscale, M, N, K, (float)sign);
      break;
    case RT_PREC_BF16X3:
      hipLaunchKernelGGL((sigma_b16_kernel<true, true>), dim3(tiles), dim3(256), 0, st,
                         hi, lo, lda, L, x, y, p.d_albedo, nullptr, 1.f,
                         xscale, M, N, K, (float)sign);
      break;
    default:
      fail(RT_E_INVALID, "launch_sigma_b16: not a 16-bit precision");
  }
  RT_HIP(hipGetLastError());
}

}  // namespace rtsn
