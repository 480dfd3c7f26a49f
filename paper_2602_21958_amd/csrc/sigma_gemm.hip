// Scattering step Sigma as one dense GEMM on the matrix cores of gfx950.
//
// Paper Sec. 3.3: Sigma is block diagonal over spatial points with the same
// N_r x N_r block Gamma Psi W at every point when the scattering coefficients
// are point independent (eq. Sigma); up to the per-point factor 1 - eps_i
// this block is Mhat.  In the ray-major layout the scattering of all points
// is therefore C = Mhat (N_r x N_r) * L (N_r x N_s), with the operator
// epilogue fused:
//     y[k, i] = xs * x[k, i] + sign * (1 - eps_i) * C[k, i].
//
// FP64 / FP32 path: v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32 (one
// operand element per lane).  Workgroup tile 128 x 128, K tile 16, four
// waves in a 2 x 2 arrangement each owning a 64 x 64 sub-tile (4 x 4 MFMA
// blocks).  Mhat is kept transposed in HBM so that both operand tiles are
// [k][m] / [k][n] row segments, loaded with 16-byte vectors and stored to LDS
// unchanged; the next K tile is prefetched into registers while the current
// one is multiplied from a double-buffered LDS ring.  Tiles are assigned so
// that consecutive workgroups on the same XCD share the same column strip of
// L (L2 reuse).
#include <cstdlib>

#include "gemm_dev.h"

namespace rtsn {

using gemm::TileDots;

namespace {

template <typename T, int BK, bool DOTS>
__global__ __launch_bounds__(256) void sigma_gemm_kernel(
    const T* __restrict__ A, int lda, const T* __restrict__ B, const T* X, T* Y,
    const double* __restrict__ albedo, const double* __restrict__ xscale, int M, int N, int K,
    double sign, TileDots dots) {
  using namespace gemm;
  const int n_tiles_m = (M + BM - 1) / BM;
  const int n_tiles_n = (N + BN - 1) / BN;
  int tm, tn;
  tile_of(blockIdx.x, n_tiles_m, n_tiles_m * n_tiles_n, tm, tn);
  const double xs = (X != nullptr && xscale != nullptr) ? *xscale : 1.0;
  gemm_tile<T, BK, DOTS>(A, lda, B, X, Y, albedo, xs, M, N, K, tm * BM, tn * BN, sign, dots,
                         tn * n_tiles_m + tm);
}

template <typename T>
void launch_gemm_core(const T* mhat, int lda, const T* L, const T* x, T* y,
                      const double* albedo, const double* xscale, int M, int N, int K,
                      double sign, hipStream_t st, TileDots* dots) {
  const int tiles = ((M + gemm::BM - 1) / gemm::BM) * ((N + gemm::BN - 1) / gemm::BN);
  if (dots) {
    if (dots->ldp < tiles) fail(RT_E_INVALID, "fused dots: too few partial slots");
    dots->ldp = tiles;   // one slot per tile, all written
  }
  const TileDots d = dots ? *dots : TileDots{};
#define RT_SIGMA_LAUNCH(BKV, DV)                                                              \
  hipLaunchKernelGGL((sigma_gemm_kernel<T, BKV, DV>), dim3(tiles), dim3(256), 0, st, mhat,   \
                     lda, L, x, y, albedo, xscale, M, N, K, sign, d)
  // K stage 16 (a stage of 32 was measured slower)
  if (dots) RT_SIGMA_LAUNCH(16, true); else RT_SIGMA_LAUNCH(16, false);
#undef RT_SIGMA_LAUNCH
  RT_HIP(hipGetLastError());
}

template <typename T>
void launch_sigma_t(const Problem& p, const T* mhat, const T* L, const T* x, T* y,
                    const double* xscale, double sign, hipStream_t st, TileDots* dots) {
  ProfScope prof(sizeof(T) == 8 ? RT_KCLASS_SIGMA : RT_KCLASS_SIGMA_LO, st);
  launch_gemm_core<T>(mhat, p.lda_mhat, L, x, y, p.d_albedo, xscale, p.n_r, (int)p.n_s,
                      p.n_r, sign, st, dots);
}

}  // namespace

void launch_gemm_f64(const Problem& p, const double* A, const double* L, int N,
                     const double* x, double* y, const double* albedo, const double* xscale,
                     double sign, hipStream_t st) {
  launch_gemm_core<double>(A, p.lda_mhat, L, x, y, albedo, xscale, p.n_r, N, p.n_r, sign, st,
                           nullptr);
}

void launch_gemm_f32(const Problem& p, const float* A, const float* L, int N, const float* x,
                     float* y, const double* albedo, const double* xscale, double sign,
                     hipStream_t st) {
  launch_gemm_core<float>(A, p.lda_mhat, L, x, y, albedo, xscale, p.n_r, N, p.n_r, sign, st,
                          nullptr);
}

void launch_sigma_f64(const Problem& p, const double* L, const double* x, double* y,
                      const double* xscale, double sign, hipStream_t st, TileDots* dots) {
  launch_sigma_t<double>(p, p.d_mhat64, L, x, y, xscale, sign, st, dots);
}

void launch_sigma_f32(const Problem& p, const float* L, const float* x, float* y,
                      const double* xscale, double sign, hipStream_t st, TileDots* dots) {
  launch_sigma_t<float>(p, p.d_mhat32, L, x, y, xscale, sign, st, dots);
}

int sigma_dot_slots(const Problem& p, int precision) {
  if (precision == RT_PREC_FP64 || precision == RT_PREC_FP32)
    return ((p.n_r + gemm::BM - 1) / gemm::BM) * (int)((p.n_s + gemm::BN - 1) / gemm::BN);
  // 16-bit: the smallest candidate tile is 128 x 128 over mp16 rows
  return (p.mp16 / 128) * (int)((p.n_s + 127) / 128);
}

}  // namespace rtsn
