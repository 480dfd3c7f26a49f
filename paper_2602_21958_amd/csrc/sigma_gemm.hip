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
// blocks).  A (Mhat) is staged transposed in LDS ([k][m]), B (L) as loaded
// ([k][n]); the next K tile is prefetched into registers while the current
// one is multiplied.  Tiles are assigned so that consecutive workgroups on
// the same XCD share the same column strip of L (L2 reuse).
#include "rt_internal.h"

namespace rtsn {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Result element r of lane l sits at row dr(l, r), column l % 16 of the
// 16 x 16 block: f64 interleaves rows (l/16 + 4r), f32 stacks them (4(l/16) + r).
template <> struct Mfma<double> {
  using acc_t = d4_t;
  static __device__ __forceinline__ int dr(int lane, int r) { return (lane >> 4) + 4 * r; }
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  using acc_t = f4_t;
  static __device__ __forceinline__ int dr(int lane, int r) { return 4 * (lane >> 4) + r; }
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int PAD = 16;  // LDS row padding (elements) against bank conflicts

// Map a linear workgroup id to (m tile, n tile): workgroups are dealt to the
// 8 XCDs round-robin, so regroup ids per XCD and walk m fastest.
__device__ __forceinline__ void tile_of(int bid, int n_tiles_m, int n_tiles, int& tm, int& tn) {
  const int xcd = bid & 7;
  const int local = bid >> 3;
  const int per_xcd = (n_tiles + 7) >> 3;
  int t = xcd * per_xcd + local;
  if ((n_tiles & 7) != 0) t = bid;  // uneven split: keep the plain order
  tm = t % n_tiles_m;
  tn = t / n_tiles_m;
}

template <typename T>
__global__ __launch_bounds__(256) void sigma_gemm_kernel(
    const T* __restrict__ A, const T* __restrict__ B, const T* X,
    T* Y, const double* __restrict__ albedo, const double* __restrict__ xscale,
    int M, int N, int K, double sign) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc_t;
  __shared__ T As[BK][BM + PAD];
  __shared__ T Bs[BK][BN + PAD];

  const int n_tiles_m = (M + BM - 1) / BM;
  const int n_tiles_n = (N + BN - 1) / BN;
  int tm, tn;
  tile_of(blockIdx.x, n_tiles_m, n_tiles_m * n_tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // global -> register staging assignment
  const int a_m = tid >> 1, a_k = (tid & 1) * 8;     // A: 128 rows x 16 k
  const int b_k = tid >> 4, b_n = (tid & 15) * 8;    // B: 16 k x 128 cols
  T ra[8], rb[8];

  auto load_tile = [&](int k0) {
    const int gm = m0 + a_m;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int gk = k0 + a_k + j;
      ra[j] = (gm < M && gk < K) ? A[(size_t)gm * K + gk] : T(0);
    }
    const int gk = k0 + b_k;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int gn = n0 + b_n + j;
      rb[j] = (gk < K && gn < N) ? B[(size_t)gk * N + gn] : T(0);
    }
  };

  acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  load_tile(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int j = 0; j < 8; ++j) As[a_k + j][a_m] = ra[j];
#pragma unroll
    for (int j = 0; j < 8; ++j) Bs[b_k][b_n + j] = rb[j];
    __syncthreads();
    if (k0 + BK < K) load_tile(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const int c = lane & 15;
      T af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[kr][wm * 64 + i * 16 + c];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[kr][wn * 64 + j * 16 + c];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = MF::mma(af[i], bf[j], acc[i][j]);
    }
    __syncthreads();
  }

  // epilogue
  const double xs = (X != nullptr && xscale != nullptr) ? *xscale : 1.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int col = n0 + wn * 64 + j * 16 + (lane & 15);
    if (col >= N) continue;
    const double alb = sign * albedo[col];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 64 + i * 16 + MF::dr(lane, r);
        if (row < M) {
          const size_t idx = (size_t)row * N + col;
          double v = alb * (double)acc[i][j][r];
          if (X != nullptr) v += xs * (double)X[idx];
          Y[idx] = (T)v;
        }
      }
    }
  }
}

template <typename T>
void launch_sigma_t(const Problem& p, const T* mhat, const T* L, const T* x, T* y,
                    const double* xscale, double sign, hipStream_t st) {
  const int M = p.n_r, N = (int)p.n_s, K = p.n_r;
  const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  ProfScope prof(RT_KCLASS_SIGMA, st);
  hipLaunchKernelGGL((sigma_gemm_kernel<T>), dim3(tiles), dim3(256), 0, st, mhat, L, x, y,
                     p.d_albedo, xscale, M, N, K, sign);
  RT_HIP(hipGetLastError());
}

}  // namespace

void launch_sigma_f64(const Problem& p, const double* L, const double* x, double* y,
                      const double* xscale, double sign, hipStream_t st) {
  launch_sigma_t<double>(p, p.d_mhat64, L, x, y, xscale, sign, st);
}

void launch_sigma_f32(const Problem& p, const float* L, const float* x, float* y,
                      const double* xscale, double sign, hipStream_t st) {
  launch_sigma_t<float>(p, p.d_mhat32, L, x, y, xscale, sign, st);
}

}  // namespace rtsn
