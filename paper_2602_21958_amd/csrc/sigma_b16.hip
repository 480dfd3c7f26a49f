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

#include "rt_internal.h"

namespace rtsn {

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 64;
constexpr int LDK = BK + 8;  // LDS row length (elements): 144 B rows

template <bool IS_BF16> struct Op16;
template <> struct Op16<true> {
  static __device__ __forceinline__ uint16_t bits(float v) {
    return __bfloat16_as_ushort(__float2bfloat16(v));
  }
  static __device__ __forceinline__ float value(uint16_t b) {
    return __bfloat162float(__ushort_as_bfloat16(b));
  }
  static __device__ __forceinline__ f32x4_t mma(uint4 a, uint4 b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                   __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
  }
};
template <> struct Op16<false> {
  static __device__ __forceinline__ uint16_t bits(float v) {
    return __half_as_ushort(__float2half(v));
  }
  static __device__ __forceinline__ float value(uint16_t b) {
    return __half2float(__ushort_as_half(b));
  }
  static __device__ __forceinline__ f32x4_t mma(uint4 a, uint4 b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8_t, a),
                                                  __builtin_bit_cast(f16x8_t, b), c, 0, 0, 0);
  }
};

__device__ __forceinline__ void tile_of(int bid, int n_tiles_m, int n_tiles, int& tm, int& tn) {
  const int xcd = bid & 7;
  const int local = bid >> 3;
  const int per_xcd = (n_tiles + 7) >> 3;
  int t = xcd * per_xcd + local;
  if ((n_tiles & 7) != 0) t = bid;
  tm = t % n_tiles_m;
  tn = t / n_tiles_m;
}

__device__ __forceinline__ uint32_t pack2(uint16_t lo, uint16_t hi) {
  return (uint32_t)lo | ((uint32_t)hi << 16);
}

// IS_BF16: bf16 (true) or fp16 operands.  SPLIT: three-product split bf16.
// B is uint16_t L (not SPLIT) or float L (SPLIT).
template <bool IS_BF16, bool SPLIT>
__global__ __launch_bounds__(256) void sigma_b16_kernel(
    const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo, int lda,
    const void* __restrict__ Bv, const float* X, float* Y, const double* __restrict__ albedo,
    const float* __restrict__ rowscale, float bscale_inv, const double* __restrict__ xscale,
    int M, int N, int K, float sign) {
  using OP = Op16<IS_BF16>;
  constexpr int NA = SPLIT ? 2 : 1;
  __shared__ __align__(16) uint16_t As[NA][BM][LDK];
  __shared__ __align__(16) uint16_t Bs[NA][BN][LDK];

  const int n_tiles_m = (M + BM - 1) / BM;
  const int n_tiles_n = (N + BN - 1) / BN;
  int tm, tn;
  tile_of(blockIdx.x, n_tiles_m, n_tiles_m * n_tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // B staging: thread owns 8 k-rows x 4 points
  const int b_k = (tid >> 5) * 8;
  const int b_n = (tid & 31) * 4;
  const bool b_vec = (N % 4) == 0;

  uint4 ra[NA][4];
  uint16_t rb[NA][8][4];

  auto load_tile = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = tid + 256 * i;
      const int row = c >> 3, kc = (c & 7) * 8;
      const int gm = m0 + row, gk = k0 + kc;
      const bool ok = gm < M && gk < lda;
      const size_t off = (size_t)gm * lda + gk;
      ra[0][i] = ok ? *reinterpret_cast<const uint4*>(Ahi + off) : make_uint4(0, 0, 0, 0);
      if constexpr (SPLIT)
        ra[1][i] = ok ? *reinterpret_cast<const uint4*>(Alo + off) : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int gk = k0 + b_k + kk;
      const int gn = n0 + b_n;
      if constexpr (SPLIT) {
        const float* B = static_cast<const float*>(Bv);
        float v[4];
        if (gk < K && b_vec && gn + 3 < N) {
          const float4 q = *reinterpret_cast<const float4*>(B + (size_t)gk * N + gn);
          v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            v[j] = (gk < K && gn + j < N) ? B[(size_t)gk * N + gn + j] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint16_t h = Op16<true>::bits(v[j]);
          rb[0][kk][j] = h;
          rb[1][kk][j] = Op16<true>::bits(v[j] - Op16<true>::value(h));
        }
      } else {
        const uint16_t* B = static_cast<const uint16_t*>(Bv);
        if (gk < K && b_vec && gn + 3 < N) {
          const uint2 q = *reinterpret_cast<const uint2*>(B + (size_t)gk * N + gn);
          rb[0][kk][0] = q.x & 0xffff; rb[0][kk][1] = q.x >> 16;
          rb[0][kk][2] = q.y & 0xffff; rb[0][kk][3] = q.y >> 16;
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            rb[0][kk][j] = (gk < K && gn + j < N) ? B[(size_t)gk * N + gn + j] : (uint16_t)0;
        }
      }
    }
  };

  f32x4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  load_tile(0);
  for (int k0 = 0; k0 < lda; k0 += BK) {
#pragma unroll
    for (int s = 0; s < NA; ++s) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = tid + 256 * i;
        *reinterpret_cast<uint4*>(&As[s][c >> 3][(c & 7) * 8]) = ra[s][i];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint4 w;
        w.x = pack2(rb[s][0][j], rb[s][1][j]);
        w.y = pack2(rb[s][2][j], rb[s][3][j]);
        w.z = pack2(rb[s][4][j], rb[s][5][j]);
        w.w = pack2(rb[s][6][j], rb[s][7][j]);
        *reinterpret_cast<uint4*>(&Bs[s][b_n + j][b_k]) = w;
      }
    }
    __syncthreads();
    if (k0 + BK < lda) load_tile(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      const int kq = kk + 8 * (lane >> 4);
      const int c = lane & 15;
      uint4 af[NA][4], bf[NA][4];
#pragma unroll
      for (int s = 0; s < NA; ++s) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          af[s][i] = *reinterpret_cast<const uint4*>(&As[s][wm * 64 + i * 16 + c][kq]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          bf[s][j] = *reinterpret_cast<const uint4*>(&Bs[s][wn * 64 + j * 16 + c][kq]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j] = OP::mma(af[0][i], bf[0][j], acc[i][j]);
          if constexpr (SPLIT) {
            acc[i][j] = OP::mma(af[0][i], bf[1][j], acc[i][j]);
            acc[i][j] = OP::mma(af[1][i], bf[0][j], acc[i][j]);
          }
        }
    }
    __syncthreads();
  }

  const float xs = (X != nullptr && xscale != nullptr) ? (float)*xscale : 1.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int col = n0 + wn * 64 + j * 16 + (lane & 15);
    if (col >= N) continue;
    const float alb = sign * (float)albedo[col] * bscale_inv;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        if (row < M) {
          const size_t idx = (size_t)row * N + col;
          float v = alb * (rowscale ? rowscale[row] : 1.f) * acc[i][j][r];
          if (X != nullptr) v += xs * X[idx];
          Y[idx] = v;
        }
      }
    }
  }
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
  const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
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
