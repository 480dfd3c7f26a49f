// Device body of the 16-bit (bf16 / fp16 / split-bf16) MFMA scattering GEMM
// tile, shared by the single-problem and the grouped kernels (see
// sigma_b16.hip).
#pragma once

#include "rt_internal.h"

namespace rtsn {
namespace gemm16 {


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
// One 128 x 128 output tile at (m0, n0); xs multiplies x in the epilogue.
template <bool IS_BF16, bool SPLIT>
__device__ __forceinline__ void gemm16_tile(
    const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo, int lda,
    const void* __restrict__ Bv, const float* X, float* Y, const double* __restrict__ albedo,
    const float* __restrict__ rowscale, float bscale_inv, float xs, int M, int N, int K,
    int m0, int n0, float sign) {
  using OP = Op16<IS_BF16>;
  constexpr int NA = SPLIT ? 2 : 1;
  __shared__ __align__(16) uint16_t As[NA][BM][LDK];
  __shared__ __align__(16) uint16_t Bs[NA][BN][LDK];
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

}  // namespace gemm16
}  // namespace rtsn
