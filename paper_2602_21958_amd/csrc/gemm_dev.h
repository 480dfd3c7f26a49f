// Device body of the FP64 / FP32 MFMA scattering GEMM tile, shared by the
// single-problem and the grouped (batched) kernels (see sigma_gemm.hip).
#pragma once

#include "rt_internal.h"

namespace rtsn {
namespace gemm {


typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));

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

constexpr int BM = 128, BN = 128;
constexpr int PAD = 16;   // LDS row padding (elements)
// Mhat is stored transposed, element (k, k') at k' * lda + k, with lda a
// multiple of MPAD >= n_r and KPAD-row padding (zeros) below n_r.
constexpr int MPAD = 128;
constexpr int KPAD = 32;

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

// Optional Arnoldi dot products fused into the epilogue: with the tile's
// final outputs y still in registers, partial sums of V_q . y over the tile
// are formed for q < nv and stored to part[q * ldp + slot] (one slot per
// tile; fixed summation order).
struct TileDots {
  const void* V;     // basis base (element type of the GEMM output)
  int64_t stride;    // elements between basis vectors
  int nv;            // number of basis vectors
  double* part;
  int ldp;           // slots per vector
};

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// 16-byte native vector of T
template <typename T> struct Vec16;
template <> struct Vec16<double> { using type = d2_t; static constexpr int n = 2; };
template <> struct Vec16<float> { using type = f4_t; static constexpr int n = 4; };

// Stages between a K stage's global loads and its MFMAs: FP64 loads two
// stages ahead from two register sets (one 16-stage of FP64 MFMAs does not
// cover the load latency: 4.88 -> 4.48 ms on the 32^3 box, identical
// results); FP32 keeps one stage, which leaves it at 4 waves per SIMD.
template <typename T> constexpr int kPrefetch = sizeof(T) == 8 ? 2 : 1;

// One 128 x 128 output tile at (m0, n0) computed by a 256-thread workgroup,
// K staged BK at a time.  At: Mhat transposed ([k'][k], leading dimension
// lda, zero rows up to a multiple of KPAD >= K).  xs multiplies x in the
// epilogue (ignored when X is null).  Both operand tiles arrive [k][m] /
// [k][n] with 16-byte loads of consecutive addresses and are stored to LDS
// as loaded; later K stages are loaded into registers (PD stages ahead)
// while the current one is multiplied from a double-buffered LDS ring (one
// barrier per stage).
template <typename T, int BK, bool DOTS = false, int PD = kPrefetch<T>>
__device__ __forceinline__ void gemm_tile(const T* __restrict__ At, int lda,
                                          const T* __restrict__ B, const T* X, T* Y,
                                          const double* __restrict__ albedo, double xs, int M,
                                          int N, int K, int m0, int n0, double sign,
                                          TileDots dots = {}, int slot = 0) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc_t;
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  constexpr int A_CH = BK * BM / VN / 256;   // 16-byte chunks per thread
  constexpr int B_CH = BK * BN / VN / 256;
  constexpr int A_PER_ROW = BM / VN;
  constexpr int B_PER_ROW = BN / VN;
  static_assert(A_CH >= 1 && B_CH >= 1, "tile too small");
  static_assert(KPAD % BK == 0, "K stage must divide the row padding of Mhat");
  __shared__ __align__(16) T As[2][BK][BM + PAD];
  __shared__ __align__(16) T Bs[2][BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const bool b_vec = (N % VN) == 0;
  const int Kp = (K + BK - 1) / BK * BK;

  static_assert(PD == 1 || PD == 2, "prefetch distance");
  V ra[A_CH], rb[B_CH], ra2[A_CH], rb2[B_CH];

  auto gload = [&](int k0, V (&ra)[A_CH], V (&rb)[B_CH]) {
#pragma unroll
    for (int i = 0; i < A_CH; ++i) {
      const int c = tid + 256 * i;
      const int row = c / A_PER_ROW, mc = (c % A_PER_ROW) * VN;
      ra[i] = *reinterpret_cast<const V*>(At + (size_t)(k0 + row) * lda + m0 + mc);
    }
#pragma unroll
    for (int i = 0; i < B_CH; ++i) {
      const int c = tid + 256 * i;
      const int row = c / B_PER_ROW, nc = (c % B_PER_ROW) * VN;
      const int gk = k0 + row, gn = n0 + nc;
      if (gk < K && b_vec && gn + VN - 1 < N) {
        rb[i] = *reinterpret_cast<const V*>(B + (size_t)gk * N + gn);
      } else {
        V v;
#pragma unroll
        for (int e = 0; e < VN; ++e)
          v[e] = (gk < K && gn + e < N) ? B[(size_t)gk * N + gn + e] : T(0);
        rb[i] = v;
      }
    }
  };
  auto lstore = [&](int buf, const V (&ra)[A_CH], const V (&rb)[B_CH]) {
#pragma unroll
    for (int i = 0; i < A_CH; ++i) {
      const int c = tid + 256 * i;
      *reinterpret_cast<V*>(&As[buf][c / A_PER_ROW][(c % A_PER_ROW) * VN]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < B_CH; ++i) {
      const int c = tid + 256 * i;
      *reinterpret_cast<V*>(&Bs[buf][c / B_PER_ROW][(c % B_PER_ROW) * VN]) = rb[i];
    }
  };

  acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  const int nst = Kp / BK;
  // MFMAs of one K stage from LDS buffer buf
  auto stage = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const int c = lane & 15;
      T af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[buf][kr][wm * 64 + i * 16 + c];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[buf][kr][wn * 64 + j * 16 + c];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = MF::mma(af[i], bf[j], acc[i][j]);
    }
  };

  __syncthreads();   // a persistent caller may still read LDS of its previous tile
  gload(0, ra, rb);
  if constexpr (PD == 2) gload(min(1, nst - 1) * BK, ra2, rb2);
  lstore(0, ra, rb);
  __syncthreads();
  if constexpr (PD == 1) {
    for (int s = 0; s < nst; ++s) {
      const int buf = s & 1;
      gload(min(s + 1, nst - 1) * BK, ra, rb);   // the last stage reloads itself (unused)
      __builtin_amdgcn_sched_barrier(0);         // keep the loads ahead of the MFMAs
      stage(buf);
      __builtin_amdgcn_sched_barrier(0);
      lstore(buf ^ 1, ra, rb);
      __syncthreads();
    }
  } else {
    // the two register sets in turn: during stage s the set holding stage
    // s + 1 goes to LDS while the other receives stage s + 2 (loads past the
    // last stage reload it, unused)
    int s = 0;
    for (; s + 1 < nst; s += 2) {
      gload(min(s + 2, nst - 1) * BK, ra, rb);
      __builtin_amdgcn_sched_barrier(0);
      stage(0);
      __builtin_amdgcn_sched_barrier(0);
      lstore(1, ra2, rb2);
      __syncthreads();
      gload(min(s + 3, nst - 1) * BK, ra2, rb2);
      __builtin_amdgcn_sched_barrier(0);
      stage(1);
      __builtin_amdgcn_sched_barrier(0);
      lstore(0, ra, rb);
      __syncthreads();
    }
    if (s < nst) {   // odd stage count: the last stage is in buffer 0
      stage(0);
      __syncthreads();
    }
  }

  // epilogue (the final values stay in acc for the fused dots; zero outside)
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int col = n0 + wn * 64 + j * 16 + (lane & 15);
    const double alb = col < N ? sign * albedo[col] : 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 64 + i * 16 + MF::dr(lane, r);
        if (row < M && col < N) {
          const size_t idx = (size_t)row * N + col;
          double v = alb * (double)acc[i][j][r];
          if (X != nullptr) v += xs * (double)X[idx];
          const T t = (T)v;
          Y[idx] = t;
          acc[i][j][r] = t;
        } else {
          acc[i][j][r] = 0;
        }
      }
    }
  }
  if constexpr (DOTS) {
    // LDS is free: the K loop ended with a barrier after its last reads
    double* red = reinterpret_cast<double*>(&As[0][0][0]);
    const T* V = static_cast<const T*>(dots.V);
    for (int q = 0; q < dots.nv; ++q) {
      const T* Vq = V + (size_t)q * dots.stride;
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = m0 + wm * 64 + i * 16 + MF::dr(lane, r);
            if (row < M && col < N)
              s += (double)Vq[(size_t)row * N + col] * (double)acc[i][j][r];
          }
        }
        __builtin_amdgcn_sched_barrier(0);   // bound the loads in flight
      }
      s = wave_sum_d(s);
      if (lane == 0) red[q * 4 + wave] = s;
    }
    __syncthreads();
    for (int q = tid; q < dots.nv; q += 256)
      dots.part[(size_t)q * dots.ldp + slot] =
          (red[q * 4] + red[q * 4 + 1]) + (red[q * 4 + 2] + red[q * 4 + 3]);
  }
}

}  // namespace gemm
}  // namespace rtsn
