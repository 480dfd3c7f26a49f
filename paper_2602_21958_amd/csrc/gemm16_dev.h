// Device body of the 16-bit (bf16 / fp16 / split-bf16) MFMA scattering GEMM
// tile, shared by the single-problem kernels (sigma_b16.hip) and the grouped
// kernel of the batch engine (batch.hip).
//
//   Y[m, n] = ymul (xs X[m, n] + sign * albedo[n] * rowfac[m] * sum_k A[m, k] B[k, n])
//
// Operand layouts (16-bit values, zero padded):
//   A (Mhat)      "k8": element (m, k) at ((k / 8) * Mp + m) * 8 + k % 8, k < Kp
//   B (Lambda's   "k4": element (k, n) at ((k / 4) * Np + n) * 4 + k % 4
//      output)
// with Mp, Np multiples of 256 and Kp a multiple of 64.  A 16-byte chunk of A
// is 8 consecutive k of one row, the operand of one MFMA lane; a 16-byte
// chunk of B holds 4 consecutive k of two neighbouring points, and the two
// k4 groups a lane needs are staged one LDS block apart so that one
// ds_read2_b64 fetches them.  Global memory is read in 16-byte chunks, 64
// lanes on 1 KB of contiguous memory, into registers one K stage ahead, then
// stored into a double-buffered LDS ring (one barrier per stage).
//
// MFMA: v_mfma_f32_16x16x32 (F32 = false) or v_mfma_f32_32x32x16 (F32 =
// true) on bf16 or fp16.  A lane's 8 operand values are 8 consecutive k for
// both A and B, so the k order inside an instruction is the natural one.
//
// MODE_I8 (exact integer products for the error-free split of an FP64
// GEMM): the same layouts and tile with each 16-bit element holding two
// consecutive int8 values (k even in the low byte), on
// v_mfma_i32_16x16x64_i8 / v_mfma_i32_32x32x32_i8, whose lane operands are
// the same 16 bytes (16 consecutive k); accumulation in int32 is exact while
// K * 128^2 < 2^31.  The epilogue writes acc mod imod in [0, imod) as bytes.
#pragma once

#include <type_traits>

#include "gemm_dev.h"
#include "rt_internal.h"

namespace rtsn {
namespace g16 {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

enum { MODE_BF16 = 0, MODE_FP16 = 1, MODE_SPLIT = 2, MODE_I8 = 3 };
typedef int i32x4_t __attribute__((ext_vector_type(4)));
typedef int i32x16_t __attribute__((ext_vector_type(16)));

constexpr int kMAlign = 256;   // Mp, Np multiple of this
constexpr int kKAlign = 64;    // Kp multiple of this

__host__ __device__ constexpr int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

template <bool IS_BF16, bool BIG> struct Mma;
template <> struct Mma<true, false> {
  using acc_t = f32x4_t;
  static __device__ __forceinline__ acc_t run(u32x4_t a, u32x4_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                   __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
  }
};
template <> struct Mma<false, false> {
  using acc_t = f32x4_t;
  static __device__ __forceinline__ acc_t run(u32x4_t a, u32x4_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8_t, a),
                                                  __builtin_bit_cast(f16x8_t, b), c, 0, 0, 0);
  }
};
template <> struct Mma<true, true> {
  using acc_t = f32x16_t;
  static __device__ __forceinline__ acc_t run(u32x4_t a, u32x4_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                   __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
  }
};
template <> struct Mma<false, true> {
  using acc_t = f32x16_t;
  static __device__ __forceinline__ acc_t run(u32x4_t a, u32x4_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, a),
                                                  __builtin_bit_cast(f16x8_t, b), c, 0, 0, 0);
  }
};

template <bool BIG> struct MmaI8;
template <> struct MmaI8<false> {
  using acc_t = i32x4_t;
  static __device__ __forceinline__ acc_t run(u32x4_t a, u32x4_t b, acc_t c) {
    return __builtin_amdgcn_mfma_i32_16x16x64_i8(__builtin_bit_cast(i32x4_t, a),
                                                 __builtin_bit_cast(i32x4_t, b), c, 0, 0, 0);
  }
};
template <> struct MmaI8<true> {
  using acc_t = i32x16_t;
  static __device__ __forceinline__ acc_t run(u32x4_t a, u32x4_t b, acc_t c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(i32x4_t, a),
                                                 __builtin_bit_cast(i32x4_t, b), c, 0, 0, 0);
  }
};

// Tile configuration: BM x BN output tile, WGM x WGN waves, K stage BK,
// BIG = 32x32x16 instructions (else 16x16x32), PP = ping-pong schedule
// (tile_pp; eight waves in two groups).
template <int BM_, int BN_, int WGM_, int WGN_, int BK_, bool BIG_, bool PP_ = false>
struct Cfg {
  static constexpr int BM = BM_, BN = BN_, WGM = WGM_, WGN = WGN_, BK = BK_;
  static constexpr bool BIG = BIG_, PP = PP_;
  static constexpr int NW = WGM * WGN, NT = 64 * NW;
  static constexpr int WM = BM / WGM, WN = BN / WGN;
  static constexpr int MI = BIG ? 32 : 16;           // instruction tile
  static constexpr int TI = WM / MI, TJ = WN / MI;
  static constexpr int HB = BN / 128;                // 128-point halves of a B stage block row
  static constexpr int RB = BM / 64;                 // 64-row blocks of an A stage
  static constexpr int BLKA = 1024;
  static constexpr int BLKB = 1024 + 64 / HB;        // padding spreads the two k4 reads over all banks
  static constexpr int A_BLK = (BK / 8) * RB;        // 1 KB blocks per stage and operand part
  static constexpr int B_BLK = (BK / 4) * HB;
  static constexpr int ASB = A_BLK * BLKA, BSB = B_BLK * BLKB;
  static constexpr int AU = A_BLK / NW, BU = B_BLK / NW;
  static_assert(A_BLK % NW == 0 && B_BLK % NW == 0, "stage loads must split evenly over waves");
  static_assert(TI >= 1 && TJ >= 1 && BM % 64 == 0 && BN % 128 == 0 && BK % 32 == 0, "shape");
  template <int MODE> static constexpr int lds_bytes() {
    return 2 * (MODE == MODE_SPLIT ? 2 : 1) * (ASB + BSB);
  }
};

// Global loads of one K stage (k4 groups kg4 .. kg4 + BK/4 - 1) into
// registers: wave w loads the 1 KB blocks w, w + NW, ... of A and of B.
template <typename C, int NP>
__device__ __forceinline__ void stage_gload(u32x4_t (&ra)[NP][C::AU], u32x4_t (&rb)[NP][C::BU],
                                            const uint16_t* const (&Ap)[2],
                                            const uint16_t* const (&Bp)[2], int Mp, int Np,
                                            int m0, int n0, int kg4, int wave, int lane) {
  const int kg8 = kg4 >> 1;
#pragma unroll
  for (int s = 0; s < NP; ++s) {
#pragma unroll
    for (int u = 0; u < C::AU; ++u) {
      const int b = wave + C::NW * u;
      const int g8 = b / C::RB, rbk = b % C::RB;
      ra[s][u] = *reinterpret_cast<const u32x4_t*>(
          Ap[s] + ((size_t)(kg8 + g8) * Mp + m0 + rbk * 64 + lane) * 8);
    }
#pragma unroll
    for (int u = 0; u < C::BU; ++u) {
      const int b = wave + C::NW * u;
      const int g4 = b / C::HB, hb = b % C::HB;
      rb[s][u] = *reinterpret_cast<const u32x4_t*>(
          Bp[s] + ((size_t)(kg4 + g4) * Np + n0 + hb * 128 + 2 * lane) * 4);
    }
  }
}

// The same blocks stored into one LDS stage buffer (parts hi, lo one after
// the other); the two k4 groups of a B block row sit one LDS block apart.
template <typename C, int NP>
__device__ __forceinline__ void stage_lstore(const u32x4_t (&ra)[NP][C::AU],
                                             const u32x4_t (&rb)[NP][C::BU], uint8_t* st_lds,
                                             int wave, int lane) {
#pragma unroll
  for (int s = 0; s < NP; ++s) {
    uint8_t* As = st_lds + s * (C::ASB + C::BSB);
    uint8_t* Bs = As + C::ASB;
#pragma unroll
    for (int u = 0; u < C::AU; ++u) {
      const int b = wave + C::NW * u;
      *reinterpret_cast<u32x4_t*>(As + b * C::BLKA + 16 * lane) = ra[s][u];
    }
#pragma unroll
    for (int u = 0; u < C::BU; ++u) {
      const int b = wave + C::NW * u;
      const int g4 = b / C::HB, hb = b % C::HB;
      *reinterpret_cast<u32x4_t*>(
          Bs + ((g4 >> 1) * 2 * C::HB + hb * 2 + (g4 & 1)) * C::BLKB + 16 * lane) = rb[s][u];
    }
  }
}

// Operand fragments of instruction step h of a stage for wave (wm, wn):
// lane roles 16x16x32 -> 4 groups of 16 lanes (k8 chunk kgrp, row/col rc);
// 32x32x16 -> 2 groups of 32 lanes.
template <typename C, int NP>
__device__ __forceinline__ void stage_frags(const uint8_t* st_lds, int h, int kgrp, int rc, int wm,
                                            int wn, u32x4_t (&bf)[NP][C::TJ],
                                            u32x4_t (&af)[NP][C::TI]) {
  constexpr int KCH = (C::BIG ? 16 : 32) / 8;    // k8 chunks per instruction
  const int c8 = KCH * h + kgrp;                 // k8 chunk of this lane within the stage
#pragma unroll
  for (int s = 0; s < NP; ++s) {
    const uint8_t* As = st_lds + s * (C::ASB + C::BSB);
    const uint8_t* Bs = As + C::ASB;
#pragma unroll
    for (int j = 0; j < C::TJ; ++j) {
      const int n = wn * C::WN + C::MI * j + rc;
      const uint8_t* p0 = Bs + (c8 * 2 * C::HB + (n >> 7) * 2) * C::BLKB + (n & 127) * 8;
      const uint2 lo = *reinterpret_cast<const uint2*>(p0);
      const uint2 hi = *reinterpret_cast<const uint2*>(p0 + C::BLKB);
      bf[s][j] = u32x4_t{lo.x, lo.y, hi.x, hi.y};
    }
#pragma unroll
    for (int i = 0; i < C::TI; ++i) {
      const int m = wm * C::WM + C::MI * i + rc;
      af[s][i] = *reinterpret_cast<const u32x4_t*>(As + (c8 * C::RB + (m >> 6)) * C::BLKA +
                                                  (m & 63) * 16);
    }
  }
}

// Epilogue of one wave's WM x WN part of an output tile.  Float modes:
// Y = ymul (xs X + sign albedo[col] colmul rowscale[row] acc), with the stored
// values left in acc (zero outside M x N) for fused dots.  MODE_I8: the exact
// integer products reduced to [0, imod), stored as bytes.
template <int MODE, typename C, typename TY, typename ACC>
__device__ __forceinline__ void write_tile(ACC (&acc)[C::TI][C::TJ], int lane, int wm, int wn,
                                           const TY* X, TY* Y,
                                           const double* __restrict__ albedo,
                                           const float* __restrict__ rowscale, float colmul,
                                           float xs, float sign, int M, int N, int m0, int n0,
                                           float ymul, int imod) {
  constexpr int NR = C::BIG ? 16 : 4;
  const int kgrp = C::BIG ? (lane >> 5) : (lane >> 4);
  const int rc = C::BIG ? (lane & 31) : (lane & 15);
#pragma unroll
  for (int j = 0; j < C::TJ; ++j) {
    const int col = n0 + wn * C::WN + C::MI * j + rc;
    float cf = 0.f;
    if constexpr (MODE != MODE_I8) cf = col < N ? sign * (float)albedo[col] * colmul : 0.f;
#pragma unroll
    for (int i = 0; i < C::TI; ++i) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int row = m0 + wm * C::WM + C::MI * i +
                        (C::BIG ? 8 * (r >> 2) + 4 * kgrp + (r & 3) : 4 * kgrp + r);
        if constexpr (MODE == MODE_I8) {
          if (row < M && col < N) {
            int v = acc[i][j][r] % imod;
            v += v < 0 ? imod : 0;
            Y[(size_t)row * N + col] = (TY)v;
          }
        } else {
          if (row < M && col < N) {
            const size_t idx = (size_t)row * N + col;
            float v = cf * (rowscale ? rowscale[row] : 1.f) * acc[i][j][r];
            if (X != nullptr) v += xs * (float)X[idx];
            const TY t = (TY)(ymul * v);
            Y[idx] = t;
            acc[i][j][r] = (float)t;
          } else {
            acc[i][j][r] = 0.f;
          }
        }
      }
    }
  }
}

// One output tile at (m0, n0).  lds: Cfg::lds_bytes<MODE>() bytes, 16-byte
// aligned.  Caller guarantees m0 + BM <= Mp, n0 + BN <= Np, K4p % (BK/4) == 0.
// The function starts with a barrier, so a persistent caller may reuse lds.
// TY: element type of X and Y (float, or _Float16 for a scaled fp16 Krylov
// basis); ymul multiplies the whole output (the basis scale; 1 otherwise).
template <int MODE, typename C, bool DOTS = false, typename TY = float>
__device__ __forceinline__ void tile(const uint16_t* __restrict__ Ahi,
                                     const uint16_t* __restrict__ Alo, int Mp,
                                     const uint16_t* __restrict__ Bhi,
                                     const uint16_t* __restrict__ Blo, int Np, int K4p,
                                     const TY* X, TY* Y, const double* __restrict__ albedo,
                                     const float* __restrict__ rowscale, float colmul, float xs,
                                     float sign, int M, int N, int m0, int n0, uint8_t* lds,
                                     gemm::TileDots dots = {}, int slot = 0, float ymul = 1.f,
                                     int imod = 0) {
  static_assert(!DOTS || sizeof(TY) == 4, "fused dots need an FP32 output");
  constexpr bool SPLIT = MODE == MODE_SPLIT;
  constexpr int NP = SPLIT ? 2 : 1;   // operand parts (hi, lo)
  using MM = typename std::conditional<MODE == MODE_I8, MmaI8<C::BIG>,
                                       Mma<MODE != MODE_FP16, C::BIG>>::type;
  using acc_t = typename MM::acc_t;
  constexpr int NR = C::BIG ? 16 : 4;
  constexpr int STAGE = NP * (C::ASB + C::BSB);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / C::WGN, wn = wave % C::WGN;

  u32x4_t ra[NP][C::AU], rb[NP][C::BU];
  const uint16_t* const Ap[2] = {Ahi, Alo};
  const uint16_t* const Bp[2] = {Bhi, Blo};
  auto gload = [&](int kg4) {
    stage_gload<C, NP>(ra, rb, Ap, Bp, Mp, Np, m0, n0, kg4, wave, lane);
  };
  auto lstore = [&](int buf) { stage_lstore<C, NP>(ra, rb, lds + buf * STAGE, wave, lane); };

  acc_t acc[C::TI][C::TJ];
#pragma unroll
  for (int i = 0; i < C::TI; ++i)
#pragma unroll
    for (int j = 0; j < C::TJ; ++j)
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[i][j][r] = 0;

  const int kgrp = C::BIG ? (lane >> 5) : (lane >> 4);
  const int rc = C::BIG ? (lane & 31) : (lane & 15);
  constexpr int KSTEP = C::BIG ? 16 : 32;      // k per instruction

  const int nst = K4p / (C::BK / 4);
  __syncthreads();   // lds may still be read by a previous tile of this workgroup
  gload(0);
  lstore(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    gload(min(st + 1, nst - 1) * (C::BK / 4));   // the last stage reloads itself (unused)
    __builtin_amdgcn_sched_barrier(0);           // keep the loads ahead of the MFMAs
    // fragments of instruction step h, read one step ahead into two
    // alternating register sets, so that the MFMAs of step h run while the
    // LDS reads of step h + 1 are in flight
    constexpr int H = C::BK / KSTEP;
    u32x4_t bfr[2][NP][C::TJ], afr[2][NP][C::TI];
    auto read_frags = [&](int h, u32x4_t (&bf)[NP][C::TJ], u32x4_t (&af)[NP][C::TI]) {
      stage_frags<C, NP>(lds + buf * STAGE, h, kgrp, rc, wm, wn, bf, af);
    };
    read_frags(0, bfr[0], afr[0]);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      if (h + 1 < H) read_frags(h + 1, bfr[(h + 1) & 1], afr[(h + 1) & 1]);
      const auto& bf = bfr[h & 1];
      const auto& af = afr[h & 1];
#pragma unroll
      for (int i = 0; i < C::TI; ++i) {
#pragma unroll
        for (int j = 0; j < C::TJ; ++j) {
          acc[i][j] = MM::run(af[0][i], bf[0][j], acc[i][j]);
          if constexpr (SPLIT) {
            acc[i][j] = MM::run(af[0][i], bf[1][j], acc[i][j]);
            acc[i][j] = MM::run(af[1][i], bf[0][j], acc[i][j]);
          }
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    lstore(buf ^ 1);
    __syncthreads();
  }

  write_tile<MODE, C, TY>(acc, lane, wm, wn, X, Y, albedo, rowscale, colmul, xs, sign, M, N, m0,
                          n0, ymul, imod);
  if constexpr (MODE != MODE_I8) {
  if constexpr (DOTS) {
    // LDS is free: the K loop ended with a barrier after its last reads
    double* red = reinterpret_cast<double*>(lds);
    const float* V = static_cast<const float*>(dots.V);
    for (int q = 0; q < dots.nv; ++q) {
      const float* Vq = V + (size_t)q * dots.stride;
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < C::TJ; ++j) {
        const int col = n0 + wn * C::WN + C::MI * j + rc;
#pragma unroll
        for (int i = 0; i < C::TI; ++i) {
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const int row = m0 + wm * C::WM + C::MI * i +
                            (C::BIG ? 8 * (r >> 2) + 4 * kgrp + (r & 3) : 4 * kgrp + r);
            if (row < M && col < N)
              s += (double)Vq[(size_t)row * N + col] * (double)acc[i][j][r];
          }
        }
        __builtin_amdgcn_sched_barrier(0);   // bound the loads in flight
      }
      s = gemm::wave_sum_d(s);
      if (lane == 0) red[q * C::NW + wave] = s;
    }
    __syncthreads();
    for (int q = tid; q < dots.nv; q += C::NT) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < C::NW; ++w) t += red[q * C::NW + w];
      dots.part[(size_t)q * dots.ldp + slot] = t;
    }
  }
  }
}

// Workgroup barrier that orders LDS accesses only: global loads issued
// before it stay in flight.  The scheduling fences keep every instruction on
// its side of the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  __builtin_amdgcn_sched_barrier(0);
}

// The tile of `tile` (same operands, layouts, epilogue and k order per
// output) with a ping-pong schedule for eight waves, two per SIMD.  Waves
// 0-3 (rows 0 .. BM/2 - 1) and 4-7 (the other half) form two groups that
// run the same K loop one phase apart, every phase ended by a workgroup
// barrier, so that on each SIMD one wave issues only matrix instructions on
// fragments already in its registers while the other moves data:
//   M(s): read all fragments of stage s from LDS buffer s & 1; store the
//         registers loaded in M(s - 2) (this wave's share of stage s + 1)
//         into buffer (s + 1) & 1; load its share of stage s + 3 from global
//         memory into those registers;
//   C(s): the MFMAs of stage s, at raised wave priority.
// Group 0 runs M(s) in phase 2s and C(s) in phase 2s + 1, group 1 one phase
// later.  Stage s + 1 is written in phases 2s and 2s + 1 (half by each
// group) and first read in phase 2s + 2; buffer s & 1 is read in phases 2s
// and 2s + 1 and rewritten from phase 2s + 2 on.  Not for the split mode or
// fused dots.
template <int MODE, typename C, typename TY = float>
__device__ __forceinline__ void tile_pp(const uint16_t* __restrict__ A, int Mp,
                                        const uint16_t* __restrict__ B, int Np, int K4p,
                                        const TY* X, TY* Y, const double* __restrict__ albedo,
                                        const float* __restrict__ rowscale, float colmul,
                                        float xs, float sign, int M, int N, int m0, int n0,
                                        uint8_t* lds, float ymul = 1.f, int imod = 0) {
  static_assert(C::PP && C::NW == 8 && C::WGM == 2 && MODE != MODE_SPLIT,
                "ping-pong: two groups of four waves, one per row half");
  using MM = typename std::conditional<MODE == MODE_I8, MmaI8<C::BIG>,
                                       Mma<MODE != MODE_FP16, C::BIG>>::type;
  using acc_t = typename MM::acc_t;
  constexpr int NR = C::BIG ? 16 : 4;
  constexpr int STAGE = C::ASB + C::BSB;
  constexpr int KSTEP = C::BIG ? 16 : 32;
  constexpr int H = C::BK / KSTEP;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave / C::WGN, wn = wave % C::WGN;
  const int grp = wm;
  const int kgrp = C::BIG ? (lane >> 5) : (lane >> 4);
  const int rc = C::BIG ? (lane & 31) : (lane & 15);
  const uint16_t* const Ap[2] = {A, nullptr};
  const uint16_t* const Bp[2] = {B, nullptr};

  // two register sets for the global loads: the set stored in M(s) holds
  // stage s + 1 and is reloaded with stage s + 3, so loads have two phase
  // pairs to arrive
  u32x4_t ra[2][1][C::AU], rb[2][1][C::BU];
  u32x4_t af[H][1][C::TI], bf[H][1][C::TJ];
  acc_t acc[C::TI][C::TJ];
#pragma unroll
  for (int i = 0; i < C::TI; ++i)
#pragma unroll
    for (int j = 0; j < C::TJ; ++j)
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[i][j][r] = 0;

  const int nst = K4p / (C::BK / 4);
  constexpr int KG = C::BK / 4;
  lds_barrier();   // lds may still be read by a previous tile of this workgroup
  stage_gload<C, 1>(ra[0], rb[0], Ap, Bp, Mp, Np, m0, n0, 0, wave, lane);
  stage_lstore<C, 1>(ra[0], rb[0], lds, wave, lane);
  if (nst > 1) stage_gload<C, 1>(ra[0], rb[0], Ap, Bp, Mp, Np, m0, n0, KG, wave, lane);
  if (nst > 2) stage_gload<C, 1>(ra[1], rb[1], Ap, Bp, Mp, Np, m0, n0, 2 * KG, wave, lane);
  lds_barrier();
  if (grp == 1) lds_barrier();
  auto stage = [&](int s, u32x4_t (&rA)[1][C::AU], u32x4_t (&rB)[1][C::BU]) {
    const uint8_t* cur = lds + (s & 1) * STAGE;
#pragma unroll
    for (int h = 0; h < H; ++h) stage_frags<C, 1>(cur, h, kgrp, rc, wm, wn, bf[h], af[h]);
    if (s + 1 < nst) stage_lstore<C, 1>(rA, rB, lds + ((s + 1) & 1) * STAGE, wave, lane);
    if (s + 3 < nst) stage_gload<C, 1>(rA, rB, Ap, Bp, Mp, Np, m0, n0, (s + 3) * KG, wave, lane);
    lds_barrier();
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int i = 0; i < C::TI; ++i)
#pragma unroll
        for (int j = 0; j < C::TJ; ++j) acc[i][j] = MM::run(af[h][0][i], bf[h][0][j], acc[i][j]);
    __builtin_amdgcn_s_setprio(0);
    lds_barrier();
  };
  for (int s = 0; s < nst; s += 2) {
    stage(s, ra[0], rb[0]);
    if (s + 1 < nst) stage(s + 1, ra[1], rb[1]);
  }
  if (grp == 0) lds_barrier();
  write_tile<MODE, C, TY>(acc, lane, wm, wn, X, Y, albedo, rowscale, colmul, xs, sign, M, N, m0,
                          n0, ymul, imod);
}

// Workgroups are dealt to the 8 XCDs round-robin: give each XCD a contiguous
// range of tiles, ordered GM row tiles at a time so that the tiles in flight
// on one XCD share operand rows and columns in its L2.  Returns false for the
// few padding workgroups of a grid of 8 * ceil(T / 8).
__device__ __forceinline__ bool tile_of(int bid, int Mt, int Nt, int GM, int& tm, int& tn) {
  const int T = Mt * Nt;
  const int per = (T + 7) >> 3;
  const int t = (bid & 7) * per + (bid >> 3);
  if (t >= T) return false;
  const int gsz = GM * Nt;
  const int grp = t / gsz, in = t % gsz;
  const int gm0 = grp * GM;
  const int gmw = min(GM, Mt - gm0);
  tm = gm0 + in % gmw;
  tn = in / gmw;
  return true;
}

}  // namespace g16
}  // namespace rtsn
