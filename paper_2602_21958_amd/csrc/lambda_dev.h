// Device bodies of the formal solver Lambda shared by the single-problem and
// the batched kernels (see lambda.hip for the method).
#pragma once

#include "rt_internal.h"

namespace rtsn {
namespace lam {


template <typename C> struct Series;
template <> struct Series<double> { static constexpr int terms = 16; };
template <> struct Series<float> { static constexpr int terms = 9; };

// 1/n! for n = 0..17
static __device__ __constant__ double kInvFactN[18] = {
    1.0, 1.0, 1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0,
    1.0 / 40320.0, 1.0 / 362880.0, 1.0 / 3628800.0, 1.0 / 39916800.0, 1.0 / 479001600.0,
    1.0 / 6227020800.0, 1.0 / 87178291200.0, 1.0 / 1307674368000.0, 1.0 / 20922789888000.0,
    1.0 / 355687428096000.0};

// Weights of one linear short-characteristics step of optical length d:
// e = e^{-d}, a = (1 - e)/d - e, c = 1 - (1 - e)/d.  One transcendental at
// most: below d = 1/2 all three come from their Taylor polynomials,
//   e = sum_n (-d)^n/n!,  c = sum_{n>=1} (-1)^{n+1} d^n/(n+1)!,
//   a = sum_{n>=1} (-1)^{n+1} n d^n/(n+1)!;
// above it e = exp(-d) and q = (1 - e)/d has no cancellation.
template <typename C>
__device__ __forceinline__ void sc_weights(C d, C& e, C& a, C& c) {
  if (d < C(0.5)) {
    constexpr int T = Series<C>::terms;
    C cs = C(0), as = C(0), es = C(0);
#pragma unroll
    for (int n = T; n >= 1; --n) {
      const C sg = (n & 1) ? C(1) : C(-1);
      const C f = C(kInvFactN[n + 1]);
      cs = cs * d + sg * f;
      as = as * d + sg * C(n) * f;
      es = es * d + (-sg) * C(kInvFactN[n]);   // coefficient of d^n in e^{-d}
    }
    c = cs * d;
    a = as * d;
    e = es * d + C(1);
  } else {
    e = exp(-d);
    const C q = (C(1) - e) / d;
    a = q - e;
    c = C(1) - q;
  }
}

template <typename T> __device__ __forceinline__ T to_out(double v);
template <> __device__ __forceinline__ double to_out<double>(double v) { return v; }
template <> __device__ __forceinline__ float to_out<float>(double v) { return (float)v; }
template <typename T> __device__ __forceinline__ T to_outf(float v);
template <> __device__ __forceinline__ float to_outf<float>(float v) { return v; }
template <> __device__ __forceinline__ double to_outf<double>(float v) { return v; }
template <> __device__ __forceinline__ __hip_bfloat16 to_outf<__hip_bfloat16>(float v) {
  return __float2bfloat16(v);
}
template <> __device__ __forceinline__ __half to_outf<__half>(float v) { return __float2half(v); }

template <typename C, typename LT>
__device__ __forceinline__ LT store_val(C v) {
  if constexpr (sizeof(C) == 8) return to_out<LT>(v);
  else return to_outf<LT>(v);
}

// Where a ray's values go.  PlainOut: element i of the ray at o[i] (the
// ray-major vector layout).  K4Out: the 16-bit B operand of the scattering
// GEMM, element i of ray k at base[((k / 4) * Np + i) * 4 + k % 4]; the
// pointers are already offset to the ray, so element i is at [4 i].
template <typename LT>
struct PlainOut {
  LT* o;
  template <typename C>
  __device__ __forceinline__ void put(size_t i, C v) const { o[i] = store_val<C, LT>(v); }
};

enum { K4_BF16 = 0, K4_FP16 = 1, K4_SPLIT = 2 };

__device__ __forceinline__ uint16_t bf16_rne(float v) {
  return __bfloat16_as_ushort(__float2bfloat16(v));
}

template <int MODE>
struct K4Out {
  uint16_t* hi;
  uint16_t* lo;   // SPLIT only: v - bf16(v), rounded to bf16
  template <typename C>
  __device__ __forceinline__ void put(size_t i, C cv) const {
    const float v = (float)cv;
    if constexpr (MODE == K4_FP16) {
      hi[4 * i] = __half_as_ushort(__float2half(v));
    } else {
      const uint16_t h = bf16_rne(v);
      hi[4 * i] = h;
      if constexpr (MODE == K4_SPLIT)
        lo[4 * i] = bf16_rne(v - __bfloat162float(__ushort_as_bfloat16(h)));
    }
  }
};

// 16-bit operand of ray k inside a k4 buffer (Np points per k4 group).
template <int MODE>
__device__ __forceinline__ K4Out<MODE> k4_ray(uint16_t* hi, uint16_t* lo, int k, int64_t Np) {
  const size_t off = ((size_t)(k >> 2) * Np) * 4 + (k & 3);
  return K4Out<MODE>{hi + off, lo ? lo + off : nullptr};
}

// ---------------------------------------------------------------------------
// One slab ray, swept by one 64-lane wavefront (all lanes of the wave call
// this together).  sk: the ray's nz source values; out: where its nz output
// values go.
template <typename VT, typename OUT, typename C>
__device__ __forceinline__ void slab_ray(const VT* __restrict__ sk, const OUT out,
                                         const double* __restrict__ dt, double mu, double fac,
                                         int nz, C i_in, C sc, int scheme, float out_mul,
                                         int lane) {
  const double g = fac / fabs(mu);
  const bool down = mu < 0.0;
  const int L = (nz + 63) >> 6;
  const int q0 = lane * L;

  // affine map of sweep position q: I_q = e I_{q-1} + b
  auto elem = [&](int q, C& e, C& b) {
    if (q == 0) { e = C(0); b = i_in; return; }
    const int m = down ? q : nz - 1 - q;      // memory index of this node
    const int mp = down ? q - 1 : nz - q;     // memory index of the upwind node
    const int iv = down ? q - 1 : m;          // interval index
    const C d = C(dt[iv] * g);
    const C s0 = sc * C(sk[m]);
    if (scheme == RT_FORMAL_IMPLICIT_EULER) {
      const C inv = C(1) / (C(1) + d);
      e = inv;
      b = d * s0 * inv;
    } else {
      C a, c;
      sc_weights<C>(d, e, a, c);
      b = a * (sc * C(sk[mp])) + c * s0;
    }
  };

  C A = C(1), B = C(0);
  for (int j = 0; j < L; ++j) {
    const int q = q0 + j;
    if (q >= nz) break;
    C e, b;
    elem(q, e, b);
    B = e * B + b;
    A = e * A;
  }
  // inclusive scan of the composites (later o earlier)
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const C Ap = __shfl_up(A, off, 64);
    const C Bp = __shfl_up(B, off, 64);
    if (lane >= off) {
      B = A * Bp + B;
      A = A * Ap;
    }
  }
  C I = __shfl_up(B, 1, 64);  // intensity just before this lane's chunk
  if (lane == 0) I = C(0);
  for (int j = 0; j < L; ++j) {
    const int q = q0 + j;
    if (q >= nz) break;
    C e, b;
    elem(q, e, b);
    I = e * I + b;
    out.put(down ? q : nz - 1 - q, I * C(out_mul));
  }
}

// ---------------------------------------------------------------------------
// One box ray (ordinate stencil st, frequency factor fac), swept plane by
// plane by a whole 256-thread workgroup; smem holds 3 P values of type C.
// sk: the ray's nz*P source values; out: where its nz*P output values go.
constexpr int kBoxThreads = 256;

template <typename VT, typename OUT, typename C, int kBoxMaxPts, int NT = kBoxThreads>
__device__ __forceinline__ void box_ray(const VT* __restrict__ sk, const OUT out,
                                        const double* __restrict__ kline, const BoxStencil st,
                                        C fac, int nx, int ny, int nz, C i_in, C sc,
                                        float out_mul, C* smem) {
  const int P = nx * ny;
  C* lI = smem;
  C* lS = lI + P;
  C* lK = lS + P;
  const C path = C(st.path);
  const C tx = C(st.tx), ty = C(st.ty);
  const size_t plane_stride = (size_t)P;

  const int npt = (P + NT - 1) / NT;
  C Iv[kBoxMaxPts], Sv[kBoxMaxPts], Kv[kBoxMaxPts];
  // upwind bilinear source offsets per owned point (fixed for the ordinate)
  int n00[kBoxMaxPts], n01[kBoxMaxPts], n10[kBoxMaxPts], n11[kBoxMaxPts];
#pragma unroll
  for (int j = 0; j < kBoxMaxPts; ++j) {
    if (j >= npt) break;
    const int p = threadIdx.x + j * NT;
    if (p < P) {
      const int x = p % nx, y = p / nx;
      int xa = x + st.i0; if (xa >= nx) xa -= nx;
      int xb = xa + 1;    if (xb >= nx) xb -= nx;
      int ya = y + st.j0; if (ya >= ny) ya -= ny;
      int yb = ya + 1;    if (yb >= ny) yb -= ny;
      n00[j] = ya * nx + xa;
      n01[j] = ya * nx + xb;
      n10[j] = yb * nx + xa;
      n11[j] = yb * nx + xb;
    } else {
      n00[j] = n01[j] = n10[j] = n11[j] = 0;
    }
  }
  const C w00 = (C(1) - ty) * (C(1) - tx), w01 = (C(1) - ty) * tx;
  const C w10 = ty * (C(1) - tx), w11 = ty * tx;

  // source and opacity of the next plane are loaded one plane ahead
  C Sn[kBoxMaxPts], Kn[kBoxMaxPts];
  auto load_plane = [&](int t) {
    const int z = st.up ? t : nz - 1 - t;
    const VT* sz = sk + (size_t)z * plane_stride;
    const double* kz = kline + (size_t)z * plane_stride;
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      if (j >= npt) break;
      const int p = threadIdx.x + j * NT;
      if (p < P) {
        Sn[j] = sc * C(sz[p]);
        Kn[j] = C(kz[p]);
      }
    }
  };
  load_plane(0);
  for (int t = 0; t < nz; ++t) {
    const int z = st.up ? t : nz - 1 - t;
    const size_t oz = (size_t)z * plane_stride;
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      if (j >= npt) break;
      Sv[j] = Sn[j];
      Kv[j] = Kn[j];
    }
    if (t + 1 < nz) load_plane(t + 1);
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      if (j >= npt) break;
      const int p = threadIdx.x + j * NT;
      if (p >= P) break;
      const C s0 = Sv[j];
      const C k0 = Kv[j];
      C I;
      if (t == 0) {
        I = i_in;
      } else {
        const C ku = w00 * lK[n00[j]] + w01 * lK[n01[j]] + w10 * lK[n10[j]] + w11 * lK[n11[j]];
        const C Iu = w00 * lI[n00[j]] + w01 * lI[n01[j]] + w10 * lI[n10[j]] + w11 * lI[n11[j]];
        const C Su = w00 * lS[n00[j]] + w01 * lS[n01[j]] + w10 * lS[n10[j]] + w11 * lS[n11[j]];
        const C d = C(0.5) * (ku + k0) * path * fac;
        C e, a, c;
        sc_weights<C>(d, e, a, c);
        I = e * Iu + a * Su + c * s0;
      }
      out.put(oz + p, I * C(out_mul));
      Iv[j] = I;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      if (j >= npt) break;
      const int p = threadIdx.x + j * NT;
      if (p >= P) break;
      lI[p] = Iv[j];
      lS[p] = Sv[j];
      lK[p] = Kv[j];
    }
    __syncthreads();
  }
}

}  // namespace lam
}  // namespace rtsn
