// Device bodies of the formal solver Lambda shared by the single-problem and
// the batched kernels (see lambda.hip for the method).
#pragma once

#include "rt_internal.h"

namespace rtsn {
namespace lam {


// Terms of the series for phi_2(d) = sum_{m>=0} (-d)^m / (m+2)! below d = 1/2:
// the first omitted term is below the type's unit roundoff relative to
// phi_2 >= 0.42 there.
template <typename C> struct Series;
template <> struct Series<double> { static constexpr int terms = 14; };
template <> struct Series<float> { static constexpr int terms = 8; };

// 1/n! for n = 0..17
static __device__ __constant__ double kInvFactN[18] = {
    1.0, 1.0, 1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0,
    1.0 / 40320.0, 1.0 / 362880.0, 1.0 / 3628800.0, 1.0 / 39916800.0, 1.0 / 479001600.0,
    1.0 / 6227020800.0, 1.0 / 87178291200.0, 1.0 / 1307674368000.0, 1.0 / 20922789888000.0,
    1.0 / 355687428096000.0};

// e^{-d} in FP64 for d >= 0: Cody-Waite range reduction and a Taylor
// series.  d = n ln2 + r with n = rint(d / ln2) and |r| <= ln2 / 2, ln2
// split into a head whose low 12 significand bits are zero (n head is exact
// for n < 2^12) and a tail; e^{-r} = sum_{k=0}^{13} (-r)^k / k!, whose first
// omitted term is below 5e-18 of the sum; the result is scaled by 2^-n.  d is
// clamped at 800, past which e^{-d} is 0 in FP64 anyway.  The coefficients
// come from kInvFactN (scalar registers), so each Horner step is one FMA.
__device__ __forceinline__ double exp_neg_f64(double d) {
  constexpr double kInvLn2 = 0x1.71547652b82fep+0;
  constexpr double kLn2Hi = 0x1.62e42fefa3000p-1;
  constexpr double kLn2Lo = 0x1.3de6af278ece6p-42;
  const double dc = fmin(d, 800.0);
  const double mn = rint(dc * -kInvLn2);   // -n (rint is odd: same n)
  double r = fma(mn, kLn2Hi, dc);
  r = fma(mn, kLn2Lo, r);
  double p = kInvFactN[13];
#pragma unroll
  for (int k = 12; k >= 0; --k) p = fma(p, -r, kInvFactN[k]);
  return ldexp(p, (int)mn);
}

// num / d in FP64 for d >= 1/2 and |num| <= 1 (no operand near the exponent
// limits, so no scaling): the hardware reciprocal refined by two Newton
// steps, then one residual correction of the quotient (within 1 ulp).
__device__ __forceinline__ double div_f64_normal(double num, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  const double q = num * r;
  return fma(fma(-d, q, num), r, q);
}

// Weights of one linear short-characteristics step of optical length d:
// e = e^{-d}, a = (1 - e)/d - e, c = 1 - (1 - e)/d.  With q = (1 - e)/d the
// three follow from c alone: q = 1 - c, e = 1 - d q = 1 - d + d c and
// a = q - e = d - (1 + d) c, none of which cancels for d <= 1/2, where
// c = d phi_2(d) comes from its series (one Horner chain).  Above 1/2,
// e = exp(-d) and q = (1 - e)/d have no cancellation (FP64: exp_neg_f64 and
// div_f64_normal).  FP32 uses the hardware exponential and reciprocal (about
// 1 ulp each).
//
// BR: keep the two ranges as a branch that a wavefront whose lanes all fall
// on one side skips the other side of (an empty volatile asm statement on
// each side stops the compiler from evaluating both and selecting).  In a
// box sweep the 64 points of a wavefront lie in one plane of one ray, with
// nearly equal optical steps, so most wavefronts run one side (32^3 box:
// FP64 0.299 -> 0.247 ms, FP32 0.141 -> 0.130 ms).  Slab rays put the whole
// depth range in one wavefront and evaluate both sides and select.
template <typename C, bool BR = false>
__device__ __forceinline__ void sc_weights(C d, C& e, C& a, C& c) {
  if (d < C(0.5)) {
    if constexpr (BR) asm volatile("" : "+v"(d));
    constexpr int T = Series<C>::terms;
    C ph = C(kInvFactN[T + 1]);
#pragma unroll
    for (int m = T - 2; m >= 0; --m) ph = ph * (-d) + C(kInvFactN[m + 2]);
    c = d * ph;
    e = (C(1) - d) + d * c;
    a = d - (C(1) + d) * c;
  } else {
    if constexpr (BR) asm volatile("" : "+v"(d));
    C q;
    if constexpr (sizeof(C) == 8) {
      e = exp_neg_f64(d);
      q = div_f64_normal(C(1) - e, d);
    } else {
      e = __expf(-d);
      q = __fdividef(C(1) - e, d);
    }
    a = q - e;
    c = C(1) - q;
  }
}

// Quadratic short characteristics: with the source the parabola through the
// upwind (s_u), local (s_0) and downwind (s_d) values, the integral form of
// the transfer equation over the upwind interval of optical length du gives
// I_0 = e^{-du} I_u + pu s_u + p0 s_0 + pd s_d, where integrating each Lagrange
// basis polynomial (abscissa t = optical depth back from the local point:
// du upwind, -dd downwind) against e^{-t} over [0, du] gives
//   pu = (w2 + dd w1) / (du (du + dd)),
//   p0 = (w2 - (du - dd) w1 - du dd w0) / (-du dd),
//   pd = (w2 - du w1) / (dd (du + dd)),
// with the moments w_k = int_0^du t^k e^{-t} dt.  Above du = 1/2 the moments
// follow from e^{-du} by integration by parts (w0 = 1 - e, w1 = w0 - du e,
// w2 = 2 w1 - du^2 e); below, from their Taylor series
// w_k = du^{k+1} sum_m (-du)^m / (m! (k + m + 1)), whose first omitted term
// (m = 16 in FP64, 9 in FP32) is below the unit roundoff of the sum.
constexpr double mom_coef(int k, int m) {
  double f = 1.0;
  for (int j = 2; j <= m; ++j) f *= j;
  return 1.0 / (f * (k + m + 1));
}
#define RT_MC(k) {mom_coef(k, 0), mom_coef(k, 1), mom_coef(k, 2), mom_coef(k, 3), \
  mom_coef(k, 4), mom_coef(k, 5), mom_coef(k, 6), mom_coef(k, 7), mom_coef(k, 8), \
  mom_coef(k, 9), mom_coef(k, 10), mom_coef(k, 11), mom_coef(k, 12), mom_coef(k, 13), \
  mom_coef(k, 14), mom_coef(k, 15)}
static __device__ __constant__ double kMomCoef[3][16] = {RT_MC(0), RT_MC(1), RT_MC(2)};
#undef RT_MC

template <typename C>
__device__ __forceinline__ void qsc_weights(C du, C dd, C& e, C& pu, C& p0, C& pd) {
  C w0, w1, w2;
  if (du < C(0.5)) {
    constexpr int T = sizeof(C) == 8 ? 16 : 9;
    C s0 = C(kMomCoef[0][T - 1]), s1 = C(kMomCoef[1][T - 1]), s2 = C(kMomCoef[2][T - 1]);
#pragma unroll
    for (int m = T - 2; m >= 0; --m) {
      s0 = s0 * (-du) + C(kMomCoef[0][m]);
      s1 = s1 * (-du) + C(kMomCoef[1][m]);
      s2 = s2 * (-du) + C(kMomCoef[2][m]);
    }
    const C d2 = du * du;
    w0 = du * s0;
    w1 = d2 * s1;
    w2 = d2 * du * s2;
    e = C(1) - w0;
  } else {
    if constexpr (sizeof(C) == 8) e = exp_neg_f64(du);
    else e = __expf(-du);
    w0 = C(1) - e;
    w1 = w0 - du * e;
    w2 = C(2) * w1 - du * du * e;
  }
  const C sum = du + dd;
  pu = (w2 + dd * w1) / (du * sum);
  p0 = (w2 - (du - dd) * w1 - du * dd * w0) / (-du * dd);
  pd = (w2 - du * w1) / (dd * sum);
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
  static constexpr bool kScaled = false;   // no output scale (out_mul is 1)
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
  static constexpr bool kScaled = true;    // fp16 operands carry an output scale
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

// Outputs of F consecutive rays k0 .. k0 + F - 1.
template <typename LT>
struct PlainOuts {
  static constexpr bool kScaled = false;
  LT* o;          // ray k0
  size_t stride;  // elements per ray
  template <typename C>
  __device__ __forceinline__ void put(int f, size_t i, C v) const {
    o[(size_t)f * stride + i] = store_val<C, LT>(v);
  }
  // element base + i: base the same for the whole wavefront, i per lane
  template <typename C>
  __device__ __forceinline__ void put(int f, size_t base, int i, C v) const {
    LT* r = o + (size_t)f * stride + base;
    r[(unsigned)i] = store_val<C, LT>(v);
  }
};

template <int MODE>
struct K4Outs {
  static constexpr bool kScaled = true;
  uint16_t* hi;   // k4 buffer parts (not offset)
  uint16_t* lo;
  int64_t Np;
  int k0;
  template <typename C>
  __device__ __forceinline__ void put(int f, size_t i, C v) const {
    const int k = k0 + f;
    const size_t off = ((size_t)(k >> 2) * Np) * 4 + (k & 3);
    K4Out<MODE>{hi + off, lo ? lo + off : nullptr}.put(i, v);
  }
  // element base + i: base the same for the whole wavefront, i per lane
  template <typename C>
  __device__ __forceinline__ void put(int f, size_t base, int i, C v) const {
    const int k = k0 + f;
    const size_t off = ((size_t)(k >> 2) * Np + base) * 4 + (k & 3);
    K4Out<MODE>{hi + off, lo ? lo + off : nullptr}.put((unsigned)i, v);
  }
};

// v times the output scale om where the output type takes one (a plain
// output is never scaled, which saves a multiply per unknown).
template <typename OUT, typename C>
__device__ __forceinline__ C scaled_out(C v, C om) {
  if constexpr (OUT::kScaled) return v * om;
  else return v;
}

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
    } else if (scheme == RT_FORMAL_QUADRATIC_SC && q + 1 < nz) {
      const int md = down ? q + 1 : m - 1;      // memory index of the downwind node
      const int ivd = down ? q : m - 1;         // downwind interval index
      const C dd = C(dt[ivd] * g);
      C pu, p0, pd;
      qsc_weights<C>(d, dd, e, pu, p0, pd);
      b = pu * (sc * C(sk[mp])) + p0 * s0 + pd * (sc * C(sk[md]));
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
    out.put(down ? q : nz - 1 - q, scaled_out<OUT>(I, C(out_mul)));
  }
}

// ---------------------------------------------------------------------------
// Box sweep of F rays that share one ordinate (frequencies nu0 .. nu0 + nf - 1,
// nf <= F), plane by plane, by a whole NT-thread workgroup.  The upwind
// stencil, the interpolated opacity and the step's optical depth up to the
// frequency factor are computed once per point and used by all F rays; the
// previous plane's intensities and sources (per ray) and opacity sit in LDS,
// (2F + 1) values per point.  PP: two such sets, written by alternate planes,
// so that a plane needs one barrier (its writes go to the set the next plane
// reads, while the set it reads is not written); otherwise one set and two
// barriers per plane.  The next plane's sources and opacity are loaded a
// plane ahead and kept as loaded (no arithmetic on them before they are
// used, so the loads stay in flight over a plane).  Every thread takes up to
// kBoxMaxPts points of each plane (point threadIdx.x + j NT).
//
// Both forms keep each plane in LDS with one halo column and row (copies of
// column 0 and row 0: box_halo), so that the four corners of every upwind
// stencil are a, a + 1, a + W and a + W + 1 (W = nx + 1) with no wrap and
// one index per point serves them all; the stencil indices are re-formed
// inside the plane loop (an empty asm statement stops the compiler from
// hoisting every derived address out of the loop, which spilled).  The sums
// of products are explicit FMA chains, so that every launch shape rounds
// alike (the compiler's own contraction may fuse a different product from
// one instantiation to the next).
//
// Two forms, by compute type:
// * FP32 (box_rays_halo): a slot past the plane computes on the plane's
//   last point and is neither stored nor written to LDS, so no load sits
//   under a branch.  Loads and stores to global memory share one wait
//   counter, which is waited down to zero whenever both kinds are
//   outstanding; so the intensities of plane t are stored at the start of
//   plane t + 1, right after the wait for its sources and next to the loads
//   of plane t + 2, and the wait of every plane finds both a plane old
//   (quadratic sweeps, which read downwind values from global memory in
//   mid-plane, store at the end of the plane).  A point's 2F + 1 values
//   sit side by side, so that one address serves a stencil row (paired
//   LDS reads).  64^2 planes: 5.2 -> 4.1 ms per box64 sweep (fp16 operand).
// * FP64 (box_rays_sep): separate opacity, intensity and source planes, a
//   uniform exit per slot, stores at the end of each plane, and bilinear
//   weights formed on the host (scalar registers): 64 VGPRs at two points
//   per thread (eight waves per SIMD on 32^2 planes) and 101 at four with no
//   spill (10.5 -> 8.9 ms per box64 sweep).  The FP32 form's layout and
//   deferred stores hold more FP64 registers: 0.243 against 0.215 ms per
//   box32 sweep, 12.8 against 10.5 ms on box64.
//
// src(f): the ray's nz*P source values; fac[f]: phi_nu + r of ray f;
// out.put(f, i, v) stores value i of ray f.
constexpr int kBoxThreads = 256;

// Points of an LDS plane with its halo row and column.
constexpr size_t box_halo(int nx, int ny) { return (size_t)(nx + 1) * (ny + 1); }

// LDS elements of type C that box_rays needs, for halo planes of PH values.
constexpr size_t box_lds_elems(int F, size_t PH, bool pp) { return (size_t)(pp ? 2 : 1) * (2 * F + 1) * PH; }

//
// QUAD: quadratic short characteristics (qsc_weights): every plane but the
// last also takes the source at the downwind point, on the next plane
// downstream at the opposite displacement (st.di0, st.dj0, st.dtx, st.dty),
// and the opacity there for the downwind interval; both are bilinear
// interpolations read from global memory (the plane was just read into the
// L2 as the next plane's local values).
template <typename VT, typename OUT, typename C, int F, int kBoxMaxPts, int NT = kBoxThreads,
          bool PP = false, bool QUAD = false>
__device__ __forceinline__ void box_rays_halo(const VT* __restrict__ s0, size_t ray_stride, int nf,
                                         const OUT& out, const double* __restrict__ kline,
                                         const BoxStencil st, const C* fac, int nx, int ny,
                                         int nz, C i_in, C sc, float out_mul, C* smem) {
  const int P = nx * ny;
  constexpr int V = 2 * F + 1;           // values per LDS point: K, I [F], S [F]
  const int W = nx + 1;                  // LDS points per row
  const int WV = W * V;                  // LDS row pitch in elements
  const size_t PH = box_halo(nx, ny);
  const size_t set = (size_t)V * PH;
  const C hpath = C(0.5) * C(st.path);   // exact: (a / 2) path = a (path / 2)
  const C tx = C(st.tx), ty = C(st.ty);
  const size_t plane_stride = (size_t)P;
  constexpr bool kDefer = !QUAD;

  // slot j: point pc[j] (clamped to the plane); nb[j]: LDS element of its
  // upwind stencil's first corner; hq[j]: its own LDS element, with bit 20
  // set on column 0 and bit 21 on row 0 (the values the halo repeats)
  int pc[kBoxMaxPts], nb[kBoxMaxPts], hq[kBoxMaxPts];
  bool live[kBoxMaxPts];
#pragma unroll
  for (int j = 0; j < kBoxMaxPts; ++j) {
    const int p = threadIdx.x + j * NT;
    live[j] = p < P;
    pc[j] = live[j] ? p : P - 1;
    const int x = pc[j] % nx, y = pc[j] / nx;
    int xa = x + st.i0; if (xa >= nx) xa -= nx;
    int ya = y + st.j0; if (ya >= ny) ya -= ny;
    nb[j] = (ya * W + xa) * V;
    hq[j] = (y * W + x) * V | (x == 0 ? 1 << 20 : 0) | (y == 0 ? 1 << 21 : 0);
  }
  const C w00 = (C(1) - ty) * (C(1) - tx), w01 = (C(1) - ty) * tx;
  const C w10 = ty * (C(1) - tx), w11 = ty * tx;
  const C om = C(out_mul);
  // downwind stencil (QUAD)
  int d00[QUAD ? kBoxMaxPts : 1], d01[QUAD ? kBoxMaxPts : 1];
  int d10[QUAD ? kBoxMaxPts : 1], d11[QUAD ? kBoxMaxPts : 1];
  C v00 = C(0), v01 = C(0), v10 = C(0), v11 = C(0);
  if constexpr (QUAD) {
    const C dtx = C(st.dtx), dty = C(st.dty);
    v00 = (C(1) - dty) * (C(1) - dtx);
    v01 = (C(1) - dty) * dtx;
    v10 = dty * (C(1) - dtx);
    v11 = dty * dtx;
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      const int x = pc[j] % nx, y = pc[j] / nx;
      int xa = x + st.di0; if (xa >= nx) xa -= nx;
      int xb = xa + 1;     if (xb >= nx) xb -= nx;
      int ya = y + st.dj0; if (ya >= ny) ya -= ny;
      int yb = ya + 1;     if (yb >= ny) yb -= ny;
      d00[j] = ya * nx + xa;
      d01[j] = ya * nx + xb;
      d10[j] = yb * nx + xa;
      d11[j] = yb * nx + xb;
    }
  }
  // source of ray slot f (slots past nf repeat the last ray and are not stored)
  const VT* src[F];
#pragma unroll
  for (int f = 0; f < F; ++f) src[f] = s0 + (size_t)(f < nf ? f : nf - 1) * ray_stride;
  auto plane_of = [&](int t) { return st.up ? t : nz - 1 - t; };

  // sources and opacity of the next plane, loaded one plane ahead
  VT Sn[F][kBoxMaxPts];
  double Kn[kBoxMaxPts];
  C Sv[F][kBoxMaxPts], Iv[F][kBoxMaxPts], Kv[kBoxMaxPts];
  auto load_plane = [&](int t) {
    const size_t oz = (size_t)plane_of(t) * plane_stride;
    const double* kz = kline + oz;
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) Kn[j] = kz[(unsigned)pc[j]];
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      // unsigned lane offsets: one 32-bit offset register from a uniform base
      const unsigned q = (unsigned)pc[j];
#pragma unroll
      for (int f = 0; f < F; ++f) {
        const VT* sz = src[f] + oz;
        Sn[f][j] = sz[q];
      }
    }
  };
  // the intensities of plane t, held in Iv
  auto store_plane = [&](int t) {
    const size_t oz = (size_t)plane_of(t) * plane_stride;
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      if (!live[j]) continue;
#pragma unroll
      for (int f = 0; f < F; ++f)
        if (f < nf) out.put(f, oz, pc[j], scaled_out<OUT>(Iv[f][j], om));
    }
  };
  load_plane(0);
  for (int t = 0; t < nz; ++t) {
    const int z = plane_of(t);
    // the set the previous plane wrote, and the one this plane writes
    const C* rd = smem + (PP ? (size_t)((t + 1) & 1) * set : 0);
    C* wr = smem + (PP ? (size_t)(t & 1) * set : 0);
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      Kv[j] = C(Kn[j]);
#pragma unroll
      for (int f = 0; f < F; ++f) Sv[f][j] = sc * C(Sn[f][j]);
    }
    if constexpr (kDefer) {
      if (t > 0) store_plane(t - 1);
    }
    // the last plane loads itself again (in the L2), keeping the loads unconditional
    load_plane(t + 1 < nz ? t + 1 : t);
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      C I[F];
      if (t == 0) {
#pragma unroll
        for (int f = 0; f < F; ++f) I[f] = i_in;
      } else {
        int a = nb[j];
        asm volatile("" : "+v"(a));    // addresses from a are formed here, not kept live
        const C* r0 = rd + a;          // stencil rows
        const C* r1 = r0 + WV;
        // value c of the four corners
        auto interp = [&](int c) {
          return fma(w11, r1[V + c], fma(w10, r1[c], fma(w01, r0[V + c], w00 * r0[c])));
        };
        const C ku = interp(0);
        const C base = (ku + Kv[j]) * hpath;
        if (QUAD && t + 1 < nz) {
          const int zd = st.up ? z + 1 : z - 1;
          const double* kd = kline + (size_t)zd * plane_stride;
          const C kdn = fma(v11, C(kd[d11[j]]),
                            fma(v10, C(kd[d10[j]]), fma(v01, C(kd[d01[j]]), v00 * C(kd[d00[j]]))));
          const C based = (kdn + Kv[j]) * hpath;
#pragma unroll
          for (int f = 0; f < F; ++f) {
            const VT* sd = src[f] + (size_t)zd * plane_stride;
            const C Iu = interp(1 + f);
            const C Su = interp(1 + F + f);
            const C Sd = sc * fma(v11, C(sd[d11[j]]),
                                  fma(v10, C(sd[d10[j]]),
                                      fma(v01, C(sd[d01[j]]), v00 * C(sd[d00[j]]))));
            C e, pu, p0, pd;
            qsc_weights<C>(base * fac[f], based * fac[f], e, pu, p0, pd);
            I[f] = fma(pd, Sd, fma(p0, Sv[f][j], fma(pu, Su, e * Iu)));
          }
        } else {
#pragma unroll
          for (int f = 0; f < F; ++f) {
            const C Iu = interp(1 + f);
            const C Su = interp(1 + F + f);
            C e, a, c;
            sc_weights<C, true>(base * fac[f], e, a, c);   // branch form
            I[f] = fma(c, Sv[f][j], fma(a, Su, e * Iu));
          }
        }
      }
#pragma unroll
      for (int f = 0; f < F; ++f) Iv[f][j] = I[f];
    }
    if constexpr (!kDefer) store_plane(t);
    if constexpr (!PP) __syncthreads();   // every read of the one set is done
    auto put_lds = [&](int q, int j) {
      C* w = wr + q;
      w[0] = Kv[j];
#pragma unroll
      for (int f = 0; f < F; ++f) {
        w[1 + f] = Iv[f][j];
        w[1 + F + f] = Sv[f][j];
      }
    };
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      if (!live[j]) continue;
      int h = hq[j];
      asm volatile("" : "+v"(h));    // as for the reads
      const int q = h & 0xfffff;
      put_lds(q, j);
      if (h & (1 << 20)) put_lds(q + nx * V, j);                // halo column
      if (h & (1 << 21)) put_lds(q + ny * WV, j);               // halo row
      if ((h >> 20) == 3) put_lds(q + ny * WV + nx * V, j);     // halo corner
    }
    __syncthreads();
  }
  if constexpr (kDefer) store_plane(nz - 1);
}

template <typename VT, typename OUT, typename C, int F, int kBoxMaxPts, int NT = kBoxThreads,
          bool PP = false, bool QUAD = false>
__device__ __forceinline__ void box_rays_sep(const VT* __restrict__ s0, size_t ray_stride, int nf,
                                         const OUT& out, const double* __restrict__ kline,
                                         const BoxStencil st, const C* fac, int nx, int ny,
                                         int nz, C i_in, C sc, float out_mul, C* smem) {
  const int P = nx * ny;
  const int W = nx + 1;                 // LDS points per row (halo column)
  const size_t PH = box_halo(nx, ny);
  const size_t set = (size_t)(2 * F + 1) * PH;   // one set: K [PH], I [F][PH], S [F][PH]
  const C hpath = C(st.hpath);   // exact: (a / 2) path = a (path / 2)
  const size_t plane_stride = (size_t)P;

  const int npt = (P + NT - 1) / NT;
  // slot j: nb[j], the LDS index of its upwind stencil's first corner (the
  // others at + 1, + W, + W + 1); hq[j], its own LDS index, with bit 20 set on
  // column 0 and bit 21 on row 0 (the values the halo repeats)
  int nb[kBoxMaxPts], hq[kBoxMaxPts];
#pragma unroll
  for (int j = 0; j < kBoxMaxPts; ++j) {
    if (j >= npt) break;
    const int p = threadIdx.x + j * NT;
    nb[j] = hq[j] = 0;
    if (p < P) {
      const int x = p % nx, y = p / nx;
      int xa = x + st.i0; if (xa >= nx) xa -= nx;
      int ya = y + st.j0; if (ya >= ny) ya -= ny;
      nb[j] = ya * W + xa;
      hq[j] = (y * W + x) | (x == 0 ? 1 << 20 : 0) | (y == 0 ? 1 << 21 : 0);
    }
  }
  const C w00 = C(st.w00), w01 = C(st.w01), w10 = C(st.w10), w11 = C(st.w11);
  const C om = C(out_mul);
  // downwind stencil (QUAD)
  int d00[QUAD ? kBoxMaxPts : 1], d01[QUAD ? kBoxMaxPts : 1];
  int d10[QUAD ? kBoxMaxPts : 1], d11[QUAD ? kBoxMaxPts : 1];
  C v00 = C(0), v01 = C(0), v10 = C(0), v11 = C(0);
  if constexpr (QUAD) {
    const C dtx = C(st.dtx), dty = C(st.dty);
    v00 = (C(1) - dty) * (C(1) - dtx);
    v01 = (C(1) - dty) * dtx;
    v10 = dty * (C(1) - dtx);
    v11 = dty * dtx;
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      if (j >= npt) break;
      const int p = threadIdx.x + j * NT;
      const int x = p % nx, y = p / nx;
      int xa = x + st.di0; if (xa >= nx) xa -= nx;
      int xb = xa + 1;     if (xb >= nx) xb -= nx;
      int ya = y + st.dj0; if (ya >= ny) ya -= ny;
      int yb = ya + 1;     if (yb >= ny) yb -= ny;
      const bool in = p < P;
      d00[j] = in ? ya * nx + xa : 0;
      d01[j] = in ? ya * nx + xb : 0;
      d10[j] = in ? yb * nx + xa : 0;
      d11[j] = in ? yb * nx + xb : 0;
    }
  }

  // sources and opacity of the next plane, loaded one plane ahead
  VT Sn[F][kBoxMaxPts];
  double Kn[kBoxMaxPts];
  C Sv[F][kBoxMaxPts], Iv[F][kBoxMaxPts], Kv[kBoxMaxPts];
  auto load_plane = [&](int t) {
    const int z = st.up ? t : nz - 1 - t;
    const double* kz = kline + (size_t)z * plane_stride;
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      if (j >= npt) break;
      const int p = threadIdx.x + j * NT;
      if (p < P) {
        Kn[j] = kz[p];
#pragma unroll
        for (int f = 0; f < F; ++f)
          Sn[f][j] = f < nf ? s0[(size_t)f * ray_stride + (size_t)z * plane_stride + p] : VT(0);
      }
    }
  };
  load_plane(0);
  for (int t = 0; t < nz; ++t) {
    const int z = st.up ? t : nz - 1 - t;
    const size_t oz = (size_t)z * plane_stride;
    // the set the previous plane wrote, and the one this plane writes
    const C* rK = smem + (PP ? (size_t)((t + 1) & 1) * set : 0);
    const C* rI = rK + PH;
    const C* rS = rI + F * PH;
    C* wK = smem + (PP ? (size_t)(t & 1) * set : 0);
    C* wI = wK + PH;
    C* wS = wI + F * PH;
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      if (j >= npt) break;
      Kv[j] = C(Kn[j]);
#pragma unroll
      for (int f = 0; f < F; ++f) Sv[f][j] = sc * C(Sn[f][j]);
    }
    if (t + 1 < nz) load_plane(t + 1);
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      if (j >= npt) break;
      const int p = threadIdx.x + j * NT;
      if (p >= P) break;
      C I[F];
      if (t == 0) {
#pragma unroll
        for (int f = 0; f < F; ++f) I[f] = i_in;
      } else {
        int a = nb[j];
        asm volatile("" : "+v"(a));    // addresses from a are formed here, not kept live
        auto interp = [&](const C* v) {
          return fma(w11, v[a + W + 1], fma(w10, v[a + W], fma(w01, v[a + 1], w00 * v[a])));
        };
        const C ku = interp(rK);
        const C base = (ku + Kv[j]) * hpath;
        if (QUAD && t + 1 < nz) {
          const int zd = st.up ? z + 1 : z - 1;
          const double* kd = kline + (size_t)zd * plane_stride;
          const C kdn = fma(v11, C(kd[d11[j]]),
                            fma(v10, C(kd[d10[j]]), fma(v01, C(kd[d01[j]]), v00 * C(kd[d00[j]]))));
          const C based = (kdn + Kv[j]) * hpath;
#pragma unroll
          for (int f = 0; f < F; ++f) {
            const VT* sd = s0 + (size_t)f * ray_stride + (size_t)zd * plane_stride;
            const C Iu = interp(rI + f * PH);
            const C Su = interp(rS + f * PH);
            const C Sd = sc * fma(v11, C(sd[d11[j]]),
                                  fma(v10, C(sd[d10[j]]),
                                      fma(v01, C(sd[d01[j]]), v00 * C(sd[d00[j]]))));
            C e, pu, p0, pd;
            qsc_weights<C>(base * fac[f], based * fac[f], e, pu, p0, pd);
            I[f] = fma(pd, Sd, fma(p0, Sv[f][j], fma(pu, Su, e * Iu)));
          }
        } else {
#pragma unroll
          for (int f = 0; f < F; ++f) {
            const C Iu = interp(rI + f * PH);
            const C Su = interp(rS + f * PH);
            C e, a, c;
            sc_weights<C, true>(base * fac[f], e, a, c);   // branch form
            I[f] = fma(c, Sv[f][j], fma(a, Su, e * Iu));
          }
        }
      }
#pragma unroll
      for (int f = 0; f < F; ++f)
        if (f < nf) out.put(f, oz + p, scaled_out<OUT>(I[f], om));
#pragma unroll
      for (int f = 0; f < F; ++f) Iv[f][j] = I[f];
    }
    if constexpr (!PP) __syncthreads();   // every read of the one set is done
    auto put_lds = [&](int q, int j) {
      wK[q] = Kv[j];
#pragma unroll
      for (int f = 0; f < F; ++f) {
        wI[f * PH + q] = Iv[f][j];
        wS[f * PH + q] = Sv[f][j];
      }
    };
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      if (j >= npt) break;
      const int p = threadIdx.x + j * NT;
      if (p >= P) break;
      int h = hq[j];
      asm volatile("" : "+v"(h));    // as for the reads
      const int q = h & 0xfffff;
      put_lds(q, j);
      if (h & (1 << 20)) put_lds(q + nx, j);                // halo column
      if (h & (1 << 21)) put_lds(q + ny * W, j);            // halo row
      if ((h >> 20) == 3) put_lds(q + ny * W + nx, j);      // halo corner
    }
    __syncthreads();
  }
}


// The box sweep in the form for its compute type (see above).
template <typename VT, typename OUT, typename C, int F, int kBoxMaxPts, int NT = kBoxThreads,
          bool PP = false, bool QUAD = false>
__device__ __forceinline__ void box_rays(const VT* __restrict__ s0, size_t ray_stride, int nf,
                                         const OUT& out, const double* __restrict__ kline,
                                         const BoxStencil st, const C* fac, int nx, int ny,
                                         int nz, C i_in, C sc, float out_mul, C* smem) {
  if constexpr (sizeof(C) == 8)
    box_rays_sep<VT, OUT, C, F, kBoxMaxPts, NT, PP, QUAD>(s0, ray_stride, nf, out, kline, st, fac,
                                                          nx, ny, nz, i_in, sc, out_mul, smem);
  else
    box_rays_halo<VT, OUT, C, F, kBoxMaxPts, NT, PP, QUAD>(s0, ray_stride, nf, out, kline, st,
                                                           fac, nx, ny, nz, i_in, sc, out_mul, smem);
}

}  // namespace lam
}  // namespace rtsn
