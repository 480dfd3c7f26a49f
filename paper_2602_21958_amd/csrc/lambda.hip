// Formal solution Lambda on gfx950.
//
// Paper Sec. 3.2: rays are independent (Lambda is block diagonal in ray
// order, eq. lambda_block); along a ray the solution is a first-order linear
// recurrence I_q = e_q I_{q-1} + beta_q from the incoming boundary.
//
// * Linear short characteristics (exponential integrator from the integral
//   form of the transfer equation, Sec. 2 eq. rt_integral): over an interval
//   of optical length D, e = exp(-D), beta = a(D) s_up + c(D) s_0 with
//   a = (1 - e)/D - e and c = 1 - (1 - e)/D (Taylor series for D < 1/2).
// * Implicit Euler (eqs. ie_1 / ie_2): e = 1/(1 + D), beta = D s_0 / (1 + D).
//
// Slab: one 64-lane wavefront per ray.  The recurrence is evaluated as a
// parallel prefix over the lanes: each lane composes the affine maps of its
// chunk of depth points, the 64 composites are scanned with cross-lane
// shuffles, and each lane then replays its chunk from the scanned prefix.
// Loads of a ray's depth profile are contiguous (ray-major layout).
//
// Box: one workgroup per ray (ordinate, frequency) sweeps the planes in
// upwind order; the previous plane's intensity, source and opacity sit in
// LDS and the upwind point of every node is a fixed bilinear stencil of that
// plane (uniform grid, one offset per ordinate), with periodic wrap.
#include "rt_internal.h"

namespace rtsn {

namespace {

template <typename C> struct Series;
template <> struct Series<double> { static constexpr int terms = 16; };
template <> struct Series<float> { static constexpr int terms = 9; };

// 1/(n+1)! for n = 1..16
__device__ __constant__ double kInvFact[16] = {
    1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0,
    1.0 / 40320.0, 1.0 / 362880.0, 1.0 / 3628800.0, 1.0 / 39916800.0,
    1.0 / 479001600.0, 1.0 / 6227020800.0, 1.0 / 87178291200.0,
    1.0 / 1307674368000.0, 1.0 / 20922789888000.0, 1.0 / 355687428096000.0};

template <typename C>
__device__ __forceinline__ void sc_weights(C d, C& e, C& a, C& c) {
  e = exp(-d);
  if (d < C(0.5)) {
    // c = sum_{n>=1} (-1)^{n+1} d^n/(n+1)!,  a = sum_{n>=1} (-1)^{n+1} n d^n/(n+1)!
    constexpr int T = Series<C>::terms;
    C cs = C(0), as = C(0);
#pragma unroll
    for (int n = T; n >= 1; --n) {
      C sg = (n & 1) ? C(1) : C(-1);
      cs = cs * d + sg * C(kInvFact[n - 1]);
      as = as * d + sg * C(n) * C(kInvFact[n - 1]);
    }
    c = cs * d;
    a = as * d;
  } else {
    C q = -expm1(-d) / d;
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

// ---------------------------------------------------------------------------
// Slab sweep: blockDim = 256 (4 waves), one ray per wave.
template <typename VT, typename LT, typename C>
__global__ __launch_bounds__(256) void lambda_slab_kernel(
    const VT* __restrict__ s, LT* __restrict__ out, const double* __restrict__ dt,
    const double* __restrict__ ray_mu, const double* __restrict__ ray_fac, int n_r, int nz,
    double i_top, double i_bot, int with_bc, const double* __restrict__ scale, int scheme,
    float out_mul) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= n_r) return;  // whole wave leaves; no block barrier below
  const double mu = ray_mu[k];
  const double g = ray_fac[k] / fabs(mu);
  const bool down = mu < 0.0;
  const C sc = scale ? C(*scale) : C(1);
  const VT* sk = s + (size_t)k * nz;
  LT* ok = out + (size_t)k * nz;
  const C i_in = with_bc ? C(down ? i_top : i_bot) : C(0);
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
    ok[down ? q : nz - 1 - q] = store_val<C, LT>(I * C(out_mul));
  }
}

// ---------------------------------------------------------------------------
// Box sweep: one workgroup per ray, 256 threads, plane of P = nx*ny points
// in LDS (intensity, source, opacity of the upwind plane).
constexpr int kBoxThreads = 256;

template <typename VT, typename LT, typename C, int kBoxMaxPts>
__global__ __launch_bounds__(kBoxThreads) void lambda_box_kernel(
    const VT* __restrict__ s, LT* __restrict__ out, const double* __restrict__ kline,
    const BoxStencil* __restrict__ stencil, const double* __restrict__ ray_fac, int n_nu,
    int nx, int ny, int nz, double i_top, double i_bot, int with_bc,
    const double* __restrict__ scale, float out_mul) {
  extern __shared__ unsigned char smem_raw[];
  const int P = nx * ny;
  C* lI = reinterpret_cast<C*>(smem_raw);
  C* lS = lI + P;
  C* lK = lS + P;

  const int k = blockIdx.x;
  const int o = k / n_nu;
  const BoxStencil st = stencil[o];
  const C fac = C(ray_fac[k]);
  const C path = C(st.path);
  const C tx = C(st.tx), ty = C(st.ty);
  const C sc = scale ? C(*scale) : C(1);
  const C i_in = with_bc ? C(st.up ? i_bot : i_top) : C(0);
  const size_t plane_stride = (size_t)P;
  const VT* sk = s + (size_t)k * nz * plane_stride;
  LT* ok = out + (size_t)k * nz * plane_stride;

  const int npt = (P + kBoxThreads - 1) / kBoxThreads;
  C Iv[kBoxMaxPts], Sv[kBoxMaxPts], Kv[kBoxMaxPts];
  // upwind bilinear source offsets per owned point (fixed for the ordinate)
  int n00[kBoxMaxPts], n01[kBoxMaxPts], n10[kBoxMaxPts], n11[kBoxMaxPts];
#pragma unroll
  for (int j = 0; j < kBoxMaxPts; ++j) {
    if (j >= npt) break;
    const int p = threadIdx.x + j * kBoxThreads;
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

  for (int t = 0; t < nz; ++t) {
    const int z = st.up ? t : nz - 1 - t;
    const VT* sz = sk + (size_t)z * plane_stride;
    LT* oz = ok + (size_t)z * plane_stride;
    const double* kz = kline + (size_t)z * plane_stride;
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      if (j >= npt) break;
      const int p = threadIdx.x + j * kBoxThreads;
      if (p >= P) break;
      const C s0 = sc * C(sz[p]);
      const C k0 = C(kz[p]);
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
      oz[p] = store_val<C, LT>(I * C(out_mul));
      Iv[j] = I;
      Sv[j] = s0;
      Kv[j] = k0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBoxMaxPts; ++j) {
      if (j >= npt) break;
      const int p = threadIdx.x + j * kBoxThreads;
      if (p >= P) break;
      lI[p] = Iv[j];
      lS[p] = Sv[j];
      lK[p] = Kv[j];
    }
    __syncthreads();
  }
}

template <typename VT> struct ComputeOf;
template <> struct ComputeOf<double> { using type = double; };
template <> struct ComputeOf<float> { using type = float; };

}  // namespace

template <typename VT, typename LT>
void launch_lambda(const Problem& p, const VT* s, LT* out, bool with_bc,
                   const double* scale, hipStream_t st, float out_mul) {
  using C = typename ComputeOf<VT>::type;
  ProfScope prof(RT_KCLASS_LAMBDA, st);
  if (p.geom == RT_GEOM_SLAB) {
    dim3 grid((p.n_r + 3) / 4);
    hipLaunchKernelGGL((lambda_slab_kernel<VT, LT, C>), grid, dim3(256), 0, st, s, out,
                       p.d_dt, p.d_ray_mu, p.d_ray_fac, p.n_r, p.nz, p.i_top, p.i_bot,
                       with_bc ? 1 : 0, scale, p.formal, out_mul);
  } else {
    const int P = p.nx * p.ny;
    size_t lds = (size_t)3 * P * sizeof(C);
    int max_lds = 0;
    RT_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p.device));
    if (lds > (size_t)max_lds) fail(RT_E_INVALID, "box plane too large for LDS in this precision");
#define RT_BOX_LAUNCH(NPT)                                                                \
  hipLaunchKernelGGL((lambda_box_kernel<VT, LT, C, NPT>), dim3(p.n_r), dim3(kBoxThreads), \
                     lds, st, s, out, p.d_kline, p.d_stencil, p.d_ray_fac, p.n_nu, p.nx,   \
                     p.ny, p.nz, p.i_top, p.i_bot, with_bc ? 1 : 0, scale, out_mul)
    if (P <= kBoxThreads) RT_BOX_LAUNCH(1);
    else if (P <= 4 * kBoxThreads) RT_BOX_LAUNCH(4);
    else if (P <= 16 * kBoxThreads) RT_BOX_LAUNCH(16);
    else fail(RT_E_INVALID, "box plane larger than 4096 points");
#undef RT_BOX_LAUNCH
  }
  RT_HIP(hipGetLastError());
}

template void launch_lambda<double, double>(const Problem&, const double*, double*, bool,
                                            const double*, hipStream_t, float);
template void launch_lambda<float, float>(const Problem&, const float*, float*, bool,
                                          const double*, hipStream_t, float);
template void launch_lambda<float, __hip_bfloat16>(const Problem&, const float*,
                                                   __hip_bfloat16*, bool, const double*,
                                                   hipStream_t, float);
template void launch_lambda<float, __half>(const Problem&, const float*, __half*, bool,
                                           const double*, hipStream_t, float);

}  // namespace rtsn
