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
#include <cstdlib>

#include "lambda_dev.h"

namespace rtsn {

namespace {

using lam::kBoxThreads;

// Output of ray k: plain ray-major array of LT (K4 < 0) or the k4-interleaved
// 16-bit GEMM operand (K4 = lam::K4_BF16 / K4_FP16 / K4_SPLIT).
template <typename LT, int K4>
__device__ __forceinline__ auto ray_out(void* o0, void* o1, int k, size_t len, int64_t Np) {
  if constexpr (K4 < 0)
    return lam::PlainOut<LT>{static_cast<LT*>(o0) + (size_t)k * len};
  else
    return lam::k4_ray<K4>(static_cast<uint16_t*>(o0), static_cast<uint16_t*>(o1), k, Np);
}

template <typename VT, typename LT, typename C, int K4>
__global__ __launch_bounds__(256) void lambda_slab_kernel(
    const VT* __restrict__ s, void* out0, void* out1, int64_t Np, const double* __restrict__ dt,
    const double* __restrict__ ray_mu, const double* __restrict__ ray_fac, int n_r, int nz,
    double i_top, double i_bot, int with_bc, const double* __restrict__ scale, int scheme,
    float out_mul) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= n_r) return;  // whole wave leaves; no block barrier inside
  const double mu = ray_mu[k];
  const C sc = scale ? C(*scale) : C(1);
  const C i_in = with_bc ? C(mu < 0.0 ? i_top : i_bot) : C(0);
  lam::slab_ray<VT>(s + (size_t)k * nz, ray_out<LT, K4>(out0, out1, k, nz, Np), dt, mu,
                    ray_fac[k], nz, i_in, sc, scheme, out_mul, lane);
}

// Outputs of rays k0 .. k0 + F - 1 (plain ray-major array or k4 operand).
template <typename LT, int K4>
__device__ __forceinline__ auto rays_out(void* o0, void* o1, int k0, size_t len, int64_t Np) {
  if constexpr (K4 < 0)
    return lam::PlainOuts<LT>{static_cast<LT*>(o0) + (size_t)k0 * len, len};
  else
    return lam::K4Outs<K4>{static_cast<uint16_t*>(o0), static_cast<uint16_t*>(o1), Np, k0};
}

// Order of the groups when each writes one ray of the k4-interleaved 16-bit
// operand: the four rays of a k4 group fill alternate 2-byte slots of the
// same cache lines.  Workgroups are dealt to the 8 XCDs in turn (group b on
// XCD b % 8), each with its own L2, so in launch order the four rays would
// write parts of each line from four L2s.  Group b = 8 (4 m + r) + x sweeps
// ray 4 (8 m + x) + r instead: the rays of a k4 group run on one XCD, one
// after another in its dispatch order, and their writes meet in one L2.  A
// tail of fewer than 32 groups keeps launch order.
__device__ __forceinline__ int k4_xcd_order(int b, int n) {
  if (b >= n / 32 * 32) return b;
  const int x = b & 7, slot = b >> 3;
  return 4 * (8 * (slot >> 2) + x) + (slot & 3);
}

// One workgroup per (ordinate, chunk of F frequencies).
template <typename VT, typename LT, typename C, int K4, int F, int NPT, int NT, bool PP,
          bool QUAD>
__global__ __launch_bounds__(NT) void lambda_box_kernel(
    const VT* __restrict__ s, void* out0, void* out1, int64_t Np,
    const double* __restrict__ kline, const BoxStencil* __restrict__ stencil,
    const double* __restrict__ ray_fac, int n_nu, int nx, int ny, int nz, double i_top,
    double i_bot, int with_bc, const double* __restrict__ scale, float out_mul, int xcd_order) {
  extern __shared__ unsigned char smem_raw[];
  const int nch = (n_nu + F - 1) / F;
  const int b = xcd_order ? k4_xcd_order(blockIdx.x, gridDim.x) : blockIdx.x;
  const int o = b / nch;
  const int nu0 = (b % nch) * F;
  const int nf = min(F, n_nu - nu0);
  const int k0 = o * n_nu + nu0;
  const BoxStencil st = stencil[o];
  const size_t vol = (size_t)nx * ny * nz;
  const C sc = scale ? C(*scale) : C(1);
  const C i_in = with_bc ? C(st.up ? i_bot : i_top) : C(0);
  C fac[F];
#pragma unroll
  for (int f = 0; f < F; ++f) fac[f] = f < nf ? C(ray_fac[k0 + f]) : C(0);
  const auto outs = rays_out<LT, K4>(out0, out1, k0, vol, Np);
  lam::box_rays<VT, decltype(outs), C, F, NPT, NT, PP, QUAD>(
      s + (size_t)k0 * vol, vol, nf, outs, kline, st, fac, nx, ny, nz, i_in, sc, out_mul,
      reinterpret_cast<C*>(smem_raw));
}

template <typename VT> struct ComputeOf;
template <> struct ComputeOf<double> { using type = double; };
template <> struct ComputeOf<float> { using type = float; };
template <> struct ComputeOf<_Float16> { using type = float; };

}  // namespace

// Frequencies per box workgroup: one (a ray per group), or 0 when the ray's
// three LDS planes do not fit.  Sweeping four frequencies of an ordinate
// together shares the upwind stencil and opacity but needs 4x the per-thread
// state, and at the occupancy that leaves it was measured slower on the 32^3
// box (FP64 0.82 against 0.40 ms; FP32 0.22 against 0.19 ms); two
// frequencies per group on 64^2 planes (FP32 form, 1024 threads of 4
// points) need more than the 128 registers a thread has there (172 bytes
// spilled).
int box_chunk(size_t PH, int elem_bytes, int max_lds) {
  return 3 * PH * elem_bytes <= (size_t)max_lds ? 1 : 0;
}

// Measured with two sets against one on the 32^3 box: FP64 0.239 -> 0.226 ms
// (72 against 92 VGPRs: three groups per CU instead of two), FP32 0.144 ->
// 0.141 ms, fp16 input 0.153 -> 0.126 ms.  On 64^2 planes (1024 threads,
// one group per CU either way) the FP32 form gains too (fp16 operand
// 4.10 -> 3.89 ms per box64 sweep, bf16x3 5.43 -> 5.13 ms), while the FP64
// form's two sets would not fit in LDS.
bool box_pingpong(int F, int P, size_t PH, int elem_bytes, int max_lds) {
  if (F != 1 || lam::box_lds_elems(F, PH, true) * elem_bytes > (size_t)max_lds) return false;
  return P <= 1024 || elem_bytes == 4;
}

template <typename VT, typename LT, int K4>
void lambda_dispatch(const Problem& p, const VT* s, void* out0, void* out1, int64_t Np,
                     bool with_bc, const double* scale, hipStream_t st, float out_mul) {
  using C = typename ComputeOf<VT>::type;
  // plain outputs are stored unscaled (the kernels skip the multiply)
  if (K4 < 0 && out_mul != 1.f) fail(RT_E_INVALID, "plain Lambda output takes no output scale");
  ProfScope prof(sizeof(C) == 8 ? RT_KCLASS_LAMBDA : RT_KCLASS_LAMBDA_LO, st);
  if (p.geom == RT_GEOM_SLAB) {
    dim3 grid((p.n_r + 3) / 4);
    hipLaunchKernelGGL((lambda_slab_kernel<VT, LT, C, K4>), grid, dim3(256), 0, st, s, out0,
                       out1, Np, p.d_dt, p.d_ray_mu, p.d_ray_fac, p.n_r, p.nz, p.i_top, p.i_bot,
                       with_bc ? 1 : 0, scale, p.formal, out_mul);
  } else {
    const int P = p.nx * p.ny;
    int max_lds = 0;
    RT_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p.device));
    const size_t PH = lam::box_halo(p.nx, p.ny);
    const int F = box_chunk(PH, (int)sizeof(C), max_lds);
    if (F == 0) fail(RT_E_INVALID, "box plane too large for LDS in this precision");
    // the kernel takes PP = true only where pp sized the LDS for two sets
    const bool pp = box_pingpong(F, P, PH, (int)sizeof(C), max_lds);
    const size_t lds = lam::box_lds_elems(F, PH, pp) * sizeof(C);
    const int grid = p.n_omega * ((p.n_nu + F - 1) / F);
    // one ray per group (group index = ray index) into the k4 operand
    const int xcd = (K4 >= 0 && F == 1) ? 1 : 0;
#define RT_BOX_LAUNCH2(FF, NPT, NT, PPV, QV)                                                    \
  hipLaunchKernelGGL((lambda_box_kernel<VT, LT, C, K4, FF, NPT, NT, PPV, QV>), dim3(grid),      \
                     dim3(NT), lds, st, s, out0, out1, Np, p.d_kline, p.d_stencil, p.d_ray_fac, \
                     p.n_nu, p.nx, p.ny, p.nz, p.i_top, p.i_bot, with_bc ? 1 : 0, scale,        \
                     out_mul, xcd)
#define RT_BOX_LAUNCH1(FF, NPT, NT, PPV)                                \
  if (p.formal == RT_FORMAL_QUADRATIC_SC) RT_BOX_LAUNCH2(FF, NPT, NT, PPV, true); \
  else RT_BOX_LAUNCH2(FF, NPT, NT, PPV, false)
#define RT_BOX_LAUNCH(FF, NPT, NT)       \
  if (pp) { RT_BOX_LAUNCH1(FF, NPT, NT, true); } \
  else { RT_BOX_LAUNCH1(FF, NPT, NT, false); }
    // planes up to 256 points: 256 threads; up to 1024 points: 512 threads of
    // 2 points each (FP64 with two LDS sets: 64 VGPRs, three groups per CU;
    // 256 threads of 4 points or 1024 threads of 1 point measured slower on
    // the 32^3 box); up to 4096 points: 1024 threads of 4 points (FP64: 101
    // VGPRs, 16 waves per CU; 512 threads of 8 points took 250 VGPRs and
    // more time); the FP32 form computes all its point slots, so planes of
    // up to 2048 points take two
    if (P <= 256) { RT_BOX_LAUNCH(1, 1, 256); }
    else if (P <= 1024) { RT_BOX_LAUNCH(1, 2, 512); }
    else if (P <= 2048) { RT_BOX_LAUNCH(1, 2, 1024); }
    else if (P <= 4096) { RT_BOX_LAUNCH(1, 4, 1024); }
    else {
      fail(RT_E_INVALID, "box plane larger than 4096 points");
    }
#undef RT_BOX_LAUNCH
#undef RT_BOX_LAUNCH1
#undef RT_BOX_LAUNCH2
  }
  RT_HIP(hipGetLastError());
}

template <typename VT, typename LT>
void launch_lambda(const Problem& p, const VT* s, LT* out, bool with_bc,
                   const double* scale, hipStream_t st, float out_mul) {
  lambda_dispatch<VT, LT, -1>(p, s, out, nullptr, 0, with_bc, scale, st, out_mul);
}

template <typename VT>
void lambda_k4(const Problem& p, int precision, const VT* s, uint16_t* hi, uint16_t* lo,
               const double* scale, hipStream_t st) {
  const int64_t Np = p.np16;
  switch (precision) {
    case RT_PREC_BF16:
      lambda_dispatch<VT, float, lam::K4_BF16>(p, s, hi, nullptr, Np, false, scale, st, 1.f);
      break;
    case RT_PREC_FP16:
      lambda_dispatch<VT, float, lam::K4_FP16>(p, s, hi, nullptr, Np, false, scale, st,
                                               fp16_lambda_scale(p.n));
      break;
    case RT_PREC_BF16X3:
      lambda_dispatch<VT, float, lam::K4_SPLIT>(p, s, hi, lo, Np, false, scale, st, 1.f);
      break;
    default:
      fail(RT_E_INVALID, "launch_lambda_k4: not a 16-bit precision");
  }
}

void launch_lambda_k4(const Problem& p, int precision, const float* s, uint16_t* hi,
                      uint16_t* lo, const double* scale, hipStream_t st) {
  lambda_k4<float>(p, precision, s, hi, lo, scale, st);
}

void launch_lambda_k4(const Problem& p, int precision, const _Float16* s, uint16_t* hi,
                      uint16_t* lo, const double* scale, hipStream_t st) {
  lambda_k4<_Float16>(p, precision, s, hi, lo, scale, st);
}

template void launch_lambda<double, double>(const Problem&, const double*, double*, bool,
                                            const double*, hipStream_t, float);
template void launch_lambda<float, float>(const Problem&, const float*, float*, bool,
                                          const double*, hipStream_t, float);

}  // namespace rtsn
