// Batched solver kernels: many independent problems (slots) advance together.
//
// Every kernel is persistent: a fixed grid loops over a device-side work list
// whose length is also on the device, so the launch sequence of one engine
// step has fixed arguments and can be captured once in a hipGraph and
// replayed while the host rewrites the lists.  Work is decomposed per slot
// only (rays, 128 x 128 GEMM tiles, 4096-element chunks), so a slot's
// arithmetic, including the order of every reduction, does not depend on the
// other slots in the batch.
//
// Per slot, one engine step is one Arnoldi step of restarted GMRES on
// A_lo d = r / ||r|| (Lambda, Sigma GEMM with fused epilogue, dots, update,
// Givens); a cycle ends after `restart` steps or when |g_{j+1}| reaches the
// slot's target, with x += ||r|| V y and an FP64 residual r = b - A_64 x.
// With FP64 vectors and operator this is plain restarted GMRES; with FP32
// vectors and a low-precision operator it is FP64 iterative refinement.
#include "batch.h"
#include "gemm16_dev.h"
#include "gemm_dev.h"
#include "lambda_dev.h"

namespace rtsn {

namespace {

constexpr int TB = 256;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum G per-thread values over the block; thread g < cnt writes out[g*stride].
template <int G>
__device__ __forceinline__ void block_sum_store(double (&acc)[G], double* out, int stride,
                                                int cnt) {
  __shared__ double red[G][TB / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const double v = wsum(acc[g]);
    if (lane == 0) red[g][wave] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < G && (int)threadIdx.x < cnt) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < TB / 64; ++w) s += red[threadIdx.x][w];
    out[(size_t)threadIdx.x * stride] = s;
  }
  __syncthreads();
}

template <typename TV> struct ComputeOf;
template <> struct ComputeOf<double> { using type = double; };
template <> struct ComputeOf<float> { using type = float; };
template <> struct ComputeOf<_Float16> { using type = float; };

// ------------------------------------------------------------------ Lambda
// OUTER: x (FP64) -> L (FP64), no input scale.  Otherwise V_j (scaled by
// vscale_j) -> L (type LT; with K4 >= 0 the k4 16-bit GEMM operand, times
// l_scale for fp16).
template <typename LT, int K4>
__device__ __forceinline__ auto slot_out(const SlotDev& s, int k, size_t len) {
  if constexpr (K4 < 0)
    return lam::PlainOut<LT>{static_cast<LT*>(s.L) + (size_t)k * len};
  else
    return lam::k4_ray<K4>(s.l16, K4 == lam::K4_SPLIT ? s.l16 + (size_t)s.kp16 * s.np16 : nullptr,
                           k, s.np16);
}

template <typename VT, typename LT, typename C, int K4, bool OUTER>
__global__ __launch_bounds__(TB) void bk_lambda_slab(const SlotDev* __restrict__ slots,
                                                     const SlotStat* __restrict__ stat,
                                                     const Item* __restrict__ items,
                                                     const int* __restrict__ counts) {
  const int cnt = counts[0];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const Item w = items[it];
    const SlotDev& s = slots[w.slot];
    const int k = w.a + wave;
    if (k >= s.n_r) continue;  // per wave; slab_ray has no block barrier
    const VT* src;
    C sc;
    float om;
    if constexpr (OUTER) {
      src = reinterpret_cast<const VT*>(s.x);
      sc = C(1);
      om = 1.f;
    } else {
      // preconditioned slots sweep u = P^-1 v_j (same scale)
      const int j = stat[w.slot].j;
      src = s.prq ? static_cast<const VT*>(s.pu) : static_cast<const VT*>(s.V) + (size_t)j * s.n;
      sc = C(s.gs->vscale[j]);
      om = s.l_scale;
    }
    lam::slab_ray<VT>(src + (size_t)k * s.nz, slot_out<LT, K4>(s, k, s.nz), s.dt, s.ray_mu[k],
                      s.ray_fac[k], s.nz, C(0), sc, s.formal, om, lane);
  }
}

// Box items: rays k0 .. k0 + nf - 1 of one ordinate (Item a = k0, b = nf).
template <typename LT, int K4>
__device__ __forceinline__ auto slot_outs(const SlotDev& s, int k0, size_t len) {
  if constexpr (K4 < 0)
    return lam::PlainOuts<LT>{static_cast<LT*>(s.L) + (size_t)k0 * len, len};
  else
    return lam::K4Outs<K4>{s.l16, K4 == lam::K4_SPLIT ? s.l16 + (size_t)s.kp16 * s.np16 : nullptr,
                           s.np16, k0};
}

template <typename VT, typename LT, typename C, int K4, int F, int NPT, int NT, bool PP, bool OUTER>
__global__ __launch_bounds__(NT) void bk_lambda_box(const SlotDev* __restrict__ slots,
                                                    const SlotStat* __restrict__ stat,
                                                    const Item* __restrict__ items,
                                                    const int* __restrict__ counts) {
  extern __shared__ unsigned char smem_raw[];
  const int cnt = counts[1];
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const Item w = items[it];
    const SlotDev& s = slots[w.slot];
    const int k0 = w.a, nf = w.b;
    const size_t vol = (size_t)s.n_s;
    const VT* src;
    C sc;
    float om;
    if constexpr (OUTER) {
      src = reinterpret_cast<const VT*>(s.x);
      sc = C(1);
      om = 1.f;
    } else {
      const int j = stat[w.slot].j;
      src = s.prq ? static_cast<const VT*>(s.pu) : static_cast<const VT*>(s.V) + (size_t)j * s.n;
      sc = C(s.gs->vscale[j]);
      om = s.l_scale;
    }
    C fac[F];
#pragma unroll
    for (int f = 0; f < F; ++f) fac[f] = f < nf ? C(s.ray_fac[k0 + f]) : C(0);
    const auto outs = slot_outs<LT, K4>(s, k0, vol);
    lam::box_rays<VT, decltype(outs), C, F, NPT, NT, PP>(
        src + (size_t)k0 * vol, vol, nf, outs, s.kline, s.stencil[k0 / s.n_nu], fac, s.nx,
        s.ny, s.nz, C(0), sc, om, reinterpret_cast<C*>(smem_raw));
  }
}

// ------------------------------------------------------------------- GEMMs
// OUTER: r = x - (1 - eps) Mhat L (FP64).  Otherwise
// V_{j+1} = vscale_j V_j - (1 - eps) Mhat L.
template <typename T, bool OUTER>
__global__ __launch_bounds__(TB) void bk_gemm(const SlotDev* __restrict__ slots,
                                              const SlotStat* __restrict__ stat,
                                              const Item* __restrict__ items,
                                              const int* __restrict__ counts) {
  const int cnt = counts[2];
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const Item w = items[it];
    const SlotDev& s = slots[w.slot];
    const T* A;
    const T* X;
    T* Y;
    double xs;
    if constexpr (OUTER) {
      A = reinterpret_cast<const T*>(s.mhat64);
      X = reinterpret_cast<const T*>(s.x);
      Y = reinterpret_cast<T*>(s.r);
      xs = 1.0;
    } else {
      const int j = stat[w.slot].j;
      if constexpr (sizeof(T) == 8)
        A = reinterpret_cast<const T*>(s.mhat64);
      else
        A = reinterpret_cast<const T*>(s.mhat32);
      // Arnoldi on K: the step reads no V_j; preconditioned (K' = I - A
      // P^-1) it adds nd = v_j - u
      X = s.prq ? static_cast<const T*>(s.pnd) : nullptr;
      Y = static_cast<T*>(s.V) + (size_t)(j + 1) * s.n;
      xs = s.gs->vscale[j];
    }
    // Arnoldi steps on K: y = +(1 - eps) Mhat L (+ xs nd)
    const double sign = OUTER ? -1.0 : 1.0;
    gemm::gemm_tile<T, 16>(A, s.lda_mhat, static_cast<const T*>(s.L), X, Y, s.albedo, xs,
                           s.n_r, (int)s.n_s, s.n_r, w.a, w.b, sign);
  }
}

// 16-bit operands, one tile shape for every slot (tiles of the lists are
// 128 x 128): V_{j+1} = vscale_j V_j - (1 - eps) Mhat L.  Two tile bodies
// are candidates for the engine's tuner (32x32x16 with K stage 32, and
// 16x16x32 with K stage 64).
using BatchCfg16a = g16::Cfg<128, 128, 2, 2, 32, true>;
using BatchCfg16b = g16::Cfg<128, 128, 2, 2, 64, false>;

// TY: basis element type (float, or _Float16 stored times the slot's basis
// scale vs, which multiplies the whole output).
template <int MODE, typename C, typename TY>
__global__ __launch_bounds__(C::NT) void bk_gemm16(const SlotDev* __restrict__ slots,
                                                   const SlotStat* __restrict__ stat,
                                                   const Item* __restrict__ items,
                                                   const int* __restrict__ counts) {
  __shared__ __align__(16) uint8_t lds[C::template lds_bytes<MODE>()];
  const int cnt = counts[2];
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const Item w = items[it];
    const SlotDev& s = slots[w.slot];
    const int j = stat[w.slot].j;
    TY* Y = static_cast<TY*>(s.V) + (size_t)(j + 1) * s.n;
    const uint16_t* ahi = MODE == g16::MODE_FP16 ? s.a8_f16 : s.a8_hi;
    const uint16_t* blo = MODE == g16::MODE_SPLIT ? s.l16 + (size_t)s.kp16 * s.np16 : nullptr;
    const TY* X = s.prq ? static_cast<const TY*>(s.pnd) : nullptr;
    g16::tile<MODE, C, false, TY>(ahi, s.a8_lo, s.mp16, s.l16, blo, (int)s.np16, s.kp16 / 4, X,
                                  Y, s.albedo, MODE == g16::MODE_FP16 ? s.f16_rowscale : nullptr,
                                  1.f / s.l_scale, (float)s.gs->vscale[j],
                                  1.f, s.n_r,
                                  (int)s.n_s, w.a, w.b, lds, gemm::TileDots{}, 0, s.vs);
  }
}

// --------------------------------------------------------------- Arnoldi
// 16-byte vectors of the basis type (used when a slot's length keeps every
// basis vector 16-byte aligned).
template <typename TV> struct BVec;
template <> struct BVec<float> {
  typedef float T __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};
template <> struct BVec<double> {
  typedef double T __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};
template <> struct BVec<_Float16> {
  typedef _Float16 T __attribute__((ext_vector_type(8)));
  static constexpr int n = 8;
};
// arithmetic of the update: FP64 for FP64 / FP32 bases, FP32 for fp16
template <typename TV> struct BAcc { using type = double; };
template <> struct BAcc<_Float16> { using type = float; };

template <typename TV>
__device__ __forceinline__ double vdot(typename BVec<TV>::T a, typename BVec<TV>::T b) {
  if constexpr (sizeof(TV) == 2) {   // products of halves are exact in FP32
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < BVec<TV>::n; ++q) s += (float)a[q] * (float)b[q];
    return (double)s;
  } else {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < BVec<TV>::n; ++q) s += (double)a[q] * (double)b[q];
    return s;
  }
}

// Dots of the slot's basis with w over one kChunk-element chunk.
template <typename TV>
__global__ __launch_bounds__(TB) void bk_mdot(const SlotDev* __restrict__ slots,
                                              const SlotStat* __restrict__ stat,
                                              const Item* __restrict__ items,
                                              const int* __restrict__ counts) {
  using VT = typename BVec<TV>::T;
  constexpr int W = BVec<TV>::n;
  const int cnt = counts[3];
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const Item w = items[it];
    const SlotDev& s = slots[w.slot];
    const int j = stat[w.slot].j;
    const TV* V = static_cast<const TV*>(s.V);
    const TV* wv = V + (size_t)(j + 1) * s.n;
    const int64_t e0 = (int64_t)w.a * kChunk;
    const int64_t e1 = e0 + kChunk < s.n ? e0 + kChunk : s.n;
    const bool vec = (s.n % W) == 0;   // uniform per slot
    for (int i0 = 0; i0 <= j; i0 += 16) {
      double acc[16];
#pragma unroll
      for (int g = 0; g < 16; ++g) acc[g] = 0.0;
      if (vec) {
        const VT* wq = reinterpret_cast<const VT*>(wv);
        for (int64_t e = e0 / W + threadIdx.x; e < e1 / W; e += TB) {
          const VT x = wq[e];
#pragma unroll
          for (int g = 0; g < 16; ++g)
            if (i0 + g <= j)
              acc[g] += vdot<TV>(reinterpret_cast<const VT*>(V + (size_t)(i0 + g) * s.n)[e], x);
        }
      } else {
        for (int64_t e = e0 + threadIdx.x; e < e1; e += TB) {
          const double x = (double)wv[e];
#pragma unroll
          for (int g = 0; g < 16; ++g)
            if (i0 + g <= j) acc[g] += (double)V[(size_t)(i0 + g) * s.n + e] * x;
        }
      }
      const int c = j + 1 - i0 < 16 ? j + 1 - i0 : 16;
      block_sum_store<16>(acc, s.partial + (size_t)i0 * s.nch + w.a, s.nch, c);
    }
  }
}

__global__ __launch_bounds__(TB) void bk_reduce_rows(const SlotDev* __restrict__ slots,
                                                     const SlotStat* __restrict__ stat,
                                                     const int* __restrict__ list,
                                                     const int* __restrict__ counts) {
  const int cnt = counts[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const int si = list[it];
    const SlotDev& s = slots[si];
    const int j = stat[si].j;
    for (int i = wave; i <= j; i += TB / 64) {
      double v = 0.0;
      for (int c = lane; c < s.nch; c += 64) v += s.partial[(size_t)i * s.nch + c];
      v = wsum(v);
      if (lane == 0) s.gs->h[i] = s.gs->vscale[i] * v;
    }
  }
}

template <typename TV>
__global__ __launch_bounds__(TB) void bk_update(const SlotDev* __restrict__ slots,
                                                const SlotStat* __restrict__ stat,
                                                const Item* __restrict__ items,
                                                const int* __restrict__ counts) {
  using AT = typename BAcc<TV>::type;
  __shared__ AT coef[kMaxRestart + 1];
  const int cnt = counts[3];
  using VT = typename BVec<TV>::T;
  constexpr int W = BVec<TV>::n;
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const Item w = items[it];
    const SlotDev& s = slots[w.slot];
    const int j = stat[w.slot].j;
    __syncthreads();   // coef of the previous item is no longer read
    for (int i = threadIdx.x; i <= j; i += TB) coef[i] = (AT)(s.gs->h[i] * s.gs->vscale[i]);
    __syncthreads();
    TV* V = static_cast<TV*>(s.V);
    TV* wv = V + (size_t)(j + 1) * s.n;
    const int64_t e0 = (int64_t)w.a * kChunk;
    const int64_t e1 = e0 + kChunk < s.n ? e0 + kChunk : s.n;
    double nrm = 0.0;
    if ((s.n % W) == 0) {   // uniform per slot
      VT* wq = reinterpret_cast<VT*>(wv);
      for (int64_t e = e0 / W + threadIdx.x; e < e1 / W; e += TB) {
        const VT x = wq[e];
        AT v[W];
#pragma unroll
        for (int q = 0; q < W; ++q) v[q] = (AT)x[q];
        for (int i = 0; i <= j; ++i) {
          const VT b = reinterpret_cast<const VT*>(V + (size_t)i * s.n)[e];
#pragma unroll
          for (int q = 0; q < W; ++q) v[q] -= coef[i] * (AT)b[q];
        }
        VT r;
#pragma unroll
        for (int q = 0; q < W; ++q) {
          r[q] = (TV)v[q];
          nrm += (double)r[q] * (double)r[q];
        }
        wq[e] = r;
      }
    } else {
      for (int64_t e = e0 + threadIdx.x; e < e1; e += TB) {
        AT v = (AT)wv[e];
        for (int i = 0; i <= j; ++i) v -= coef[i] * (AT)V[(size_t)i * s.n + e];
        const TV q = (TV)v;
        wv[e] = q;
        nrm += (double)q * (double)q;
      }
    }
    double a[1] = {nrm};
    block_sum_store<1>(a, s.partial + (size_t)(s.restart + 1) * s.nch + w.a, 1, 1);
  }
}

__global__ __launch_bounds__(64) void bk_givens(const SlotDev* __restrict__ slots,
                                                SlotStat* __restrict__ stat,
                                                const int* __restrict__ list,
                                                const int* __restrict__ counts) {
  const int cnt = counts[4];
  const int lane = threadIdx.x;
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const int si = list[it];
    const SlotDev& s = slots[si];
    SlotStat& z = stat[si];
    double v = 0.0;
    for (int c = lane; c < s.nch; c += 64) v += s.partial[(size_t)(s.restart + 1) * s.nch + c];
    v = wsum(v);
    if (lane == 0) {
      GmresState* gs = s.gs;
      const int j = z.j;
      const double hn = sqrt(v);
      double* col = gs->R + (size_t)j * (kMaxRestart + 1);
      // vs A v_j = vs v_j - vs K v_j
      for (int i = 0; i <= j; ++i) col[i] = (i == j ? (double)s.vs : 0.0) - gs->h[i];
      col[j + 1] = -hn;
      const double raw_diag = col[j];
      for (int i = 0; i < j; ++i) {
        const double t1 = gs->cs[i] * col[i] + gs->sn[i] * col[i + 1];
        col[i + 1] = -gs->sn[i] * col[i] + gs->cs[i] * col[i + 1];
        col[i] = t1;
      }
      double c = 1.0, sn = 0.0;
      if (col[j + 1] != 0.0) {
        const double hh = hypot(col[j], col[j + 1]);
        c = col[j] / hh;
        sn = col[j + 1] / hh;
      }
      gs->cs[j] = c;
      gs->sn[j] = sn;
      col[j] = c * col[j] + sn * col[j + 1];
      col[j + 1] = 0.0;
      gs->g[j + 1] = -sn * gs->g[j];
      gs->g[j] = c * gs->g[j];
      const int breakdown = !(hn > 1e-14 * fabs(raw_diag) + 1e-300);
      gs->vscale[j + 1] = breakdown ? 0.0 : 1.0 / hn;
      const double resid = fabs(gs->g[j + 1]);
      z.resid = resid;
      z.breakdown = breakdown;
      z.nonfinite = !isfinite(hn) || !isfinite(resid);
      z.j = j + 1;
      z.iters += 1;
      // resid is relative to g_0 = vs (the basis scale; 1 unless fp16)
      z.cycle_done = (j + 1 >= s.restart) || resid <= z.target * (double)s.vs || breakdown ||
                     z.nonfinite;
    }
  }
}

// ------------------------------------------------------------- cycle end
__global__ __launch_bounds__(64) void bk_solve_r(const SlotDev* __restrict__ slots,
                                                 const SlotStat* __restrict__ stat,
                                                 const int* __restrict__ list,
                                                 const int* __restrict__ counts) {
  const int cnt = counts[4];
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    if (threadIdx.x != 0) continue;
    const int si = list[it];
    GmresState* gs = slots[si].gs;
    const int k = stat[si].j;
    const double rn = stat[si].rn;
    for (int i = k - 1; i >= 0; --i) {
      double v = gs->g[i];
      for (int l = i + 1; l < k; ++l) v -= gs->R[(size_t)l * (kMaxRestart + 1) + i] * gs->y[l];
      gs->y[i] = v / gs->R[(size_t)i * (kMaxRestart + 1) + i];
    }
    for (int i = 0; i < k; ++i) gs->coef[i] = gs->y[i] * gs->vscale[i] * rn;
  }
}

template <typename TV>
__global__ __launch_bounds__(TB) void bk_combine(const SlotDev* __restrict__ slots,
                                                 const SlotStat* __restrict__ stat,
                                                 const Item* __restrict__ items,
                                                 const int* __restrict__ counts) {
  __shared__ double coef[kMaxRestart + 1];
  const int cnt = counts[3];
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const Item w = items[it];
    const SlotDev& s = slots[w.slot];
    const int k = stat[w.slot].j;
    for (int i = threadIdx.x; i < k; i += TB) coef[i] = s.gs->coef[i];
    __syncthreads();
    const TV* V = static_cast<const TV*>(s.V);
    const int64_t e0 = (int64_t)w.a * kChunk;
    const int64_t e1 = e0 + kChunk < s.n ? e0 + kChunk : s.n;
    if (s.prq) {
      // preconditioned: d = V y into nd; x += P^-1 d follows (bk_prec_*)
      TV* d = static_cast<TV*>(s.pnd);
      for (int64_t e = e0 + threadIdx.x; e < e1; e += TB) {
        double v = 0.0;
        for (int i = 0; i < k; ++i) v += coef[i] * (double)V[(size_t)i * s.n + e];
        d[e] = (TV)v;
      }
    } else {
      for (int64_t e = e0 + threadIdx.x; e < e1; e += TB) {
        double v = s.x[e];
        for (int i = 0; i < k; ++i) v += coef[i] * (double)V[(size_t)i * s.n + e];
        s.x[e] = v;
      }
    }
    __syncthreads();
  }
}

// ----------------------------------------------- physics-based preconditioner
// The three passes of P^-1 (see precond.hip) over the chunk lists, for the
// slots with prq > 0: chunk c covers elements c kChunk .. (c + 1) kChunk - 1
// of the reduced index space (m = n_nu n_s for reduce and expand, prq m
// for the block products; both fit in n).  CYCLE selects the source: the
// basis vector v_j inside an iteration, d = V y (in nd) at a cycle end.
constexpr int kMaxPrecModes = 6;

template <typename TV, bool CYCLE>
__global__ __launch_bounds__(TB) void bk_prec_reduce(const SlotDev* __restrict__ slots,
                                                     const SlotStat* __restrict__ stat,
                                                     const Item* __restrict__ items,
                                                     const int* __restrict__ counts) {
  const int cnt = counts[3];
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const Item w = items[it];
    const SlotDev& s = slots[w.slot];
    if (s.prq == 0) continue;
    const int64_t m = (int64_t)s.n_nu * s.n_s;
    const int64_t e0 = (int64_t)w.a * kChunk;
    if (e0 >= m) continue;
    const int64_t e1 = e0 + kChunk < m ? e0 + kChunk : m;
    const TV* src = CYCLE ? static_cast<const TV*>(s.pnd)
                          : static_cast<const TV*>(s.V) + (size_t)stat[w.slot].j * s.n;
    const TV* G = static_cast<const TV*>(s.pG);
    TV* r = static_cast<TV*>(s.pr);
    const int n_om = s.n_r / s.n_nu, rq = s.prq;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += TB) {
      TV acc[kMaxPrecModes];
#pragma unroll
      for (int q = 0; q < kMaxPrecModes; ++q) acc[q] = TV(0);
      int o = 0;
      for (; o + 4 <= n_om; o += 4) {   // four loads in flight
        TV v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = src[(int64_t)(o + u) * m + e];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int q = 0; q < kMaxPrecModes; ++q)
            if (q < rq) acc[q] += G[(o + u) * rq + q] * v[u];
      }
      for (; o < n_om; ++o) {
        const TV v = src[(int64_t)o * m + e];
#pragma unroll
        for (int q = 0; q < kMaxPrecModes; ++q)
          if (q < rq) acc[q] += G[o * rq + q] * v;
      }
#pragma unroll
      for (int q = 0; q < kMaxPrecModes; ++q)
        if (q < rq) r[(int64_t)q * m + e] = acc[q];
    }
  }
}

// z[q][nu][i] = sum_k T[q][i][nu][k] r[q][k][i]: one wave per block (q, i).
// FP32 blocks of up to kMixLds rows go through LDS: the wave copies the block
// with coalesced loads into its own region (rows padded to n + 1, so that
// lanes reading one row each hit distinct banks) with r beside it, then lane
// nu sums its row.  Larger and FP64 blocks read their rows from global
// memory.  Item c of a slot takes the blocks 4 c + w, 4 c + w + 4 nch, ...
// (w the wave); the waves of a workgroup never wait for each other.
constexpr int kMixLds = 64;

template <typename TV>
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

template <typename TV>
__global__ __launch_bounds__(TB) void bk_prec_mix(const SlotDev* __restrict__ slots,
                                                  const Item* __restrict__ items,
                                                  const int* __restrict__ counts) {
  // FP32 tables only: an FP64 region would leave one workgroup per CU,
  // which measured slower than the global-memory rows
  constexpr bool kLds = sizeof(TV) == 4;
  __shared__ TV lds[kLds ? 4 : 1][kLds ? kMixLds * (kMixLds + 1) + kMixLds : 1];
  const int cnt = counts[3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  TV* L = lds[kLds ? wave : 0];
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const Item w = items[it];
    const SlotDev& s = slots[w.slot];
    if (s.prq == 0) continue;
    const int n = s.n_nu;
    const int64_t m = (int64_t)n * s.n_s, nblk = (int64_t)s.prq * s.n_s;
    const TV* T = static_cast<const TV*>(s.pT);
    const TV* r = static_cast<const TV*>(s.pr);
    TV* z = static_cast<TV*>(s.pz);
    for (int64_t b = (int64_t)w.a * 4 + wave; b < nblk; b += (int64_t)s.nch * 4) {
      const int q = (int)(b / s.n_s);
      const int64_t i = b - (int64_t)q * s.n_s;
      const TV* rq = r + (int64_t)q * m + i;
      const TV* blk = T + (size_t)b * n * n;
      TV* zq = z + (int64_t)q * m + i;
      if (kLds && n <= kMixLds) {
        TV* rl = L + n * (n + 1);
        for (int e = lane; e < n * n; e += 64) {
          const int row = e / n;
          L[row * (n + 1) + (e - row * n)] = blk[e];
        }
        if (lane < n) rl[lane] = rq[(int64_t)lane * s.n_s];
        wave_lds_sync<TV>();
        if (lane < n) {
          TV acc = TV(0);
          const TV* row = L + lane * (n + 1);
          for (int k = 0; k < n; ++k) acc += row[k] * rl[k];
          zq[(int64_t)lane * s.n_s] = acc;
        }
        wave_lds_sync<TV>();   // the next block overwrites the region
      } else {
        for (int nu = lane; nu < n; nu += 64) {
          TV acc = TV(0);
          for (int k = 0; k < n; ++k) acc += blk[(size_t)nu * n + k] * rq[(int64_t)k * s.n_s];
          zq[(int64_t)nu * s.n_s] = acc;
        }
      }
    }
  }
}

// Delta[(o, nu), i] = sum_q F[o][q] z[q][nu][i]; inside an iteration
// u = v_j + Delta and nd = -Delta, at a cycle end x += d + Delta (FP64 x)
template <typename TV, bool CYCLE>
__global__ __launch_bounds__(TB) void bk_prec_expand(const SlotDev* __restrict__ slots,
                                                     const SlotStat* __restrict__ stat,
                                                     const Item* __restrict__ items,
                                                     const int* __restrict__ counts) {
  const int cnt = counts[3];
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const Item w = items[it];
    const SlotDev& s = slots[w.slot];
    if (s.prq == 0) continue;
    const int64_t m = (int64_t)s.n_nu * s.n_s;
    const int64_t e0 = (int64_t)w.a * kChunk;
    if (e0 >= m) continue;
    const int64_t e1 = e0 + kChunk < m ? e0 + kChunk : m;
    const TV* src = CYCLE ? static_cast<const TV*>(s.pnd)
                          : static_cast<const TV*>(s.V) + (size_t)stat[w.slot].j * s.n;
    const TV* F = static_cast<const TV*>(s.pF);
    const TV* z = static_cast<const TV*>(s.pz);
    TV* u = static_cast<TV*>(s.pu);
    TV* nd = static_cast<TV*>(s.pnd);
    const int n_om = s.n_r / s.n_nu, rq = s.prq;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += TB) {
      TV zv[kMaxPrecModes];
#pragma unroll
      for (int q = 0; q < kMaxPrecModes; ++q) zv[q] = q < rq ? z[(int64_t)q * m + e] : TV(0);
      int o = 0;
      for (; o + 4 <= n_om; o += 4) {   // four loads in flight
        TV sv[4];
#pragma unroll
        for (int uu = 0; uu < 4; ++uu) sv[uu] = src[(int64_t)(o + uu) * m + e];
#pragma unroll
        for (int uu = 0; uu < 4; ++uu) {
          TV dlt = TV(0);
#pragma unroll
          for (int q = 0; q < kMaxPrecModes; ++q)
            if (q < rq) dlt += F[(o + uu) * rq + q] * zv[q];
          const int64_t at = (int64_t)(o + uu) * m + e;
          if constexpr (CYCLE) {
            s.x[at] += (double)(sv[uu] + dlt);
          } else {
            u[at] = sv[uu] + dlt;
            nd[at] = -dlt;
          }
        }
      }
      for (; o < n_om; ++o) {
        TV dlt = TV(0);
#pragma unroll
        for (int q = 0; q < kMaxPrecModes; ++q)
          if (q < rq) dlt += F[o * rq + q] * zv[q];
        const int64_t at = (int64_t)o * m + e;
        if constexpr (CYCLE) {
          s.x[at] += (double)(src[at] + dlt);
        } else {
          u[at] = src[at] + dlt;
          nd[at] = -dlt;
        }
      }
    }
  }
}

// r = b - r (r holds A x), partial norms
__global__ __launch_bounds__(TB) void bk_residual(const SlotDev* __restrict__ slots,
                                                  const Item* __restrict__ items,
                                                  const int* __restrict__ counts) {
  const int cnt = counts[3];
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const Item w = items[it];
    const SlotDev& s = slots[w.slot];
    const int64_t e0 = (int64_t)w.a * kChunk;
    const int64_t e1 = e0 + kChunk < s.n ? e0 + kChunk : s.n;
    double nrm = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += TB) {
      const double v = s.b[e] - s.r[e];
      s.r[e] = v;
      nrm += v * v;
    }
    double a[1] = {nrm};
    block_sum_store<1>(a, s.partial + (size_t)(s.restart + 1) * s.nch + w.a, 1, 1);
  }
}

__global__ __launch_bounds__(64) void bk_finish_rn(const SlotDev* __restrict__ slots,
                                                   SlotStat* __restrict__ stat,
                                                   const int* __restrict__ list,
                                                   const int* __restrict__ counts) {
  const int cnt = counts[4];
  const int lane = threadIdx.x;
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const int si = list[it];
    const SlotDev& s = slots[si];
    double v = 0.0;
    for (int c = lane; c < s.nch; c += 64) v += s.partial[(size_t)(s.restart + 1) * s.nch + c];
    v = wsum(v);
    if (lane == 0) {
      stat[si].rn = sqrt(v);
      stat[si].nonfinite = !isfinite(v);
    }
  }
}

// ----------------------------------------------------------- cycle start
template <typename TV>
__global__ __launch_bounds__(TB) void bk_v0(const SlotDev* __restrict__ slots,
                                            const SlotStat* __restrict__ stat,
                                            const Item* __restrict__ items,
                                            const int* __restrict__ counts) {
  const int cnt = counts[3];
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const Item w = items[it];
    const SlotDev& s = slots[w.slot];
    const double inv = (double)s.vs / stat[w.slot].rn;
    TV* V = static_cast<TV*>(s.V);
    const int64_t e0 = (int64_t)w.a * kChunk;
    const int64_t e1 = e0 + kChunk < s.n ? e0 + kChunk : s.n;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += TB) V[e] = (TV)(s.r[e] * inv);
  }
}

__global__ __launch_bounds__(64) void bk_init_cycle(const SlotDev* __restrict__ slots,
                                                    const int* __restrict__ list,
                                                    const int* __restrict__ counts) {
  const int cnt = counts[4];
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const SlotDev& s = slots[list[it]];
    GmresState* gs = s.gs;
    // V_0 = vs r / ||r||: g_0 = vs and unit v_0 = V_0 / vs
    for (int i = threadIdx.x; i <= kMaxRestart; i += 64) gs->g[i] = i == 0 ? (double)s.vs : 0.0;
    if (threadIdx.x == 0) gs->vscale[0] = 1.0 / (double)s.vs;
  }
}

template <typename K, typename... Args>
void persist(K kernel, int threads, size_t lds, hipStream_t st, Args... args) {
  hipLaunchKernelGGL(kernel, dim3(kPersistBlocks), dim3(threads), lds, st, args...);
  RT_HIP(hipGetLastError());
}

template <typename K, typename... Args>
void persist_grid(K kernel, int grid, int threads, size_t lds, hipStream_t st, Args... args) {
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), lds, st, args...);
  RT_HIP(hipGetLastError());
}

template <int MODE, typename TY>
void launch_b_gemm16(const SlotDev* slots, const SlotStat* stat, const WorkLists& wl,
                     const BatchTune& tune, hipStream_t st) {
  ProfScope prof(RT_KCLASS_SIGMA_LO, st);
  if (tune.cfg == 1)
    persist_grid(bk_gemm16<MODE, BatchCfg16b, TY>, tune.grid, BatchCfg16b::NT, 0, st, slots,
                 stat, wl.tiles, wl.counts);
  else
    persist_grid(bk_gemm16<MODE, BatchCfg16a, TY>, tune.grid, BatchCfg16a::NT, 0, st, slots,
                 stat, wl.tiles, wl.counts);
}

template <typename VT, typename LT, typename C, int K4, bool OUTER>
void launch_b_lambda(const SlotDev* slots, const SlotStat* stat, const WorkLists& wl,
                     hipStream_t st) {
  ProfScope prof(sizeof(C) == 8 ? RT_KCLASS_LAMBDA : RT_KCLASS_LAMBDA_LO, st);
  if (wl.h_counts[0] > 0)
    persist(bk_lambda_slab<VT, LT, C, K4, OUTER>, TB, 0, st, slots, stat, wl.lam_slab, wl.counts);
  if (wl.h_counts[1] > 0) {
    // two alternating LDS sets where they fit (the kernel takes PP = true
    // only then; PP = false needs no more than lds either way)
    const bool pp = box_pingpong(wl.box_f, wl.box_pmax, wl.box_phmax, (int)sizeof(C),
                                 wl.max_lds);
    const size_t lds = lam::box_lds_elems(wl.box_f, wl.box_phmax, pp) * sizeof(C);
#define RT_BBOX1(FF, NPT, NT, PPV)                                                          \
  persist(bk_lambda_box<VT, LT, C, K4, FF, NPT, NT, PPV, OUTER>, NT, lds, st, slots, stat, \
          wl.lam_box, wl.counts)
#define RT_BBOX(FF, NPT, NT)         \
  if (pp) RT_BBOX1(FF, NPT, NT, true); \
  else RT_BBOX1(FF, NPT, NT, false)
    if (wl.box_f == 4) {
      if (wl.box_npt <= 1) RT_BBOX1(4, 1, 256, false);
      else RT_BBOX1(4, 1, 1024, false);
    } else {
      if (wl.box_npt <= 1) { RT_BBOX(1, 1, 256); }
      else if (wl.box_npt <= 2) { RT_BBOX(1, 2, 512); }
      else { RT_BBOX(1, 4, 1024); }
    }
#undef RT_BBOX
#undef RT_BBOX1
  }
}

}  // namespace

const char* batch_gemm16_name(int cfg) {
  return cfg == 1 ? "128x128 16x16x32 K64" : "128x128 32x32x16 K32";
}

template <typename TV>
void lambda16(const SlotDev* slots, SlotStat* stat, const WorkLists& wl, int prec,
              hipStream_t st) {
  switch (prec) {
    case RT_PREC_BF16:
      launch_b_lambda<TV, float, float, lam::K4_BF16, false>(slots, stat, wl, st);
      break;
    case RT_PREC_FP16:
      launch_b_lambda<TV, float, float, lam::K4_FP16, false>(slots, stat, wl, st);
      break;
    case RT_PREC_BF16X3:
      launch_b_lambda<TV, float, float, lam::K4_SPLIT, false>(slots, stat, wl, st);
      break;
    default:
      fail(RT_E_INVALID, "b_lambda16: not a 16-bit precision");
  }
}

template <typename TV>
void gemm16(const SlotDev* slots, SlotStat* stat, const WorkLists& wl, int prec, hipStream_t st,
            const BatchTune& tune) {
  switch (prec) {
    case RT_PREC_BF16: launch_b_gemm16<g16::MODE_BF16, TV>(slots, stat, wl, tune, st); break;
    case RT_PREC_FP16: launch_b_gemm16<g16::MODE_FP16, TV>(slots, stat, wl, tune, st); break;
    case RT_PREC_BF16X3: launch_b_gemm16<g16::MODE_SPLIT, TV>(slots, stat, wl, tune, st); break;
    default: fail(RT_E_INVALID, "b_time_gemm16: not a 16-bit precision");
  }
}

void b_lambda16(const SlotDev* slots, SlotStat* stat, const WorkLists& wl, int prec,
                hipStream_t st, bool half_basis) {
  if (half_basis) lambda16<_Float16>(slots, stat, wl, prec, st);
  else lambda16<float>(slots, stat, wl, prec, st);
}

void b_time_gemm16(const SlotDev* slots, SlotStat* stat, const WorkLists& wl, int prec,
                   hipStream_t st, const BatchTune& tune, bool half_basis) {
  if (half_basis) gemm16<_Float16>(slots, stat, wl, prec, st, tune);
  else gemm16<float>(slots, stat, wl, prec, st, tune);
}

// u = P^-1 v_j and nd = v_j - u (CYCLE = false), or x += P^-1 d with d in
// nd (CYCLE = true), for the preconditioned slots of the lists
template <typename TV, bool CYCLE>
void b_precond(const SlotDev* slots, SlotStat* stat, const WorkLists& wl, hipStream_t st) {
  if constexpr (sizeof(TV) == 2) {
    fail(RT_E_INVALID, "the preconditioner needs FP64 or FP32 bases");
  } else {
    ProfScope prof(RT_KCLASS_PRECOND, st);
    persist(bk_prec_reduce<TV, CYCLE>, TB, 0, st, slots, stat, wl.chunks, wl.counts);
    persist(bk_prec_mix<TV>, TB, 0, st, slots, wl.chunks, wl.counts);
    persist(bk_prec_expand<TV, CYCLE>, TB, 0, st, slots, stat, wl.chunks, wl.counts);
  }
}

template <typename TV>
void b_inner_iteration(const SlotDev* slots, SlotStat* stat, const WorkLists& wl, int prec,
                       hipStream_t st, const BatchTune& tune) {
  using C = typename ComputeOf<TV>::type;
  if (wl.any_prec) b_precond<TV, false>(slots, stat, wl, st);
  if constexpr (sizeof(TV) == 8) {
    if (prec != RT_PREC_FP64) fail(RT_E_INVALID, "FP64 vectors need the FP64 operator");
    launch_b_lambda<double, double, double, -1, false>(slots, stat, wl, st);
    ProfScope prof(RT_KCLASS_SIGMA, st);
    persist(bk_gemm<double, false>, TB, 0, st, slots, stat, wl.tiles, wl.counts);
  } else {
    switch (prec) {
      case RT_PREC_FP32: {
        if constexpr (sizeof(TV) == 2) fail(RT_E_INVALID, "an fp16 basis needs a 16-bit operator");
        launch_b_lambda<float, float, C, -1, false>(slots, stat, wl, st);
        ProfScope prof(RT_KCLASS_SIGMA_LO, st);
        persist(bk_gemm<float, false>, TB, 0, st, slots, stat, wl.tiles, wl.counts);
        break;
      }
      case RT_PREC_BF16:
      case RT_PREC_FP16:
      case RT_PREC_BF16X3:
        lambda16<TV>(slots, stat, wl, prec, st);
        gemm16<TV>(slots, stat, wl, prec, st, tune);
        break;
      default:
        fail(RT_E_INVALID, "unknown precision");
    }
  }
  {
    ProfScope prof(RT_KCLASS_ARNOLDI, st);
    persist(bk_mdot<TV>, TB, 0, st, slots, stat, wl.chunks, wl.counts);
    persist(bk_reduce_rows, TB, 0, st, slots, stat, wl.slots, wl.counts);
    persist(bk_update<TV>, TB, 0, st, slots, stat, wl.chunks, wl.counts);
  }
  persist(bk_givens, 64, 0, st, slots, stat, wl.slots, wl.counts);
}

template <typename TV>
void b_cycle_end(const SlotDev* slots, SlotStat* stat, const WorkLists& wl, hipStream_t st) {
  persist(bk_solve_r, 64, 0, st, slots, stat, wl.slots, wl.counts);
  persist(bk_combine<TV>, TB, 0, st, slots, stat, wl.chunks, wl.counts);
  if (wl.any_prec) b_precond<TV, true>(slots, stat, wl, st);
  launch_b_lambda<double, double, double, -1, true>(slots, stat, wl, st);
  {
    ProfScope prof(RT_KCLASS_SIGMA, st);
    persist(bk_gemm<double, true>, TB, 0, st, slots, stat, wl.tiles, wl.counts);
  }
  persist(bk_residual, TB, 0, st, slots, wl.chunks, wl.counts);
  persist(bk_finish_rn, 64, 0, st, slots, stat, wl.slots, wl.counts);
}

template <typename TV>
void b_start_cycle(const SlotDev* slots, SlotStat* stat, const WorkLists& wl, hipStream_t st) {
  persist(bk_v0<TV>, TB, 0, st, slots, stat, wl.chunks, wl.counts);
  persist(bk_init_cycle, 64, 0, st, slots, wl.slots, wl.counts);
}

template void b_inner_iteration<double>(const SlotDev*, SlotStat*, const WorkLists&, int,
                                        hipStream_t, const BatchTune&);
template void b_inner_iteration<float>(const SlotDev*, SlotStat*, const WorkLists&, int,
                                       hipStream_t, const BatchTune&);
template void b_cycle_end<double>(const SlotDev*, SlotStat*, const WorkLists&, hipStream_t);
template void b_cycle_end<float>(const SlotDev*, SlotStat*, const WorkLists&, hipStream_t);
template void b_start_cycle<double>(const SlotDev*, SlotStat*, const WorkLists&, hipStream_t);
template void b_start_cycle<float>(const SlotDev*, SlotStat*, const WorkLists&, hipStream_t);
template void b_inner_iteration<_Float16>(const SlotDev*, SlotStat*, const WorkLists&, int,
                                          hipStream_t, const BatchTune&);
template void b_cycle_end<_Float16>(const SlotDev*, SlotStat*, const WorkLists&, hipStream_t);
template void b_start_cycle<_Float16>(const SlotDev*, SlotStat*, const WorkLists&, hipStream_t);

}  // namespace rtsn
