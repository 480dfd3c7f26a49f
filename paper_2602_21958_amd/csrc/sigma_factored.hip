// Scattering step in factored form for the dipole x PRD kernel.
//
// Paper Sec. 3.3 (eq. Sigma) gives the scattering block of every point as
// Gamma Psi W; Sec. 4.1 remarks that a low-rank approximation of the
// redistribution makes its application cost linear in the unknowns.  For
// the dipole phase function times a frequency redistribution the block is a
// Kronecker product with an angular factor of exact rank R (6 in 3D, 2 for
// the azimuth-averaged slab; see build_factors in setup.cpp):
//     Mhat[(o,nu),(o',nu')] = sum_q fq[o][q] fg[o'][q] * fb[nu][nu'].
// So y = xs x + sign (1 - eps_i) Mhat L is applied in three passes over the
// ray-major vectors instead of one dense N_r x N_r GEMM:
//   reduce:  W[q][nu'][i] = sum_o' fg[o'][q] L[(o' N_nu + nu') N_s + i]
//   mix:     Z[q][nu][i]  = sum_nu' fb[nu][nu'] W[q][nu'][i]
//   expand:  y[(o N_nu + nu) N_s + i] = xs x[...] + sign (1 - eps_i)
//                                       sum_q fq[o][q] Z[q][nu][i]
// Work per unknown is 2 R (reduce) + 2 R (expand) flops plus 2 R N_nu / N_omega
// (mix), so the passes are bound by HBM: reduce reads L, expand reads x and
// writes y; W and Z hold R / N_omega of a vector each.
#include <type_traits>

#include "rt_internal.h"

namespace rtsn {

namespace {

constexpr int kMaxRank = 6;
constexpr int kMixTile = 64;     // points per mix workgroup

// Vectors of V consecutive points: one 16-byte load or store per lane when
// V = 16 / sizeof(T) (the problem's point count a multiple of V, so that every
// ray's row starts 16-byte aligned), else single elements.
template <typename T, int V> struct VecOf;
template <> struct VecOf<double, 2> { typedef double __attribute__((ext_vector_type(2))) type; };
template <> struct VecOf<float, 4> { typedef float __attribute__((ext_vector_type(4))) type; };
template <> struct VecOf<double, 1> { typedef double type; };
template <> struct VecOf<float, 1> { typedef float type; };

// W = fg^T L over the ordinates; one thread per (nu', V points), grid-stride.
// The ordinate loop walks rays nu' + o' N_nu, so a wave's loads are 64 V
// consecutive points of one ray; fg is wave-uniform (scalar loads).
template <typename T, int R, int V>
__global__ __launch_bounds__(256) void fsig_reduce(const T* __restrict__ L,
                                                   const T* __restrict__ fg, T* __restrict__ W,
                                                   int n_om, int n_nu, int64_t n_s) {
  using VT = typename VecOf<T, V>::type;
  const int64_t m = (int64_t)n_nu * n_s;
  const int64_t mv = m / V;
  const int64_t ray_stride = m / V;    // in vectors
  const VT* Lv = reinterpret_cast<const VT*>(L);
  VT* Wv = reinterpret_cast<VT*>(W);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < mv;
       e += (int64_t)gridDim.x * blockDim.x) {
    VT acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = VT(0);
    const VT* src = Lv + e;
    int o = 0;
    for (; o + 4 <= n_om; o += 4) {
      VT v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = src[(int64_t)(o + u) * ray_stride];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] += fg[(o + u) * R + q] * v[u];
    }
    for (; o < n_om; ++o) {
      const VT v = src[(int64_t)o * ray_stride];
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] += fg[o * R + q] * v;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) Wv[(int64_t)q * mv + e] = acc[q];
  }
}

// Z[q] = fb W[q] over frequencies.  One workgroup per (q, tile of 64 points):
// the tile's N_nu rows of W[q] and fb are staged in LDS; thread t computes
// frequencies nu = t / 64 + 4 j of point t % 64.
template <typename T>
__global__ __launch_bounds__(256) void fsig_mix(const T* __restrict__ W, const T* __restrict__ fb,
                                                T* __restrict__ Z, int n_nu, int64_t n_s,
                                                int64_t n_tiles) {
  extern __shared__ unsigned char smem_raw[];
  T* sw = reinterpret_cast<T*>(smem_raw);          // n_nu x kMixTile
  T* sb = sw + (size_t)n_nu * kMixTile;            // n_nu x n_nu
  const int64_t m = (int64_t)n_nu * n_s;
  const int q = (int)(blockIdx.x / n_tiles);
  const int64_t i0 = (blockIdx.x - (int64_t)q * n_tiles) * kMixTile;
  const int p = threadIdx.x % kMixTile;
  const int64_t i = i0 + p;
  const bool live = i < n_s;
  const T* wq = W + (int64_t)q * m;
  for (int nu = threadIdx.x / kMixTile; nu < n_nu; nu += blockDim.x / kMixTile)
    sw[nu * kMixTile + p] = live ? wq[(int64_t)nu * n_s + i] : T(0);
  for (int e = threadIdx.x; e < n_nu * n_nu; e += blockDim.x) sb[e] = fb[e];
  __syncthreads();
  if (!live) return;
  T* zq = Z + (int64_t)q * m;
  for (int nu = threadIdx.x / kMixTile; nu < n_nu; nu += blockDim.x / kMixTile) {
    const T* b = sb + nu * n_nu;
    T acc = T(0);
    for (int k = 0; k < n_nu; ++k) acc += b[k] * sw[k * kMixTile + p];
    zq[(int64_t)nu * n_s + i] = acc;
  }
}

// y = xs x + sign (1 - eps_i) fq Z, one thread per (nu, V points), looping
// over the ordinates (fq wave-uniform).  RP > 0: the x term is instead
// xs (-Delta) with Delta = sum_q Fp[o][q] zp[q][nu][i], the preconditioner's
// correction (its RP angular modes, the same sum in the same order as the
// preconditioner's expansion, so the same values as reading its v - u = -Delta
// back from memory).
// YT = _Float16 (FP32 only): y is an fp16 basis vector, written as
// ymul times the value, rounded to nearest.
template <typename T, int V>
__device__ __forceinline__ void put_h(_Float16* y, const typename VecOf<T, V>::type& v, T ymul) {
  if constexpr (V == 1) {
    *y = (_Float16)(ymul * v);
  } else {
    typedef _Float16 __attribute__((ext_vector_type(V))) HV;
    HV h;
#pragma unroll
    for (int u = 0; u < V; ++u) h[u] = (_Float16)(ymul * v[u]);
    *reinterpret_cast<HV*>(y) = h;
  }
}

template <typename T, int R, int V, int RP, typename YT = T>
__global__ __launch_bounds__(256) void fsig_expand(const T* __restrict__ Z,
                                                   const T* __restrict__ fq,
                                                   const double* __restrict__ albedo,
                                                   const T* x, YT* y,
                                                   const double* __restrict__ xscale, T sign,
                                                   int n_om, int n_nu, int64_t n_s,
                                                   const T* __restrict__ Fp,
                                                   const T* __restrict__ zp, T ymul = T(1)) {
  using VT = typename VecOf<T, V>::type;
  constexpr bool kHalf = !std::is_same<YT, T>::value;
  const int64_t m = (int64_t)n_nu * n_s;
  const int64_t mv = m / V;
  const T xs = ((x != nullptr || RP > 0) && xscale != nullptr) ? T(*xscale) : T(1);
  const VT* Zv = reinterpret_cast<const VT*>(Z);
  const VT* xv = reinterpret_cast<const VT*>(x);
  const VT* zpv = reinterpret_cast<const VT*>(zp);
  VT* yv = reinterpret_cast<VT*>(y);   // YT = T only
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < mv;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i0 = (e * V) % n_s;     // V points of one ray row
    VT a;
    if constexpr (V == 1) {
      a = sign * T(albedo[i0]);
    } else {
#pragma unroll
      for (int u = 0; u < V; ++u) a[u] = sign * T(albedo[i0 + u]);
    }
    VT z[R];
#pragma unroll
    for (int q = 0; q < R; ++q) z[q] = a * Zv[(int64_t)q * mv + e];
    VT zc[RP > 0 ? RP : 1];
    if constexpr (RP > 0) {
#pragma unroll
      for (int q = 0; q < RP; ++q) zc[q] = zpv[(int64_t)q * mv + e];
    }
    for (int o = 0; o < n_om; ++o) {
      VT s = VT(0);
#pragma unroll
      for (int q = 0; q < R; ++q) s += fq[o * R + q] * z[q];
      const int64_t at = (int64_t)o * mv + e;
      if constexpr (RP > 0) {
        VT d = VT(0);
#pragma unroll
        for (int q = 0; q < RP; ++q) d += Fp[o * RP + q] * zc[q];
        const VT val = xs * (-d) + s;
        if constexpr (kHalf) put_h<T, V>(y + at * V, val, ymul);
        else yv[at] = val;
      } else {
        const VT val = x ? xs * xv[at] + s : s;
        if constexpr (kHalf) put_h<T, V>(y + at * V, val, ymul);
        else yv[at] = val;
      }
    }
  }
}

int stream_grid(int64_t m) {
  const int64_t blocks = (m + 255) / 256;
  return (int)std::min<int64_t>(blocks, 8192);
}

template <typename T, typename YT = T>
void launch_factored(const Problem& p, const T* fq, const T* fg, const T* fb, const T* L,
                     const T* x, YT* y, T* work, const double* xscale, double sign,
                     hipStream_t st, const T* Fp = nullptr, const T* zp = nullptr, int rp = 0,
                     T ymul = T(1)) {
  const int R = p.tab.frank;
  const int n_om = p.n_omega, n_nu = p.n_nu;
  const int64_t n_s = p.n_s, m = (int64_t)n_nu * n_s;
  T* W = work;
  T* Z = work + (size_t)R * m;
  ProfScope prof(sizeof(T) == 8 ? RT_KCLASS_SIGMA : RT_KCLASS_SIGMA_LO, st);
  constexpr int VV = 16 / sizeof(T);
  const bool vec = n_s % VV == 0;
  const int g = stream_grid(vec ? m / VV : m);
#define RT_FSIG(KER, RR, ...)                                                              \
  if (vec) hipLaunchKernelGGL((KER<T, RR, VV>), dim3(g), dim3(256), 0, st, __VA_ARGS__); \
  else hipLaunchKernelGGL((KER<T, RR, 1>), dim3(g), dim3(256), 0, st, __VA_ARGS__)
  if (R == 6) {
    RT_FSIG(fsig_reduce, 6, L, fg, W, n_om, n_nu, n_s);
  } else if (R == 2) {
    RT_FSIG(fsig_reduce, 2, L, fg, W, n_om, n_nu, n_s);
  } else {
    fail(RT_E_INVALID, "factored scattering: unsupported angular rank");
  }
  const int64_t tiles = (n_s + kMixTile - 1) / kMixTile;
  const size_t lds = ((size_t)n_nu * kMixTile + (size_t)n_nu * n_nu) * sizeof(T);
  hipLaunchKernelGGL((fsig_mix<T>), dim3((unsigned)(R * tiles)), dim3(256), lds, st, W, fb, Z,
                     n_nu, n_s, tiles);
#define RT_FSIG_X(RR, PP)                                                                     \
  if (vec)                                                                                    \
    hipLaunchKernelGGL((fsig_expand<T, RR, VV, PP, YT>), dim3(g), dim3(256), 0, st, Z, fq,    \
                       p.d_albedo, x, y, xscale, T(sign), n_om, n_nu, n_s, Fp, zp, ymul);     \
  else                                                                                        \
    hipLaunchKernelGGL((fsig_expand<T, RR, 1, PP, YT>), dim3(g), dim3(256), 0, st, Z, fq,     \
                       p.d_albedo, x, y, xscale, T(sign), n_om, n_nu, n_s, Fp, zp, ymul)
#define RT_FSIG_R(RR)                                   \
  switch (rp) {                                         \
    case 0: RT_FSIG_X(RR, 0); break;                    \
    case 1: RT_FSIG_X(RR, 1); break;                    \
    case 2: RT_FSIG_X(RR, 2); break;                    \
    case 3: RT_FSIG_X(RR, 3); break;                    \
    case 4: RT_FSIG_X(RR, 4); break;                    \
    case 5: RT_FSIG_X(RR, 5); break;                    \
    case 6: RT_FSIG_X(RR, 6); break;                    \
    default: fail(RT_E_INVALID, "preconditioner: mode count"); \
  }
  if (R == 6) {
    RT_FSIG_R(6);
  } else {
    RT_FSIG_R(2);
  }
#undef RT_FSIG_R
#undef RT_FSIG_X
#undef RT_FSIG
  RT_HIP(hipGetLastError());
}

}  // namespace

size_t factored_work_elems(const Problem& p) {
  return (size_t)2 * p.tab.frank * (size_t)p.n_nu * (size_t)p.n_s;
}

// LDS of the mix pass: the tile of W and the frequency block.
bool factored_fits(const Problem& p, int elem_bytes) {
  int max_lds = 0;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p.device) !=
      hipSuccess)
    return false;
  const size_t lds = ((size_t)p.n_nu * kMixTile + (size_t)p.n_nu * p.n_nu) * elem_bytes;
  return p.tab.frank > 0 && p.tab.frank <= kMaxRank && lds <= (size_t)max_lds;
}

void launch_sigma_factored_f64(const Problem& p, const double* L, const double* x, double* y,
                               double* work, const double* xscale, double sign, hipStream_t st) {
  launch_factored<double>(p, p.d_fq64, p.d_fg64, p.d_fb64, L, x, y, work, xscale, sign, st);
}

void launch_sigma_factored_f32(const Problem& p, const float* L, const float* x, float* y,
                               float* work, const double* xscale, double sign, hipStream_t st) {
  launch_factored<float>(p, p.d_fq32, p.d_fg32, p.d_fb32, L, x, y, work, xscale, sign, st);
}

void launch_sigma_factored_pre_f64(const Problem& p, const double* L, const double* Fp,
                                   const double* zp, int rp, double* y, double* work,
                                   const double* xscale, hipStream_t st) {
  launch_factored<double>(p, p.d_fq64, p.d_fg64, p.d_fb64, L, nullptr, y, work, xscale, +1.0, st,
                          Fp, zp, rp);
}

void launch_sigma_factored_pre_f32(const Problem& p, const float* L, const float* Fp,
                                   const float* zp, int rp, float* y, float* work,
                                   const double* xscale, hipStream_t st) {
  launch_factored<float>(p, p.d_fq32, p.d_fg32, p.d_fb32, L, nullptr, y, work, xscale, +1.0, st,
                         Fp, zp, rp);
}

void launch_sigma_factored_pre_h(const Problem& p, const float* L, const float* Fp,
                                 const float* zp, int rp, _Float16* y, float ymul, float* work,
                                 const double* xscale, hipStream_t st) {
  launch_factored<float, _Float16>(p, p.d_fq32, p.d_fg32, p.d_fb32, L, nullptr, y, work, xscale,
                                   +1.0, st, Fp, zp, rp, ymul);
}

}  // namespace rtsn
