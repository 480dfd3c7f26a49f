// Physics-based preconditioner of the source-function system (Sec. 6 remarks
// that physics-based preconditioning can still cut iteration counts; the
// classic physics-based choice keeps the local part of Lambda, as in
// accelerated Lambda iteration).  Here the local part is the response of a
// point to a unit source on its own plane, averaged over directions, and it
// is kept with the point's full scattering block (Sec. 3.3, eq. Sigma):
//
//   Dbar[nu][i] = sum_o w_o (Lambda_0 1_z)[(o, nu), i] / sum_o w_o   (i on plane z)
//   P_i         = Id - (1 - eps_i) Mhat diag_k(Dbar[nu(k)][i])
//
// (with linear short characteristics Lambda_0 1_z restricted to plane z is
// the diagonal of Lambda_0).  GMRES runs on A P^-1 (right preconditioning:
// the residual, and so the stopping test, is that of A x = b).
//
// For the dipole x PRD kernel Mhat = P_A kron P_B with the angular block
// P_A = fq fg^T (rank <= 6) and the frequency block P_B = fb.  P_A is
// similar to the symmetric S = W^1/2 P_A W^-1/2 (W = diag(w_o)); with
// S = U Lam U^T, F = W^-1/2 U and G = W^1/2 U (G^T F = Id) over the nonzero
// eigenvalues,
//   P_i^-1 = Id + sum_q (F_q kron Id) T_iq (G_q^T kron Id),
//   T_iq   = (Id - (1 - eps_i) lam_q P_B diag(Dbar[:, i]))^-1 - Id,
// applied in three passes over the ray-major vectors: reduce r = G^T x over
// the ordinates, the per-point N_nu x N_nu blocks z = T r, and expand
// x + F z.  Set-up: one FP64 formal solution per plane for Dbar, a Jacobi
// eigen-solve of S on the host, and one in-LDS Gauss-Jordan inversion with
// partial pivoting per (point, mode).
#include <algorithm>
#include <type_traits>
#include <cmath>
#include <vector>

#include "rt_internal.h"

namespace rtsn {

namespace {

constexpr int kMaxModes = 6;
constexpr int kMixPts = 64;   // points per mix workgroup

// s[k, i] = v for every ray k and the points i0 .. i0 + P - 1 of one plane
template <typename T>
__global__ __launch_bounds__(256) void plane_fill(T* s, int n_r, int64_t n_s, int64_t i0, int P,
                                                  T v) {
  const int64_t m = (int64_t)n_r * P;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / P);
    s[(int64_t)k * n_s + i0 + (e - (int64_t)k * P)] = v;
  }
}

// dbar[nu][i] = sum_o wbar_o L[(o n_nu + nu), i] for the plane's points
__global__ __launch_bounds__(256) void plane_average(const double* __restrict__ L,
                                                     const double* __restrict__ wbar,
                                                     double* __restrict__ dbar, int n_om,
                                                     int n_nu, int64_t n_s, int64_t i0, int P) {
  const int64_t m = (int64_t)n_nu * P;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int nu = (int)(e / P);
    const int64_t i = i0 + (e - (int64_t)nu * P);
    double a = 0.0;
    for (int o = 0; o < n_om; ++o) a += wbar[o] * L[((int64_t)o * n_nu + nu) * n_s + i];
    dbar[(int64_t)nu * n_s + i] = a;
  }
}

// T[q][i] = (Id - albedo_i lam_q fb diag(dbar[:, i]))^-1 - Id, one wave per
// (q, i): in-place Gauss-Jordan with partial pivoting on the matrix in LDS
// (rows padded to n + 1 doubles), lane r owning rows r and r + 64; the row
// interchanges are undone as column interchanges of the inverse at the end.
template <typename TO>
__global__ __launch_bounds__(64) void build_blocks(const double* __restrict__ fb,
                                                   const double* __restrict__ lam,
                                                   const double* __restrict__ albedo,
                                                   const double* __restrict__ dbar, TO* T, int n,
                                                   int64_t n_s, int64_t first) {
  extern __shared__ double a[];                 // n x (n + 1)
  int* perm = reinterpret_cast<int*>(a + (size_t)n * (n + 1));
  const int ld = n + 1;
  const int lane = threadIdx.x;
  const int64_t item = first + blockIdx.x;      // q * n_s + i
  const int q = (int)(item / n_s);
  const int64_t i = item - (int64_t)q * n_s;
  const double c = albedo[i] * lam[q];
  for (int e = lane; e < n * n; e += 64) {
    const int r = e / n, k = e - r * n;
    a[r * ld + k] = (r == k ? 1.0 : 0.0) - c * fb[e] * dbar[(int64_t)k * n_s + i];
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // pivot: the largest |a[r][k]| over r >= k (ties: the smallest r)
    double best = -1.0;
    int bi = k;
    for (int r = k + lane; r < n; r += 64) {
      const double v = fabs(a[r * ld + k]);
      if (v > best) {
        best = v;
        bi = r;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) perm[k] = bi;
    if (bi != k)
      for (int j = lane; j < n; j += 64) {
        const double t = a[k * ld + j];
        a[k * ld + j] = a[bi * ld + j];
        a[bi * ld + j] = t;
      }
    __syncthreads();
    const double inv = 1.0 / a[k * ld + k];
    double f[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = lane + 64 * h;
      f[h] = (r < n && r != k) ? a[r * ld + k] : 0.0;
    }
    __syncthreads();
    for (int j = lane; j < n; j += 64) a[k * ld + j] = (j == k) ? inv : a[k * ld + j] * inv;
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = lane + 64 * h;
      if (r < n && r != k) {
        for (int j = 0; j < n; ++j)
          if (j != k) a[r * ld + j] -= f[h] * a[k * ld + j];
        a[r * ld + k] = -f[h] * inv;
      }
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int pk = perm[k];
    if (pk != k)
      for (int r = lane; r < n; r += 64) {
        const double t = a[r * ld + k];
        a[r * ld + k] = a[r * ld + pk];
        a[r * ld + pk] = t;
      }
    __syncthreads();
  }
  TO* out = T + (size_t)item * n * n;
  for (int e = lane; e < n * n; e += 64) {
    const int r = e / n, k = e - r * n;
    out[e] = TO(a[r * ld + k] - (r == k ? 1.0 : 0.0));
  }
}

// W consecutive values of T moved as one access: 16 bytes (4 floats or 2
// doubles) in the streaming kernels below, or one value where the arrays do
// not allow it (m not a multiple of the width, or a vector not 16-byte
// aligned).
template <typename T> constexpr int kVec16 = 16 / (int)sizeof(T);

template <typename T, int W>
__device__ __forceinline__ void vload(const T* p, T (&v)[W]) {
  if constexpr (W == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  } else if constexpr (W == 2) {
    const double2 t = *reinterpret_cast<const double2*>(p);
    v[0] = t.x; v[1] = t.y;
  } else {
    v[0] = *p;
  }
}

// 8 fp16 values (16 bytes) widened to T
template <typename T>
__device__ __forceinline__ void vload_h8(const _Float16* p, T (&v)[8]) {
  typedef _Float16 __attribute__((ext_vector_type(8))) H8;
  const H8 t = *reinterpret_cast<const H8*>(p);
#pragma unroll
  for (int w = 0; w < 8; ++w) v[w] = T(t[w]);
}

template <typename T, int W>
__device__ __forceinline__ void vstore(T* p, const T (&v)[W]) {
  if constexpr (W == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  } else if constexpr (W == 2) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
  } else {
    *p = v[0];
  }
}

// r[q][nu][i] = sum_o G[o][q] x[(o n_nu + nu) n_s + i]: each thread takes W
// consecutive entries (m a multiple of W), eight ordinates' loads issued
// together.
// XT: type of x (T, or fp16 basis vectors read one value per thread; four
// per 8-byte load measured no faster: 271 against 261 ms of preconditioner
// per box64 solve).
template <typename T, int RQ, int W, typename XT = T>
__global__ __launch_bounds__(256) void prec_reduce(const XT* __restrict__ x,
                                                   const T* __restrict__ G, T* __restrict__ r,
                                                   int n_om, int64_t m) {
  static_assert(std::is_same<XT, T>::value || W == 1, "converted input: one value per thread");
  const int64_t mv = m / W;
  for (int64_t ev = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; ev < mv;
       ev += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = ev * W;
    T acc[RQ][W];
#pragma unroll
    for (int q = 0; q < RQ; ++q)
#pragma unroll
      for (int w = 0; w < W; ++w) acc[q][w] = T(0);
#pragma unroll 8
    for (int o = 0; o < n_om; ++o) {
      T v[W];
      if constexpr (std::is_same<XT, T>::value) vload<T, W>(x + (int64_t)o * m + e, v);
      else v[0] = T(x[(int64_t)o * m + e]);
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        const T g = G[o * RQ + q];
#pragma unroll
        for (int w = 0; w < W; ++w) acc[q][w] += g * v[w];
      }
    }
#pragma unroll
    for (int q = 0; q < RQ; ++q) vstore<T, W>(r + (int64_t)q * m + e, acc[q]);
  }
}

// z[q][nu][i] = sum_nu' T[q][i][nu][nu'] r[q][nu'][i]: one workgroup per (q,
// tile of kMixPts points) with the tile of r in LDS; thread (point, rows
// nu = t / kMixPts + 4 j).  A lane walks its point's block row by row, so
// each cache line of T is read once.
template <typename T>
__global__ __launch_bounds__(256) void prec_mix(const T* __restrict__ Tb,
                                                const T* __restrict__ r, T* __restrict__ z,
                                                int n_nu, int64_t n_s, int64_t tiles) {
  extern __shared__ unsigned char smem_raw[];
  T* rl = reinterpret_cast<T*>(smem_raw);        // n_nu x kMixPts
  const int q = (int)(blockIdx.x / tiles);
  const int64_t i0 = (blockIdx.x - (int64_t)q * tiles) * kMixPts;
  const int p = threadIdx.x % kMixPts;
  const int64_t i = i0 + p;
  const bool live = i < n_s;
  const int64_t m = (int64_t)n_nu * n_s;
  const T* rq = r + (int64_t)q * m;
  for (int nu = threadIdx.x / kMixPts; nu < n_nu; nu += blockDim.x / kMixPts)
    rl[nu * kMixPts + p] = live ? rq[(int64_t)nu * n_s + i] : T(0);
  __syncthreads();
  if (!live) return;
  const T* tb = Tb + ((int64_t)q * n_s + i) * n_nu * n_nu;
  T* zq = z + (int64_t)q * m;
  for (int nu = threadIdx.x / kMixPts; nu < n_nu; nu += blockDim.x / kMixPts) {
    const T* row = tb + (int64_t)nu * n_nu;
    T acc = T(0);
    for (int k = 0; k < n_nu; ++k) acc += row[k] * rl[k * kMixPts + p];
    zq[(int64_t)nu * n_s + i] = acc;
  }
}

// LDS accesses of one wavefront ordered around a wave barrier.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// The same product, one wavefront per block (q, i): the block's n x n
// values (contiguous) are read by all 64 lanes in 16-byte vectors, VPL per
// lane, all issued before the first is used and none under a branch (a lane
// past the block reloads its last vector; n a multiple of the vector width,
// so that a vector lies in one row), into LDS rows padded to n + 1
// (conflict-free column walks); then lane nu forms row nu against
// r[q][.][i] (broadcast from LDS).  Four wavefronts per group, each with its
// own LDS region of n (n + 1) + n values.  Wavefront k of a pass takes block
// mix_order(k): groups are dealt to the 8 XCDs in turn, each with its own L2,
// and the order puts the 32 consecutive points whose r and z values share a
// 128-byte line on the waves of one XCD, so each line is fetched and
// written back whole by one L2 (in launch order, by eight).
__device__ __forceinline__ int64_t mix_order(int64_t k, int64_t nfull) {
  if (k >= nfull) return k;
  const int64_t base = k & ~(int64_t)255;
  const int g = (int)((k >> 2) & 63), w = (int)(k & 3);   // group in the chunk, wave
  return base + 32 * (g & 7) + 4 * (g >> 3) + w;
}

// TT: type of the stored blocks (T, or fp16 widened to T as it is staged).
template <typename T, int VPL, typename TT = T>
__global__ __launch_bounds__(256) void prec_mix_wave(const TT* __restrict__ Tb,
                                                     const T* __restrict__ r, T* __restrict__ z,
                                                     int n, int64_t n_s, int64_t nblk) {
  constexpr int W = 16 / (int)sizeof(TT);
  extern __shared__ unsigned char smem_raw[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T* L = reinterpret_cast<T*>(smem_raw) + (size_t)wave * (n * (n + 1) + n);
  T* rl = L + n * (n + 1);
  const int64_t m = (int64_t)n * n_s;
  const int nvr = n / W, nv = n * nvr;   // vectors per row, per block
  // row of vector ev: (ev + 1/2) / nvr rounded down, exact in FP32 here
  // (ev < 1024, nvr <= 16: the quotient stays 1/32 away from an integer)
  const float inv_nvr = 1.0f / (float)nvr;
  const int64_t nfull = nblk & ~(int64_t)255;
  const int64_t stride = (int64_t)gridDim.x * 4;
  // software pipeline: the loads of the next block and the store of the
  // previous block's row are issued together, after the wait for this
  // block's loads, so that both have a whole block's work to complete (loads
  // and stores share one wait counter, which is waited down to zero while
  // both are outstanding)
  typedef TT __attribute__((ext_vector_type(W))) RV;   // 16 bytes
  RV raw[VPL];
  T rv;
  auto fetch = [&](int64_t kk) {
    const int64_t bb = mix_order(kk, nfull);
    const int qq = (int)(bb / n_s);
    const int64_t ii = bb - (int64_t)qq * n_s;
    const TT* blk = Tb + (size_t)bb * n * n;
#pragma unroll
    for (int t = 0; t < VPL; ++t)
      raw[t] = *reinterpret_cast<const RV*>(blk + (size_t)min(lane + 64 * t, nv - 1) * W);
    rv = r[(int64_t)qq * m + (int64_t)min(lane, n - 1) * n_s + ii];
  };
  int64_t k = (int64_t)blockIdx.x * 4 + wave;
  if (k >= nblk) return;   // the whole wavefront
  fetch(k);
  int64_t zat = -1;        // where the previous block's row goes
  T zval = T(0);
  for (; k < nblk; k += stride) {
    RV cur[VPL];
#pragma unroll
    for (int t = 0; t < VPL; ++t) cur[t] = raw[t];
    const T rcur = rv;
    if (zat >= 0 && lane < n) z[zat] = zval;
    // the last block reloads itself, which keeps the loads unconditional
    fetch(k + stride < nblk ? k + stride : k);
    const int64_t b = mix_order(k, nfull);
    const int q = (int)(b / n_s);
    const int64_t i = b - (int64_t)q * n_s;
#pragma unroll
    for (int t = 0; t < VPL; ++t) {
      const int ev = lane + 64 * t;
      if (ev < nv) {
        const int row = (int)(((float)ev + 0.5f) * inv_nvr);
        T* dst = L + row * (n + 1) + (ev - row * nvr) * W;
#pragma unroll
        for (int w = 0; w < W; ++w) dst[w] = T(cur[t][w]);
      }
    }
    if (lane < n) rl[lane] = rcur;
    wave_lds_sync();
    if (lane < n) {
      const T* row = L + lane * (n + 1);
      T acc = T(0);
      for (int kk = 0; kk < n; ++kk) acc += row[kk] * rl[kk];
      zval = acc;
      zat = (int64_t)q * m + (int64_t)lane * n_s + i;
    }
    wave_lds_sync();   // the next block overwrites the region
  }
  if (zat >= 0 && lane < n) z[zat] = zval;
}

// Delta[(o, nu), i] = sum_q F[o][q] z[q][nu][i];
//   ACC = false: u = x + Delta and nd = -Delta (u = P^-1 x, nd = x - u);
//   ACC = true:  u += x + Delta (accumulate P^-1 x into u).
// W consecutive entries per thread, as in prec_reduce.
template <typename T, int RQ, bool ACC, int W, typename XT = T>
__global__ __launch_bounds__(256) void prec_expand(const T* __restrict__ z,
                                                   const T* __restrict__ F, const XT* x, T* u,
                                                   T* nd, int n_om, int64_t m) {
  const int64_t mv = m / W;
  for (int64_t ev = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; ev < mv;
       ev += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = ev * W;
    T zv[RQ][W];
#pragma unroll
    for (int q = 0; q < RQ; ++q) vload<T, W>(z + (int64_t)q * m + e, zv[q]);
#pragma unroll 4
    for (int o = 0; o < n_om; ++o) {
      T d[W];
#pragma unroll
      for (int w = 0; w < W; ++w) d[w] = T(0);
#pragma unroll
      for (int q = 0; q < RQ; ++q) {
        const T f = F[o * RQ + q];
#pragma unroll
        for (int w = 0; w < W; ++w) d[w] += f * zv[q][w];
      }
      const int64_t at = (int64_t)o * m + e;
      T xv[W], uv[W];
      if constexpr (std::is_same<XT, T>::value) {
        vload<T, W>(x + at, xv);
      } else if constexpr (W == 1) {
        xv[0] = T(x[at]);
      } else {
        typedef XT __attribute__((ext_vector_type(W))) XV;
        const XV t = *reinterpret_cast<const XV*>(x + at);
#pragma unroll
        for (int w = 0; w < W; ++w) xv[w] = T(t[w]);
      }
      if constexpr (ACC) {
        vload<T, W>(u + at, uv);
#pragma unroll
        for (int w = 0; w < W; ++w) uv[w] += xv[w] + d[w];
        vstore<T, W>(u + at, uv);
      } else {
        T nv[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
          uv[w] = xv[w] + d[w];
          nv[w] = -d[w];
        }
        vstore<T, W>(u + at, uv);
        if (nd) vstore<T, W>(nd + at, nv);   // null: the caller forms v - u itself
      }
    }
  }
}

int grid_for(int64_t m) { return (int)std::min<int64_t>((m + 255) / 256, 8192); }

// Cyclic Jacobi eigen-solve of a symmetric n x n matrix (row-major, in
// place): eigenvalues on the diagonal of a, eigenvectors in the columns of v.
void jacobi_eigen(std::vector<double>& a, std::vector<double>& v, int n) {
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        (i == j ? diag : off) += a[(size_t)i * n + j] * a[(size_t)i * n + j];
    if (off <= 1e-30 * diag) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) /
                         (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {   // rows p, q
          const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
          a[(size_t)k * n + p] = c * akp - s * akq;
          a[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // columns p, q
          const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
          a[(size_t)p * n + k] = c * apk - s * aqk;
          a[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
          v[(size_t)k * n + p] = c * vkp - s * vkq;
          v[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

template <typename T>
T* dcopy(const std::vector<double>& h) {
  std::vector<T> t(h.begin(), h.end());
  void* d = nullptr;
  RT_HIP(hipMalloc(&d, std::max<size_t>(1, t.size()) * sizeof(T)));
  RT_HIP(hipMemcpy(d, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice));
  return static_cast<T*>(d);
}

// angular modes (host): F, G, lam over the nonzero eigenvalues of P_A
void angular_modes(Problem& p) {
  const Tables& t = p.tab;
  const int n_om = p.n_omega, R = t.frank;
  std::vector<double> s((size_t)n_om * n_om), v;
  for (int o = 0; o < n_om; ++o)
    for (int o2 = 0; o2 < n_om; ++o2) {
      double pa = 0.0;   // P_A[o][o2] = sum_a fq[o][a] fg[o2][a]
      for (int a = 0; a < R; ++a) pa += t.fq[(size_t)o * R + a] * t.fg[(size_t)o2 * R + a];
      s[(size_t)o * n_om + o2] = pa * std::sqrt(t.w_o[o] / t.w_o[o2]);
    }
  // symmetrise the rounding of the two products
  for (int o = 0; o < n_om; ++o)
    for (int o2 = o + 1; o2 < n_om; ++o2) {
      const double m = 0.5 * (s[(size_t)o * n_om + o2] + s[(size_t)o2 * n_om + o]);
      s[(size_t)o * n_om + o2] = s[(size_t)o2 * n_om + o] = m;
    }
  jacobi_eigen(s, v, n_om);
  double mx = 0.0;
  for (int o = 0; o < n_om; ++o) mx = std::max(mx, std::fabs(s[(size_t)o * n_om + o]));
  p.prec_lam.clear();
  std::vector<int> keep;
  for (int o = 0; o < n_om; ++o)
    if (std::fabs(s[(size_t)o * n_om + o]) > 1e-12 * mx) keep.push_back(o);
  if ((int)keep.size() > kMaxModes)
    fail(RT_E_INVALID, "preconditioner: angular block of rank above six");
  const int rq = (int)keep.size();
  p.prec_rq = rq;
  p.prec_F.assign((size_t)n_om * rq, 0.0);
  p.prec_G.assign((size_t)n_om * rq, 0.0);
  for (int q = 0; q < rq; ++q) {
    p.prec_lam.push_back(s[(size_t)keep[q] * n_om + keep[q]]);
    for (int o = 0; o < n_om; ++o) {
      const double u = v[(size_t)o * n_om + keep[q]];
      const double sw = std::sqrt(t.w_o[o]);
      p.prec_F[(size_t)o * rq + q] = u / sw;
      p.prec_G[(size_t)o * rq + q] = u * sw;
    }
  }
}

// Dbar by one FP64 formal solution per plane of a unit source on that plane
void build_dbar(Problem& p, hipStream_t st) {
  const int64_t n = p.n, n_s = p.n_s;
  const int P = p.geom == RT_GEOM_BOX ? p.nx * p.ny : 1;
  const int planes = (int)(n_s / P);
  double* s = nullptr;
  RT_HIP(hipMalloc(&s, (size_t)n * sizeof(double)));
  double* L = static_cast<double*>(problem_lbuf(p, (size_t)n * sizeof(double)));
  if (!p.d_prec_dbar) RT_HIP(hipMalloc(&p.d_prec_dbar, (size_t)p.n_nu * n_s * sizeof(double)));
  double wsum = 0.0;
  for (double w : p.tab.w_o) wsum += w;
  std::vector<double> wb(p.tab.w_o);
  for (double& w : wb) w /= wsum;
  double* d_wb = dcopy<double>(wb);
  RT_HIP(hipMemsetAsync(s, 0, (size_t)n * sizeof(double), st));
  const int gf = grid_for((int64_t)p.n_r * P), ga = grid_for((int64_t)p.n_nu * P);
  for (int z = 0; z < planes; ++z) {
    const int64_t i0 = (int64_t)z * P;
    hipLaunchKernelGGL(plane_fill<double>, dim3(gf), dim3(256), 0, st, s, p.n_r, n_s, i0, P, 1.0);
    launch_lambda<double, double>(p, s, L, false, nullptr, st);
    hipLaunchKernelGGL(plane_average, dim3(ga), dim3(256), 0, st, L, d_wb, p.d_prec_dbar,
                       p.n_omega, p.n_nu, n_s, i0, P);
    hipLaunchKernelGGL(plane_fill<double>, dim3(gf), dim3(256), 0, st, s, p.n_r, n_s, i0, P, 0.0);
  }
  RT_HIP(hipGetLastError());
  RT_HIP(hipStreamSynchronize(st));
  RT_HIP(hipFree(s));
  RT_HIP(hipFree(d_wb));
}

template <typename TO>
void build_T(Problem& p, TO** out, hipStream_t st) {
  const int n = p.n_nu, rq = p.prec_rq;
  const int64_t items = (int64_t)rq * p.n_s;
  RT_HIP(hipMalloc((void**)out, (size_t)items * n * n * sizeof(TO)));
  double* d_fb = dcopy<double>(p.tab.fb);
  double* d_lam = dcopy<double>(p.prec_lam);
  const size_t lds = (size_t)n * (n + 1) * sizeof(double) + (size_t)n * sizeof(int) + 16;
  // launches of at most 2^20 workgroups
  for (int64_t f = 0; f < items; f += (int64_t)1 << 20) {
    const int64_t cnt = std::min<int64_t>(items - f, (int64_t)1 << 20);
    hipLaunchKernelGGL((build_blocks<TO>), dim3((unsigned)cnt), dim3(64), lds, st, d_fb, d_lam,
                       p.d_albedo, p.d_prec_dbar, *out, n, p.n_s, f);
  }
  RT_HIP(hipGetLastError());
  RT_HIP(hipStreamSynchronize(st));
  RT_HIP(hipFree(d_fb));
  RT_HIP(hipFree(d_lam));
}

template <typename T> struct PrecPtrs;
template <> struct PrecPtrs<double> {
  static double* F(Problem& p) { return p.d_prec_F64; }
  static double* G(Problem& p) { return p.d_prec_G64; }
  static double* T(Problem& p) { return p.d_prec_T64; }
};
template <> struct PrecPtrs<float> {
  static float* F(Problem& p) { return p.d_prec_F32; }
  static float* G(Problem& p) { return p.d_prec_G32; }
  static float* T(Problem& p) { return p.d_prec_T32; }
};

template <typename T>
T* work_rz(Problem& p) {
  return static_cast<T*>(p.d_prec_work);
}

// half: take the fp16 copy of the FP32 blocks where it exists (the solves
// on fp16 bases)
template <typename T, bool ACC, typename XT = T>
void apply_impl(Problem& p, const XT* x, T* u, T* nd, hipStream_t st, bool half = false) {
  using PP = PrecPtrs<T>;
  if (!PP::T(p)) fail(RT_E_INVALID, "preconditioner not prepared in this precision");
  const int rq = p.prec_rq, n_om = p.n_omega, n_nu = p.n_nu;
  const int64_t n_s = p.n_s, m = (int64_t)n_nu * n_s;
  T* r = work_rz<T>(p);
  T* z = r + (size_t)rq * m;
  ProfScope prof(RT_KCLASS_PRECOND, st);
  // 16-byte accesses where every vector allows them
  constexpr int WV = kVec16<T>;
  auto al = [](const void* q) { return q == nullptr || ((uintptr_t)q & 15) == 0; };
  const bool vec = std::is_same<XT, T>::value && m % WV == 0 && al(x) && al(u) && al(r);
  const int g = grid_for(vec ? m / WV : m);
  // the expansion runs one value per thread: 16-byte accesses measured
  // slower there (box64, FP32: 3.89 against 3.75 ms)
  const int ge = grid_for(m);
#define RT_PREC_RQ(RR)                                                                           \
  case RR:                                                                                       \
    if (vec)                                                                                     \
      hipLaunchKernelGGL((prec_reduce<T, RR, std::is_same<XT, T>::value ? WV : 1, XT>), dim3(g), \
                         dim3(256), 0, st, x, PP::G(p), r, n_om, m);                             \
    else                                                                                         \
      hipLaunchKernelGGL((prec_reduce<T, RR, 1, XT>), dim3(g), dim3(256), 0, st, x, PP::G(p), r, \
                         n_om, m);                                                               \
    break;
  switch (rq) {
    RT_PREC_RQ(1) RT_PREC_RQ(2) RT_PREC_RQ(3) RT_PREC_RQ(4) RT_PREC_RQ(5) RT_PREC_RQ(6)
    default: fail(RT_E_INVALID, "preconditioner: mode count");
  }
#undef RT_PREC_RQ
  const size_t wave_lds = 4 * ((size_t)n_nu * (n_nu + 1) + n_nu) * sizeof(T);
  // vectors per lane of the wavefront product: 4, 9 or 16
  const int vpl = (int)(((int64_t)n_nu * n_nu / kVec16<T> + 63) / 64);
  // FP32 tables only (FP64 on the 32^3 box: 22.4 against 20.8 ms of
  // preconditioner per solve with the point-tile product)
  const bool wave_mix = sizeof(T) == 4 && n_nu <= 64 && n_nu % kVec16<T> == 0 && vpl <= 16 &&
                        wave_lds <= 65536;
  // the fp16 blocks: 8 values per 16-byte vector, so n_nu a multiple of 8
  const bool h16 = half && sizeof(T) == 4 && p.d_prec_T16 && n_nu % 8 == 0 && n_nu <= 64 &&
                   wave_lds <= 65536;
  if (h16) {
    const int64_t nblk = (int64_t)rq * n_s;
    const int grid = (int)std::min<int64_t>((nblk + 3) / 4, 4096);
    const int vph = (int)(((int64_t)n_nu * n_nu / 8 + 63) / 64);   // 2, 5 or 8 at 32, 48, 64
#define RT_MIXH(V)                                                                            \
  hipLaunchKernelGGL((prec_mix_wave<T, V, _Float16>), dim3(grid), dim3(256), wave_lds, st,    \
                     p.d_prec_T16, r, z, n_nu, n_s, nblk)
    if (vph <= 2) RT_MIXH(2);
    else if (vph <= 5) RT_MIXH(5);
    else RT_MIXH(8);
#undef RT_MIXH
  } else if (wave_mix) {
    const int64_t nblk = (int64_t)rq * n_s;
    // a multiple of 64 groups keeps every pass on whole 256-wave chunks
    const int grid = (int)std::min<int64_t>((nblk + 3) / 4, 4096);
#define RT_MIX(V)                                                                            \
  hipLaunchKernelGGL((prec_mix_wave<T, V>), dim3(grid), dim3(256), wave_lds, st, PP::T(p), r, \
                     z, n_nu, n_s, nblk)
    if (vpl <= 4) RT_MIX(4);
    else if (vpl <= 9) RT_MIX(9);
    else RT_MIX(16);
#undef RT_MIX
  } else {
    const int64_t tiles = (n_s + kMixPts - 1) / kMixPts;
    hipLaunchKernelGGL((prec_mix<T>), dim3((unsigned)(rq * tiles)), dim3(256),
                       (size_t)n_nu * kMixPts * sizeof(T), st, PP::T(p), r, z, n_nu, n_s, tiles);
  }
  // fp16 input: 4 values per thread (8-byte loads, 16-byte stores of u),
  // where x and u allow it
  constexpr bool kHalfIn = !std::is_same<XT, T>::value && sizeof(T) == 4;
  const bool vh = kHalfIn && !ACC && nd == nullptr && m % 4 == 0 &&
                  ((uintptr_t)x & 7) == 0 && ((uintptr_t)u & 15) == 0;
#define RT_PREC_RQ(RR)                                                                       \
  case RR:                                                                                   \
    if (vh)                                                                                  \
      hipLaunchKernelGGL((prec_expand<T, RR, ACC, kHalfIn ? 4 : 1, XT>),                     \
                         dim3(grid_for(m / 4)), dim3(256), 0, st, z, PP::F(p), x, u, nd,     \
                         n_om, m);                                                           \
    else                                                                                     \
      hipLaunchKernelGGL((prec_expand<T, RR, ACC, 1, XT>), dim3(ge), dim3(256), 0, st, z,    \
                         PP::F(p), x, u, nd, n_om, m);                                       \
    break;
  switch (rq) {
    RT_PREC_RQ(1) RT_PREC_RQ(2) RT_PREC_RQ(3) RT_PREC_RQ(4) RT_PREC_RQ(5) RT_PREC_RQ(6)
    default: fail(RT_E_INVALID, "preconditioner: mode count");
  }
#undef RT_PREC_RQ
  RT_HIP(hipGetLastError());
}

}  // namespace

size_t precond_table_bytes(const Problem& p, int elem_bytes) {
  const int rq = p.tab.frank;   // an upper bound before the eigen-solve
  return (size_t)rq * p.n_s * p.n_nu * p.n_nu * elem_bytes +
         (size_t)p.n_nu * p.n_s * sizeof(double) +
         (size_t)(2 * rq * (size_t)p.n_nu * p.n_s + 2 * (size_t)p.n) * elem_bytes;
}

void precond_check(const Problem& p) {
  if (p.tab.frank == 0 || p.n_classes > 1)
    fail(RT_E_INVALID, "the preconditioner needs the dipole x PRD kernel, one for all points");
  int max_lds = 0;
  RT_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p.device));
  if ((size_t)p.n_nu * (p.n_nu + 1) * sizeof(double) + (size_t)p.n_nu * sizeof(int) + 16 >
      (size_t)max_lds)
    fail(RT_E_INVALID, "preconditioner: too many frequencies for the in-LDS block inversion");
}

void precond_prepare_local(Problem& p, hipStream_t st) {
  precond_check(p);
  if (p.prec_rq == 0) {
    angular_modes(p);
    p.d_prec_F64 = dcopy<double>(p.prec_F);
    p.d_prec_G64 = dcopy<double>(p.prec_G);
    p.d_prec_F32 = dcopy<float>(p.prec_F);
    p.d_prec_G32 = dcopy<float>(p.prec_G);
  }
  if (!p.d_prec_dbar) build_dbar(p, st);
}

void precond_prepare(Problem& p, int elem_bytes, hipStream_t st) {
  if (elem_bytes != 8 && elem_bytes != 4) fail(RT_E_INVALID, "preconditioner precision");
  precond_prepare_local(p, st);
  if (elem_bytes == 8 && !p.d_prec_T64) build_T<double>(p, &p.d_prec_T64, st);
  if (elem_bytes == 4 && !p.d_prec_T32) build_T<float>(p, &p.d_prec_T32, st);
  // work: r and z (rq n_nu n_s each) and the u / nd vectors, in the wider type
  const size_t bytes = (size_t)(2 * (size_t)p.prec_rq * p.n_nu * p.n_s + 2 * (size_t)p.n) *
                       (p.d_prec_T64 ? 8 : 4);
  if (bytes > p.prec_work_bytes) {
    hipFree(p.d_prec_work);
    p.d_prec_work = nullptr;
    p.prec_work_bytes = 0;
    RT_HIP(hipMalloc(&p.d_prec_work, bytes));
    p.prec_work_bytes = bytes;
  }
}

template <typename T>
T* precond_u(Problem& p) {
  return work_rz<T>(p) + 2 * (size_t)p.prec_rq * p.n_nu * p.n_s;
}
template <typename T>
T* precond_nd(Problem& p) {
  return precond_u<T>(p) + (size_t)p.n;
}

template <typename T>
void precond_apply(Problem& p, const T* x, T* u, T* nd, hipStream_t st) {
  apply_impl<T, false>(p, x, u, nd, st);
}

bool precond_fused(const Problem& p, int precision) {
  return (precision == RT_PREC_FP64 || precision == RT_PREC_FP32) &&
         p.sigma_form == RT_SIGMA_FACTORED && p.n_classes <= 1;
}

template <typename T>
const T* precond_modes_F(Problem& p) {
  return PrecPtrs<T>::F(p);
}
template <typename T>
const T* precond_modes_z(Problem& p) {
  return work_rz<T>(p) + (size_t)p.prec_rq * p.n_nu * p.n_s;
}
template const double* precond_modes_F<double>(Problem&);
template const float* precond_modes_F<float>(Problem&);
template const double* precond_modes_z<double>(Problem&);
template const float* precond_modes_z<float>(Problem&);

template <typename T>
void precond_apply_add(Problem& p, const T* d, T* y, hipStream_t st) {
  apply_impl<T, true>(p, d, y, nullptr, st);
}

void precond_apply_h(Problem& p, const _Float16* x, float* u, hipStream_t st) {
  apply_impl<float, false, _Float16>(p, x, u, nullptr, st, true);
}

void precond_apply_add_h(Problem& p, const float* d, float* y, hipStream_t st) {
  apply_impl<float, true>(p, d, y, nullptr, st, true);
}

__global__ __launch_bounds__(256) void t16_convert(const float* __restrict__ a,
                                                   _Float16* __restrict__ h, int64_t count,
                                                   unsigned* __restrict__ bad) {
  unsigned any = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float v = a[e];
    any |= !(fabsf(v) <= 65504.0f);   // out of fp16's range, or not finite
    h[e] = (_Float16)v;
  }
  if (any) atomicOr(bad, 1u);
}

void precond_prepare_h(Problem& p, hipStream_t st) {
  precond_prepare(p, 4, st);
  if (p.d_prec_T16 || p.prec_t16_tried) return;
  p.prec_t16_tried = true;
  const int64_t count = (int64_t)p.prec_rq * p.n_s * p.n_nu * p.n_nu;
  _Float16* h = nullptr;
  unsigned* bad = nullptr;
  RT_HIP(hipMalloc(&h, (size_t)count * sizeof(_Float16)));
  RT_HIP(hipMalloc(&bad, sizeof(unsigned)));
  RT_HIP(hipMemsetAsync(bad, 0, sizeof(unsigned), st));
  hipLaunchKernelGGL(t16_convert, dim3(grid_for(count)), dim3(256), 0, st, p.d_prec_T32, h,
                     count, bad);
  RT_HIP(hipGetLastError());
  unsigned hb = 0;
  RT_HIP(hipMemcpyAsync(&hb, bad, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  RT_HIP(hipStreamSynchronize(st));
  hipFree(bad);
  if (hb) hipFree(h);   // an entry outside fp16: keep the FP32 blocks
  else p.d_prec_T16 = h;
}

template double* precond_u<double>(Problem&);
template float* precond_u<float>(Problem&);
template double* precond_nd<double>(Problem&);
template float* precond_nd<float>(Problem&);
template void precond_apply<double>(Problem&, const double*, double*, double*, hipStream_t);
template void precond_apply<float>(Problem&, const float*, float*, float*, hipStream_t);
template void precond_apply_add<double>(Problem&, const double*, double*, hipStream_t);
template void precond_apply_add<float>(Problem&, const float*, float*, hipStream_t);

}  // namespace rtsn
