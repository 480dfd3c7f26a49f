// FP64 scattering GEMM emulated with exact int8 matrix-core products: the
// error-free splitting of Ozaki et al. in its integer-modular form (Ozaki,
// Uchino and Imamura, "Ozaki Scheme II: a GEMM-oriented emulation of
// floating-point matrix multiplication using an integer modular technique").
// Not a passage of the radiative-transfer paper: a published method for the
// same product y = xs x + sign (1 - eps) Mhat L (Sec. 3.3, eq. Sigma).
//
//   1. Scale each row k of Mhat by 2^ea_k and each column i of L by 2^fb_i so
//      that their entries round to integers A', B' of at most kBits bits
//      (Mhat once per problem, L per call).
//   2. For each modulus m_l of a set of pairwise coprime moduli <= 256 whose
//      product M exceeds 2 K 2^(2 kBits), take the residues of A' and B' as
//      int8 and form C_l = A'_l B'_l on the int8 MFMA (int32 accumulation,
//      exact while K 128^2 < 2^31); keep C_l mod m_l.
//   3. The Chinese remainder theorem gives A' B' mod M exactly, hence A' B'
//      itself (|A' B'| < M / 2); scaling back by 2^-(ea_k + fb_i) gives the
//      product with only the rounding of step 1 (relative 2^-kBits of a row's
//      and a column's largest entry) and of the final conversion to FP64.
//
// Residue operands use the 16-bit GEMM's layouts with each 16-bit element
// holding two consecutive int8 k values (gemm16_dev.h, MODE_I8).
#include <cmath>
#include <vector>

#include "gemm16_dev.h"

namespace rtsn {

namespace {

using namespace g16;

constexpr int kMods = 15;
// pairwise coprime: 2^8, 3*5*17, 11*23, 251, 13*19, 241, 239, 233, 229, 227,
// 223, 7*31, 211, 199, 197; product about 2^117.8
constexpr int kMod[kMods] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217,
                             211, 199, 197};
// integer bits of the scaled operands: |A' B'| <= K 2^102 < 2^116 < M / 2 for
// K <= 2^14 (n_rays <= 16384)
constexpr int kBits = 51;

typedef unsigned __int128 u128;

// Tables of Garner's mixed-radix reconstruction, with P_l = m_0 ... m_{l-1}:
// pmod[j][l] = P_j mod m_l (j < l) and pinv[l] = P_l^-1 mod m_l.
constexpr int inv_mod(int a, int m) {
  a %= m;
  for (int t = 1; t < m; ++t)
    if ((a * t) % m == 1) return t;
  return 0;
}
struct GarnerTable {
  int pmod[kMods][kMods];
  int pinv[kMods];
  constexpr GarnerTable() : pmod{}, pinv{} {
    for (int l = 0; l < kMods; ++l) {
      int pl = 1 % kMod[l];                      // P_j mod m_l, j = 0, 1, ...
      for (int j = 0; j < l; ++j) {
        pmod[j][l] = pl;
        pl = (pl * kMod[j]) % kMod[l];
      }
      pinv[l] = inv_mod(pl, kMod[l]);
    }
  }
};
constexpr GarnerTable kGarner{};

struct Crt {
  uint64_t m_lo, m_hi;   // M = product of the moduli
};

Crt make_crt() {
  u128 M = 1;
  for (int l = 0; l < kMods; ++l) M *= (u128)kMod[l];
  return Crt{(uint64_t)M, (uint64_t)(M >> 64)};
}

// signed residue of v mod m in [-128, 127] (m <= 256)
__host__ __device__ __forceinline__ int sres(int64_t v, int m) {
  int r = (int)(v % m);
  if (r < 0) r += m;
  return r >= 128 ? r - m : r;
}

// The same for |v| <= 2^51 in 32-bit arithmetic: v = h 2^34 + c 2^17 + l with
// 0 <= c, l < 2^17 and |h| <= 2^17, so v = h (2^34 mod m) + c (2^17 mod m) + l
// (mod m), a sum below 2^26 in magnitude made non-negative by adding 2^18 m.
struct Limbs {
  int h, c, l;
};
__device__ __forceinline__ Limbs limbs_of(int64_t v) {
  return Limbs{(int)(v >> 34), (int)((v >> 17) & 0x1ffff), (int)(v & 0x1ffff)};
}
template <int M>
__device__ __forceinline__ int sres_limbs(Limbs v) {
  constexpr int c2 = (int)((1LL << 34) % M), c1 = (1 << 17) % M;
  const uint32_t s = (uint32_t)(v.h * c2 + v.c * c1 + v.l + (M << 18));
  const int r = (int)(s % (uint32_t)M);
  return r >= 128 ? r - M : r;
}

constexpr int kNoExp = -(1 << 30);

__global__ __launch_bounds__(256) void oz_fill(int* a, int64_t n, int v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// Column exponents: pe_i = max over k of the binary exponent p of L[k, i]
// (|L[k, i]| < 2^p), kNoExp for an all-zero column.  Threads over points,
// blockIdx.y over chunks of rows, combined with atomicMax.
__global__ __launch_bounds__(256) void oz_colexp(const double* __restrict__ L, int* pe, int n_r,
                                                 int64_t n_s, int rows_per_chunk) {
  const int k0 = blockIdx.y * rows_per_chunk;
  const int k1 = min(n_r, k0 + rows_per_chunk);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_s;
       i += (int64_t)gridDim.x * blockDim.x) {
    double mx = 0.0;
    for (int k = k0; k < k1; ++k) mx = fmax(mx, fabs(L[(int64_t)k * n_s + i]));
    if (mx > 0.0) {
      int p = 0;
      (void)frexp(mx, &p);
      atomicMax(pe + i, p);
    }
  }
}

__device__ __forceinline__ int col_shift(int pe) { return pe == kNoExp ? 0 : kBits - pe; }

// B'_l residues in the k4-virtual int8 layout: byte ((k / 8) Np + i) 8 + k % 8
// of part l.  One thread per (group of 8 k, point i).
template <int L0>
__device__ __forceinline__ void store_residues(uint8_t* dst, int64_t part, const Limbs (&b)[8]) {
  if constexpr (L0 < kMods) {
    constexpr int M = kMod[L0];
    uint32_t w0 = 0, w1 = 0;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      w0 |= (uint32_t)(uint8_t)(int8_t)sres_limbs<M>(b[kk]) << (8 * kk);
      w1 |= (uint32_t)(uint8_t)(int8_t)sres_limbs<M>(b[kk + 4]) << (8 * kk);
    }
    *reinterpret_cast<uint2*>(dst + (int64_t)L0 * part) = make_uint2(w0, w1);
    store_residues<L0 + 1>(dst, part, b);
  }
}

__global__ __launch_bounds__(256) void oz_split_b(const double* __restrict__ L,
                                                  const int* __restrict__ pe, uint8_t* Bres,
                                                  int n_r, int64_t n_s, int64_t Np, int kg8,
                                                  int64_t part) {
  const int64_t m = (int64_t)kg8 * n_s;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(e / n_s);
    const int64_t i = e - (int64_t)g * n_s;
    const int f = col_shift(pe[i]);
    Limbs b[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = 8 * g + kk;
      const double v = k < n_r ? L[(int64_t)k * n_s + i] : 0.0;
      b[kk] = limbs_of((int64_t)rint(ldexp(v, f)));   // |b| <= 2^51
    }
    store_residues<0>(Bres + ((int64_t)g * Np + i) * 8, part, b);
  }
}

// y = xs x + sign (1 - eps_i) 2^-(ea_k + fb_i) CRT(c_0 .. c_14) for V
// consecutive elements of one ray row per thread.  Garner's algorithm gives
// mixed-radix digits v_l in [0, m_l) with A' B' mod M = sum_l v_l P_l:
//   v_l = (c_l - sum_{j<l} v_j (P_j mod m_l)) P_l^-1 mod m_l,
// the inner sum in plain 32-bit integers (below 2^20) and one reduction per
// digit.  The value is then assembled as X_lo + P_8 X_hi from two 64-bit
// Horner sums over digits 0..7 and 8..14; the centred representative (above
// M / 2 means negative) is A' B' itself.
template <int V>
__device__ __forceinline__ void garner_digits(const uint8_t* __restrict__ Cres, int64_t part,
                                              int64_t e, uint32_t (&v)[kMods][V]) {
#pragma unroll
  for (int l = 0; l < kMods; ++l) {
    uint32_t c[V];
    if constexpr (V == 4) {
      const uint32_t w = *reinterpret_cast<const uint32_t*>(Cres + (int64_t)l * part + e);
#pragma unroll
      for (int u = 0; u < 4; ++u) c[u] = (w >> (8 * u)) & 0xffu;
    } else {
      c[0] = Cres[(int64_t)l * part + e];
    }
    constexpr uint32_t bias = 8192u;   // 8192 m_l > 14 * 255^2 >= the inner sum
#pragma unroll
    for (int u = 0; u < V; ++u) {
      uint32_t sum = 0;
#pragma unroll
      for (int j = 0; j < l; ++j) sum += v[j][u] * (uint32_t)kGarner.pmod[j][l];
      const uint32_t t = c[u] + bias * (uint32_t)kMod[l] - sum;
      v[l][u] = (t * (uint32_t)kGarner.pinv[l]) % (uint32_t)kMod[l];
    }
  }
}

__device__ __forceinline__ double crt_value(const uint32_t (&d)[kMods], Crt c, uint64_t p8) {
  uint64_t lo = d[7], hi = d[kMods - 1];
#pragma unroll
  for (int l = 6; l >= 0; --l) lo = lo * (uint64_t)kMod[l] + d[l];
#pragma unroll
  for (int l = kMods - 2; l >= 8; --l) hi = hi * (uint64_t)kMod[l] + d[l];
  const u128 M = ((u128)c.m_hi << 64) | c.m_lo;
  const u128 r = (u128)hi * p8 + lo;
  const bool neg = r > (M >> 1);
  const u128 mag = neg ? M - r : r;
  const double val = ldexp((double)(uint64_t)(mag >> 64), 64) + (double)(uint64_t)mag;
  return neg ? -val : val;
}

template <int V>
__global__ __launch_bounds__(256) void oz_crt(const uint8_t* __restrict__ Cres, int64_t part,
                                              const int* __restrict__ ea,
                                              const int* __restrict__ fb,
                                              const double* __restrict__ albedo, const double* x,
                                              double* y, const double* __restrict__ xscale,
                                              double sign, int64_t n_s, Crt c, uint64_t p8) {
  const int64_t nv = part / V;
  const double xs = (x != nullptr && xscale != nullptr) ? *xscale : 1.0;
  for (int64_t ev = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; ev < nv;
       ev += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = ev * V;
    uint32_t v[kMods][V];
    garner_digits<V>(Cres, part, e, v);
    const int k = (int)(e / n_s);
    const int64_t i = e - (int64_t)k * n_s;    // V points of ray k
#pragma unroll
    for (int u = 0; u < V; ++u) {
      uint32_t d[kMods];
#pragma unroll
      for (int l = 0; l < kMods; ++l) d[l] = v[l][u];
      const double val = ldexp(crt_value(d, c, p8), -(ea[k] + col_shift(fb[i + u])));
      const double t = sign * albedo[i + u] * val;
      y[e + u] = x ? xs * x[e + u] + t : t;
    }
  }
}

int grid_of(int64_t m) { return (int)std::min<int64_t>((m + 255) / 256, 16384); }

template <int MODE, typename C>
__global__ __launch_bounds__(C::NT) void oz_gemm_kernel(const uint16_t* __restrict__ A, int Mp,
                                                        const uint16_t* __restrict__ B, int Np,
                                                        int K4p, uint8_t* Y, int M, int N,
                                                        int imod) {
  __shared__ __align__(16) uint8_t lds[C::template lds_bytes<MODE>()];
  const int Mt = Mp / C::BM;
  int tm, tn;
  if (!tile_of(blockIdx.x, Mt, (N + C::BN - 1) / C::BN, 8, tm, tn)) return;
  tile<MODE, C, false, uint8_t>(A, nullptr, Mp, B, nullptr, Np, K4p, nullptr, Y, nullptr, nullptr,
                                1.f, 1.f, 1.f, M, N, tm * C::BM, tn * C::BN, lds, {}, 0, 1.f,
                                imod);
}

using OzCfg = Cfg<128, 128, 2, 2, 32, true>;

}  // namespace

// Kv: virtual (int8-pair) K of the residue operands, a multiple of 64.
static int oz_kv(const Problem& p) { return (int)round_up((p.n_r + 1) / 2, 64); }

void ozaki_prepare(Problem& p) {
  if (p.d_oz_a) return;
  const int n_r = p.n_r, Mp = p.mp16, Kv = oz_kv(p);
  const size_t part = (size_t)Mp * Kv;   // uint16 elements per modulus
  std::vector<uint16_t> a((size_t)kMods * part, 0);
  std::vector<int> ea(Mp, 0);
  for (int k = 0; k < n_r; ++k) {
    double mx = 0.0;
    for (int kp = 0; kp < n_r; ++kp) mx = std::max(mx, std::fabs(p.tab.mhat[(size_t)k * n_r + kp]));
    int e = 0;
    if (mx > 0.0) (void)std::frexp(mx, &e);
    ea[k] = mx > 0.0 ? kBits - e : 0;
    for (int kp = 0; kp < n_r; ++kp) {
      const int64_t v = (int64_t)std::nearbyint(std::ldexp(p.tab.mhat[(size_t)k * n_r + kp], ea[k]));
      const int kv = kp / 2;
      const size_t at = ((size_t)(kv / 8) * Mp + k) * 8 + kv % 8;
      for (int l = 0; l < kMods; ++l) {
        const uint16_t byte = (uint8_t)(int8_t)sres(v, kMod[l]);
        a[(size_t)l * part + at] |= (uint16_t)(byte << (8 * (kp % 2)));
      }
    }
  }
  int64_t tot = 0;
  void* d = nullptr;
  RT_HIP(hipMalloc(&d, a.size() * sizeof(uint16_t)));
  RT_HIP(hipMemcpy(d, a.data(), a.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
  p.d_oz_a = static_cast<uint16_t*>(d);
  tot += (int64_t)(a.size() * sizeof(uint16_t));
  RT_HIP(hipMalloc(&d, ea.size() * sizeof(int)));
  RT_HIP(hipMemcpy(d, ea.data(), ea.size() * sizeof(int), hipMemcpyHostToDevice));
  p.d_oz_ea = static_cast<int*>(d);
  p.bytes_problem += tot + (int64_t)(ea.size() * sizeof(int));
}

size_t ozaki_work_bytes(const Problem& p) {
  const size_t kv = (size_t)oz_kv(p);
  return (size_t)p.n_s * sizeof(int) + 256 +                 // column scales
         (size_t)kMods * 2 * kv * (size_t)p.np16 +            // B residues
         (size_t)kMods * (size_t)p.n_r * (size_t)p.n_s;       // C residues
}

void launch_sigma_ozaki(const Problem& p, const double* L, const double* x, double* y,
                        void* work, const double* xscale, double sign, hipStream_t st) {
  static const Crt crt = make_crt();
  const int n_r = p.n_r;
  const int64_t n_s = p.n_s;
  const int Kv = oz_kv(p);
  const int64_t Np = p.np16;
  uint8_t* w8 = static_cast<uint8_t*>(work);
  int* fb = reinterpret_cast<int*>(w8);
  uint8_t* Bres = w8 + round_up((int64_t)n_s * sizeof(int), 256);
  const int64_t bpart = 2 * (int64_t)Kv * Np;   // bytes per modulus
  uint8_t* Cres = Bres + kMods * bpart;
  const int64_t cpart = (int64_t)n_r * n_s;
  ProfScope prof(RT_KCLASS_SIGMA, st);
  hipLaunchKernelGGL(oz_fill, dim3(grid_of(n_s)), dim3(256), 0, st, fb, n_s, kNoExp);
  const int chunks = std::max(1, std::min(64, n_r / 64));
  hipLaunchKernelGGL(oz_colexp, dim3(grid_of(n_s), chunks), dim3(256), 0, st, L, fb, n_r, n_s,
                     (n_r + chunks - 1) / chunks);
  const int kg8 = 2 * Kv / 8;
  hipLaunchKernelGGL(oz_split_b, dim3(grid_of((int64_t)kg8 * n_s)), dim3(256), 0, st, L, fb,
                     Bres, n_r, n_s, Np, kg8, bpart);
  const int Mt = p.mp16 / OzCfg::BM, Nt = (int)((n_s + OzCfg::BN - 1) / OzCfg::BN);
  if ((int64_t)Nt * OzCfg::BN > Np || (Kv / 4) % (OzCfg::BK / 4))
    fail(RT_E_INVALID, "emulated FP64 GEMM: operand padding does not fit the tile");
  const int grid = 8 * ((Mt * Nt + 7) / 8);
  const size_t apart = (size_t)p.mp16 * Kv;
  for (int l = 0; l < kMods; ++l)
    hipLaunchKernelGGL((oz_gemm_kernel<MODE_I8, OzCfg>), dim3(grid), dim3(OzCfg::NT), 0, st,
                       p.d_oz_a + l * apart, p.mp16,
                       reinterpret_cast<const uint16_t*>(Bres + l * bpart), (int)Np, Kv / 4,
                       Cres + l * cpart, n_r, (int)n_s, kMod[l]);
  static const uint64_t p8 = [] {
    uint64_t q = 1;
    for (int l = 0; l < 8; ++l) q *= (uint64_t)kMod[l];
    return q;
  }();
  if (n_s % 4 == 0)
    hipLaunchKernelGGL((oz_crt<4>), dim3(grid_of(cpart / 4)), dim3(256), 0, st, Cres, cpart,
                       p.d_oz_ea, fb, p.d_albedo, x, y, xscale, sign, n_s, crt, p8);
  else
    hipLaunchKernelGGL((oz_crt<1>), dim3(grid_of(cpart)), dim3(256), 0, st, Cres, cpart,
                       p.d_oz_ea, fb, p.d_albedo, x, y, xscale, sign, n_s, crt, p8);
  RT_HIP(hipGetLastError());
}

}  // namespace rtsn
