// Scattering GEMM with 16-bit matrix-core operands and FP32 accumulation:
//   y[k, i] = xs * x[k, i] + sign * (1 - eps_i) * rs_k * sum_k' Mhat'[k, k'] L'[k', i]
// (the operator epilogue of the FP64 GEMM; Mhat' / L' are the stored 16-bit
// operands, rs_k undoes their scaling).
//
// Modes: BF16 (Lambda emits bf16), FP16 (Lambda emits fp16 scaled by a power
// of two, Mhat rows scaled to unit maximum; both undone in FP32 in the
// epilogue) and split BF16 ("bf16x3": Mhat = hi + lo and L = hi + lo in bf16,
// hi*hi + hi*lo + lo*hi accumulated).
//
// Operand layouts and the tile body are in gemm16_dev.h.  The tile shape is
// chosen per problem and mode by timing the candidates below on the
// problem's own operands the first time the mode is used (the tile choice
// changes the speed only: every candidate accumulates each output in the same
// k order up to the MFMA's internal order).  RTSN_GEMM16_CFG=<index> forces a
// candidate.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>

#include "gemm16_dev.h"
#include "lambda_dev.h"

namespace rtsn {

namespace {

using namespace g16;

template <int MODE, typename C, int OCC, bool DOTS, typename TY>
__global__ __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(1, OCC))) void sigma16_kernel(
    const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo, int Mp,
    const uint16_t* __restrict__ Bhi, const uint16_t* __restrict__ Blo, int64_t Np, int K4p,
    const TY* X, TY* Y, const double* __restrict__ albedo, const float* __restrict__ rowscale,
    float colmul, const double* __restrict__ xscale, float sign, int M, int N, int GM,
    gemm::TileDots dots, float ymul) {
  __shared__ __align__(16) uint8_t lds[C::template lds_bytes<MODE>()];
  const int Mt = Mp / C::BM;
  int tm, tn;
  if (!tile_of(blockIdx.x, Mt, (N + C::BN - 1) / C::BN, GM, tm, tn)) return;
  const float xs = (X != nullptr && xscale != nullptr) ? (float)*xscale : 1.f;
  if constexpr (C::PP) {
    static_assert(!DOTS, "the ping-pong tile has no fused dots");
    tile_pp<MODE, C, TY>(Ahi, Mp, Bhi, (int)Np, K4p, X, Y, albedo, rowscale, colmul, xs, sign, M,
                         N, tm * C::BM, tn * C::BN, lds, ymul);
  } else {
    tile<MODE, C, DOTS, TY>(Ahi, Alo, Mp, Bhi, Blo, (int)Np, K4p, X, Y, albedo, rowscale, colmul,
                            xs, sign, M, N, tm * C::BM, tn * C::BN, lds, dots, tn * Mt + tm,
                            ymul);
  }
}

// Candidate tile shapes (BM x BN, waves, K stage, instruction) and the
// occupancy each is compiled for.  The split mode stages twice the operands,
// so its widest candidate uses the shorter K stage.
using C0 = Cfg<256, 256, 2, 4, 64, true>;
using C0s = Cfg<256, 256, 2, 4, 32, true>;
using C1 = Cfg<256, 128, 2, 2, 32, false>;
using C2 = Cfg<128, 128, 2, 2, 32, true>;
using C3 = Cfg<128, 128, 2, 2, 64, false>;
using C4 = Cfg<256, 256, 2, 4, 32, true, true>;   // ping-pong (not split, no fused dots)
constexpr int kNumCfg = 5;
const char* const kCfgName[kNumCfg] = {"256x256 32x32x16 K64", "256x128 16x16x32 K32",
                                       "128x128 32x32x16 K32", "128x128 16x16x32 K64",
                                       "256x256 32x32x16 K32 ping-pong"};
// candidates a mode can run (the ping-pong tile has one operand part)
bool cfg_allowed(int mode, int cfg) { return cfg != 4 || mode != MODE_SPLIT; }

struct Args {
  const uint16_t *ahi, *alo;
  int Mp;
  const uint16_t *bhi, *blo;
  int64_t Np;
  int K4p;
  const void* x;   // float, or _Float16 when half_xy
  void* y;
  bool half_xy;
  float ymul;
  const double* albedo;
  const float* rowscale;
  float colmul;
  const double* xscale;
  float sign;
  int M, N;
  gemm::TileDots* dots;
};

template <int MODE, typename C, int OCC>
void launch_cfg(const Args& a, hipStream_t st) {
  const int Mt = a.Mp / C::BM, Nt = (a.N + C::BN - 1) / C::BN;
  if (a.Mp % C::BM || a.K4p % (C::BK / 4) || (int64_t)Nt * C::BN > a.Np)
    fail(RT_E_INVALID, "16-bit GEMM: operand padding does not fit the tile");
  const int T = Mt * Nt;
  const int grid = 8 * ((T + 7) / 8);
  const float* xf = static_cast<const float*>(a.x);
  float* yf = static_cast<float*>(a.y);
  if (a.half_xy) {
    if (a.dots) fail(RT_E_INVALID, "fused dots need an FP32 output");
    hipLaunchKernelGGL((sigma16_kernel<MODE, C, OCC, false, _Float16>), dim3(grid), dim3(C::NT),
                       0, st, a.ahi, a.alo, a.Mp, a.bhi, a.blo, a.Np, a.K4p,
                       static_cast<const _Float16*>(a.x), static_cast<_Float16*>(a.y), a.albedo,
                       a.rowscale, a.colmul, a.xscale, a.sign, a.M, a.N, 8, gemm::TileDots{},
                       a.ymul);
  } else if (a.dots) {
    if constexpr (C::PP) {
      fail(RT_E_INVALID, "fused dots: not with the ping-pong tile");
    } else {
      if (a.dots->ldp < T) fail(RT_E_INVALID, "fused dots: too few partial slots");
      a.dots->ldp = T;   // one slot per tile, all written
      hipLaunchKernelGGL((sigma16_kernel<MODE, C, OCC, true, float>), dim3(grid), dim3(C::NT),
                         0, st, a.ahi, a.alo, a.Mp, a.bhi, a.blo, a.Np, a.K4p, xf, yf, a.albedo,
                         a.rowscale, a.colmul, a.xscale, a.sign, a.M, a.N, 8, *a.dots, a.ymul);
    }
  } else {
    hipLaunchKernelGGL((sigma16_kernel<MODE, C, OCC, false, float>), dim3(grid), dim3(C::NT), 0,
                       st, a.ahi, a.alo, a.Mp, a.bhi, a.blo, a.Np, a.K4p, xf, yf, a.albedo,
                       a.rowscale, a.colmul, a.xscale, a.sign, a.M, a.N, 8, gemm::TileDots{},
                       a.ymul);
  }
}

template <int MODE>
void launch_index(int cfg, const Args& a, hipStream_t st) {
  switch (cfg) {
    case 0:
      if constexpr (MODE == MODE_SPLIT) launch_cfg<MODE, C0s, 2>(a, st);
      else launch_cfg<MODE, C0, 2>(a, st);
      break;
    case 1: launch_cfg<MODE, C1, 2>(a, st); break;
    case 2: launch_cfg<MODE, C2, 4>(a, st); break;
    case 3: launch_cfg<MODE, C3, 2>(a, st); break;
    default:
      // the ping-pong tile: not for the split mode, and fused dots take the
      // 128 x 128 tile
      if constexpr (MODE == MODE_SPLIT) launch_cfg<MODE, C0s, 2>(a, st);
      else if (a.dots) launch_cfg<MODE, C2, 4>(a, st);
      else launch_cfg<MODE, C4, 2>(a, st);
      break;
  }
}

void launch_mode(int mode, int cfg, const Args& a, hipStream_t st) {
  if (mode == MODE_BF16) launch_index<MODE_BF16>(cfg, a, st);
  else if (mode == MODE_FP16) launch_index<MODE_FP16>(cfg, a, st);
  else launch_index<MODE_SPLIT>(cfg, a, st);
}

// Persistent tuning cache (RTSN_TUNE_CACHE=<file>): one line per tuned
// problem shape, "<arch> <mode> <M> <N> <cfg>", read before timing and
// appended after; a shape found there is not timed again (no stream
// synchronisation, no scratch allocation).  Unset: nothing is read or
// written.
std::mutex g_cache_mu;

std::string cache_key(int device, int mode, int M, int N) {
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "";
  char buf[160];
  std::snprintf(buf, sizeof buf, "%s %d %d %d", prop.gcnArchName, mode, M, N);
  return buf;
}

int cache_lookup(const std::string& key) {
  const char* path = std::getenv("RTSN_TUNE_CACHE");
  if (!path || key.empty()) return -1;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  FILE* f = std::fopen(path, "r");
  if (!f) return -1;
  char line[256];
  int found = -1;
  while (std::fgets(line, sizeof line, f)) {
    std::string s(line);
    const size_t sp = s.find_last_of(' ');
    if (sp == std::string::npos) continue;
    if (s.compare(0, sp, key) == 0 && sp == key.size()) {
      const int c = std::atoi(s.c_str() + sp + 1);
      if (c >= 0 && c < kNumCfg) found = c;   // the last entry wins
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const std::string& key, int cfg) {
  const char* path = std::getenv("RTSN_TUNE_CACHE");
  if (!path || key.empty()) return;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "%s %d\n", key.c_str(), cfg);
    std::fclose(f);
  }
}

// Time every candidate on a column slice of the real operands and epilogue
// input (scratch output) and keep the fastest.
int autotune(const Problem& p, int mode, const Args& full, hipStream_t st) {
  if (const char* e = std::getenv("RTSN_GEMM16_CFG")) {
    const int c = std::atoi(e);
    if (c >= 0 && c < kNumCfg && cfg_allowed(mode, c)) return c;
  }
  const std::string key = cache_key(p.device, mode, full.M, full.N);
  if (const int c = cache_lookup(key); c >= 0) return c;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  RT_HIP(hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone) return 2;   // cannot time inside a capture
  Args a = full;
  a.dots = nullptr;
  if (a.half_xy) {   // time the FP32-output form (same tile body)
    a.half_xy = false;
    a.x = nullptr;
    a.xscale = nullptr;
    a.ymul = 1.f;
  }
  const int64_t want = round_up(std::max<int64_t>(4096, (int64_t(1) << 27) / std::max(1, a.M)), 256);
  // the slice keeps the leading dimension N of x: rows of the slice are
  // strided, so time full rows when the slice would not be contiguous
  a.N = (int)std::min<int64_t>(a.N, want);
  if (a.N != full.N) {
    a.x = nullptr;
    a.xscale = nullptr;
  }
  float* scratch = nullptr;
  RT_HIP(hipMalloc(&scratch, (size_t)a.M * a.N * sizeof(float)));
  a.y = scratch;
  hipEvent_t e0, e1;
  RT_HIP(hipEventCreate(&e0));
  RT_HIP(hipEventCreate(&e1));
  int best = 2;
  float best_ms = 1e30f;
  for (int c = 0; c < kNumCfg; ++c) {
    if (!cfg_allowed(mode, c)) continue;
    launch_mode(mode, c, a, st);   // warm-up
    float ms = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      RT_HIP(hipEventRecord(e0, st));
      launch_mode(mode, c, a, st);
      RT_HIP(hipEventRecord(e1, st));
      RT_HIP(hipEventSynchronize(e1));
      float t = 0.f;
      RT_HIP(hipEventElapsedTime(&t, e0, e1));
      ms = std::min(ms, t);
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  RT_HIP(hipEventDestroy(e0));
  RT_HIP(hipEventDestroy(e1));
  RT_HIP(hipFree(scratch));
  cache_store(key, best);
  return best;
}

template <int MODE>
__global__ __launch_bounds__(256) void to_k4_kernel(const float* __restrict__ L, uint16_t* hi,
                                                   uint16_t* lo, int n_r, int64_t n_s,
                                                   int64_t Np, float mul) {
  const int64_t n = (int64_t)n_r * n_s;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / n_s);
    const int64_t i = e - (int64_t)k * n_s;
    lam::k4_ray<MODE>(hi, lo, k, Np).put(i, L[e] * mul);
  }
}

}  // namespace

void convert_to_k4(const Problem& p, int precision, const float* L, uint16_t* hi, uint16_t* lo,
                   hipStream_t st) {
  const dim3 grid(2048), block(256);
  switch (precision) {
    case RT_PREC_BF16:
      hipLaunchKernelGGL(to_k4_kernel<lam::K4_BF16>, grid, block, 0, st, L, hi, lo, p.n_r,
                         p.n_s, p.np16, 1.f);
      break;
    case RT_PREC_FP16:
      hipLaunchKernelGGL(to_k4_kernel<lam::K4_FP16>, grid, block, 0, st, L, hi, lo, p.n_r,
                         p.n_s, p.np16, fp16_lambda_scale(p.n));
      break;
    case RT_PREC_BF16X3:
      hipLaunchKernelGGL(to_k4_kernel<lam::K4_SPLIT>, grid, block, 0, st, L, hi, lo, p.n_r,
                         p.n_s, p.np16, 1.f);
      break;
    default:
      fail(RT_E_INVALID, "convert_to_k4: not a 16-bit precision");
  }
  RT_HIP(hipGetLastError());
}

// Power-of-two scale applied to Lambda's fp16 output: about sqrt(n), which
// brings the entries of Lambda of a unit-norm vector of n entries near 1,
// capped at 2^14.  The cap keeps every entry finite: Lambda's weights are
// non-negative and sum to at most 1 along a ray, so |Lambda v| <= max |v| <= 1
// and the scaled output stays below 2^14, a quarter of fp16's largest value.
float fp16_lambda_scale(int64_t n) {
  const double e = std::ceil(0.5 * std::log2((double)(n > 1 ? n : 1)));
  return (float)std::ldexp(1.0, std::min((int)e, 14));
}

// Scale of an fp16 Krylov basis (stored vectors are 2^11 times the unit-norm
// ones).  Transfer weights are non-negative with row sums <= 1, so for the
// physical kernels (|(1 - eps) Mhat|_inf about 1, refused above 2) an
// operator output for a unit vector has entries of at most about 2, stored
// below 2^12; the Gram-Schmidt update subtracts multiples h_i of unit
// vectors, with |h_i| <= |A v_j|_2, in practice of order one, which leaves
// a factor of about 16 below fp16's largest value.  An overflow would show
// as a non-finite value and stop the solve with RT_E_NONFINITE.  The
// smallest normal fp16 value stands for 3e-8 of a unit vector.
float fp16_basis_scale(int64_t) { return 2048.f; }

const char* gemm16_config_name(int cfg) {
  return (cfg >= 0 && cfg < kNumCfg) ? kCfgName[cfg] : "untuned";
}

namespace {

void launch_b16(Problem& p, int precision, const uint16_t* l_hi, const uint16_t* l_lo,
                const void* x, void* y, bool half_xy, float ymul, const double* xscale,
                double sign, hipStream_t st, gemm::TileDots* dots) {
  Args a{};
  a.half_xy = half_xy;
  a.ymul = ymul;
  int mode;
  switch (precision) {
    case RT_PREC_BF16:
      mode = MODE_BF16;
      a.ahi = p.d_a8_bf16;
      a.colmul = 1.f;
      break;
    case RT_PREC_FP16:
      mode = MODE_FP16;
      a.ahi = p.d_a8_f16;
      a.rowscale = p.d_f16_rowscale;
      a.colmul = 1.f / fp16_lambda_scale(p.n);
      break;
    case RT_PREC_BF16X3:
      mode = MODE_SPLIT;
      a.ahi = p.d_a8_bf16;
      a.alo = p.d_a8_bf16_lo;
      a.blo = l_lo;
      a.colmul = 1.f;
      break;
    default:
      fail(RT_E_INVALID, "launch_sigma_b16: not a 16-bit precision");
  }
  a.Mp = p.mp16;
  a.bhi = l_hi;
  a.Np = p.np16;
  a.K4p = p.kp16 / 4;
  a.x = x;
  a.y = y;
  a.albedo = p.d_albedo;
  a.xscale = xscale;
  a.sign = (float)sign;
  a.M = p.n_r;
  a.N = (int)p.n_s;
  a.dots = nullptr;
  if (p.g16_cfg[mode] < 0) p.g16_cfg[mode] = autotune(p, mode, a, st);
  a.dots = dots;
  ProfScope prof(RT_KCLASS_SIGMA_LO, st);
  launch_mode(mode, p.g16_cfg[mode], a, st);
  RT_HIP(hipGetLastError());
}

}  // namespace

void launch_sigma_b16(Problem& p, int precision, const uint16_t* l_hi, const uint16_t* l_lo,
                      const float* x, float* y, const double* xscale, double sign,
                      hipStream_t st, gemm::TileDots* dots) {
  launch_b16(p, precision, l_hi, l_lo, x, y, false, 1.f, xscale, sign, st, dots);
}

void launch_sigma_b16_h(Problem& p, int precision, const uint16_t* l_hi, const uint16_t* l_lo,
                        const _Float16* x, _Float16* y, float ymul, const double* xscale,
                        double sign, hipStream_t st) {
  launch_b16(p, precision, l_hi, l_lo, x, y, true, ymul, xscale, sign, st, nullptr);
}

}  // namespace rtsn
