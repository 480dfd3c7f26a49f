// Scattering step with per-point classes.
//
// Paper Sec. 3.3: Sigma is block diagonal over the spatial points, with the
// block Gamma Psi_[i] W of point i (eq. Sigma); the block may differ from
// point to point.  When the points fall into classes that share a block, the
// scattering of one class is a dense GEMM of its Mhat with the columns of L
// that belong to the class.  The columns are gathered into a contiguous
// operand (ray-major, the class's points in increasing order), multiplied by
// the same MFMA GEMM as the one-kernel path with the class's albedo in its
// epilogue, and scattered back as y = xs x + sign * result.
#include "rt_internal.h"

namespace rtsn {

namespace {

// G[k][j] = L[k][idx[j]] for k < n_r, j < nc.
template <typename T>
__global__ __launch_bounds__(256) void gather_cols(const T* __restrict__ L,
                                                   const int32_t* __restrict__ idx, T* G,
                                                   int n_r, int64_t n_s, int64_t nc) {
  const int64_t m = (int64_t)n_r * nc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / nc, j = e - k * nc;
    G[e] = L[k * n_s + idx[j]];
  }
}

// y[k][idx[j]] = xs x[k][idx[j]] + sign R[k][j]   (x may be null: no x term).
template <typename T>
__global__ __launch_bounds__(256) void scatter_cols(const T* __restrict__ R,
                                                    const int32_t* __restrict__ idx,
                                                    const T* x, T* y,
                                                    const double* __restrict__ xscale, T sign,
                                                    int n_r, int64_t n_s, int64_t nc) {
  const int64_t m = (int64_t)n_r * nc;
  const T xs = (x != nullptr && xscale != nullptr) ? T(*xscale) : T(1);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / nc, j = e - k * nc;
    const int64_t at = k * n_s + idx[j];
    const T v = sign * R[e];
    y[at] = x ? xs * x[at] + v : v;
  }
}

int grid_of(int64_t m) { return (int)std::min<int64_t>((m + 255) / 256, 8192); }

template <typename T>
void classes_t(const Problem& p, const T* cmhat, const T* L, const T* x, T* y, T* work,
               const double* xscale, double sign, hipStream_t st,
               void (*gemm)(const Problem&, const T*, const T*, int, const T*, T*,
                            const double*, const double*, double, hipStream_t)) {
  ProfScope prof(sizeof(T) == 8 ? RT_KCLASS_SIGMA : RT_KCLASS_SIGMA_LO, st);
  int64_t max_nc = 0;
  for (int c = 0; c < p.n_classes; ++c)
    max_nc = std::max(max_nc, p.class_off[c + 1] - p.class_off[c]);
  T* G = work;
  T* R = work + (size_t)p.n_r * max_nc;
  for (int c = 0; c < p.n_classes; ++c) {
    const int64_t off = p.class_off[c], nc = p.class_off[c + 1] - off;
    if (nc == 0) continue;
    const int32_t* idx = p.d_cidx + off;
    const int64_t m = (int64_t)p.n_r * nc;
    hipLaunchKernelGGL(gather_cols<T>, dim3(grid_of(m)), dim3(256), 0, st, L, idx, G, p.n_r,
                       p.n_s, nc);
    gemm(p, cmhat + (size_t)c * p.class_mhat_stride, G, (int)nc, nullptr, R, p.d_calb + off,
         nullptr, +1.0, st);
    hipLaunchKernelGGL(scatter_cols<T>, dim3(grid_of(m)), dim3(256), 0, st, R, idx, x, y,
                       xscale, T(sign), p.n_r, p.n_s, nc);
  }
  RT_HIP(hipGetLastError());
}

}  // namespace

size_t classes_work_elems(const Problem& p) {
  int64_t max_nc = 0;
  for (int c = 0; c < p.n_classes; ++c)
    max_nc = std::max(max_nc, p.class_off[c + 1] - p.class_off[c]);
  return (size_t)2 * p.n_r * (size_t)max_nc;
}

void launch_sigma_classes_f64(const Problem& p, const double* L, const double* x, double* y,
                              double* work, const double* xscale, double sign, hipStream_t st) {
  classes_t<double>(p, p.d_cmhat64, L, x, y, work, xscale, sign, st, launch_gemm_f64);
}

void launch_sigma_classes_f32(const Problem& p, const float* L, const float* x, float* y,
                              float* work, const double* xscale, double sign, hipStream_t st) {
  classes_t<float>(p, p.d_cmhat32, L, x, y, work, xscale, sign, st, launch_gemm_f32);
}

}  // namespace rtsn
