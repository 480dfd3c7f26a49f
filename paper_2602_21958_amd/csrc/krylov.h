// Device-side Krylov state and the launchers of krylov.hip.
#pragma once

#include "rt_internal.h"

namespace rtsn {

constexpr int kMaxRestart = 128;
constexpr int kPairRows = kMaxRestart + 2;   // two-step Arnoldi: rows per dot block
constexpr int kReduceBlocks = 1024;  // dots; the update pass uses twice as many

// GMRES state kept in device memory.  The fields before h are what the host
// reads back.  resid / breakdown / nonfinite describe the step at which the
// cycle stops (stop_k, 1-based; 0 while it continues) once that step has
// run, so steps launched past it change none of them.
struct GmresState {
  double resid;        // |g_{j+1}| after the last Givens step up to the stop
  double beta;         // norm computed by finish_norm
  int breakdown;       // h_{j+1,j} vanished (lucky breakdown)
  int nonfinite;       // NaN/Inf met
  int stop_k;          // first step whose residual estimate met the tolerance,
                       // broke down or was not finite (0: none yet)
  int pad;
  double log[kMaxRestart];   // |g_{j+1}| of every step j of the cycle
  double h[kMaxRestart + 1];
  double R[(size_t)kMaxRestart * (kMaxRestart + 1)];  // column j at j*(kMaxRestart+1)
  double cs[kMaxRestart], sn[kMaxRestart];
  double g[kMaxRestart + 1];
  double y[kMaxRestart];
  double coef[kMaxRestart + 1];
  double vscale[kMaxRestart + 1];
};

struct BicgState {
  double rho, alpha, omega, beta;
  double snorm, rnorm;
  int iter, breakdown;
};

template <typename TV>
void k_mdot(const TV* V, int64_t n, int cnt, const TV* w, double* partial, hipStream_t st);
// Same with an explicit number nb of partial slots per row.
void k_reduce_rows_nb(const double* partial, int nb, int nrows, const double* scale, double* out,
                      hipStream_t st);
void k_reduce_rows(const double* partial, int64_t n, int nrows, const double* scale, double* out,
                   hipStream_t st);
template <typename TV>
void k_update(const TV* V, int64_t n, int cnt, const double* h, const double* vscale, TV* w,
              double* partial, hipStream_t st);
template <typename TV, typename TX>
void k_combine(const TV* V, int64_t n, int cnt, const double* coef, TX* x, hipStream_t st);
template <typename TB, typename TA, typename TR>
void k_residual(const TB* b, const TA* ax, int64_t n, TR* r, double* partial, hipStream_t st);
template <typename T>
void k_norm_partial(const T* x, int64_t n, double* partial, hipStream_t st);
void k_finish_norm(const double* partial, int64_t n, GmresState* gs, int start_cycle,
                   hipStream_t st);
void k_finish_norm_simple(const double* partial, int64_t n, double* out, hipStream_t st);
// Givens step j; tol: residual-estimate threshold that stops the cycle.
// kdiag != 0: h and the norm are those of Arnoldi on c K where c A =
// c I - c K and kdiag = c (K v_j = sum_i h_i v_i + beta v_{j+1}); the step
// uses the column kdiag e_j - h, -beta of c A.
void k_givens(const double* partial, int64_t n, GmresState* gs, int j, double tol,
              hipStream_t st, double kdiag = 0.0);
void k_solve_r(GmresState* gs, int k, hipStream_t st);
// Two Arnoldi steps on K at once (FP64 basis): u1 = K v_j in slot j + 1 and
// u2 = K u1 in slot j + 2 become v_{j+1}, v_{j+2} (stored unnormalised with
// their scales) with one dots pass and one update pass over v_0..v_j.
// pair: 8 + 4 kPairRows doubles; hk: kPairRows^2 doubles (K's Hessenberg
// columns of the cycle).
// Slot of the pair workspace (8 + 4 kPairRows doubles) that the pair kernels
// leave alone (they use 0, 1 and 8 on): a caller's device scalar.
constexpr int kPairUser = 2;
template <typename TV>
void k_mdot2(const TV* V, int64_t n, int cnt, const TV* u1, const TV* u2, double* partial,
             hipStream_t st);
void k_pair_coef(const double* partial, int64_t n, int j, const double* vscale, double* pair,
                 hipStream_t st);
template <typename TV>
void k_update2(const TV* V, int64_t n, int cnt, const double* pair, TV* u1, TV* u2,
               double* partial, hipStream_t st);
// Z <- Z - rho P1 with rho = P1 . Z / |P1|^2 from the update's sums (the
// P1 component that nu's rounding leaves); |Z|^2 recomputed.
template <typename TV>
void k_pair_fix(TV* p1, TV* z, int64_t n, double* pair, double* partial, hipStream_t st);
void k_givens2(const double* partial, int64_t n, GmresState* gs, int j, double tol,
               const double* pair, double* hk, hipStream_t st, double kdiag = 1.0,
               double sigma = 1.0);
template <typename T>
void k_dots4(const T* a0, const T* b0, const T* a1, const T* b1, int cnt, int64_t n,
             double* partial, hipStream_t st);
template <typename T>
void k_bicg_p(const T* r, const T* v, T* p, int64_t n, const BicgState* bs, hipStream_t st);
template <typename T>
void k_bicg_s(T* r, const T* v, int64_t n, const BicgState* bs, double* partial, hipStream_t st);
template <typename T, typename TX>
void k_bicg_xr(TX* x, const T* p, T* r, const T* t, int64_t n, const BicgState* bs,
               int only_alpha, double* partial, hipStream_t st);
void k_bicg_scalar(const double* partial, int64_t n, int stage, BicgState* bs, hipStream_t st);
template <typename TS, typename TD>
void k_convert(const TS* a, TD* b, int64_t n, double scale, hipStream_t st);
void k_axpy_f64(double* x, const float* d, int64_t n, const double* scale, hipStream_t st);
int reduce_blocks(int64_t n);

// Solver workspace, allocated on first use and kept with the problem.
struct Workspace {
  int restart = 0;
  bool mixed = false;
  size_t bytes = 0;
  void* V = nullptr;            // (restart + 1) * n basis (double; float or fp16 if mixed)
  size_t vbytes = 0;
  double* partial = nullptr;    // partial_elems partial sums
  size_t partial_elems = 0;
  int dot_slots = 0;            // slots per vector of the dots fused into the GEMM
  GmresState* gs = nullptr;
  BicgState* bs = nullptr;
  double* scal = nullptr;       // small device scalars
  double* r64 = nullptr;        // n FP64: residual / BiCGStab vectors
  double* ax64 = nullptr;       // n FP64: A x
  double* bic = nullptr;        // 4 n FP64 for BiCGStab (rhat, p, v, t)
  float* d32 = nullptr;         // n: inner correction (mixed)
  float* t32 = nullptr;         // n: scaled residual, inner right-hand side (mixed)
  float* a32 = nullptr;         // n: inner operator output (mixed)
  double* pair = nullptr;       // two-step Arnoldi coefficients (8 + 4 kPairRows)
  double* hk = nullptr;         // K's Hessenberg columns of a cycle (kPairRows^2)
  GmresState* host = nullptr;   // pinned status mirror
  ~Workspace();
};

// basis_elem: bytes per basis element (0: 8 for FP64, 4 for mixed)
size_t workspace_bytes(const Problem& p, int restart, bool mixed, bool bicgstab,
                       int basis_elem = 0);

rt_status solve(Problem& p, const rt_solver_opts& o, const double* b, double* x, int x_is_guess,
                rt_solve_stats* stats, hipStream_t st);

}  // namespace rtsn
