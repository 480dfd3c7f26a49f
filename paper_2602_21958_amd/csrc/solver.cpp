// Krylov solvers driven from the host, all vector work on the device.
//
// * Restarted GMRES(m) (Saad-Schultz) with classical Gram-Schmidt Arnoldi,
//   Givens rotations and a true-residual check at the end of each cycle; the
//   paper's solver (Sec. 5 set-up; Sec. 5.3 restart 30).  The host reads one
//   scalar per Arnoldi step (|g_{j+1}|) and one per cycle (true residual).
// * Mixed precision: FP64 iterative refinement around a low-precision inner
//   GMRES: r = b - A_64 x in FP64, inner solve of A_lo d = r / ||r|| with an
//   FP32 basis (FP64 dot accumulation) and the operator in FP32 / BF16 /
//   FP16 / split-BF16 arithmetic, then x += ||r|| d.  Optionally (basis_fp16)
//   the inner basis is kept in fp16, scaled to entries of order one.
// * BiCGStab (van der Vorst), FP64, scalars kept on the device.
#include <algorithm>
#include <type_traits>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstring>

#include "gemm_dev.h"
#include "krylov.h"

namespace rtsn {

Workspace::~Workspace() {
  hipFree(V);
  hipFree(partial);
  hipFree(gs);
  hipFree(bs);
  hipFree(scal);
  hipFree(r64);
  hipFree(ax64);
  hipFree(bic);
  hipFree(d32);
  hipFree(t32);
  hipFree(a32);
  if (host) hipHostFree(host);
}

size_t workspace_bytes(const Problem& p, int restart, bool mixed, bool bicgstab,
                       int basis_elem) {
  const size_t n = (size_t)p.n;
  if (basis_elem <= 0) basis_elem = mixed ? 4 : 8;
  size_t b = sizeof(double) * (size_t)(kMaxRestart + 1) * 2 * kReduceBlocks + sizeof(GmresState) +
             sizeof(BicgState) + 64 * sizeof(double);
  b += (size_t)(bicgstab ? 1 : restart + 1) * n * basis_elem;   // BiCGStab keeps no basis
  b += (mixed ? 1 : 2) * n * sizeof(double);  // r64 (+ ax64 for FP64 GMRES)
  if (mixed) b += 2 * n * sizeof(float);
  if (bicgstab) b += 4 * n * sizeof(double);
  b += n * lambda_elem_bytes(mixed ? RT_PREC_FP32 : RT_PREC_FP64);  // operator L buffer
  return b;
}

namespace {

template <typename T>
T* dalloc(size_t count, size_t& total) {
  void* ptr = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(&ptr, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(RT_E_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  total += count * sizeof(T);
  return static_cast<T*>(ptr);
}

// Arnoldi inner products in their own streaming pass (default) or fused into
// the Sigma GEMM's epilogue (RTSN_FUSED_DOTS=1).  The fused form reads the
// same basis bytes but all tiles reach their epilogue together, so the reads
// come as one burst that the MFMA phase does not hide: measured slower (box
// 32^3 FP64: 8.2 ms per fused GEMM against 4.97 ms GEMM + 1.03 ms dots).
bool fuse_dots_env() {
  const char* e = std::getenv("RTSN_FUSED_DOTS");
  return e && e[0] == '1';
}



// basis_elem: bytes per basis element (8 FP64, 4 FP32, 2 fp16)
Workspace& ensure_workspace(Problem& p, int restart, bool mixed, bool bicgstab, int basis_elem) {
  Workspace* ws = p.ws;
  const size_t vbytes = (size_t)(bicgstab ? 1 : restart + 1) * (size_t)p.n * basis_elem;
  const bool ok = ws && ws->restart >= restart && ws->mixed == mixed && ws->vbytes >= vbytes &&
                  (!bicgstab || ws->bic != nullptr);
  if (ok) return *ws;
  delete p.ws;
  p.ws = nullptr;
  ws = new Workspace();
  p.ws = ws;
  const size_t n = (size_t)p.n;
  size_t tot = 0;
  ws->restart = restart;
  ws->mixed = mixed;
  ws->V = dalloc<char>(vbytes, tot);
  ws->vbytes = vbytes;
  // partial sums: reduction kernels use (kMaxRestart + 1) x 2 kReduceBlocks;
  // the dots fused into the Sigma GEMM one slot per output tile and basis
  // vector (the 16-bit GEMM's smallest tile gives the most slots)
  ws->dot_slots = sigma_dot_slots(p, RT_PREC_BF16);
  ws->partial_elems = std::max({(size_t)(kMaxRestart + 1) * 2 * kReduceBlocks,
                                (size_t)2 * kPairRows * kReduceBlocks,
                                (size_t)(restart + 1) * ws->dot_slots});
  ws->partial = dalloc<double>(ws->partial_elems, tot);
  ws->gs = dalloc<GmresState>(1, tot);
  ws->pair = dalloc<double>(8 + 4 * kPairRows, tot);
  ws->hk = dalloc<double>((size_t)kPairRows * kPairRows, tot);
  ws->bs = dalloc<BicgState>(1, tot);
  ws->scal = dalloc<double>(64, tot);
  ws->r64 = dalloc<double>(n, tot);
  if (!mixed) ws->ax64 = dalloc<double>(n, tot);
  if (mixed) {
    ws->d32 = dalloc<float>(n, tot);
    ws->t32 = dalloc<float>(n, tot);
  }
  if (bicgstab) ws->bic = dalloc<double>(4 * n, tot);
  RT_HIP(hipHostMalloc((void**)&ws->host, sizeof(GmresState), hipHostMallocDefault));
  RT_HIP(hipMemset(ws->gs, 0, sizeof(GmresState)));
  ws->bytes = tot;
  return *ws;
}

struct Status {
  double resid, beta;
  int breakdown, nonfinite;
};

Status read_status(Workspace& ws, hipStream_t st) {
  RT_HIP(hipMemcpyAsync(ws.host, ws.gs, offsetof(GmresState, h), hipMemcpyDeviceToHost, st));
  RT_HIP(hipStreamSynchronize(st));
  return Status{ws.host->resid, ws.host->beta, ws.host->breakdown, ws.host->nonfinite};
}

// Arnoldi steps launched between two status reads.  A read is a host round
// trip, which dominates the step time of small problems; steps launched past
// the cycle's stopping step are discarded (the cycle keeps its first stop_k
// steps, whose basis vectors, Hessenberg columns and g entries later steps do
// not touch), so the results are those of reading after every step.  Large
// problems read after every step: a discarded step would cost more than the
// read.  RTSN_STATUS_EVERY overrides.
int status_every(int64_t n) {
  if (const char* e = std::getenv("RTSN_STATUS_EVERY")) return std::max(1, std::atoi(e));
  return n <= (int64_t(1) << 22) ? 4 : 1;
}

struct StepRead {
  int k;        // steps of the cycle to keep
  bool stop;    // the cycle met its tolerance, broke down (or hit a non-finite value)
};

// Status read after `done` steps of the cycle: the steps to keep, the new
// residual estimates appended to hist (relative to bnorm); fails on a
// non-finite value at or before the stopping step.
StepRead read_steps(Workspace& ws, hipStream_t st, int done, int& logged,
                    std::vector<double>* hist, double bnorm) {
  const Status g = read_status(ws, st);
  const int stop_k = ws.host->stop_k;
  const int k = stop_k > 0 ? std::min(stop_k, done) : done;
  if (hist)
    for (int q = logged; q < k; ++q) hist->push_back(ws.host->log[q] / bnorm);
  logged = k;
  if (g.nonfinite) fail(RT_E_NONFINITE, "non-finite value in the Arnoldi process");
  return StepRead{k, stop_k > 0};
}

double read_scalar(const double* d, hipStream_t st, Workspace& ws) {
  double* h = reinterpret_cast<double*>(ws.host);
  RT_HIP(hipMemcpyAsync(h, d, sizeof(double), hipMemcpyDeviceToHost, st));
  RT_HIP(hipStreamSynchronize(st));
  return *h;
}

template <typename TV>
double vec_norm(const TV* v, int64_t n, Workspace& ws, hipStream_t st) {
  k_norm_partial<TV>(v, n, ws.partial, st);
  k_finish_norm_simple(ws.partial, n, ws.scal, st);
  return read_scalar(ws.scal, st, ws);
}

struct CoreResult {
  int iters = 0;
  int cycles = 0;
  double beta = 0;  // last true residual norm (operator of the core's precision)
};

// GMRES(m) on A_prec x = b with vectors of type TV.  x is overwritten; if
// x_zero it starts from 0.  Returns RT_OK / RT_NOT_CONVERGED.
// With single_cycle the solve stops after one restart cycle and skips the
// true-residual recomputation (inner solves of iterative refinement, whose
// low-precision operator is not exactly linear).
// With pre (right preconditioning, A P^-1 y = b, x = P^-1 y) the Arnoldi
// operator is K' = I - A P^-1 instead of K = I - A, so the Hessenberg
// bookkeeping is unchanged: with u = P^-1 v and P = Id - (1 - eps) Mhat Dbar,
// K' v = v - A u = K u - (u - v), formed as one operator application on u
// whose epilogue adds nd = v - u (operator_apply_kx).  The cycle end adds
// P^-1 (V y) to x.
template <typename TV>
rt_status gmres_core(Problem& p, int prec, const TV* b, TV* x, bool x_zero, int m, double rtol,
                     int max_iters, double bnorm, Workspace& ws, TV* tmp, hipStream_t st,
                     std::vector<double>* hist, CoreResult& res, bool single_cycle = false,
                     bool two = false, bool pre = false) {
  const int64_t n = p.n;
  TV* V = static_cast<TV*>(ws.V);
  GmresState* gs = ws.gs;
  // the fused dots live in the dense GEMM's epilogue
  const bool fuse_dots =
      !pre && fuse_dots_env() &&
      (p.sigma_form == RT_SIGMA_DENSE || (prec != RT_PREC_FP64 && prec != RT_PREC_FP32));
  // y = K (xs v) or K' (xs v)
  auto step_op = [&](const TV* v, TV* y, const double* xs) {
    if (pre) {
      TV* u = precond_u<TV>(p);
      // the factored expansion forms v - u from the preconditioner's modes
      TV* nd = precond_fused(p, prec) ? nullptr : precond_nd<TV>(p);
      precond_apply<TV>(p, v, u, nd, st);
      operator_apply_kx(p, prec, u, nd, y, xs, st);
    } else {
      operator_apply_k(p, prec, v, y, xs, st);
    }
  };
  if (x_zero) {
    RT_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(TV), st));
    RT_HIP(hipMemcpyAsync(V, b, (size_t)n * sizeof(TV), hipMemcpyDeviceToDevice, st));
    k_norm_partial<TV>(V, n, ws.partial, st);
  } else {
    operator_apply(p, prec, x, tmp, nullptr, st);
    k_residual<TV, TV, TV>(b, tmp, n, V, ws.partial, st);
  }
  k_finish_norm(ws.partial, n, gs, 1, st);
  Status s = read_status(ws, st);
  if (!std::isfinite(s.beta)) fail(RT_E_NONFINITE, "non-finite residual");
  res.beta = s.beta;
  if (hist) hist->push_back(s.beta / bnorm);
  const int every = status_every(n);
  while (s.beta > rtol * bnorm && res.iters < max_iters) {
    res.cycles++;
    int k = 0, logged = 0;
    const bool pairs = (std::is_same<TV, double>::value || std::is_same<TV, float>::value) &&
                       !fuse_dots && two;
    for (int j = 0; j < m; ++j) {
      TV* vj = V + (size_t)j * n;
      TV* w = V + (size_t)(j + 1) * n;
      if (pairs && j + 1 < m && res.iters + 2 <= max_iters) {
        // steps j and j + 1: u1 = K v_j, u2 = K u1, one dots and one update pass
        TV* u1 = V + (size_t)(j + 1) * n;
        TV* u2 = V + (size_t)(j + 2) * n;
        step_op(vj, u1, gs->vscale + j);
        step_op(u1, u2, nullptr);
        k_mdot2<TV>(V, n, j + 2, u1, u2, ws.partial, st);
        k_pair_coef(ws.partial, n, j, gs->vscale, ws.pair, st);
        k_update2<TV>(V, n, j + 1, ws.pair, u1, u2, ws.partial, st);
        k_pair_fix<TV>(u1, u2, n, ws.pair, ws.partial, st);
        k_givens2(ws.partial, n, gs, j, rtol * bnorm, ws.pair, ws.hk, st);
        res.iters += 2;
        ++j;
        k = j + 1;
        if (k < m && res.iters < max_iters && k % every != 0 && (k - 1) % every != 0) continue;
        const StepRead r = read_steps(ws, st, k, logged, hist, bnorm);
        res.iters -= k - r.k;
        k = r.k;
        if (r.stop || res.iters >= max_iters) break;
        continue;
      }
      // Arnoldi on K = I - A (same Krylov space; A's Hessenberg column is
      // e_j - h, -beta): the operator has no x term, the GEMM reads no v_j
      if (fuse_dots) {
        // h_q = vscale_q V_q . w, summed over the GEMM's output tiles in its epilogue
        gemm::TileDots d{V, n, j + 1, ws.partial, ws.dot_slots};
        operator_apply_k(p, prec, vj, w, gs->vscale + j, st, &d);   // sets d.ldp
        k_reduce_rows_nb(ws.partial, d.ldp, j + 1, gs->vscale, gs->h, st);
      } else {
        step_op(vj, w, gs->vscale + j);
        k_mdot<TV>(V, n, j + 1, w, ws.partial, st);
        k_reduce_rows(ws.partial, n, j + 1, gs->vscale, gs->h, st);
      }
      k_update<TV>(V, n, j + 1, gs->h, gs->vscale, w, ws.partial, st);
      k_givens(ws.partial, n, gs, j, rtol * bnorm, st, 1.0);
      res.iters++;
      k = j + 1;
      if (k < m && res.iters < max_iters && k % every != 0) continue;
      const StepRead r = read_steps(ws, st, k, logged, hist, bnorm);
      res.iters -= k - r.k;
      k = r.k;
      if (r.stop || res.iters >= max_iters) break;
    }
    k_solve_r(gs, k, st);
    if (pre) {
      TV* d = precond_nd<TV>(p);
      RT_HIP(hipMemsetAsync(d, 0, (size_t)n * sizeof(TV), st));
      k_combine<TV, TV>(V, n, k, gs->coef, d, st);
      precond_apply_add<TV>(p, d, x, st);
    } else {
      k_combine<TV, TV>(V, n, k, gs->coef, x, st);
    }
    if (single_cycle) {
      res.beta = ws.host->resid;
      return res.beta <= rtol * bnorm ? RT_OK : RT_NOT_CONVERGED;
    }
    operator_apply(p, prec, x, tmp, nullptr, st);
    k_residual<TV, TV, TV>(b, tmp, n, V, ws.partial, st);
    k_finish_norm(ws.partial, n, gs, 1, st);
    s = read_status(ws, st);
    if (!std::isfinite(s.beta)) fail(RT_E_NONFINITE, "non-finite residual");
    res.beta = s.beta;
    if (s.beta > rtol * bnorm && res.iters < max_iters && hist) hist->push_back(s.beta / bnorm);
  }
  return s.beta <= rtol * bnorm ? RT_OK : RT_NOT_CONVERGED;
}

// One GMRES(m) cycle of the refinement's inner solve A_lo d = r / ||r|| with
// the basis in fp16.  Stored basis vectors are S times the FP32 basis's
// (S = fp16_basis_scale: entries of a unit vector would mostly be fp16
// subnormals otherwise): the cycle runs Arnoldi on the operator S A with
// right-hand side S r / ||r||, whose Hessenberg matrix is S times A's and
// whose least-squares solution y, and hence d = sum y_i v_i, is the unscaled
// one.  Returns the inner iteration count.
//
// pre: the preconditioned FP32 operator with factored scattering (u = P^-1 v
// in FP32, v - u formed in the factored expansion, the result rounded into
// the fp16 basis at S times its value); the cycle end adds P^-1 (V y).
int inner_cycle_fp16(Problem& p, int prec, const double* r64, double rn, float* d, int m,
                     double itol, int cap, Workspace& ws, hipStream_t st, bool two,
                     bool pre) {
  const int64_t n = p.n;
  _Float16* V = static_cast<_Float16*>(ws.V);   // the FP32 basis's memory, half used
  GmresState* gs = ws.gs;
  const float S = fp16_basis_scale(n);
  k_convert<double, _Float16>(r64, V, n, (double)S / rn, st);
  RT_HIP(hipMemsetAsync(d, 0, (size_t)n * sizeof(float), st));
  k_norm_partial<_Float16>(V, n, ws.partial, st);
  k_finish_norm(ws.partial, n, gs, 1, st);
  // 1 / S on the device for the pairs' second application (read_status
  // below waits for the copy while inv_s lives)
  const double inv_s = 1.0 / (double)S;
  RT_HIP(hipMemcpyAsync(ws.pair + kPairUser, &inv_s, sizeof(double), hipMemcpyHostToDevice, st));
  const Status s0 = read_status(ws, st);
  if (!(s0.beta > 0.0) || !std::isfinite(s0.beta))
    fail(RT_E_NONFINITE, "fp16 basis: right-hand side out of range");
  int k = 0, logged = 0;
  const int steps = std::min(m, cap), every = status_every(n);
  const bool pairs = two;
  // w = S K v (K' v preconditioned) with v scaled by xs
  auto op_h = [&](const _Float16* v, _Float16* w, const double* xs) {
    if (pre) {
      float* u = precond_u<float>(p);
      precond_apply_h(p, v, u, st);
      operator_apply_kxh(p, u, w, xs, S, st);
    } else {
      operator_apply_h(p, prec, v, w, xs, S, st, true);
    }
  };
  for (int j = 0; j < steps; ++j) {
    _Float16* w = V + (size_t)(j + 1) * n;
    if (pairs && j + 1 < steps) {
      // steps j and j + 1: u1 = S K v_j as in a single step, u2 = K u1 (not
      // S K u1, which would leave fp16's range), so the pair's second
      // Hessenberg column carries the factor S (sigma of k_givens2).  u2 is
      // formed as S K (u1 / S): the 16-bit Lambda output's scale assumes an
      // input of unit size, which u1 / S has and u1 does not.
      _Float16* u2 = V + (size_t)(j + 2) * n;
      op_h(V + (size_t)j * n, w, gs->vscale + j);
      op_h(w, u2, ws.pair + kPairUser);
      k_mdot2<_Float16>(V, n, j + 2, w, u2, ws.partial, st);
      k_pair_coef(ws.partial, n, j, gs->vscale, ws.pair, st);
      k_update2<_Float16>(V, n, j + 1, ws.pair, w, u2, ws.partial, st);
      k_pair_fix<_Float16>(w, u2, n, ws.pair, ws.partial, st);
      k_givens2(ws.partial, n, gs, j, itol * s0.beta, ws.pair, ws.hk, st, (double)S, (double)S);
      ++j;
      k = j + 1;
      if (k < steps && k % every != 0 && (k - 1) % every != 0) continue;
      const StepRead r = read_steps(ws, st, k, logged, nullptr, 1.0);
      k = r.k;
      if (r.stop) break;
      continue;
    }
    // Arnoldi on S K: S A = S I - S K
    op_h(V + (size_t)j * n, w, gs->vscale + j);
    k_mdot<_Float16>(V, n, j + 1, w, ws.partial, st);
    k_reduce_rows(ws.partial, n, j + 1, gs->vscale, gs->h, st);
    k_update<_Float16>(V, n, j + 1, gs->h, gs->vscale, w, ws.partial, st);
    k_givens(ws.partial, n, gs, j, itol * s0.beta, st, (double)S);
    k = j + 1;
    if (k < steps && k % every != 0) continue;
    const StepRead r = read_steps(ws, st, k, logged, nullptr, 1.0);
    k = r.k;
    if (r.stop) break;
  }
  k_solve_r(gs, k, st);
  if (pre) {
    float* t = precond_nd<float>(p);   // free: the fused step writes no v - u
    RT_HIP(hipMemsetAsync(t, 0, (size_t)n * sizeof(float), st));
    k_combine<_Float16, float>(V, n, k, gs->coef, t, st);
    precond_apply_add_h(p, t, d, st);
  } else {
    k_combine<_Float16, float>(V, n, k, gs->coef, d, st);
  }
  return k;
}

rt_status bicgstab_fp64(Problem& p, const double* b, double* x, bool x_zero, double rtol,
                        int max_iters, double bnorm, Workspace& ws, hipStream_t st,
                        std::vector<double>* hist, CoreResult& res) {
  const int64_t n = p.n;
  double* r = ws.r64;
  double* rhat = ws.bic;
  double* pv = ws.bic + n;
  double* v = ws.bic + 2 * n;
  double* t = ws.bic + 3 * n;
  BicgState* bs = ws.bs;
  if (x_zero) {
    RT_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), st));
    RT_HIP(hipMemcpyAsync(r, b, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
  } else {
    operator_apply(p, RT_PREC_FP64, x, ws.ax64, nullptr, st);
    k_residual<double, double, double>(b, ws.ax64, n, r, ws.partial, st);
  }
  RT_HIP(hipMemcpyAsync(rhat, r, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
  RT_HIP(hipMemsetAsync(pv, 0, (size_t)n * sizeof(double), st));
  RT_HIP(hipMemsetAsync(v, 0, (size_t)n * sizeof(double), st));
  BicgState init{1.0, 1.0, 1.0, 0.0, 0.0, 0.0, 0, 0};
  RT_HIP(hipMemcpyAsync(bs, &init, sizeof(init), hipMemcpyHostToDevice, st));
  double rn = vec_norm<double>(r, n, ws, st);
  res.beta = rn;
  if (hist) hist->push_back(rn / bnorm);
  BicgState hs{};
  auto read_bs = [&]() {
    RT_HIP(hipMemcpyAsync(ws.host, bs, sizeof(BicgState), hipMemcpyDeviceToHost, st));
    RT_HIP(hipStreamSynchronize(st));
    std::memcpy(&hs, ws.host, sizeof(BicgState));
  };
  int it = 0;
  while (rn > rtol * bnorm && it < max_iters) {
    k_dots4<double>(rhat, r, nullptr, nullptr, 1, n, ws.partial, st);
    k_bicg_scalar(ws.partial, n, 0, bs, st);
    k_bicg_p<double>(r, v, pv, n, bs, st);
    operator_apply(p, RT_PREC_FP64, pv, v, nullptr, st);
    k_dots4<double>(rhat, v, nullptr, nullptr, 1, n, ws.partial, st);
    k_bicg_scalar(ws.partial, n, 1, bs, st);
    k_bicg_s<double>(r, v, n, bs, ws.partial, st);  // r now holds s
    k_finish_norm_simple(ws.partial, n, ws.scal, st);
    const double sn = read_scalar(ws.scal, st, ws);
    read_bs();
    it++;
    if (hs.breakdown) return RT_E_BREAKDOWN;
    if (sn <= rtol * bnorm) {
      k_bicg_xr<double, double>(x, pv, r, t, n, bs, 1, ws.partial, st);
      rn = sn;
      if (hist) hist->push_back(rn / bnorm);
      break;
    }
    operator_apply(p, RT_PREC_FP64, r, t, nullptr, st);
    k_dots4<double>(t, r, t, t, 2, n, ws.partial, st);
    k_bicg_scalar(ws.partial, n, 2, bs, st);
    k_bicg_xr<double, double>(x, pv, r, t, n, bs, 0, ws.partial, st);
    k_finish_norm_simple(ws.partial, n, ws.scal, st);
    rn = read_scalar(ws.scal, st, ws);
    read_bs();
    if (!std::isfinite(rn)) fail(RT_E_NONFINITE, "non-finite residual");
    if (hist) hist->push_back(rn / bnorm);
    if (hs.breakdown) return RT_E_BREAKDOWN;
    // next iteration's scalar stage uses iter > 0
    int one = 1;
    RT_HIP(hipMemcpyAsync(&bs->iter, &one, sizeof(int), hipMemcpyHostToDevice, st));
  }
  res.iters = it;
  // true residual
  operator_apply(p, RT_PREC_FP64, x, ws.ax64, nullptr, st);
  k_residual<double, double, double>(b, ws.ax64, n, ws.r64, ws.partial, st);
  k_finish_norm_simple(ws.partial, n, ws.scal, st);
  res.beta = read_scalar(ws.scal, st, ws);
  return res.beta <= rtol * bnorm ? RT_OK : RT_NOT_CONVERGED;
}

// Inner solve of the refinement with BiCGStab (van der Vorst 1992) in FP32
// vectors and the low-precision operator, FP64 dot products: A_lo d = r32
// (r32 of unit norm on entry; overwritten) from d = 0 until the recursive
// residual estimate is below itol or after cap iterations, or at a
// breakdown (d then holds the last iterate, which the outer FP64 residual
// judges).  Returns the iterations taken.
int bicgstab_inner_f32(Problem& p, int prec, float* r, float* d, double itol, int cap,
                       Workspace& ws, hipStream_t st) {
  const int64_t n = p.n;
  float* rhat = reinterpret_cast<float*>(ws.bic);
  float* pv = rhat + n;
  float* v = rhat + 2 * n;
  float* t = rhat + 3 * n;
  BicgState* bs = ws.bs;
  RT_HIP(hipMemsetAsync(d, 0, (size_t)n * sizeof(float), st));
  RT_HIP(hipMemcpyAsync(rhat, r, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st));
  RT_HIP(hipMemsetAsync(pv, 0, (size_t)n * sizeof(float), st));
  RT_HIP(hipMemsetAsync(v, 0, (size_t)n * sizeof(float), st));
  BicgState init{1.0, 1.0, 1.0, 0.0, 0.0, 0.0, 0, 0};
  RT_HIP(hipMemcpyAsync(bs, &init, sizeof(init), hipMemcpyHostToDevice, st));
  BicgState hs{};
  auto read_bs = [&]() {
    RT_HIP(hipMemcpyAsync(ws.host, bs, sizeof(BicgState), hipMemcpyDeviceToHost, st));
    RT_HIP(hipStreamSynchronize(st));
    std::memcpy(&hs, ws.host, sizeof(BicgState));
  };
  int it = 0;
  while (it < cap) {
    k_dots4<float>(rhat, r, nullptr, nullptr, 1, n, ws.partial, st);
    k_bicg_scalar(ws.partial, n, 0, bs, st);
    k_bicg_p<float>(r, v, pv, n, bs, st);
    operator_apply(p, prec, pv, v, nullptr, st);
    k_dots4<float>(rhat, v, nullptr, nullptr, 1, n, ws.partial, st);
    k_bicg_scalar(ws.partial, n, 1, bs, st);
    k_bicg_s<float>(r, v, n, bs, ws.partial, st);   // r now holds s
    k_finish_norm_simple(ws.partial, n, ws.scal, st);
    const double sn = read_scalar(ws.scal, st, ws);
    read_bs();
    it++;
    if (hs.breakdown || !std::isfinite(sn)) break;
    if (sn <= itol) {
      k_bicg_xr<float, float>(d, pv, r, t, n, bs, 1, ws.partial, st);
      break;
    }
    operator_apply(p, prec, r, t, nullptr, st);
    k_dots4<float>(t, r, t, t, 2, n, ws.partial, st);
    k_bicg_scalar(ws.partial, n, 2, bs, st);
    k_bicg_xr<float, float>(d, pv, r, t, n, bs, 0, ws.partial, st);
    k_finish_norm_simple(ws.partial, n, ws.scal, st);
    const double rn = read_scalar(ws.scal, st, ws);
    read_bs();
    if (hs.breakdown || !std::isfinite(rn) || rn <= itol) break;
    int one = 1;
    RT_HIP(hipMemcpyAsync(&bs->iter, &one, sizeof(int), hipMemcpyHostToDevice, st));
  }
  return it;
}

}  // namespace

rt_status solve(Problem& p, const rt_solver_opts& o, const double* b_in, double* x,
                int x_is_guess, rt_solve_stats* stats, hipStream_t st) {
  auto t0 = std::chrono::steady_clock::now();
  const bool mixed = o.precision != RT_PREC_FP64;
  const bool bicg = o.krylov == RT_KRYLOV_BICGSTAB;
  const bool pre = o.precond == RT_PRECOND_LOCAL;
  if (pre) {
    if (o.basis_fp16) precond_prepare_h(p, st);
    else precond_prepare(p, mixed ? 4 : 8, st);
  }
  Workspace& ws = ensure_workspace(p, o.restart, mixed, bicg,
                                   !mixed ? 8 : (o.basis_fp16 ? 2 : 4));
  const int64_t n = p.n;
  p.history.clear();
  std::vector<double>* hist = o.record_history ? &p.history : nullptr;

  const double* b = b_in;
  const double bnorm = vec_norm<double>(b, n, ws, st);
  rt_status status = RT_OK;
  CoreResult res;
  int outer = 0;
  if (bnorm == 0.0) {
    RT_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), st));
    RT_HIP(hipStreamSynchronize(st));
    if (hist) hist->push_back(0.0);
  } else if (!mixed && !bicg) {
    status = gmres_core<double>(p, RT_PREC_FP64, b, x, !x_is_guess, o.restart, o.rtol,
                                o.max_iters, bnorm, ws, ws.ax64, st, hist, res, false,
                                o.two_step != 0, pre);
    outer = res.cycles;
  } else if (!mixed && bicg) {
    status = bicgstab_fp64(p, b, x, !x_is_guess, o.rtol, o.max_iters, bnorm, ws, st, hist, res);
  } else {
    if (bicg && o.basis_fp16) fail(RT_E_INVALID, "an fp16 basis is a GMRES option");
    // FP64 iterative refinement: r = b - A_64 x; inner A_lo d = r/||r|| (one
    // GMRES(m) cycle); x += ||r|| d.  Stops at rtol, at max_outer, or after
    // three steps without residual reduction.
    if (!x_is_guess) RT_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), st));
    double rn;
    if (!x_is_guess) {
      RT_HIP(hipMemcpyAsync(ws.r64, b, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
      rn = bnorm;
    } else {
      operator_apply(p, RT_PREC_FP64, x, ws.r64, nullptr, st);
      k_residual<double, double, double>(b, ws.r64, n, ws.r64, ws.partial, st);
      k_finish_norm_simple(ws.partial, n, ws.scal, st);
      rn = read_scalar(ws.scal, st, ws);
    }
    if (hist) hist->push_back(rn / bnorm);
    int total_inner = 0, stalls = 0;
    while (rn > o.rtol * bnorm && outer < o.max_outer && total_inner < o.max_iters) {
      outer++;
      float* r32 = ws.t32;
      if (!o.basis_fp16) k_convert<double, float>(ws.r64, r32, n, 1.0 / rn, st);
      double itol = o.inner_rtol;
      const double need = o.rtol * bnorm / rn;
      if (need > itol) itol = need;
      const int cap = std::min(o.restart, o.max_iters - total_inner);
      if (bicg) {
        // inner BiCGStab on the FP32 residual, at most `restart` iterations
        total_inner += bicgstab_inner_f32(p, o.precision, r32, ws.d32, itol, cap, ws, st);
      } else if (o.basis_fp16) {
        total_inner += inner_cycle_fp16(p, o.precision, ws.r64, rn, ws.d32, o.restart, itol, cap,
                                        ws, st, o.two_step != 0, pre);
      } else {
        // a pair's second application takes u1 = K v_j unnormalised; the
        // 16-bit operators' fp16 Lambda scale assumes entries of at most
        // about one, which |(1 - eps) Mhat|_inf <= 2 keeps (the physical
        // kernels give about 1); above that the steps go one at a time.
        // Preconditioned, both steps feed P^-1 of a vector of about unit
        // size to Lambda, as a single step does (an fp16 overflow would stop
        // the solve with RT_E_NONFINITE).
        const bool pairs = o.two_step != 0 &&
                           (o.precision == RT_PREC_FP32 || p.scatter_inf <= 2.0);
        CoreResult ir;
        gmres_core<float>(p, o.precision, r32, ws.d32, true, o.restart, itol, cap, 1.0, ws,
                          nullptr, st, nullptr, ir, /*single_cycle=*/true, pairs, pre);
        total_inner += ir.iters;
      }
      RT_HIP(hipMemcpyAsync(ws.scal + 1, &rn, sizeof(double), hipMemcpyHostToDevice, st));
      k_axpy_f64(x, ws.d32, n, ws.scal + 1, st);
      operator_apply(p, RT_PREC_FP64, x, ws.r64, nullptr, st);
      k_residual<double, double, double>(b, ws.r64, n, ws.r64, ws.partial, st);
      k_finish_norm_simple(ws.partial, n, ws.scal, st);
      const double rn_new = read_scalar(ws.scal, st, ws);
      if (!std::isfinite(rn_new)) fail(RT_E_NONFINITE, "non-finite residual");
      stalls = rn_new >= 0.9 * rn ? stalls + 1 : 0;
      rn = rn_new;
      if (hist) hist->push_back(rn / bnorm);
      if (stalls >= 3) break;
    }
    res.iters = total_inner;
    res.beta = rn;
    status = rn <= o.rtol * bnorm ? RT_OK : RT_NOT_CONVERGED;
  }
  RT_HIP(hipStreamSynchronize(st));
  auto t1 = std::chrono::steady_clock::now();
  if (stats) {
    stats->iters = res.iters;
    stats->outer_iters = outer;
    stats->relres = bnorm > 0 ? res.beta / bnorm : 0.0;
    stats->converged = status == RT_OK;
    stats->ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    stats->history_len = (int)p.history.size();
    stats->history = p.history.empty() ? nullptr : p.history.data();
  }
  return status;
}

}  // namespace rtsn
