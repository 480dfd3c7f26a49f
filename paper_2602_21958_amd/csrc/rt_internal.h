// Internal declarations of the rtsn library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <shared_mutex>
#include <string>
#include <vector>

#include "rtsn.h"

namespace rtsn {

// --------------------------------------------------------------------------
// Errors: internal code throws RtError; the ABI layer converts to rt_status.
struct RtError {
  rt_status code;
  std::string msg;
};
[[noreturn]] void fail(rt_status code, const std::string& msg);
void set_last_error(const std::string& msg);
bool profile_enabled();
// Held shared by problem create/destroy (device allocations) and exclusively
// while a batch engine captures a hipGraph, so no allocation from another
// thread lands inside a capture.
std::shared_mutex& capture_mutex();
void hip_check(hipError_t e, const char* what);
#define RT_HIP(call) ::rtsn::hip_check((call), #call)

// --------------------------------------------------------------------------
// Host-side discretisation tables (FP64), built in setup.cpp.
struct Tables {
  std::vector<double> mu_o, w_o;        // per ordinate: direction cosine, weight
  std::vector<double> om_x, om_y;       // per ordinate horizontal components (box)
  std::vector<double> x_nu, w_nu, phi;  // per frequency
  std::vector<double> mu_ray, w_ray, phi_ray, fac_ray;  // per ray k = o*n_nu+nu
  std::vector<double> mhat;             // n_r x n_r row-major
  // Factored form of Mhat for the dipole x PRD kernel (frank = 0 otherwise):
  // Mhat[(o,nu),(o',nu')] = sum_q fq[o][q] fg[o'][q] * fb[nu][nu'], with
  // fq (n_om x frank) the angular basis, fg (n_om x frank) the weighted
  // coefficients and fb (n_nu x n_nu) the frequency block
  // diag(1/(phi + r)) P_nu diag(w_nu).
  int frank = 0;
  std::vector<double> fq, fg, fb;
};

void build_tables(const rt_problem_desc& d, Tables& t);
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Upwind stencil of one box ordinate (plane-to-plane short characteristics).
struct BoxStencil {
  int i0, j0;       // upwind cell offsets, reduced mod nx / ny (>= 0)
  int up;           // 1: sweep bottom -> top (mu > 0), 0: top -> bottom
  int pad;
  double tx, ty;    // bilinear fractions
  double path;      // dz / |mu|
  // downwind point (quadratic short characteristics): the opposite
  // displacement on the next plane downstream
  int di0, dj0;
  double dtx, dty;
  // FP64 forms of the bilinear weights (1-ty)(1-tx), (1-ty)tx, ty(1-tx), ty tx
  // and of path / 2, formed once here so that an FP64 sweep reads them from
  // scalar registers instead of holding them in vector ones
  double w00, w01, w10, w11, hpath;
};

// --------------------------------------------------------------------------
// Device-resident problem.
struct Workspace;

struct Problem {
  int device = 0;
  int geom = RT_GEOM_SLAB;
  int nx = 1, ny = 1, nz = 2;
  int n_mu = 2, n_az = 1, n_nu = 1, n_omega = 2, n_r = 2;
  int64_t n_s = 0, n = 0;
  int formal = RT_FORMAL_LINEAR_SC;
  double r = 0, i_top = 0, i_bot = 0;
  Tables tab;
  std::vector<BoxStencil> stencil;      // box: per ordinate

  // device data
  double* d_mhat64 = nullptr;           // Mhat transposed: (k, k') at k' * lda_mhat + k
  float* d_mhat32 = nullptr;            // same layout
  int lda_mhat = 0;                     // n_r rounded up to a multiple of 128
  // 16-bit copies of Mhat for the MFMA GEMM, "k8" layout: element (k, k') at
  // ((k' / 8) * mp16 + k) * 8 + k' % 8, zero padded to mp16 rows and kp16
  // columns.
  uint16_t* d_a8_bf16 = nullptr;        // bf16 (hi part of the split)
  uint16_t* d_a8_bf16_lo = nullptr;     // bf16 of Mhat - hi
  uint16_t* d_a8_f16 = nullptr;         // fp16, rows scaled to unit maximum
  float* d_f16_rowscale = nullptr;      // n_r: undo factor per row k
  int mp16 = 0, kp16 = 0;               // n_r rounded up to 256 / to 64
  int64_t np16 = 0;                     // n_s rounded up to 256
  // 16-bit B operand (Lambda output), "k4" layout: element (k, i) at
  // ((k / 4) * np16 + i) * 4 + k % 4; two parts (hi, lo) of kp16 * np16
  // values each.  Zero-filled at allocation: padding rows must stay zero.
  uint16_t* d_l16 = nullptr;
  int g16_cfg[3] = {-1, -1, -1};        // tuned tile configuration per 16-bit mode
  double scatter_inf = 0;               // max_k sum_k' |(1 - eps) Mhat[k, k']| (about 1
                                        // for the physical kernels; an fp16 basis is
                                        // refused above 2)
  double* d_albedo = nullptr;           // n_s: 1 - eps_i
  double* d_thermal = nullptr;          // n: t
  double* d_dt = nullptr;               // slab: nz-1 depth increments
  double* d_kline = nullptr;            // box: n_s
  double* d_ray_mu = nullptr;           // n_r
  double* d_ray_fac = nullptr;          // n_r: phi_nu + r
  BoxStencil* d_stencil = nullptr;      // box: n_omega
  double* d_rhs = nullptr;              // physical right-hand side (lazily built)
  void* d_lbuf = nullptr;               // scratch for Lambda output (apply_operator)
  size_t lbuf_bytes = 0;
  // factored scattering form (dipole x PRD kernels): factors of Mhat in FP64
  // and FP32 (see Tables), the form FP64 / FP32 applications use, and the
  // lazily allocated W / Z work vectors of the factored passes
  double *d_fq64 = nullptr, *d_fg64 = nullptr, *d_fb64 = nullptr;
  float *d_fq32 = nullptr, *d_fg32 = nullptr, *d_fb32 = nullptr;
  int sigma_form = RT_SIGMA_DENSE;
  void* d_fwork = nullptr;
  size_t fwork_bytes = 0;
  // per-point scattering classes (n_classes > 1): one transposed Mhat per
  // class (class_mhat_stride elements apart), the points sorted by class
  // (d_cidx, class c at class_off[c] .. class_off[c + 1]) with their albedo
  // in that order (d_calb), and the gathered operand / product work buffer
  int n_classes = 1;
  size_t class_mhat_stride = 0;
  double* d_cmhat64 = nullptr;
  float* d_cmhat32 = nullptr;
  int32_t* d_cidx = nullptr;
  double* d_calb = nullptr;
  std::vector<int64_t> class_off;
  void* d_cwork = nullptr;
  size_t cwork_bytes = 0;
  // emulated FP64 scattering (RT_SIGMA_OZAKI): residues of the scaled Mhat
  // for every modulus in the 16-bit GEMM's A layout, the row scales, and the
  // per-call work (column scales, B and C residues)
  uint16_t* d_oz_a = nullptr;
  int* d_oz_ea = nullptr;
  void* d_ozwork = nullptr;
  size_t ozwork_bytes = 0;
  // physics-based preconditioner (precond.hip), built by precond_prepare:
  // the kept angular modes (prec_rq <= 6 eigenvalues of the angular block,
  // F and G n_omega x prec_rq), the direction-averaged plane response Dbar
  // (n_nu x n_s, FP64), the per-point blocks T (prec_rq x n_s blocks of
  // n_nu x n_nu, FP64 and / or FP32) and the apply's work (r, z and the
  // u, nd vectors)
  int prec_rq = 0;
  std::vector<double> prec_lam, prec_F, prec_G;
  double* d_prec_dbar = nullptr;
  double *d_prec_F64 = nullptr, *d_prec_G64 = nullptr, *d_prec_T64 = nullptr;
  float *d_prec_F32 = nullptr, *d_prec_G32 = nullptr, *d_prec_T32 = nullptr;
  // fp16 copy of the FP32 blocks for the solves on fp16 bases (null when an
  // entry falls outside fp16's range; prec_t16_tried then stops a retry)
  _Float16* d_prec_T16 = nullptr;
  bool prec_t16_tried = false;
  void* d_prec_work = nullptr;
  size_t prec_work_bytes = 0;
  Workspace* ws = nullptr;
  int64_t bytes_problem = 0;
  std::vector<double> history;

  ~Problem();
};

void problem_build(Problem& p, const rt_problem_desc& d);
void* problem_lbuf(Problem& p, size_t bytes);

// --------------------------------------------------------------------------
// Kernel launchers.  Vector types: V = double (FP64) or float (others).
// Lambda output type LT: double, float, __hip_bfloat16 or __half.
// out = Lambda(scale * s) * out_mul (+ boundary term if with_bc)
template <typename VT, typename LT>
void launch_lambda(const Problem& p, const VT* s, LT* out, bool with_bc,
                   const double* scale, hipStream_t st, float out_mul = 1.f);
// Lambda (no boundary term) of an FP32 vector into the k4 16-bit operand of
// the scattering GEMM (hi; lo for BF16X3), scaled for FP16.
void launch_lambda_k4(const Problem& p, int precision, const float* s, uint16_t* hi,
                      uint16_t* lo, const double* scale, hipStream_t st);
// Same for an fp16 vector (a Krylov basis vector stored in half precision).
void launch_lambda_k4(const Problem& p, int precision, const _Float16* s, uint16_t* hi,
                      uint16_t* lo, const double* scale, hipStream_t st);
float fp16_lambda_scale(int64_t n);
// Power-of-two scale of an fp16 Krylov basis of vectors of n entries.
float fp16_basis_scale(int64_t n);
// Frequencies swept together by one box workgroup for planes of PH values in
// LDS (the plane with its halo row and column).
int box_chunk(size_t PH, int elem_bytes, int max_lds);
// Whether box sweeps of F frequencies per group on planes of P points (PH in
// LDS) keep two alternating LDS sets (one barrier per plane): F == 1,
// P <= 1024 or 4-byte values, and 2 (2F + 1) PH elements within max_lds
// bytes.
bool box_pingpong(int F, int P, size_t PH, int elem_bytes, int max_lds);
// Size in elements of one part of the k4 operand; allocation of the
// problem's (zeroed) two-part buffer.
int64_t l16_part_elems(const Problem& p);
uint16_t* problem_l16(Problem& p, hipStream_t st);
const char* gemm16_config_name(int cfg);
// FP32 ray-major L -> k4 16-bit operand (rounded like Lambda's output).
void convert_to_k4(const Problem& p, int precision, const float* L, uint16_t* hi, uint16_t* lo,
                   hipStream_t st);

namespace gemm { struct TileDots; }
// y = xs * x + sign * albedo .* (Mhat L); x may be null (then xs ignored).
// With dots, the GEMM also forms partial sums of V_q . y (q < dots->nv) in
// dots->part[q * ldp + tile]: dots->ldp holds the capacity on entry
// (sigma_dot_slots gives the largest count any tile shape needs) and the
// number of tiles, every slot written, on return.
void launch_sigma_f64(const Problem& p, const double* L, const double* x, double* y,
                      const double* xscale, double sign, hipStream_t st,
                      gemm::TileDots* dots = nullptr);
void launch_sigma_f32(const Problem& p, const float* L, const float* x, float* y,
                      const double* xscale, double sign, hipStream_t st,
                      gemm::TileDots* dots = nullptr);
// 16-bit operands: L16 = k4 operand (hi, lo parts for BF16X3).
void launch_sigma_b16(Problem& p, int precision, const uint16_t* l_hi, const uint16_t* l_lo,
                      const float* x, float* y, const double* xscale, double sign,
                      hipStream_t st, gemm::TileDots* dots = nullptr);
// Same with x and y in fp16 and the whole output multiplied by ymul.
void launch_sigma_b16_h(Problem& p, int precision, const uint16_t* l_hi, const uint16_t* l_lo,
                        const _Float16* x, _Float16* y, float ymul, const double* xscale,
                        double sign, hipStream_t st);
int sigma_dot_slots(const Problem& p, int precision);

// Operator y = A (xs x) in the given precision, using the problem's L buffer;
// with dots, also the partial sums of V_q . y (see launch_sigma_f64).
void operator_apply(Problem& p, int precision, const void* x, void* y,
                    const double* xscale, hipStream_t st,
                    gemm::TileDots* dots = nullptr);
// The scattering part alone, y = K (xs x) with K = (1 - eps) Mhat Lambda =
// I - A (no x term: the GEMM epilogue reads no x).
void operator_apply_k(Problem& p, int precision, const void* x, void* y,
                      const double* xscale, hipStream_t st,
                      gemm::TileDots* dots = nullptr);
// 16-bit operator precisions on an fp16 basis: y = ymul A (xs x), or with
// kform y = ymul K (xs x) (no x term).
void operator_apply_h(Problem& p, int precision, const _Float16* x, _Float16* y,
                      const double* xscale, float ymul, hipStream_t st, bool kform = false);
// rt_apply_operator's arithmetic (FP64 / FP32, dense scattering form) with
// the formal solution held in a fixed device array instead of the problem's
// buffer; no device memory is allocated.
void operator_apply_noalloc(Problem& p, int precision, const void* x, void* y, hipStream_t st);
size_t lambda_elem_bytes(int precision);
// Factored scattering (sigma_factored.hip): y = xs x + sign (1 - eps) Mhat L
// through the rank-R angular and the frequency factors; work holds
// factored_work_elems(p) elements.  factored_fits: the mix pass's LDS fits.
size_t factored_work_elems(const Problem& p);
bool factored_fits(const Problem& p, int elem_bytes);
void launch_sigma_factored_f64(const Problem& p, const double* L, const double* x, double* y,
                               double* work, const double* xscale, double sign, hipStream_t st);
void launch_sigma_factored_f32(const Problem& p, const float* L, const float* x, float* y,
                               float* work, const double* xscale, double sign, hipStream_t st);
// The same with the preconditioner's correction as the x term: y = xs (-Delta)
// + (1 - eps) Mhat L with Delta = sum_q Fp[o][q] zp[q][nu][i] (rp modes), i.e.
// the preconditioned step's v - u formed in the expansion (precond_fused).
void launch_sigma_factored_pre_f64(const Problem& p, const double* L, const double* Fp,
                                   const double* zp, int rp, double* y, double* work,
                                   const double* xscale, hipStream_t st);
void launch_sigma_factored_pre_f32(const Problem& p, const float* L, const float* Fp,
                                   const float* zp, int rp, float* y, float* work,
                                   const double* xscale, hipStream_t st);
// ... into an fp16 basis vector: y = ymul (xs (-Delta) + (1 - eps) Mhat L),
// rounded to fp16
void launch_sigma_factored_pre_h(const Problem& p, const float* L, const float* Fp,
                                 const float* zp, int rp, _Float16* y, float ymul, float* work,
                                 const double* xscale, hipStream_t st);
// y = ymul K' (xs v) into an fp16 basis vector for the preconditioned step
// with FP32 factored scattering: u = P^-1 v (FP32) already formed, v - u from
// the preconditioner's modes
void operator_apply_kxh(Problem& p, const float* u, _Float16* y, const double* xscale,
                        float ymul, hipStream_t st);
// Scattering with per-point classes (sigma_classes.hip): for each class,
// gather its points' columns of L, one GEMM with the class's Mhat and
// albedo, and scatter y = xs x + sign (result) to the class's columns.
// work holds 2 n_r max_c(class size) elements.
void launch_sigma_classes_f64(const Problem& p, const double* L, const double* x, double* y,
                              double* work, const double* xscale, double sign, hipStream_t st);
void launch_sigma_classes_f32(const Problem& p, const float* L, const float* x, float* y,
                              float* work, const double* xscale, double sign, hipStream_t st);
size_t classes_work_elems(const Problem& p);
// Physics-based preconditioner (precond.hip).  precond_prepare builds the
// tables for vectors of elem_bytes (8 FP64, 4 FP32) if missing (RT_E_INVALID
// without the dipole x PRD kernel for all points); precond_apply writes
// u = P^-1 x and nd = x - u; precond_apply_add adds P^-1 d to y.
// precond_u / precond_nd: two n-vectors of the apply's work for callers.
void precond_prepare(Problem& p, int elem_bytes, hipStream_t st);
// the angular modes and Dbar only
void precond_prepare_local(Problem& p, hipStream_t st);
// RT_E_INVALID unless the problem can take the preconditioner
void precond_check(const Problem& p);
size_t precond_table_bytes(const Problem& p, int elem_bytes);
template <typename T> void precond_apply(Problem& p, const T* x, T* u, T* nd, hipStream_t st);
template <typename T> void precond_apply_add(Problem& p, const T* d, T* y, hipStream_t st);
// The solves on fp16 bases: precond_prepare_h adds an fp16 copy of the FP32
// blocks (where every entry fits); precond_apply_h forms u = P^-1 x for an
// fp16 basis vector x (FP32 u; v - u is left to the factored expansion, as
// with precond_fused) and precond_apply_add_h adds P^-1 d to y, both with the
// fp16 blocks where they exist, so that the steps and the cycle end apply
// the same preconditioner.
void precond_prepare_h(Problem& p, hipStream_t st);
void precond_apply_h(Problem& p, const _Float16* x, float* u, hipStream_t st);
void precond_apply_add_h(Problem& p, const float* d, float* y, hipStream_t st);
template <typename T> T* precond_u(Problem& p);
template <typename T> T* precond_nd(Problem& p);
// Whether the preconditioned step operator in this precision forms v - u in
// the scattering expansion (factored form in FP64 / FP32, one kernel for all
// points); then precond_apply may take nd = nullptr, and operator_apply_kx
// reads the last application's modes (precond_modes) instead of nd.
bool precond_fused(const Problem& p, int precision);
// the angular mode matrix F (n_omega x prec_rq) and the last application's
// mode values z (prec_rq x n_nu x n_s) of the tables in T
template <typename T> const T* precond_modes_F(Problem& p);
template <typename T> const T* precond_modes_z(Problem& p);
// y = xs * nd + K (xs * u): the preconditioned step operator K' = I - A P^-1
// applied to v with u = P^-1 v and nd = v - u (see solver.cpp); with
// precond_fused, nd is not read (may be null) and v - u comes from the
// preconditioner's modes
void operator_apply_kx(Problem& p, int precision, const void* u, const void* nd, void* y,
                       const double* xscale, hipStream_t st);
// Emulated FP64 scattering (sigma_ozaki.hip): ozaki_prepare builds the Mhat
// residues once; launch_sigma_ozaki computes y = xs x + sign (1 - eps) Mhat L
// with work of ozaki_work_bytes(p) bytes.
void ozaki_prepare(Problem& p);
size_t ozaki_work_bytes(const Problem& p);
void launch_sigma_ozaki(const Problem& p, const double* L, const double* x, double* y,
                        void* work, const double* xscale, double sign, hipStream_t st);
// RT_E_INVALID naming `what` when the problem has per-point classes.
void require_one_kernel(const Problem& p, const char* what);
// Dense GEMM y = xs x + sign albedo .* (A L) with explicit operands: A
// transposed (lda), L and y N columns wide (sigma_gemm.hip).
void launch_gemm_f64(const Problem& p, const double* A, const double* L, int N,
                     const double* x, double* y, const double* albedo, const double* xscale,
                     double sign, hipStream_t st);
void launch_gemm_f32(const Problem& p, const float* A, const float* L, int N, const float* x,
                     float* y, const double* albedo, const double* xscale, double sign,
                     hipStream_t st);
// Scattering step of FP64 / FP32 applications in the problem's form (dense
// GEMM or factored); fused dots need the dense GEMM.
void apply_sigma_f64(Problem& p, const double* L, const double* x, double* y,
                     const double* xscale, double sign, hipStream_t st,
                     gemm::TileDots* dots = nullptr);
void apply_sigma_f32(Problem& p, const float* L, const float* x, float* y,
                     const double* xscale, double sign, hipStream_t st,
                     gemm::TileDots* dots = nullptr);
const double* physical_rhs(Problem& p, hipStream_t st);

// Kernel timing (rt_profile_*): RAII scope recording a start/stop event pair
// on `st` around the launches it encloses when profiling is enabled.
class ProfScope {
 public:
  ProfScope(int kclass, hipStream_t st);
  ~ProfScope();

 private:
  int kclass_;
  hipStream_t st_;
  hipEvent_t start_ = nullptr;
};

}  // namespace rtsn
