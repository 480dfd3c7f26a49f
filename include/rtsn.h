/*
 * rtsn.h - C ABI of the MI355X (gfx950) matrix-free S_N radiative-transfer
 * library.
 *
 * The library solves the discrete linear radiative-transfer problem of
 * Benedusi, Riva, Belluzzi and Serra-Capizzano, "Analysis of eigenvalue
 * clustering leads to optimal scaling in numerical radiative transfer"
 * (arXiv:2602.21958), written in source-function form:
 *
 *     A s = s - (1 - eps) Mhat Lambda_0 s = b,
 *     b   = (1 - eps) Mhat I_bc + t,
 *
 * where Lambda_0 is the formal solution with zero incoming radiation
 * (Sec. 3.2, eqs. ie_1/ie_2 and eq. lambda_block), Mhat the scattering block
 * diag(1/(phi_nu + r)) Psi diag(w_o w_nu) shared by all spatial points
 * (Sec. 3.3, eq. Sigma), I_bc the boundary intensity propagated through the
 * medium (Sec. 3.1, the I_in vector) and t the thermal source (eq. S).  This
 * is the system (Id - Lambda Sigma) I = Lambda t + I_in of eq.
 * RT_sys_algebraic after the substitution I = Lambda_0 s + I_bc; both forms
 * have the same spectrum (Sec. 3.5).
 *
 * Conventions
 * -----------
 * Vector layout ("ray-major", the permuted ordering X~ = P X of Sec. 3.1):
 *   element [k * n_points + i], ray k = o * n_nu + nu (frequency fastest,
 *   Sec. 3.1 ray ordering), ordinate o (slab: inclination index, mu
 *   ascending; box: o = m * n_az + b, inclination-major), point i
 *   (slab: depth index, 0 = top; box: i = (z * ny + y) * nx + x, z = 0 is
 *   the bottom plane).
 * Device pointers: every vector argument marked "device" is memory of the
 *   problem's device (hipMalloc'd or torch CUDA memory); "host" arrays are
 *   ordinary CPU memory.  The library never frees caller memory and keeps no
 *   pointer to it after the call returns.
 * Streams: `stream` is a hipStream_t passed as void* (NULL = null stream).
 *   Calls are asynchronous on that stream unless stated otherwise.
 * Errors: every call returns an rt_status; on failure rt_last_error() gives a
 *   message (thread-local).  No C++ exception and no abort crosses the ABI.
 *   Invalid arguments are rejected on the host before any kernel launch.
 * Threading: one problem is used by one host thread at a time.
 */
#ifndef RTSN_H
#define RTSN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RTSN_VERSION 1

typedef enum {
  RT_OK = 0,
  RT_NOT_CONVERGED = 1,   /* solver hit max_iters; x holds the last iterate */
  RT_E_INVALID = -1,      /* bad argument (sizes, pointers, enum values)     */
  RT_E_NOMEM = -2,        /* device allocation failed                        */
  RT_E_DEVICE = -3,       /* HIP runtime error                               */
  RT_E_BREAKDOWN = -4,    /* BiCGStab breakdown (rho or omega vanished)      */
  RT_E_NONFINITE = -5,    /* NaN/Inf in an input or in a residual            */
  RT_E_BUSY = -6          /* batch: queue full / ticket still pending        */
} rt_status;

typedef struct rt_problem_s* rt_problem;
typedef struct rt_batch_s* rt_batch;

enum { RT_GEOM_SLAB = 0, RT_GEOM_BOX = 1 };
enum { RT_KERNEL_DIPOLE_PRD = 0, RT_KERNEL_EXPLICIT = 1 };
enum { RT_FORMAL_LINEAR_SC = 0, RT_FORMAL_IMPLICIT_EULER = 1, RT_FORMAL_QUADRATIC_SC = 2 };

/* Arithmetic of one operator application.
 *   FP64  : vectors double; Lambda and Sigma in FP64 (Sigma on FP64 MFMA).
 *   FP32  : vectors float;  Lambda FP32; Sigma FP32 MFMA.
 *   BF16  : vectors float;  Lambda FP32 emitting bf16; Sigma bf16 MFMA with
 *           FP32 accumulation; epilogue FP32.
 *   FP16  : as BF16 with fp16 operands (kernel-matrix rows scaled to unit
 *           maximum and Lambda output scaled by a power of two to stay in
 *           fp16 range; both undone in FP32).
 *   BF16X3: as BF16 but the kernel matrix and Lambda output are split into
 *           hi + lo bf16 parts and three products are accumulated (about
 *           16 significant bits).                                            */
enum { RT_PREC_FP64 = 0, RT_PREC_FP32 = 1, RT_PREC_BF16 = 2, RT_PREC_FP16 = 3,
       RT_PREC_BF16X3 = 4 };

/* Problem description (Sec. 2 model, Sec. 3.1 grids, Sec. 5 set-up).  All
 * pointers are host pointers; the library copies what it needs at create.   */
typedef struct {
  int geom;               /* RT_GEOM_SLAB or RT_GEOM_BOX                          */
  int nx, ny, nz;         /* spatial nodes; slab: nx = ny = 1, nz >= 2;
                             box: nx, ny >= 1 (periodic), nz >= 2; the box edge
                             is 1 in x, y and z: x_i = i/nx, z_k = k/(nz-1)      */
  const double* depth;    /* slab: nz frequency-integrated line optical depths t,
                             strictly increasing, index 0 = top; the optical depth
                             of ray (mu, nu) between nodes is (phi_nu + r) dt/|mu|
                             (Sec. 5 set-up, tau = phi t / mu)                     */
  const double* k_line;   /* box: nz*ny*nx line opacity per unit length (> 0),
                             C order (z, y, x), z = 0 bottom                      */
  int n_mu;               /* total inclinations (even): n_mu/2 Gauss-Legendre
                             nodes per hemisphere (Sec. 5 set-up)                  */
  int n_az;               /* azimuths (box; equidistant, (b+1/2) 2pi/n_az);
                             slab: 1                                               */
  int n_nu;               /* frequencies, equispaced on [-x_max, x_max], trapezoid
                             weights; Doppler profile exp(-x^2) normalised to unit
                             discrete area; n_nu = 1 is monochromatic (phi = 1)    */
  double x_max;
  double r;               /* continuum / line opacity ratio: chi = k (phi + r)     */
  double eps;             /* photon destruction probability (used if eps_field
                             is NULL)                                              */
  const double* eps_field;/* optional n_points per-point eps                       */
  double planck;          /* thermal source B (used if planck_field is NULL)       */
  const double* planck_field; /* optional n_points per-point B                     */
  double i_top, i_bot;    /* incoming intensity at the top (mu < 0) and bottom
                             (mu > 0) boundaries (eq. bc)                          */
  int kernel;             /* RT_KERNEL_DIPOLE_PRD or RT_KERNEL_EXPLICIT            */
  const double* kernel_matrix; /* EXPLICIT: n_rays*n_rays symmetric Psi, row-major
                             in ray order (Sec. 3.3, the block Psi_[i])            */
  double coh_frac;        /* DIPOLE_PRD: weight c of the coherent part            */
  double coh_width2;      /* DIPOLE_PRD: w2 in exp(-(x - x')^2 / w2)               */
  int formal;             /* RT_FORMAL_LINEAR_SC (box and slab),
                             RT_FORMAL_IMPLICIT_EULER (slab only, eqs. ie_1/ie_2)
                             or RT_FORMAL_QUADRATIC_SC: the integral form of the
                             transfer equation (Sec. 2, eq. rt_integral) with the
                             source taken as the parabola through the upwind,
                             local and downwind values (Sec. 5.3: the production
                             code's quadratic integrator); the last node of a
                             ray, which has no downwind node, takes the linear
                             step                                                 */
  /* Per-point scattering classes (Sec. 3.3: the block Psi_[i] of eq. Sigma may
   * differ from point to point).  n_classes <= 1: one kernel for every point
   * (the fields below are ignored).  n_classes > 1: point i scatters with the
   * block of class point_class[i]; DIPOLE_PRD kernels take the coherent
   * fraction class_coh_frac[c] per class (coh_width2 shared), EXPLICIT ones
   * the symmetric matrix class_kernels[c * n_rays^2 ...] (row-major; then
   * kernel_matrix is ignored).  FP64 and FP32 applications only, dense
   * scattering form; not in the batch engine.                               */
  int n_classes;
  const int32_t* point_class;   /* n_points ids in [0, n_classes)              */
  const double* class_coh_frac; /* DIPOLE_PRD: n_classes values in [0, 1]      */
  const double* class_kernels;  /* EXPLICIT: n_classes * n_rays * n_rays       */
} rt_problem_desc;

typedef struct {
  int64_t n_unknowns;     /* n_rays * n_points                                     */
  int64_t n_rays;         /* n_mu * n_az * n_nu                                    */
  int64_t n_points;       /* nx * ny * nz                                          */
  int64_t bytes_problem;  /* device bytes held by the problem itself               */
  int64_t bytes_solve_fp64;  /* extra device bytes of an FP64 GMRES(restart) solve
                                with the restart passed to rt_problem_footprint,
                                including the work buffer of the problem's
                                current scattering form (rt_problem_set_sigma) */
  int64_t bytes_solve_mixed; /* same for a mixed-precision (FP32 basis) solve.
                                Neither counts the preconditioner's tables
                                (rt_apply_precond: R' n_frequencies^2 n_points
                                values of the solve's precision, plus an fp16
                                copy for solves on an fp16 basis) nor its two
                                work vectors.                                   */
  int32_t sigma_rank;     /* angular rank of the factored scattering form (6 for
                             the 3D dipole, 2 for the slab's azimuth average; 0:
                             no factored form, explicit kernel)                  */
  int32_t sigma_form;     /* RT_SIGMA_DENSE or RT_SIGMA_FACTORED                  */
} rt_problem_info;

/* rt_problem_create: build quadratures, the redistribution kernel (dipole x
 * PRD with a Sinkhorn-scaled coherent part, Sec. 2 normalisation), Mhat, t
 * and 1 - eps on the host in FP64, and copy them to `device`.
 * Errors: RT_E_INVALID (sizes, missing arrays, non-increasing depth,
 * non-positive opacity, odd n_mu, implicit Euler in a box), RT_E_NONFINITE
 * (NaN/Inf inputs), RT_E_NOMEM, RT_E_DEVICE.  *out is NULL on failure.     */
rt_status rt_problem_create(const rt_problem_desc* desc, int device, rt_problem* out);

/* Release all device memory of the problem (and of its solver workspace).   */
rt_status rt_problem_destroy(rt_problem p);

/* Sizes and device footprint of a problem; restart = GMRES restart length
 * used for the solve estimates.                                             */
rt_status rt_problem_footprint(rt_problem p, int restart, rt_problem_info* info);

/* Copy the FP64 scattering block Mhat (n_rays x n_rays, row-major) and the
 * per-ray quadrature data to host arrays (any may be NULL): mu_ray (ray
 * direction cosine), w_ray (w_o w_nu), phi_ray (profile).  Synchronous.     */
rt_status rt_problem_tables(rt_problem p, double* mhat, double* mu_ray,
                            double* w_ray, double* phi_ray);

/* Formal solution (Sec. 3.2, eq. lambda_block; box: plane-to-plane upwind
 * short characteristics with bilinear interpolation, the short-
 * characteristics counterpart of the ray partition of Sec. 3.4):
 *   I = Lambda_0 (scale * s) + (with_bc ? I_bc : 0).
 * s, I: device, ray-major, n_unknowns elements of the precision's vector
 * type (double for FP64, float otherwise).  `scale` is an optional device
 * double (NULL = 1).  I must not alias s.  Errors: RT_E_INVALID.            */
rt_status rt_apply_lambda(rt_problem p, int precision, const void* s, void* I,
                          int with_bc, const double* scale, void* stream);

/* Scattering step (Sec. 3.3, eq. Sigma), as a GEMM shared by all points:
 *   y = x - (1 - eps) * Mhat * L      (x != NULL)
 *   y = (1 - eps) * Mhat * L          (x == NULL)
 * L, x, y: device, ray-major, vector type of the precision (for BF16/FP16/
 * BF16X3 L is float and is rounded to the 16-bit type inside).  y may alias
 * x.  Errors: RT_E_INVALID.                                                 */
rt_status rt_apply_sigma(rt_problem p, int precision, const void* L,
                         const void* x, void* y, void* stream);

/* Operator application y = A x = x - (1 - eps) Mhat Lambda_0 x (Sec. 3.5,
 * eq. A_N in source-function form).  x, y: device, ray-major, vector type of
 * the precision; y must not alias x.  Uses an internal device buffer for
 * Lambda_0 x.  Errors: RT_E_INVALID, RT_E_NOMEM.                            */
rt_status rt_apply_operator(rt_problem p, int precision, const void* x, void* y,
                            void* stream);

/* rt_apply_operator without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arithmetic, kernels and result as
 * rt_apply_operator; Lambda_0 x is held in a fixed 64 MiB device array of the
 * library instead of the problem's buffer.  One such array exists per GPU
 * for the life of the process and every call on that GPU shares it: calls
 * that overlap on one GPU (other streams, other threads, other problems)
 * race and must be serialised by the caller.  No entry of the array needs to
 * be cleared between calls (Lambda writes all n entries before the GEMM
 * reads them).  precision: RT_PREC_FP64 or RT_PREC_FP32 only, with the dense
 * scattering form (rt_problem_set_sigma).
 * Errors: RT_E_INVALID for other precisions or the factored form, for
 * n_unknowns * element size above 64 MiB (8 388 608 FP64 / 16 777 216 FP32
 * unknowns), null or aliased vectors; RT_E_DEVICE if the array's address
 * cannot be taken.                                                          */
rt_status rt_apply_operator_noalloc(rt_problem p, int precision, const void* x, void* y,
                                    void* stream);

/* How FP64 and FP32 applications compute the scattering step (Sec. 3.3,
 * eq. Sigma).  RT_SIGMA_DENSE (default): one dense N_r x N_r GEMM shared by
 * all points on the matrix cores, valid for any kernel Psi.
 * RT_SIGMA_FACTORED (dipole x PRD kernels only): Mhat is the Kronecker
 * product of an angular factor of exact rank R (R = 6 in 3D, where
 * 3/4 (1 + (O.O')^2) = q(O)^T C q(O') over the six quadratic monomials of O;
 * R = 2 for the slab's azimuth average) and the frequency block
 * diag(1/(phi + r)) P_nu diag(w_nu); the step runs as a reduction to R
 * angular moments, a frequency mix and an expansion, about
 * 4 R + 2 R N_nu / N_omega flops per unknown instead of 2 N_r (the low-rank
 * application that Sec. 4.1 remarks on; Sec. 5.1 notes the same rank
 * structure for a Legendre-series kernel), bound by HBM.  The 16-bit
 * precisions and the batch engine always use the dense GEMM.  Applies to
 * every later call on p (operator, Sigma, right-hand side, solves); the
 * physical right-hand side is rebuilt.  Synchronises the device.
 * RT_SIGMA_OZAKI (any kernel): FP64 applications emulate the dense FP64
 * GEMM with exact int8 matrix-core products (error-free splitting in the
 * integer-modular form of Ozaki, Uchino and Imamura, a published method, not
 * the paper's): M-hat's rows and L's columns scaled to 51-bit integers, their
 * residues modulo 15 pairwise coprime moduli <= 256 multiplied exactly in
 * int32, the product rebuilt by the Chinese remainder theorem; error about
 * 2^-51 of the largest entries of a row of M-hat and a column of L.  FP32
 * applications use the dense FP32 GEMM.  Work memory per problem:
 * 4 n_points + 30 ceil(n_rays / 128) 64 n_points_padded + 15 n_rays n_points
 * bytes (box64: 48 GB).
 * Errors: RT_E_INVALID (unknown form; factored with an explicit kernel or
 * with more frequencies than the mix pass's LDS holds, about 120; factored
 * or emulated with per-point classes).                                      */
enum { RT_SIGMA_DENSE = 0, RT_SIGMA_FACTORED = 1, RT_SIGMA_OZAKI = 2 };
rt_status rt_problem_set_sigma(rt_problem p, int form);

/* Right-hand side of the source-function system, b = (1 - eps) Mhat I_bc + t:
 * the scattering (Sec. 3.3, eq. Sigma) of the boundary radiation propagated
 * through the medium (the I_in vector of Sec. 3.1, eq. RT_sys_algebraic)
 * plus the thermal part of the source (Sec. 2, eq. S).  b: device, FP64,
 * ray-major, n_unknowns entries, caller-owned.  Built on the first call (or
 * solve) and kept with the problem; asynchronous on the stream.
 * Errors: RT_E_INVALID (null), RT_E_NOMEM.                                   */
rt_status rt_rhs(rt_problem p, double* b, void* stream);

/* Full intensity I = Lambda_0 s + I_bc of a source function s: the formal
 * solution with the boundary radiation (Sec. 3.2, eq. lambda_block, plus the
 * I_in vector of Sec. 3.1), e.g. the emergent spectrum of a solution.
 * s, I: device, FP64, ray-major, n_unknowns entries; I must not alias s.
 * Errors: RT_E_INVALID.                                                     */
rt_status rt_intensity(rt_problem p, const double* s, double* I, void* stream);

enum { RT_KRYLOV_GMRES = 0, RT_KRYLOV_BICGSTAB = 1 };

typedef struct {
  int krylov;             /* RT_KRYLOV_GMRES (default) or RT_KRYLOV_BICGSTAB (van der
                             Vorst; FP64 vectors in FP64 precision; in the mixed
                             precisions the inner solve of each refinement step,
                             on FP32 vectors with FP64 dot products; keeps no
                             basis)                                                */
  int restart;            /* GMRES restart length m (1..128; default 30); with
                             BiCGStab in a mixed precision, the iteration cap of
                             each inner solve                                     */
  int max_iters;          /* total inner iterations cap (default 10000)             */
  double rtol;            /* stop when ||b - A x||_2 <= rtol ||b||_2 (true residual,
                             FP64)                                                   */
  int precision;          /* RT_PREC_FP64: plain FP64 Krylov; any other value:
                             FP64 outer iterative refinement around an inner
                             solve of A_lo d = r in that precision                 */
  double inner_rtol;      /* mixed: inner relative tolerance (default 1e-3)         */
  int max_outer;          /* mixed: outer refinement cap (default 50)               */
  int record_history;     /* keep the per-iteration residual estimates              */
  int basis_fp16;         /* mixed with a 16-bit operator precision (RT_PREC_BF16,
                             RT_PREC_FP16, RT_PREC_BF16X3), or with RT_PREC_FP32
                             preconditioned (precond = RT_PRECOND_LOCAL) on the
                             factored scattering form (rt_problem_set_sigma):
                             keep the inner Krylov basis in fp16, stored times
                             2^11, which halves the bytes of every Arnoldi pass
                             (default 0: FP32 basis).  An inner cycle then gains
                             at most about kappa 2^-11: on ill-conditioned
                             problems the refinement takes more outer steps.
                             RT_E_INVALID with any other combination, or when a
                             row of
                             (1 - eps) |Mhat| sums to more than 2 (possible
                             only with an explicit kernel; the physical kernels
                             give about 1), which the basis scale assumes.      */
  int two_step;           /* GMRES (the FP64 solve, and the inner cycles of
                             mixed precision on FP32 or fp16 bases): take the
                             Arnoldi steps in pairs,
                             u1 = K v_j and u2 = K u1 with K = I - A,
                             orthogonalised together with one pass over the
                             basis for the dots and one for the update instead
                             of two each, plus one pass over the pair that
                             removes the new vector's component along the first
                             (default 1; 0: one step per pass).  Same Krylov
                             spaces and iterates in exact arithmetic.  Ignored
                             in BiCGStab.                                         */
  int precond;            /* RT_PRECOND_NONE (default: the unpreconditioned solve
                             the paper analyses) or RT_PRECOND_LOCAL: GMRES on
                             A P^-1 with the physics-based preconditioner of
                             rt_apply_precond (Sec. 6 remark on physics-based
                             preconditioning), FP64 or on the FP32 basis of the
                             mixed inner cycles, or on an fp16 basis with FP32
                             operators on the factored scattering form (see
                             basis_fp16); right preconditioning, so the
                             residual and stopping test are those of A x = b.
                             Dipole x PRD kernels with one kernel for all points;
                             not with BiCGStab or an fp16 basis of 16-bit
                             operators (RT_E_INVALID).
                             The first preconditioned solve in a precision builds
                             the preconditioner's tables (see rt_apply_precond)
                             and synchronises the device.                       */
} rt_solver_opts;

enum { RT_PRECOND_NONE = 0, RT_PRECOND_LOCAL = 1 };

typedef struct {
  int iters;              /* total Krylov iterations (inner iterations if mixed)    */
  int outer_iters;        /* refinement steps (mixed) or restart cycles (FP64)      */
  int converged;          /* 1 if the true relative residual <= rtol                */
  double relres;          /* final true relative residual, FP64 operator            */
  double ms;              /* wall time of the call                                  */
  int history_len;        /* number of entries in history                           */
  const double* history;  /* relative residual estimates (library-owned, valid until
                             the next call on this problem)                          */
} rt_solve_stats;

/* Fill opts with defaults (GMRES(30), rtol 1e-8, FP64).                     */
void rt_solver_opts_default(rt_solver_opts* opts);

/* Physics-based preconditioner (Sec. 6 remarks that physics-based
 * preconditioning can still cut iteration counts; Sec. 3.3 eq. Sigma for the
 * scattering block): y = P^-1 x with P block diagonal over points,
 *   P_i = Id - (1 - eps_i) Mhat diag_k(Dbar[nu(k)][i]),
 *   Dbar[nu][i] = sum_o w_o (Lambda_0 1_z)[(o, nu), i] / sum_o w_o,
 * where 1_z is a unit source on the plane z of point i (the slab: the depth
 * point), so Lambda_0 1_z restricted to that plane is the local part of the
 * formal solution (its diagonal with linear short characteristics or
 * implicit Euler).  For the dipole x PRD kernel P_i^-1 is applied through the
 * nonzero eigenvalues of the angular block (6 in 3D, 2 in the slab) as that
 * many N_nu x N_nu blocks per point.  x, y: device vectors of n_unknowns
 * FP64 (precision RT_PREC_FP64) or FP32 (RT_PREC_FP32), ray-major; y must not
 * alias x.  The first call in a precision builds the tables: one FP64 formal
 * solution per plane for Dbar, then the blocks (6 N_nu^2 n_points values of
 * the precision) and two work vectors; they stay with the problem.  Errors:
 * RT_E_INVALID (other precisions, null or aliased vectors, an explicit kernel
 * or per-point classes, more frequencies than the in-LDS inversion holds,
 * about 140), RT_E_NOMEM.                                                    */
rt_status rt_apply_precond(rt_problem p, int precision, const void* x, void* y, void* stream);

/* Dbar of rt_apply_precond (host array of n_frequencies x n_points doubles,
 * frequency-major), built if missing.  Synchronises the device.            */
rt_status rt_precond_local(rt_problem p, double* dbar);

/* Solve A s = b (restarted GMRES, Sec. 5 and Sec. 5.3; or BiCGStab).
 * b: device FP64 or NULL (then the physical right-hand side rt_rhs is used).
 * x: device FP64, n_unknowns; on entry the initial guess if x_is_guess,
 * otherwise ignored (x0 = 0); on exit the solution s.
 * The Krylov workspace is allocated on first use and kept on the device with
 * the problem (re-used by later solves).  Synchronises the stream.
 * Returns RT_OK, RT_NOT_CONVERGED (x valid), RT_E_BREAKDOWN,
 * RT_E_NONFINITE, RT_E_INVALID or RT_E_NOMEM.                                */
rt_status rt_solve(rt_problem p, const rt_solver_opts* opts, const double* b,
                   double* x, int x_is_guess, rt_solve_stats* stats, void* stream);

/* ---------------------------------------------------------------------------
 * Batched solves and serving (many independent problems on one device).
 * A batch engine owns a device-memory budget; submitted solves are admitted
 * when their footprint (rt_problem_footprint) fits and a slot is free,
 * otherwise queued.  Admitted solves advance together, one Krylov iteration
 * of every active slot per engine step; a slot freed by a finished solve is
 * given to the next queued request at the next step boundary.
 * ------------------------------------------------------------------------- */

/* Create an engine on `device`.  precision: the operator precision of every
 * solve in this engine (RT_PREC_FP64: plain restarted GMRES with FP64
 * vectors; otherwise FP64 iterative refinement around one-cycle inner GMRES
 * with FP32 vectors).  hbm_budget: bytes reserved at create for the solves'
 * workspaces (bases, residuals, scratch); max_slots: most concurrently
 * admitted solves; queue_cap: most queued requests; use_graph: replay the
 * inner step as a captured hipGraph.  Errors: RT_E_INVALID, RT_E_NOMEM.     */
rt_status rt_batch_create(int device, int precision, int64_t hbm_budget,
                          int max_slots, int queue_cap, int use_graph,
                          rt_batch* out);

/* Flags of rt_batch_create_ex.  RT_BATCH_BASIS_FP16: the inner Krylov bases
 * are fp16, scaled like rt_solver_opts.basis_fp16 (16-bit operator
 * precisions only); every submitted request must then set basis_fp16.      */
enum { RT_BATCH_BASIS_FP16 = 1 };

/* rt_batch_create with flags (0 or RT_BATCH_BASIS_FP16).  Errors as
 * rt_batch_create; RT_E_INVALID for unknown flags or an fp16 basis with a
 * precision other than RT_PREC_BF16, RT_PREC_FP16, RT_PREC_BF16X3.         */
rt_status rt_batch_create_ex(int device, int precision, int64_t hbm_budget,
                             int max_slots, int queue_cap, int use_graph,
                             int flags, rt_batch* out);

/* Submit a solve of problem p (which must stay alive until completion) for
 * its physical right-hand side.  opts->precision must equal the engine's;
 * GMRES only.  x_out: device FP64 n_unknowns of p, caller-owned; the engine
 * iterates in it from admission on and it holds the solution at completion.
 * Non-blocking; *ticket identifies the request.  RT_E_BUSY if the queue is
 * full; RT_E_INVALID if the problem can never fit the budget or if
 * opts->basis_fp16 differs from the engine's basis (set iff it was created
 * with RT_BATCH_BASIS_FP16).  opts->precond = RT_PRECOND_LOCAL runs the
 * solve preconditioned (see rt_solver_opts) on FP64 or FP32 bases (not in
 * an fp16-basis engine; RT_E_INVALID also where rt_apply_precond would
 * refuse the problem); its tables are built on the problem at admission
 * (once per problem and precision, synchronising the engine's stream) and
 * held by the problem outside the engine's budget, which holds the
 * preconditioner's four work vectors (2 n_unknowns and 2 * 6 n_frequencies
 * n_points elements of the basis type).  The engine applies the scattering
 * as the dense GEMM whatever form rt_problem_set_sigma chose for p (the same
 * operator; the factored and emulated forms are single-problem options).   */
rt_status rt_batch_submit(rt_batch b, rt_problem p, const rt_solver_opts* opts,
                          double* x_out, uint64_t* ticket);

/* Advance every admitted solve by one engine step (admit, iterate, retire).
 * Returns the number of solves still admitted or queued in *pending.         */
rt_status rt_batch_step(rt_batch b, int* pending);

/* RT_OK with stats when the ticket has finished, RT_E_BUSY while pending.    */
rt_status rt_batch_poll(rt_batch b, uint64_t ticket, rt_solve_stats* stats);

/* Step the engine until every submitted request has finished.               */
rt_status rt_batch_wait_all(rt_batch b);

/* Device bytes the engine reserves from its budget for one solve of p with
 * the given restart length (what admission checks against free memory).    */
rt_status rt_batch_footprint(rt_batch b, rt_problem p, int restart, int64_t* bytes);

/* Admitted solves, queued requests and arena bytes in use.                   */
rt_status rt_batch_info(rt_batch b, int* active, int* queued, int64_t* bytes_in_use);

rt_status rt_batch_destroy(rt_batch b);

/* ---------------------------------------------------------------------------
 * Kernel timing.  While enabled, every launch of the formal solver, of the
 * scattering GEMM and of the Arnoldi vector kernels (dots, update) is
 * bracketed by HIP events recorded on the stream it is launched on.  The
 * formal solver and the GEMM have one class for FP64 arithmetic (the plain
 * solve, and the outer residuals and right-hand side of a mixed solve) and
 * one for the lower precisions (FP32 sweeps, including those that emit the
 * 16-bit GEMM operand; FP32 and 16-bit GEMMs: the inner cycles).
 * rt_profile_read synchronises the recorded events and returns the number of
 * launches and their summed device time for one kernel class; `reset` clears
 * that class afterwards.  Process-wide, internally synchronised.
 * ------------------------------------------------------------------------- */
enum { RT_KCLASS_LAMBDA = 0, RT_KCLASS_SIGMA = 1, RT_KCLASS_ARNOLDI = 2,
       RT_KCLASS_LAMBDA_LO = 3, RT_KCLASS_SIGMA_LO = 4, RT_KCLASS_PRECOND = 5,
       RT_KCLASS_COUNT = 6 };

rt_status rt_profile_enable(int on);
rt_status rt_profile_read(int kclass, int64_t* launches, double* total_ms, int reset);

/* Shape the engine's grouped 16-bit scattering GEMM uses: a fixed 128x128
 * tile body (the same for every engine, so that a solve rounds identically
 * alone and in any mix) and a persistent grid size chosen at the engine's
 * first inner step by timing 512, 1024 and 2048 workgroups on the live work
 * lists.  RTSN_BATCH_GEMM16="<cfg>,<grid>" forces both.  Returns a string
 * owned by the engine ("untuned" before the first step, "" for NULL).       */
const char* rt_batch_gemm16_tile(rt_batch b);

/* Tile shape the 16-bit scattering GEMM uses for problem p in `precision`
 * (RT_PREC_BF16 / FP16 / BF16X3): chosen the first time the problem applies
 * that precision by timing the candidate shapes on the problem's own
 * operands, or forced with the environment variable RTSN_GEMM16_CFG=<index>.
 * Returns a static string ("untuned" before the first use, "" for other
 * precisions or a NULL problem).                                            */
const char* rt_gemm16_tile(rt_problem p, int precision);

/* Thread-local message of the last failed call on this thread.              */
const char* rt_last_error(void);

int rt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RTSN_H */
