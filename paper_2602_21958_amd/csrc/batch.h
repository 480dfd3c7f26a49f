// Batched solves: device-side slot descriptors, work lists and the launchers
// of batch.hip, used by the engine in batch.cpp.
#pragma once

#include "krylov.h"

namespace rtsn {

// Vector elements per reduction chunk (batch512: 2048 and 4096 equal within
// 1 % for FP32 bases, 2048 6 % faster with fp16 bases; 16384 leaves too few
// chunks for the grid, -20 %).
constexpr int kChunk = 2048;
constexpr int kPersistBlocks = 1024;  // grid of the persistent work-list kernels

// Everything one admitted solve needs on the device.  Pointers to tables are
// borrowed from the owning Problem; vectors and state live in the engine's
// arena.
struct SlotDev {
  int geom, nx, ny, nz;
  int n_r, n_nu, formal, lda_mhat;
  int mp16, kp16;               // 16-bit operand padding (see gemm16_dev.h)
  int64_t np16;
  int restart;
  int active;
  int64_t n_s, n;
  int nch;                      // reduction chunks of a length-n vector
  const double* mhat64;
  const float* mhat32;
  const uint16_t* a8_hi;        // Mhat, k8 layout: bf16 (hi part)
  const uint16_t* a8_lo;        // bf16 of Mhat - hi
  const uint16_t* a8_f16;       // fp16, rows scaled
  uint16_t* l16;                // Lambda output, k4 layout: hi part, then lo part
  const float* f16_rowscale;
  const double* albedo;
  const double* dt;
  const double* kline;
  const BoxStencil* stencil;
  const double* ray_mu;
  const double* ray_fac;
  void* V;                      // (restart + 1) * n basis vectors (TV; fp16 ones stored
                                // times vs)
  void* L;                      // n doubles of scratch (Lambda output, any type)
  double* x;                    // FP64 iterate (caller's output buffer)
  double* b;                    // FP64 right-hand side
  double* r;                    // FP64 residual / A x scratch
  double* partial;              // (kMaxRestart + 1) * nch partial sums
  GmresState* gs;
  float l_scale;                // fp16 Lambda output scale
  float vs;                     // basis scale: fp16_basis_scale for an fp16 basis,
                                // 1 otherwise
  // physics-based preconditioner (prq > 0; FP64 or FP32 bases): the angular
  // modes F, G (n_omega x prq) and the per-point blocks T (prq x n_s blocks
  // of n_nu x n_nu) borrowed from the Problem in the basis type; in the
  // arena u = P^-1 v_j and nd = v_j - u (n each; nd also holds V y at a
  // cycle end) and the reduced vectors r, z (prq n_nu n_s each)
  int prq;
  const void* pF;
  const void* pG;
  const void* pT;
  void* pu;
  void* pnd;
  void* pr;
  void* pz;
};

// Mutable per-slot scalars, written by the kernels (and by the host when a
// cycle starts); the host reads the whole array once per engine step.
struct SlotStat {
  double resid;                 // |g_{j+1}| of the current cycle (unit start)
  double rn;                    // FP64 residual norm after the last cycle end
  double target;                // the cycle stops when resid <= target
  int j;                        // Arnoldi steps done in the current cycle
  int cycle_done;
  int iters;                    // total inner iterations
  int breakdown;
  int nonfinite;
  int pad;
};

// Work-list item: slot and an index whose meaning depends on the list.
struct Item {
  int slot;
  int a, b, c;
};

struct WorkLists {
  // device arrays (capacity in items) and device counts
  Item* lam_slab = nullptr;  int cap_lam_slab = 0;
  Item* lam_box = nullptr;   int cap_lam_box = 0;
  Item* tiles = nullptr;     int cap_tiles = 0;     // tiles of the 128 x 128 GEMMs
  Item* chunks = nullptr;    int cap_chunks = 0;
  int* slots = nullptr;      int cap_slots = 0;
  int* counts = nullptr;     // [lam_slab, lam_box, tiles, chunks, slots]
  int h_counts[5] = {0, 0, 0, 0, 0};
  int box_npt = 1;           // points per thread class for box rays (1, 2, 16)
  int box_pmax = 0;          // largest box plane among the listed slots
  size_t box_phmax = 0;      // largest box plane with its LDS halo (lam::box_halo)
  int box_f = 1;             // frequencies per box item (1 or 4)
  int max_lds = 0;           // LDS bytes per workgroup of the device
  bool any_prec = false;     // some listed slot is preconditioned
  uint64_t gen = 0;          // bumped whenever a list buffer is reallocated: a graph
                             // captured with the old addresses must not be replayed
};

// Shape of the grouped 16-bit GEMM: tile body (index into the candidates of
// batch.hip) and persistent grid size.
struct BatchTune {
  int cfg = 0;
  int grid = kPersistBlocks;
};
constexpr int kBatchGemm16Cfgs = 2;
const char* batch_gemm16_name(int cfg);

// Launchers (inner: vectors TV = double, float or _Float16, operator
// precision prec)
// One Arnoldi step of every slot in the lists (operator in precision prec).
template <typename TV>
void b_inner_iteration(const SlotDev* slots, SlotStat* stat, const WorkLists& wl, int prec,
                       hipStream_t st, const BatchTune& tune = {});
// Lambda of the current basis vector followed by the grouped 16-bit GEMM in
// the given shape (the same work as the first half of an inner iteration;
// used to time the shapes).
void b_time_gemm16(const SlotDev* slots, SlotStat* stat, const WorkLists& wl, int prec,
                   hipStream_t st, const BatchTune& tune, bool half_basis);
void b_lambda16(const SlotDev* slots, SlotStat* stat, const WorkLists& wl, int prec,
                hipStream_t st, bool half_basis);
// x += rn V y, then r = b - A_64 x and rn = ||r|| for every listed slot.
template <typename TV>
void b_cycle_end(const SlotDev* slots, SlotStat* stat, const WorkLists& wl, hipStream_t st);
// V_0 = r / rn, fresh Givens state, for every listed slot.
template <typename TV>
void b_start_cycle(const SlotDev* slots, SlotStat* stat, const WorkLists& wl, hipStream_t st);

}  // namespace rtsn
