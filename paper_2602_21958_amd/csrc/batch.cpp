// Batch / serving engine: many independent solves share one device.
//
// Requests queue until a slot is free and their device footprint fits the
// engine's HBM budget (a best-fit arena carved out of one allocation at
// create).  Admitted solves advance together: each engine step runs one
// Arnoldi step of every slot that is inside a cycle, then ends the cycles
// that reached their target or the restart length (x update, FP64 true
// residual), retires converged solves, and starts new cycles.  A request that
// arrives while others run is admitted at the next step boundary; its work
// then overlaps with theirs inside the same launches.  All per-slot arithmetic
// is independent of the other slots, so a result is the same alone and in a
// mix.  The inner step is captured once in a hipGraph and replayed while the
// host rewrites the device work lists.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>

#include "batch.h"

namespace rtsn {

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Best-fit allocator over [0, size) with coalescing of freed neighbours.
class Arena {
 public:
  void init(size_t size) {
    size_ = size;
    free_.clear();
    free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t& off) {
    bytes = align_up(bytes);
    auto best = free_.end();
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes && (best == free_.end() || it->second < best->second)) best = it;
    if (best == free_.end()) return false;
    off = best->first;
    const size_t rest = best->second - bytes;
    free_.erase(best);
    if (rest) free_[off + bytes] = rest;
    used_ += bytes;
    sizes_[off] = bytes;
    return true;
  }
  void release(size_t off) {
    auto sz = sizes_.find(off);
    if (sz == sizes_.end()) return;
    size_t start = off, len = sz->second;
    used_ -= len;
    sizes_.erase(sz);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  std::map<size_t, size_t> sizes_;  // allocated offset -> length
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

enum Phase { kFree = 0, kIter = 1, kEnd = 2 };

struct Request {
  uint64_t ticket = 0;
  Problem* p = nullptr;
  rt_solver_opts o{};
  double* x_out = nullptr;
  int slot = -1;
  bool first = true;
  bool done = false;
  rt_status status = RT_OK;
  double bnorm = 0, rn = 0, t_submit = 0, t_done = 0;
  int cycles = 0, stalls = 0;
  size_t off = 0;
  std::vector<double> history;
  rt_solve_stats stats{};
};

}  // namespace

struct Engine {
  int device = 0;
  int max_lds = 0;            // LDS bytes per workgroup of the device (queried once)
  BatchTune tune;             // shape of the grouped 16-bit GEMM
  bool tuned = false;
  std::string tune_name = "untuned";
  int precision = RT_PREC_FP64;
  bool fp64 = true;
  bool basis16 = false;       // fp16 Krylov bases (16-bit operator precisions)
  bool use_graph = true;
  int max_slots = 0;
  int queue_cap = 0;
  Arena arena;
  char* base = nullptr;
  SlotDev* d_slots = nullptr;
  SlotStat* d_stat = nullptr;
  SlotStat* h_stat = nullptr;  // pinned
  std::vector<SlotDev> h_slots;
  std::vector<int> phase;
  std::vector<Request*> slot_req;
  WorkLists wl_iter, wl_end;
  Item* h_items = nullptr;     // pinned staging
  size_t h_items_cap = 0;
  hipStream_t stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  uint64_t graph_key = ~0ull;
  bool iter_dirty = true;
  int graph_failures = 0;
  uint64_t next_ticket = 1;
  std::deque<Request*> queue;
  std::map<uint64_t, Request*> requests;
  std::mutex mu;
  int64_t steps = 0;

  ~Engine();
  size_t footprint(const Problem& p, int restart, bool pre = false) const;
  void tune_gemm16();
  void admit();
  bool setup_slot(Request* r, int s);
  void release_slot(int s, rt_status st);
  void build_lists(WorkLists& wl, const std::vector<int>& set);
  void run_inner();
  int step();
};

namespace {

void wl_free(WorkLists& wl) {
  hipFree(wl.lam_slab);
  hipFree(wl.lam_box);
  hipFree(wl.tiles);
  hipFree(wl.chunks);
  hipFree(wl.slots);
  hipFree(wl.counts);
  wl = WorkLists();
}

// Grow a device list buffer; a reallocation changes its address, so it bumps
// the generation that keys the captured graph.
template <typename T>
void ensure_cap(T*& p, int& cap, int need, uint64_t& gen) {
  if (need <= cap) return;
  hipFree(p);
  p = nullptr;
  int c = std::max(std::max(need, cap * 2), 4096);
  RT_HIP(hipMalloc(&p, (size_t)c * sizeof(T)));
  cap = c;
  ++gen;
}

int nchunks(int64_t n) { return (int)((n + kChunk - 1) / kChunk); }

}  // namespace

Engine::~Engine() {
  if (stream) hipStreamSynchronize(stream);
  for (auto& kv : requests) delete kv.second;
  if (graph_exec) hipGraphExecDestroy(graph_exec);
  if (graph) hipGraphDestroy(graph);
  wl_free(wl_iter);
  wl_free(wl_end);
  hipFree(base);
  hipFree(d_slots);
  hipFree(d_stat);
  if (h_stat) hipHostFree(h_stat);
  if (h_items) hipHostFree(h_items);
  if (stream) hipStreamDestroy(stream);
}

// Arena bytes of one solve; pre adds the preconditioner's vectors (u, nd and
// the reduced r, z; its tables live with the Problem).
size_t Engine::footprint(const Problem& p, int restart, bool pre) const {
  const size_t n = (size_t)p.n;
  const size_t tv = fp64 ? sizeof(double) : (basis16 ? 2 : sizeof(float));
  size_t b = 0;
  b += align_up((size_t)(restart + 1) * n * tv);              // basis
  b += align_up(n * sizeof(double));                          // L scratch
  if (!fp64) b += align_up(2 * (size_t)l16_part_elems(p) * sizeof(uint16_t));  // 16-bit L
  b += 2 * align_up(n * sizeof(double));                      // b, r
  b += align_up((size_t)(restart + 2) * nchunks(p.n) * sizeof(double));  // partials
  b += align_up(sizeof(GmresState));
  if (pre) {
    const size_t rz = (size_t)std::max(1, p.tab.frank) * p.n_nu * p.n_s;
    b += 2 * align_up(n * tv) + 2 * align_up(rz * tv);
  }
  return b;
}

bool Engine::setup_slot(Request* r, int s) {
  Problem& p = *r->p;
  const int m = r->o.restart;
  const bool pre = r->o.precond == RT_PRECOND_LOCAL;
  const size_t fp = footprint(p, m, pre);
  size_t off = 0;
  if (!arena.alloc(fp, off)) return false;
  r->off = off;
  char* q = base + off;
  const size_t n = (size_t)p.n;
  const size_t tv = fp64 ? sizeof(double) : (basis16 ? 2 : sizeof(float));
  SlotDev d{};
  d.geom = p.geom;
  d.nx = p.nx;
  d.ny = p.ny;
  d.nz = p.nz;
  d.n_r = p.n_r;
  d.n_nu = p.n_nu;
  d.formal = p.formal;
  d.lda_mhat = p.lda_mhat;
  d.mp16 = p.mp16;
  d.kp16 = p.kp16;
  d.np16 = p.np16;
  d.restart = m;
  d.active = 1;
  d.n_s = p.n_s;
  d.n = p.n;
  d.nch = nchunks(p.n);
  d.mhat64 = p.d_mhat64;
  d.mhat32 = p.d_mhat32;
  d.a8_hi = p.d_a8_bf16;
  d.a8_lo = p.d_a8_bf16_lo;
  d.a8_f16 = p.d_a8_f16;
  d.f16_rowscale = p.d_f16_rowscale;
  d.albedo = p.d_albedo;
  d.dt = p.d_dt;
  d.kline = p.d_kline;
  d.stencil = p.d_stencil;
  d.ray_mu = p.d_ray_mu;
  d.ray_fac = p.d_ray_fac;
  d.V = q;                                      q += align_up((size_t)(m + 1) * n * tv);
  d.L = q;                                      q += align_up(n * sizeof(double));
  if (!fp64) {
    const size_t lb = 2 * (size_t)l16_part_elems(p) * sizeof(uint16_t);
    d.l16 = reinterpret_cast<uint16_t*>(q);     q += align_up(lb);
    // padding rows of the operand must read as zeros
    RT_HIP(hipMemsetAsync(d.l16, 0, lb, stream));
  }
  d.b = reinterpret_cast<double*>(q);           q += align_up(n * sizeof(double));
  d.r = reinterpret_cast<double*>(q);           q += align_up(n * sizeof(double));
  d.partial = reinterpret_cast<double*>(q);     q += align_up((size_t)(m + 2) * d.nch * 8);
  d.gs = reinterpret_cast<GmresState*>(q);      q += align_up(sizeof(GmresState));
  if (pre) {
    // the Problem's tables in the basis type (built on its first use)
    precond_prepare(p, (int)tv, stream);
    d.prq = p.prec_rq;
    d.pF = fp64 ? (const void*)p.d_prec_F64 : (const void*)p.d_prec_F32;
    d.pG = fp64 ? (const void*)p.d_prec_G64 : (const void*)p.d_prec_G32;
    d.pT = fp64 ? (const void*)p.d_prec_T64 : (const void*)p.d_prec_T32;
    const size_t rz = (size_t)std::max(1, p.tab.frank) * p.n_nu * p.n_s;
    d.pu = q;                                   q += align_up(n * tv);
    d.pnd = q;                                  q += align_up(n * tv);
    d.pr = q;                                   q += align_up(rz * tv);
    d.pz = q;                                   q += align_up(rz * tv);
  }
  d.x = r->x_out;
  // (only the fp16 k4 operand is scaled; plain outputs ignore l_scale)
  d.l_scale = precision == RT_PREC_FP16 ? fp16_lambda_scale(p.n) : 1.f;
  d.vs = basis16 ? fp16_basis_scale(p.n) : 1.f;
  h_slots[s] = d;
  RT_HIP(hipMemcpyAsync(d_slots + s, &h_slots[s], sizeof(SlotDev), hipMemcpyHostToDevice, stream));
  // right-hand side b = (1-eps) Mhat I_bc + t into the slot, x = 0
  RT_HIP(hipMemsetAsync(d.r, 0, n * sizeof(double), stream));
  launch_lambda<double, double>(p, d.r, static_cast<double*>(d.L), true, nullptr, stream);
  launch_sigma_f64(p, static_cast<const double*>(d.L), p.d_thermal, d.b, nullptr, +1.0, stream);
  RT_HIP(hipMemsetAsync(d.x, 0, n * sizeof(double), stream));
  RT_HIP(hipMemsetAsync(d.gs, 0, sizeof(GmresState), stream));
  SlotStat z{};
  std::memcpy(&h_stat[s], &z, sizeof(z));
  RT_HIP(hipMemcpyAsync(d_stat + s, &h_stat[s], sizeof(SlotStat), hipMemcpyHostToDevice, stream));
  r->slot = s;
  r->first = true;
  slot_req[s] = r;
  phase[s] = kEnd;  // first "cycle end" computes r = b and ||b||
  return true;
}

void Engine::release_slot(int s, rt_status st) {
  Request* r = slot_req[s];
  r->status = st;
  r->done = true;
  r->t_done = now_ms();
  r->stats.iters = h_stat[s].iters;
  r->stats.outer_iters = r->cycles;
  r->stats.relres = r->bnorm > 0 ? r->rn / r->bnorm : 0.0;
  r->stats.converged = st == RT_OK;
  r->stats.ms = r->t_done - r->t_submit;
  r->stats.history_len = (int)r->history.size();
  r->stats.history = r->history.empty() ? nullptr : r->history.data();
  arena.release(r->off);
  slot_req[s] = nullptr;
  phase[s] = kFree;
  h_slots[s].active = 0;
  iter_dirty = true;
}

void Engine::admit() {
  while (!queue.empty()) {
    int s = -1;
    for (int i = 0; i < max_slots; ++i)
      if (phase[i] == kFree) { s = i; break; }
    if (s < 0) return;
    Request* r = queue.front();
    if (!setup_slot(r, s)) return;  // does not fit yet: wait for memory
    queue.pop_front();
  }
}

void Engine::build_lists(WorkLists& wl, const std::vector<int>& set) {
  std::vector<Item> slab, box, tiles, chunks;
  std::vector<int> slots;
  int pmax = 0;
  size_t phmax = 0;
  for (int s : set)
    if (h_slots[s].geom != RT_GEOM_SLAB) {
      pmax = std::max(pmax, h_slots[s].nx * h_slots[s].ny);
      // LDS plane with its halo row and column
      phmax = std::max(phmax, (size_t)(h_slots[s].nx + 1) * (h_slots[s].ny + 1));
    }
  if (max_lds == 0)
    RT_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
  // frequencies per box work item: one list serves the FP64 (cycle end) and
  // the low-precision sweeps, so size it for FP64
  const int bf = pmax > 0 ? std::max(1, box_chunk(phmax, (int)sizeof(double), max_lds)) : 1;
  for (int s : set) {
    const SlotDev& d = h_slots[s];
    slots.push_back(s);
    if (d.geom == RT_GEOM_SLAB) {
      for (int k = 0; k < d.n_r; k += 4) slab.push_back(Item{s, k, 0, 0});
    } else {
      const int n_omega = d.n_r / d.n_nu;
      for (int o = 0; o < n_omega; ++o)
        for (int nu0 = 0; nu0 < d.n_nu; nu0 += bf)
          box.push_back(Item{s, o * d.n_nu + nu0, std::min(bf, d.n_nu - nu0), 0});
    }
    for (int n0 = 0; n0 < (int)d.n_s; n0 += 128)
      for (int m0 = 0; m0 < d.n_r; m0 += 128) tiles.push_back(Item{s, m0, n0, 0});
    for (int c = 0; c < d.nch; ++c) chunks.push_back(Item{s, c, 0, 0});
  }
  ensure_cap(wl.lam_slab, wl.cap_lam_slab, (int)slab.size() + 1, wl.gen);
  ensure_cap(wl.lam_box, wl.cap_lam_box, (int)box.size() + 1, wl.gen);
  ensure_cap(wl.tiles, wl.cap_tiles, (int)tiles.size() + 1, wl.gen);
  ensure_cap(wl.chunks, wl.cap_chunks, (int)chunks.size() + 1, wl.gen);
  ensure_cap(wl.slots, wl.cap_slots, (int)slots.size() + 1, wl.gen);
  if (!wl.counts) {
    RT_HIP(hipMalloc(&wl.counts, 8 * sizeof(int)));
    ++wl.gen;
  }
  // stage through pinned memory, then copy to the device lists
  const size_t total = slab.size() + box.size() + tiles.size() + chunks.size() +
                       (slots.size() + 3) / 4 + 2;
  if (total > h_items_cap) {
    if (h_items) hipHostFree(h_items);
    h_items_cap = std::max(total, h_items_cap * 2);
    RT_HIP(hipHostMalloc((void**)&h_items, h_items_cap * sizeof(Item), hipHostMallocDefault));
  }
  // the stream must not still read the staging buffer from a previous step
  RT_HIP(hipStreamSynchronize(stream));
  Item* h = h_items;
  auto put = [&](const std::vector<Item>& v, Item* dst) {
    if (v.empty()) return;
    std::memcpy(h, v.data(), v.size() * sizeof(Item));
    RT_HIP(hipMemcpyAsync(dst, h, v.size() * sizeof(Item), hipMemcpyHostToDevice, stream));
    h += v.size();
  };
  put(slab, wl.lam_slab);
  put(box, wl.lam_box);
  put(tiles, wl.tiles);
  put(chunks, wl.chunks);
  int* hs = reinterpret_cast<int*>(h);
  if (!slots.empty()) {
    std::memcpy(hs, slots.data(), slots.size() * sizeof(int));
    RT_HIP(hipMemcpyAsync(wl.slots, hs, slots.size() * sizeof(int), hipMemcpyHostToDevice,
                          stream));
  }
  h += (slots.size() + 3) / 4;
  int* hc = reinterpret_cast<int*>(h);
  hc[0] = (int)slab.size();
  hc[1] = (int)box.size();
  hc[2] = (int)tiles.size();
  hc[3] = (int)chunks.size();
  hc[4] = (int)slots.size();
  for (int i = 0; i < 5; ++i) wl.h_counts[i] = hc[i];
  RT_HIP(hipMemcpyAsync(wl.counts, hc, 5 * sizeof(int), hipMemcpyHostToDevice, stream));
  wl.any_prec = false;
  for (int s : set) wl.any_prec = wl.any_prec || h_slots[s].prq > 0;
  wl.box_pmax = pmax;
  wl.box_phmax = phmax;
  wl.box_npt = pmax <= 256 ? 1 : (pmax <= 1024 ? 2 : 16);
  wl.box_f = bf;
  wl.max_lds = max_lds;
}

// Time the grouped 16-bit GEMM's persistent grid sizes on the live work
// lists, once, before the first capture: Lambda runs once to provide the
// operand, then each size twice after a warm-up (the GEMM recomputes the same
// V_{j+1} every time).  The tile body stays fixed: a different MFMA
// instruction would round differently, and a solve must give the same bits
// alone and in any mix of other solves.  RTSN_BATCH_GEMM16 forces a body.
void Engine::tune_gemm16() {
  tuned = true;
  if (fp64 || precision == RT_PREC_FP32 || wl_iter.h_counts[2] == 0) return;
  if (const char* e = std::getenv("RTSN_BATCH_GEMM16")) {   // "<cfg>,<grid>"
    int c = 0, g = kPersistBlocks;
    if (std::sscanf(e, "%d,%d", &c, &g) >= 1 && c >= 0 && c < kBatchGemm16Cfgs && g > 0) {
      tune = BatchTune{c, g};
      tune_name = std::string(batch_gemm16_name(c)) + ", " + std::to_string(g) + " workgroups";
      return;
    }
  }
  b_lambda16(d_slots, d_stat, wl_iter, precision, stream, basis16);
  hipEvent_t e0, e1;
  RT_HIP(hipEventCreate(&e0));
  RT_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  for (int c = 0; c < 1; ++c) {
    for (int g : {512, 1024, 2048}) {
      const BatchTune t{c, g};
      b_time_gemm16(d_slots, d_stat, wl_iter, precision, stream, t, basis16);
      float ms = 1e30f;
      for (int rep = 0; rep < 2; ++rep) {
        RT_HIP(hipEventRecord(e0, stream));
        b_time_gemm16(d_slots, d_stat, wl_iter, precision, stream, t, basis16);
        RT_HIP(hipEventRecord(e1, stream));
        RT_HIP(hipEventSynchronize(e1));
        float v = 0.f;
        RT_HIP(hipEventElapsedTime(&v, e0, e1));
        ms = std::min(ms, v);
      }
      if (ms < best) {
        best = ms;
        tune = t;
      }
    }
  }
  RT_HIP(hipEventDestroy(e0));
  RT_HIP(hipEventDestroy(e1));
  tune_name = std::string(batch_gemm16_name(tune.cfg)) + ", " + std::to_string(tune.grid) +
              " workgroups";
}

void Engine::run_inner() {
  const bool profiling = profile_enabled();
  if (!tuned) tune_gemm16();
  // The captured graph bakes in the launch shape (which geometries, box class
  // and LDS size) and the addresses of the list buffers: any change of either
  // needs a new capture.
  const uint64_t key = (uint64_t)(wl_iter.h_counts[0] > 0) |
                       ((uint64_t)(wl_iter.h_counts[1] > 0) << 1) |
                       ((uint64_t)wl_iter.box_npt << 2) | ((uint64_t)wl_iter.box_pmax << 8) |
                       (wl_iter.gen << 24) | ((uint64_t)tune.cfg << 60) |
                       ((uint64_t)wl_iter.any_prec << 62);
  auto direct = [&] {
    if (fp64)
      b_inner_iteration<double>(d_slots, d_stat, wl_iter, precision, stream);
    else if (basis16)
      b_inner_iteration<_Float16>(d_slots, d_stat, wl_iter, precision, stream, tune);
    else
      b_inner_iteration<float>(d_slots, d_stat, wl_iter, precision, stream, tune);
  };
  if (use_graph && !profiling) {
    if (key != graph_key) {
      if (graph_exec) hipGraphExecDestroy(graph_exec);
      if (graph) hipGraphDestroy(graph);
      graph_exec = nullptr;
      graph = nullptr;
      graph_key = ~0ull;
      std::unique_lock<std::shared_mutex> lk(capture_mutex());
      bool ok = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed) == hipSuccess;
      if (ok) {
        try {
          direct();
        } catch (const RtError&) {
          ok = false;
        }
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(stream, &g);
        ok = ok && e == hipSuccess && g != nullptr;
        if (ok) {
          ok = hipGraphInstantiate(&graph_exec, g, nullptr, nullptr, 0) == hipSuccess;
          graph = g;
        } else if (g) {
          hipGraphDestroy(g);
        }
      }
      (void)hipGetLastError();
      if (ok) {
        graph_key = key;
      } else {
        // capture was invalidated: nothing of it ran; launch directly
        if (graph_exec) hipGraphExecDestroy(graph_exec);
        if (graph) hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
        graph_failures++;
        if (graph_failures >= 3) use_graph = false;
        direct();
        return;
      }
    }
    RT_HIP(hipGraphLaunch(graph_exec, stream));
  } else {
    direct();
  }
}

int Engine::step() {
  admit();
  steps++;
  std::vector<int> iter_set, end_set;
  for (int s = 0; s < max_slots; ++s) {
    if (phase[s] == kIter) iter_set.push_back(s);
    if (phase[s] == kEnd) end_set.push_back(s);
  }
  if (!iter_set.empty()) {
    if (iter_dirty) {
      build_lists(wl_iter, iter_set);
      iter_dirty = false;
    }
    run_inner();
    RT_HIP(hipMemcpyAsync(h_stat, d_stat, (size_t)max_slots * sizeof(SlotStat),
                          hipMemcpyDeviceToHost, stream));
    RT_HIP(hipStreamSynchronize(stream));
    for (int s : iter_set) {
      if (h_stat[s].cycle_done) {
        phase[s] = kEnd;
        end_set.push_back(s);
        iter_dirty = true;
      }
    }
  }
  if (!end_set.empty()) {
    std::sort(end_set.begin(), end_set.end());
    build_lists(wl_end, end_set);
    if (fp64)
      b_cycle_end<double>(d_slots, d_stat, wl_end, stream);
    else if (basis16)
      b_cycle_end<_Float16>(d_slots, d_stat, wl_end, stream);
    else
      b_cycle_end<float>(d_slots, d_stat, wl_end, stream);
    RT_HIP(hipMemcpyAsync(h_stat, d_stat, (size_t)max_slots * sizeof(SlotStat),
                          hipMemcpyDeviceToHost, stream));
    RT_HIP(hipStreamSynchronize(stream));
    std::vector<int> start;
    for (int s : end_set) {
      Request* r = slot_req[s];
      const double rn = h_stat[s].rn;
      if (r->first) {
        r->bnorm = rn;
        r->first = false;
      } else {
        r->cycles++;
        r->stalls = (rn >= 0.9 * r->rn && !fp64) ? r->stalls + 1 : 0;
      }
      r->rn = rn;
      const double rel = r->bnorm > 0 ? rn / r->bnorm : 0.0;
      if (r->o.record_history) r->history.push_back(rel);
      if (h_stat[s].nonfinite || !std::isfinite(rn)) {
        release_slot(s, RT_E_NONFINITE);
      } else if (r->bnorm == 0.0 || rel <= r->o.rtol) {
        release_slot(s, RT_OK);
      } else if (h_stat[s].iters >= r->o.max_iters || (!fp64 && r->cycles >= r->o.max_outer) ||
                 r->stalls >= 3) {
        release_slot(s, RT_NOT_CONVERGED);
      } else {
        double target = r->o.rtol * r->bnorm / rn;
        if (!fp64) target = std::max(target, r->o.inner_rtol);
        SlotStat& z = h_stat[s];
        z.j = 0;
        z.cycle_done = 0;
        z.target = target;
        z.breakdown = 0;
        RT_HIP(hipMemcpyAsync(d_stat + s, &h_stat[s], sizeof(SlotStat), hipMemcpyHostToDevice,
                              stream));
        start.push_back(s);
      }
    }
    if (!start.empty()) {
      build_lists(wl_end, start);
      if (fp64)
        b_start_cycle<double>(d_slots, d_stat, wl_end, stream);
      else if (basis16)
        b_start_cycle<_Float16>(d_slots, d_stat, wl_end, stream);
      else
        b_start_cycle<float>(d_slots, d_stat, wl_end, stream);
      for (int s : start) phase[s] = kIter;
      iter_dirty = true;
    }
    RT_HIP(hipStreamSynchronize(stream));
  }
  int pending = (int)queue.size();
  for (int s = 0; s < max_slots; ++s) pending += phase[s] != kFree;
  return pending;
}

}  // namespace rtsn

using namespace rtsn;

namespace {

template <typename F>
rt_status guarded_b(F&& f) {
  try {
    f();
    return RT_OK;
  } catch (const RtError& e) {
    set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return RT_E_NOMEM;
  } catch (...) {
    set_last_error("unknown error in batch engine");
    return RT_E_DEVICE;
  }
}

Engine* as_engine(rt_batch b) {
  if (!b) fail(RT_E_INVALID, "null batch handle");
  Engine* e = reinterpret_cast<Engine*>(b);
  RT_HIP(hipSetDevice(e->device));
  return e;
}

}  // namespace

extern "C" {

rt_status rt_batch_create(int device, int precision, int64_t hbm_budget, int max_slots,
                          int queue_cap, int use_graph, rt_batch* out) {
  return rt_batch_create_ex(device, precision, hbm_budget, max_slots, queue_cap, use_graph, 0,
                            out);
}

rt_status rt_batch_create_ex(int device, int precision, int64_t hbm_budget, int max_slots,
                             int queue_cap, int use_graph, int flags, rt_batch* out) {
  if (out) *out = nullptr;
  return guarded_b([&] {
    if (!out) fail(RT_E_INVALID, "null out");
    if (precision < RT_PREC_FP64 || precision > RT_PREC_BF16X3)
      fail(RT_E_INVALID, "unknown precision");
    if (flags & ~RT_BATCH_BASIS_FP16) fail(RT_E_INVALID, "unknown flags");
    const bool basis16 = (flags & RT_BATCH_BASIS_FP16) != 0;
    if (basis16 && precision != RT_PREC_BF16 && precision != RT_PREC_FP16 &&
        precision != RT_PREC_BF16X3)
      fail(RT_E_INVALID, "an fp16 basis needs a 16-bit operator precision");
    if (max_slots < 1 || max_slots > 4096) fail(RT_E_INVALID, "max_slots out of range");
    if (queue_cap < 1) fail(RT_E_INVALID, "queue_cap must be >= 1");
    if (hbm_budget < (int64_t)(1 << 20)) fail(RT_E_INVALID, "hbm_budget too small");
    int ndev = 0;
    RT_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) fail(RT_E_INVALID, "bad device index");
    RT_HIP(hipSetDevice(device));
    Engine* e = new Engine();
    try {
      e->device = device;
      e->precision = precision;
      e->fp64 = precision == RT_PREC_FP64;
      e->basis16 = basis16;
      e->use_graph = use_graph != 0;
      e->max_slots = max_slots;
      e->queue_cap = queue_cap;
      RT_HIP(hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking));
      hipError_t err = hipMalloc(&e->base, (size_t)hbm_budget);
      if (err != hipSuccess) {
        (void)hipGetLastError();
        e->base = nullptr;
        fail(RT_E_NOMEM, "cannot reserve the HBM budget");
      }
      e->arena.init((size_t)hbm_budget);
      RT_HIP(hipMalloc(&e->d_slots, (size_t)max_slots * sizeof(SlotDev)));
      RT_HIP(hipMalloc(&e->d_stat, (size_t)max_slots * sizeof(SlotStat)));
      RT_HIP(hipHostMalloc((void**)&e->h_stat, (size_t)max_slots * sizeof(SlotStat),
                           hipHostMallocDefault));
      std::memset(e->h_stat, 0, (size_t)max_slots * sizeof(SlotStat));
      RT_HIP(hipMemset(e->d_stat, 0, (size_t)max_slots * sizeof(SlotStat)));
      e->h_slots.assign(max_slots, SlotDev{});
      e->phase.assign(max_slots, kFree);
      e->slot_req.assign(max_slots, nullptr);
    } catch (...) {
      delete e;
      throw;
    }
    *out = reinterpret_cast<rt_batch>(e);
  });
}

rt_status rt_batch_submit(rt_batch b, rt_problem p, const rt_solver_opts* opts, double* x_out,
                          uint64_t* ticket) {
  return guarded_b([&] {
    Engine* e = as_engine(b);
    if (!p || !x_out || !ticket) fail(RT_E_INVALID, "null argument");
    Problem* q = reinterpret_cast<Problem*>(p);
    if (q->device != e->device) fail(RT_E_INVALID, "problem lives on another device");
    rt_solver_opts o;
    if (opts) o = *opts; else rt_solver_opts_default(&o);
    if (o.krylov != RT_KRYLOV_GMRES) fail(RT_E_INVALID, "the batch engine runs GMRES");
    require_one_kernel(*q, "the batch engine");
    if (q->geom == RT_GEOM_BOX && q->formal != RT_FORMAL_LINEAR_SC)
      fail(RT_E_INVALID, "the batch engine sweeps boxes with linear SC only");
    if (o.precision != e->precision) fail(RT_E_INVALID, "precision differs from the engine's");
    if (o.restart < 1 || o.restart > kMaxRestart) fail(RT_E_INVALID, "restart out of range");
    if (!(o.rtol > 0)) fail(RT_E_INVALID, "rtol must be > 0");
    if ((o.basis_fp16 != 0) != e->basis16)
      fail(RT_E_INVALID, "basis_fp16 differs from the engine's basis");
    if (e->basis16 && q->scatter_inf > 2.0)
      fail(RT_E_INVALID, "an fp16 basis needs max row sum of |(1-eps) Mhat| <= 2");
    if (o.precond != RT_PRECOND_NONE && o.precond != RT_PRECOND_LOCAL)
      fail(RT_E_INVALID, "unknown preconditioner");
    if (o.precond && e->basis16) fail(RT_E_INVALID, "the preconditioner needs FP64 or FP32 bases");
    if (o.precond) precond_check(*q);
    if (o.max_outer < 1) o.max_outer = 1;
    std::lock_guard<std::mutex> lk(e->mu);
    if (e->footprint(*q, o.restart, o.precond != 0) > e->arena.size())
      fail(RT_E_INVALID, "problem can never fit the engine's HBM budget");
    if ((int)e->queue.size() >= e->queue_cap) fail(RT_E_BUSY, "queue full");
    Request* r = new Request();
    r->ticket = e->next_ticket++;
    r->p = q;
    r->o = o;
    r->x_out = x_out;
    r->t_submit = now_ms();
    e->requests[r->ticket] = r;
    e->queue.push_back(r);
    *ticket = r->ticket;
  });
}

rt_status rt_batch_step(rt_batch b, int* pending) {
  return guarded_b([&] {
    Engine* e = as_engine(b);
    std::lock_guard<std::mutex> lk(e->mu);
    const int n = e->step();
    if (pending) *pending = n;
  });
}

rt_status rt_batch_poll(rt_batch b, uint64_t ticket, rt_solve_stats* stats) {
  rt_status out = RT_OK;
  rt_status g = guarded_b([&] {
    Engine* e = as_engine(b);
    std::lock_guard<std::mutex> lk(e->mu);
    auto it = e->requests.find(ticket);
    if (it == e->requests.end()) fail(RT_E_INVALID, "unknown ticket");
    Request* r = it->second;
    if (!r->done) {
      out = RT_E_BUSY;
      return;
    }
    if (stats) *stats = r->stats;
    out = r->status;
  });
  return g != RT_OK ? g : out;
}

rt_status rt_batch_wait_all(rt_batch b) {
  return guarded_b([&] {
    Engine* e = as_engine(b);
    std::lock_guard<std::mutex> lk(e->mu);
    while (e->step() > 0) {
    }
  });
}

rt_status rt_batch_info(rt_batch b, int* active, int* queued, int64_t* bytes_in_use) {
  return guarded_b([&] {
    Engine* e = as_engine(b);
    std::lock_guard<std::mutex> lk(e->mu);
    int a = 0;
    for (int s = 0; s < e->max_slots; ++s) a += e->phase[s] != kFree;
    if (active) *active = a;
    if (queued) *queued = (int)e->queue.size();
    if (bytes_in_use) *bytes_in_use = (int64_t)e->arena.used();
  });
}

const char* rt_batch_gemm16_tile(rt_batch b) {
  if (!b) return "";
  return reinterpret_cast<Engine*>(b)->tune_name.c_str();
}

rt_status rt_batch_footprint(rt_batch b, rt_problem p, int restart, int64_t* bytes) {
  return guarded_b([&] {
    Engine* e = as_engine(b);
    if (!p || !bytes) fail(RT_E_INVALID, "null argument");
    if (restart < 1 || restart > kMaxRestart) fail(RT_E_INVALID, "restart out of range");
    *bytes = (int64_t)e->footprint(*reinterpret_cast<Problem*>(p), restart);
  });
}

rt_status rt_batch_destroy(rt_batch b) {
  return guarded_b([&] {
    if (!b) return;
    Engine* e = reinterpret_cast<Engine*>(b);
    RT_HIP(hipSetDevice(e->device));
    delete e;
  });
}

}  // extern "C"
