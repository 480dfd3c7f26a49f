// Kernel timing with HIP events (rt_profile_enable / rt_profile_read).
#include <atomic>
#include <mutex>
#include <vector>

#include "rt_internal.h"

namespace rtsn {

namespace {

struct Record {
  int kclass;
  hipEvent_t start, stop;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Record> g_records;

}  // namespace

bool profile_enabled() { return g_on.load(std::memory_order_relaxed); }

ProfScope::ProfScope(int kclass, hipStream_t st) : kclass_(kclass), st_(st) {
  if (!g_on.load(std::memory_order_relaxed)) return;
  if (hipEventCreate(&start_) != hipSuccess) { start_ = nullptr; return; }
  if (hipEventRecord(start_, st_) != hipSuccess) {
    hipEventDestroy(start_);
    start_ = nullptr;
  }
}

ProfScope::~ProfScope() {
  if (!start_) return;
  hipEvent_t stop = nullptr;
  if (hipEventCreate(&stop) != hipSuccess || hipEventRecord(stop, st_) != hipSuccess) {
    if (stop) hipEventDestroy(stop);
    hipEventDestroy(start_);
    return;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_records.push_back(Record{kclass_, start_, stop});
}

}  // namespace rtsn

using namespace rtsn;

extern "C" {

rt_status rt_profile_enable(int on) {
  g_on.store(on != 0);
  return RT_OK;
}

rt_status rt_profile_read(int kclass, int64_t* launches, double* total_ms, int reset) {
  if (kclass < 0 || kclass >= RT_KCLASS_COUNT) return RT_E_INVALID;
  std::lock_guard<std::mutex> lk(g_mu);
  int64_t n = 0;
  double tot = 0.0;
  std::vector<Record> keep;
  keep.reserve(g_records.size());
  for (const Record& r : g_records) {
    if (r.kclass != kclass) {
      keep.push_back(r);
      continue;
    }
    if (hipEventSynchronize(r.stop) != hipSuccess) return RT_E_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return RT_E_DEVICE;
    tot += ms;
    ++n;
    if (reset) {
      hipEventDestroy(r.start);
      hipEventDestroy(r.stop);
    } else {
      keep.push_back(r);
    }
  }
  g_records.swap(keep);
  if (launches) *launches = n;
  if (total_ms) *total_ms = tot;
  return RT_OK;
}

}  // extern "C"
