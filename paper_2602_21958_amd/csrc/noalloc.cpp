// rt_apply_operator_noalloc: the operator application y = A x with the
// formal solution's output held in a fixed device array of this file instead
// of a buffer the library allocates, for callers that cannot allocate device
// memory.
//
// The array `scratch` below is a file-scope device variable: every GPU the
// library runs on holds its own copy, at its own address, from the time the
// code object is loaded on that GPU until the process ends.  In host code its
// name is only a host-side stand-in for the symbol, never a device address.
// The device address is taken once per device with hipGetSymbolAddress (the
// device current) and only that address is handed to kernels.
#include <mutex>

#include "rt_internal.h"

namespace rtsn {

namespace {

// Largest formal-solution buffer the entry point serves: 64 MiB, i.e.
// 8 388 608 FP64 or 16 777 216 FP32 unknowns (a 1D slab of any size in use,
// a 16^3 box of 768 rays in either precision).
constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

__attribute__((used)) static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (the device is current).
void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) fail(RT_E_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      fail(RT_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_ptr[device] = ptr;
  }
  return g_ptr[device];
}

}  // namespace

void operator_apply_noalloc(Problem& p, int precision, const void* x, void* y, hipStream_t st) {
  if (precision != RT_PREC_FP64 && precision != RT_PREC_FP32)
    fail(RT_E_INVALID,
         "rt_apply_operator_noalloc: only RT_PREC_FP64 and RT_PREC_FP32 (the 16-bit operand "
         "buffer and tile tuner of the other precisions allocate on first use)");
  require_one_kernel(p, "rt_apply_operator_noalloc");
  if (p.sigma_form != RT_SIGMA_DENSE)
    fail(RT_E_INVALID,
         "rt_apply_operator_noalloc: the factored scattering form allocates its work vectors; "
         "set RT_SIGMA_DENSE");
  const size_t elem = precision == RT_PREC_FP64 ? sizeof(double) : sizeof(float);
  const size_t need = (size_t)p.n * elem;
  if (need > kNoAllocBytes)
    fail(RT_E_INVALID, "rt_apply_operator_noalloc: the formal-solution buffer needs " +
                           std::to_string(need) + " bytes, above the fixed " +
                           std::to_string(kNoAllocBytes) + "-byte device array");
  void* L = scratch_ptr(p.device);
  // Lambda writes every one of the n entries of L before the GEMM reads
  // them, so nothing in the array needs clearing between calls.
  if (precision == RT_PREC_FP64) {
    launch_lambda<double, double>(p, static_cast<const double*>(x), static_cast<double*>(L),
                                  false, nullptr, st);
    launch_sigma_f64(p, static_cast<const double*>(L), static_cast<const double*>(x),
                     static_cast<double*>(y), nullptr, -1.0, st);
  } else {
    launch_lambda<float, float>(p, static_cast<const float*>(x), static_cast<float*>(L), false,
                                nullptr, st);
    launch_sigma_f32(p, static_cast<const float*>(L), static_cast<const float*>(x),
                     static_cast<float*>(y), nullptr, -1.0, st);
  }
}

}  // namespace rtsn
