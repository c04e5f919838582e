// Allocation-free time step (rlb_step_noalloc): every device buffer a step
// needs besides the caller's state -- the two stage arrays, the moment
// records, the quadrature tables, the work list, the node-split sums, the
// high-order equilibrium values and the flag word -- lives in one static
// device array of this file, so the call makes no allocation of any kind.
//
// The array's name is a host-side stand-in in host code; its device address
// is looked up once per device with hipGetSymbolAddress (with that device
// current) and only that address is handed to kernels.  Each GPU holds its
// own copy of the array for the life of the process; calls on one GPU share
// it, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/rlb.h"
#include "rlb_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(RLB_NOALLOC_SCRATCH_BYTES);
static_assert(kScratchBytes % 256 == 0, "scratch size is a multiple of the workspace alignment");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

// Device address of the scratch array on the current device (looked up on the
// first call on that device, with the device current).
hipError_t scratch_on_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

rlb_status rlb_step_noalloc(rlb_lattice* lat, void* state, int64_t nsteps, uint32_t* flags_device,
                            void* hip_stream) {
  rlb_status st = rlb::noalloc_validate(lat, state, nsteps, kScratchBytes);
  if (st != RLB_OK) return st;
  void* base = nullptr;
  const hipError_t e = scratch_on_current_device(&base);
  if (e != hipSuccess) return rlb::noalloc_hip_error(lat, e, "scratch address lookup");
  return rlb::noalloc_steps(lat, static_cast<char*>(base), state, reinterpret_cast<unsigned*>(flags_device), nsteps,
                            static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"
