// Allocation-free evaluation: nb_build_cells + nb_nonbonded_forces on a scratch array
// that lives in the library's own device memory, for callers that cannot allocate (code
// under HIP graph capture, tight serving loops, harnesses that forbid it).
//
// The array is a file-scope __device__ object: every GPU the library runs on holds its
// own copy, from the loading of this code until the process ends.  In host code its
// name is only a stand-in for that object, never a device address: the address of a
// device's copy comes from hipGetSymbolAddress, asked once per device (with that device
// current) and kept here.  The kernels receive that address, exactly as they receive a
// caller's workspace in nb_nonbonded_forces.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "nb_internal.h"

namespace nb {

namespace {

constexpr size_t kScratchBytes = static_cast<size_t>(NB_NOALLOC_SCRATCH_BYTES);
static_assert(kScratchBytes % 256 == 0, "whole 256-byte blocks");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up on first use on that device.
hipError_t scratch_address(void **out, std::string *why) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *why = "hipGetDevice failed";
    return e;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    *why = "device index beyond the library's table of 64";
    return hipErrorInvalidDevice;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      *why = "hipGetSymbolAddress of the scratch array failed";
      return e;
    }
    if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0) {
      *why = "scratch array address not 256-byte aligned";
      return hipErrorInvalidValue;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

nb_status noalloc_forces(const Plan &p, const nb_system *sys, double *force, double *energy, double *virial,
                         hipStream_t stream, std::string *why) {
  if (p.lay.total > kScratchBytes) {
    *why = "this batch needs " + std::to_string(p.lay.total) + " bytes of scratch, more than the " +
           std::to_string(kScratchBytes) + " of the allocation-free entry point";
    return NB_ERR_CAPACITY;
  }
  void *ws = nullptr;
  hipError_t e = scratch_address(&ws, why);
  if (e != hipSuccess) {
    *why += std::string(": ") + hipGetErrorString(e);
    return NB_ERR_HIP;
  }
  const Dev d = dev_view(p, ws);
  e = launch_build(p, d, sys, stream);
  if (e == hipSuccess) e = launch_forces(p, d, sys, force, energy, virial, stream);
  if (e != hipSuccess) {
    *why = hipGetErrorString(e);
    return NB_ERR_HIP;
  }
  return NB_OK;
}

}  // namespace nb
