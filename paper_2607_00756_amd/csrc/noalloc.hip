// bip_eels_signal_noalloc: bip_eels_signal for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).  Its workspace is a fixed device array of this
// file, so the call allocates nothing; requests that need more workspace than
// the array holds are refused.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "bip_internal.h"
#include "host_common.h"

namespace {

// Size of the workspace array: enough for the small maps, qEELS and beam
// outputs this entry point is meant for (one 128^2 specimen with a 32^2
// window and a 16 x 16 raster needs about 30 MiB).  Every device the library
// runs on holds it until the process ends.
constexpr size_t kScratchBytes = (size_t)64 << 20;

static __device__ __align__(256) char scratch[kScratchBytes];

// Device address of `scratch` on each device, looked up once per device with
// that device current (each device holds its own copy at its own address).
// In host code the name `scratch` is only a host-side stand-in: it must never
// be passed to a kernel or a copy.
std::mutex g_mu;
std::map<int, void*> g_addr;

int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return bip::hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_addr.find(dev);
  if (it == g_addr.end()) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return bip::hip_fail(e, "hipGetSymbolAddress(scratch)");
    it = g_addr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return BIP_OK;
}

}  // namespace

extern "C" {

size_t bip_noalloc_scratch_bytes(void) { return kScratchBytes; }

int bip_eels_signal_noalloc(bip_plan* p, int32_t n_ch, const float* H, const int64_t* H_off,
                            const int32_t* atom_subset, int32_t n_subset, int32_t scan_sy,
                            int32_t scan_sx, int32_t out_mode, int32_t precision, float* out,
                            void* stream) {
  void* work = nullptr;
  const int rc = scratch_address(&work);
  if (rc) return rc;
  return bip::eels_signal_impl(p, n_ch, H, H_off, atom_subset, n_subset, scan_sy, scan_sx, out_mode,
                               precision, out, work, kScratchBytes, stream);
}

}  // extern "C"
