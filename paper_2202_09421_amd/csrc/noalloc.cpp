// rte_forward_noalloc: the forward solve without a workspace argument, for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops).  Its device memory is a file-scope array that every
// GPU the library runs on holds for the life of the process.
#include <hip/hip_runtime.h>

#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "rte_internal.h"

static constexpr int64_t kScratchBytes = int64_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device ordinal, resolved on first use

// Address of this device's copy of `scratch` (host code never uses the
// array's name as an address), resolved once per device with it current.
int scratch_for_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    rte::set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    return RTE_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      rte::set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return RTE_EDEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RTE_OK;
}

}  // namespace

extern "C" int rte_forward_noalloc(rte_plan* h, const void* mu_a, const void* mu_s, double* G, void* u_final,
                                   void* stream) {
  if (!h || !mu_a || !mu_s) {
    rte::set_error("plan, mu_a and mu_s must not be NULL");
    return RTE_EINVAL;
  }
  try {
    rte::set_error("");
    rte::Plan& p = *reinterpret_cast<rte::Plan*>(h);
    const int64_t need = rte::workspace_bytes(p, false);
    if (need > kScratchBytes) {
      std::ostringstream o;
      o << "rte_forward_noalloc: this forward needs " << need << " bytes of device scratch, the static scratch "
        << "holds " << kScratchBytes << " (use rte_forward with a workspace)";
      rte::set_error(o.str());
      return RTE_ENOMEM;
    }
    void* ptr = nullptr;
    if (int rc = scratch_for_current_device(&ptr)) return rc;
    return rte::forward_into(p, mu_a, mu_s, G, u_final, ptr, kScratchBytes, static_cast<hipStream_t>(stream));
  } catch (const std::exception& e) {
    rte::set_error(e.what());
    return RTE_EINVAL;
  }
}
