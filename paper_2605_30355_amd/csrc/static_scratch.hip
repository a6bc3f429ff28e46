// static_scratch.hip -- cosm_init_static: a solver state whose device buffers
// live in a fixed array the library holds on every GPU it runs on, for callers
// that cannot allocate device memory (code under stream capture, serving loops
// with a fixed footprint, harnesses that forbid hipMalloc).
//
// The array is a file-scope __device__ variable: each device that loads the
// library gets its own copy at its own address.  Host code never passes the
// array's name to a kernel (on the host that name is only a stand-in); it
// looks up each device's address once with hipGetSymbolAddress and hands that
// pointer to cosm_init's buffer plan, exactly as a caller workspace would be.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.hpp"

namespace cosm {
namespace {

constexpr size_t kStaticScratchBytes = (size_t)32 << 20;  // 32 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};     // each device's address of scratch
bool g_in_use[kMaxDevices] = {};   // a live state holds that device's array

}  // namespace

void release_static_scratch(int32_t dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev >= 0 && dev < kMaxDevices) g_in_use[dev] = false;
}

}  // namespace cosm

using namespace cosm;

extern "C" int cosm_init_static(cosm_state **out, int32_t n, int64_t m, const int32_t *eu,
                                const int32_t *ev, const int32_t *J, const int32_t *h,
                                const int32_t *colour, int32_t num_colours, const cosm_params *p,
                                uint64_t seed, int32_t replicas, void *hip_stream) {
  clear_error();
  if (out == nullptr) return set_error(COSM_EINVAL, "out must not be NULL");
  *out = nullptr;
  size_t need = 0;
  if (int rc = cosm_workspace_bytes(n, m, num_colours, replicas, p, &need)) return rc;
  if (need > kStaticScratchBytes)
    return set_error(COSM_ERANGE, "the state needs " + std::to_string(need) +
                                      " bytes of device memory; the static scratch array holds " +
                                      std::to_string(kStaticScratchBytes));
  int dev = 0;
  COSM_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(COSM_EDEVICE, "device index out of range");
  void *ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_in_use[dev])
      return set_error(COSM_ESTATE, "a state made by cosm_init_static is still alive on this "
                                    "device (cosm_destroy it first)");
    if (g_ptr[dev] == nullptr) {
      // first call on this device (it is current): the address of its copy
      void *addr = nullptr;
      const hipError_t err = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
      if (err != hipSuccess || addr == nullptr)
        return set_error(COSM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                           hipGetErrorString(err));
      g_ptr[dev] = addr;
    }
    ptr = g_ptr[dev];
    g_in_use[dev] = true;
  }
  const int rc = init_state(out, n, m, eu, ev, J, h, colour, num_colours, p, seed, replicas,
                            hip_stream, ptr, kStaticScratchBytes, dev);
  if (rc != COSM_OK) release_static_scratch(dev);
  return rc;
}
