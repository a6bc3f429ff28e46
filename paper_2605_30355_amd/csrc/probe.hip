// probe.hip -- LDS bandwidth ceiling for the sweep's access mix (cosm_lds_probe).
//
// Each lane owns two rows of W words in its workgroup's LDS (rows of
// consecutive lanes are consecutive, so every read and write group is
// bank-conflict free), and per iteration reads both, adds one to every word
// and writes both back: the 2 reads and 2 writes per (edge, row) of the sweep
// with next to no arithmetic and no barriers, i.e. the LDS ceiling of that
// access mix.  The timed kernel runs kIters iterations; the result is LDS
// bytes moved per second.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace cosm {
namespace {

constexpr int kProbeThreads = 768;
constexpr int kIters = 4000;

template <int W>
__global__ void __launch_bounds__(kProbeThreads) k_lds_mix(float *sink, int iters) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int i = tid; i < 2 * nth * W; i += nth) lds[i] = (uint32_t)i;
  __syncthreads();
  const uint32_t bu = (uint32_t)tid * 4u * W, bv = (uint32_t)(tid + nth) * 4u * W;
  for (int it = 0; it < iters; it++) {
    uint32_t wu[W], wv[W];
    lds_load_at<W>(lds, bu, wu);
    lds_load_at<W>(lds, bv, wv);
#pragma unroll
    for (int k = 0; k < W; k++) {
      wu[k] += 1u;
      wv[k] += 1u;
    }
    lds_store_at<W>(lds, bu, wu);
    lds_store_at<W>(lds, bv, wv);
    __asm__ volatile("" ::: "memory");  // keep every iteration's LDS traffic
  }
  __syncthreads();
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < W; k++) acc += lds[tid * W + k];
  sink[(size_t)blockIdx.x * nth + tid] = (float)acc;
}

template <int W>
int run_probe(int blocks, hipStream_t st, double *gbs) {
  const size_t lds = (size_t)2 * kProbeThreads * W * 4;
  float *sink = nullptr;
  COSM_HIP_CHECK(hipMalloc(&sink, (size_t)blocks * kProbeThreads * sizeof(float)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = COSM_OK;
  float ms = 0.0f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = set_error(COSM_EDEVICE, "hipEventCreate failed");
  } else {
    hipLaunchKernelGGL((k_lds_mix<W>), dim3(blocks), dim3(kProbeThreads), lds, st, sink, 16);
    (void)hipEventRecord(e0, st);
    hipLaunchKernelGGL((k_lds_mix<W>), dim3(blocks), dim3(kProbeThreads), lds, st, sink, kIters);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.0f)
      rc = set_error(COSM_EDEVICE, "LDS probe kernel failed");
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  if (rc) return rc;
  // 2 reads + 2 writes of 4 W bytes per lane and iteration
  const double bytes = (double)blocks * kProbeThreads * kIters * 4.0 * 4.0 * W;
  *gbs = bytes / (ms * 1e-3) / 1e9;
  return COSM_OK;
}

}  // namespace
}  // namespace cosm

extern "C" int cosm_lds_probe(int32_t row_words, int32_t blocks_per_cu, void *hip_stream,
                              double *gbs_out) {
  using namespace cosm;
  clear_error();
  if (gbs_out == nullptr) return set_error(COSM_EINVAL, "gbs_out must not be NULL");
  if (blocks_per_cu != 1 && blocks_per_cu != 2)
    return set_error(COSM_EINVAL, "blocks_per_cu must be 1 or 2");
  int dev = 0, cus = 0;
  COSM_HIP_CHECK(hipGetDevice(&dev));
  COSM_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = cus * blocks_per_cu;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (row_words == 1) return run_probe<1>(blocks, st, gbs_out);
  if (row_words == 2) return run_probe<2>(blocks, st, gbs_out);
  if (row_words == 4) return run_probe<4>(blocks, st, gbs_out);
  return set_error(COSM_EINVAL, "row_words must be 1, 2 or 4");
}
