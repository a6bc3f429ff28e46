// readout_opt.hip -- optimal-bisector binarization (COSM_READOUT_OPTIMAL).
//
// The exact best line through the origin (the rank-2 rounding of Burer,
// Monteiro and Zhang, which the paper cites for its bisector readout), for
// h = 0.  With x in [0,1) turn, key_i = x_i mod 1/2 and sigma_i = +1 iff
// x_i < 1/2, the bisector at beta in [0, 1/2) gives s_i = sigma_i tau_i with
// tau_i = +1 iff beta <= key_i.  Spins only change at the distinct keys
// b_0 < b_1 < ... < b_{K-1}, so beta = b_k for k < K covers every spin
// configuration of the family (beta and beta + 1/2 give opposite spins and the
// same H).  With rank r_i of key_i among the distinct keys, an edge's product
// s_u s_v is sigma_u sigma_v, negated exactly for lo < k <= hi (lo, hi = the
// smaller and larger rank), so
//   H(k) = sum_e -J sigma_u sigma_v + sum_{e: lo < k <= hi} 2 J sigma_u sigma_v,
// a difference array over k.  The lowest H wins, the smallest k (angle) on
// ties.  Per replica: keys -> segmented radix sort (rocPRIM via hipCUB) ->
// one workgroup: ranks (block scan), difference array in LDS (int atomics),
// prefix minimum, spins.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "device_common.hpp"
#include "internal.hpp"

namespace cosm {
namespace {

constexpr int kOptThreads = 512;

// keys [R][n]: key_i as float bits (non-negative, so the bit order is the
// numeric order); vals [R][n]: i | sigma_i < 0 in bit 31.
template <int ST>
__global__ void __launch_bounds__(256) k_opt_keys(const void *phases, int32_t n, int32_t R,
                                                  uint32_t *keys, uint32_t *vals) {
  using F = Fmt<ST>;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // over [n][R]
  if (idx >= (int64_t)n * R) return;
  const int32_t i = (int32_t)(idx / R), r = (int32_t)(idx % R);
  const float x = fract1(F::to_turn(F::load_elem(phases, (size_t)idx)));
  const bool upper = x >= 0.5f;
  const float key = upper ? x - 0.5f : x;  // exact (same binade or Sterbenz)
  const size_t o = (size_t)r * n + i;
  keys[o] = __float_as_uint(key);
  vals[o] = (uint32_t)i | (upper ? 0x80000000u : 0u);
}

__global__ void k_opt_offsets(int32_t *off, int32_t n, int32_t R) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r <= R) off[r] = r * n;
}

// Inclusive scan of v over the workgroup (kOptThreads lanes); *total = sum.
__device__ __forceinline__ int64_t block_scan(int64_t v, int64_t *wsum, int64_t *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(v, off, 64);
    if (lane >= off) v += y;
  }
  __syncthreads();
  if (lane == 63) wsum[w] = v;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int k = 0; k < kOptThreads / 64; k++) {
    if (k < w) before += wsum[k];
    all += wsum[k];
  }
  *total = all;
  return v + before;
}

struct OptArgs {
  const uint32_t *keys, *vals;  // sorted per replica
  uint32_t *rank;               // [R][n] scratch: rank | sigma < 0 in bit 31
  const int32_t *eu, *ev, *J;
  int8_t *spins;
  int64_t *H, *cut;
  int32_t n, R;
  int64_t m, sumJ;
};

__global__ void __launch_bounds__(kOptThreads) k_opt_readout(const OptArgs a) {
  extern __shared__ int32_t diff[];  // [n + 1]
  __shared__ int64_t wsum[kOptThreads / 64];
  __shared__ int64_t red_v[kOptThreads / 64];
  __shared__ int32_t red_k[kOptThreads / 64];
  const int tid = threadIdx.x;
  const int32_t r = blockIdx.x, n = a.n;
  const size_t row = (size_t)r * n;
  const gptr<uint32_t> keys = as_global(a.keys) + row, vals = as_global(a.vals) + row;
  const gptr_mut<uint32_t> rank = as_global_mut(a.rank) + row;

  // 1. rank of every vertex among the distinct keys
  int64_t carry = 0;
  for (int32_t p0 = 0; p0 < n; p0 += kOptThreads) {
    const int32_t p = p0 + tid;
    int64_t flag = 0;
    if (p < n) flag = (p == 0 || keys[p] != keys[p - 1]) ? 1 : 0;
    int64_t tot;
    const int64_t inc = block_scan(flag, wsum, &tot);
    if (p < n) {
      const uint32_t v = vals[p];
      rank[v & 0x7fffffffu] = (uint32_t)(carry + inc - 1) | (v & 0x80000000u);
    }
    carry += tot;
  }
  const int32_t K = (int32_t)carry;
  for (int32_t k = tid; k <= K; k += kOptThreads) diff[k] = 0;
  __syncthreads();

  // 2. difference array of the sign changes, and H at k = 0
  int64_t base = 0;
  for (int64_t e = tid; e < a.m; e += kOptThreads) {
    const uint32_t ru = rank[as_global(a.eu)[e]], rv = rank[as_global(a.ev)[e]];
    const int32_t ss = ((ru ^ rv) >> 31) ? -1 : 1;  // sigma_u sigma_v
    const int32_t Jss = as_global(a.J)[e] * ss;
    base -= Jss;
    const int32_t qu = (int32_t)(ru & 0x7fffffffu), qv = (int32_t)(rv & 0x7fffffffu);
    if (qu != qv) {
      atomicAdd(&diff[min(qu, qv) + 1], 2 * Jss);
      atomicAdd(&diff[max(qu, qv) + 1], -2 * Jss);
    }
  }
  base = block_sum(base, wsum);  // synchronises

  // 3. H(k) = base + prefix(diff)[k]; lowest H, smallest k on ties
  int64_t best = INT64_MAX;
  int32_t bestk = 0;
  carry = 0;
  for (int32_t k0 = 0; k0 < K; k0 += kOptThreads) {
    const int32_t k = k0 + tid;
    int64_t tot;
    const int64_t inc = block_scan(k < K ? (int64_t)diff[k] : 0, wsum, &tot);
    if (k < K) {
      const int64_t h = base + carry + inc;
      if (h < best) {  // k increases within a thread: strict keeps the smallest
        best = h;
        bestk = k;
      }
    }
    carry += tot;
  }
  // workgroup argmin (value, then index)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t ov = __shfl_xor(best, off, 64);
    const int32_t ok = __shfl_xor(bestk, off, 64);
    if (ov < best || (ov == best && ok < bestk)) {
      best = ov;
      bestk = ok;
    }
  }
  const int lane = tid & 63, w = tid >> 6;
  __syncthreads();
  if (lane == 0) {
    red_v[w] = best;
    red_k[w] = bestk;
  }
  __syncthreads();
  best = red_v[0];
  bestk = red_k[0];
  for (int k = 1; k < kOptThreads / 64; k++)
    if (red_v[k] < best || (red_v[k] == best && red_k[k] < bestk)) {
      best = red_v[k];
      bestk = red_k[k];
    }

  // 4. spins of the chosen bisector: s_i = sigma_i (rank_i >= k* ? +1 : -1)
  for (int32_t i = tid; i < n; i += kOptThreads) {
    const uint32_t q = rank[i];
    const int32_t tau = (int32_t)(q & 0x7fffffffu) >= bestk ? 1 : -1;
    as_global_mut(a.spins)[row + i] = (int8_t)((q >> 31) ? -tau : tau);
  }
  if (tid == 0) {
    a.H[r] = best;
    a.cut[r] = (-a.sumJ - best) / 2;  // Eq. (14), h = 0
  }
}

}  // namespace

size_t opt_readout_temp_bytes(int32_t n, int32_t R) {
  size_t bytes = 0;
  if (hipcub::DeviceSegmentedRadixSort::SortPairs(
          nullptr, bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
          (const uint32_t *)nullptr, (uint32_t *)nullptr, n * R, R, (const int32_t *)nullptr,
          (const int32_t *)nullptr, 0, 31, (hipStream_t)0) != hipSuccess)
    return 0;
  return bytes;
}

int launch_readout_optimal(cosm_state *s) {
  const int32_t n = s->n, R = s->R;
  const int64_t nr = (int64_t)n * R;
  const DeviceBuffers &d = s->d;
  const dim3 blk(256);
  switch (s->p.storage) {
    case COSM_STORE_FP32:
      hipLaunchKernelGGL((k_opt_keys<COSM_STORE_FP32>), dim3((unsigned)((nr + 255) / 256)), blk, 0,
                         s->stream, d.phases, n, R, d.opt_keys, d.opt_vals);
      break;
    case COSM_STORE_FP16:
      hipLaunchKernelGGL((k_opt_keys<COSM_STORE_FP16>), dim3((unsigned)((nr + 255) / 256)), blk, 0,
                         s->stream, d.phases, n, R, d.opt_keys, d.opt_vals);
      break;
    case COSM_STORE_FP16_PK:
      hipLaunchKernelGGL((k_opt_keys<COSM_STORE_FP16_PK>), dim3((unsigned)((nr + 255) / 256)), blk, 0,
                         s->stream, d.phases, n, R, d.opt_keys, d.opt_vals);
      break;
    case COSM_STORE_BF16:
      hipLaunchKernelGGL((k_opt_keys<COSM_STORE_BF16>), dim3((unsigned)((nr + 255) / 256)), blk, 0,
                         s->stream, d.phases, n, R, d.opt_keys, d.opt_vals);
      break;
    case COSM_STORE_FIX16:
      hipLaunchKernelGGL((k_opt_keys<COSM_STORE_FIX16>), dim3((unsigned)((nr + 255) / 256)), blk, 0,
                         s->stream, d.phases, n, R, d.opt_keys, d.opt_vals);
      break;
    default:
      hipLaunchKernelGGL((k_opt_keys<COSM_STORE_FIX32>), dim3((unsigned)((nr + 255) / 256)), blk, 0,
                         s->stream, d.phases, n, R, d.opt_keys, d.opt_vals);
  }
  COSM_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_opt_offsets, dim3((unsigned)((R + 1 + 255) / 256)), blk, 0, s->stream,
                     d.opt_off, n, R);
  COSM_HIP_CHECK(hipGetLastError());
  size_t bytes = s->opt_temp_bytes;
  COSM_HIP_CHECK(hipcub::DeviceSegmentedRadixSort::SortPairs(
      d.opt_temp, bytes, d.opt_keys, d.opt_keys2, d.opt_vals, d.opt_vals2, (int)nr, R, d.opt_off,
      d.opt_off + 1, 0, 31, s->stream));
  OptArgs a{};
  a.keys = d.opt_keys2;
  a.vals = d.opt_vals2;
  a.rank = d.opt_vals;  // the unsorted values are no longer needed
  a.eu = d.eu;
  a.ev = d.ev;
  a.J = d.J;
  a.spins = d.spins;
  a.H = d.H;
  a.cut = d.cut;
  a.n = n;
  a.R = R;
  a.m = s->m;
  a.sumJ = s->sumJ;
  const size_t lds = ((size_t)n + 1) * 4;
  (void)hipFuncSetAttribute((const void *)k_opt_readout, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL(k_opt_readout, dim3(R), dim3(kOptThreads), lds, s->stream, a);
  COSM_HIP_CHECK(hipGetLastError());
  return COSM_OK;
}

}  // namespace cosm
