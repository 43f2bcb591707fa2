// Choosing the method (Eq. 14-17; Discussion, "Calculating Efficiencies"):
// one pass over the dense values gathers what both methods' bit counts need
// -- the exact (min, max), the sum of the unsigned element widths and the sum
// of the two's complement element widths (which one applies depends on the
// sign of the minimum, known only at the end) -- and the host derives
// Method 1's n b and Method 2's sum of (k + b_e).
#include <hip/hip_runtime.h>

#include "ccm_internal.hpp"

namespace ccm {
namespace {

constexpr int kSelThreads = 256;

__device__ __forceinline__ uint32_t bitlen_u64(uint64_t u) {
  return u ? 64u - (uint32_t)__clzll((long long)u) : 0u;
}

// Widths of one value: unsigned (Eq. 1 on the element; meaningful for v >= 0)
// and two's complement.
__device__ __forceinline__ void widths(int64_t v, uint64_t &su, uint64_t &ss) {
  const uint32_t lu = bitlen_u64((uint64_t)v);
  su += lu > 1u ? lu : 1u;
  ss += 1u + bitlen_u64((uint64_t)(v ^ (v >> 63)));
}

__global__ void k_sums_init(uint64_t *sums) {
  const int t = threadIdx.x;
  if (t < 2 * kRangeSpread * kSumStride) sums[t] = 0;
}

template <typename T>
__global__ __launch_bounds__(kSelThreads) void k_method_stats(const T *__restrict__ d, uint64_t n,
                                                              RangeSlot *slot, uint64_t *sums,
                                                              int aligned16) {
  constexpr int PER = 16 / sizeof(T);
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  uint64_t su = 0, ss = 0;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t done = 0;
  if (aligned16) {
    const uint64_t n16 = n / PER;
    const uint4 *v = reinterpret_cast<const uint4 *>(d);
    for (uint64_t i = tid; i < n16; i += stride) {
      const uint4 r = v[i];
      const T *t = reinterpret_cast<const T *>(&r);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int64_t x = (int64_t)t[q];
        lo = x < lo ? x : lo;
        hi = x > hi ? x : hi;
        widths(x, su, ss);
      }
    }
    done = n16 * PER;
  }
  for (uint64_t e = done + tid; e < n; e += stride) {
    const int64_t x = (int64_t)d[e];
    lo = x < lo ? x : lo;
    hi = x > hi ? x : hi;
    widths(x, su, ss);
  }
  // the two sums: wave sums, then one atomic pair per block into its slot
  __shared__ uint64_t s_su[kSelThreads / 64], s_ss[kSelThreads / 64];
  su = (uint64_t)wave_sum((int64_t)su);
  ss = (uint64_t)wave_sum((int64_t)ss);
  if ((threadIdx.x & 63) == 0) {
    s_su[threadIdx.x >> 6] = su;
    s_ss[threadIdx.x >> 6] = ss;
  }
  block_range_commit(lo, hi, 0, slot);  // ends with a barrier-protected fold
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t a = 0, b = 0;
#pragma unroll
    for (int w = 0; w < kSelThreads / 64; ++w) {
      a += s_su[w];
      b += s_ss[w];
    }
    uint64_t *mine = sums + 2 * kSumStride * (blockIdx.x % kRangeSpread);
    atomicAdd((unsigned long long *)&mine[0], (unsigned long long)a);
    atomicAdd((unsigned long long *)&mine[1], (unsigned long long)b);
  }
}

}  // namespace

hipError_t launch_method_stats(const void *dense, int dtype, uint64_t n, RangeSlot *slot,
                               uint64_t *sums, hipStream_t s) {
  k_sums_init<<<1, 2 * kRangeSpread * kSumStride, 0, s>>>(sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint64_t g = (n + kSelThreads * 16 - 1) / (kSelThreads * 16);
  g = g < 1 ? 1 : (g > 2048 ? 2048 : g);
  const int al = ((uintptr_t)dense % 16) == 0;
  if (dtype == CCM_I64)
    k_method_stats<int64_t><<<(unsigned)g, kSelThreads, 0, s>>>((const int64_t *)dense, n, slot,
                                                                sums, al);
  else
    k_method_stats<int32_t><<<(unsigned)g, kSelThreads, 0, s>>>((const int32_t *)dense, n, slot,
                                                                sums, al);
  return hipGetLastError();
}

}  // namespace ccm
