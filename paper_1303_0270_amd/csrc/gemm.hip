// C = A B on SM-packed operands, exact, written densely into scratch with the
// exact range of C (the max-reduction pass that fixes C's width).
//
// Generic path (any widths): 64x64 output tiles per 256-lane block, K in
// chunks of 32.  Each chunk of A (64x32) and B (32x64) is decoded from the
// packed streams straight into LDS; every lane then accumulates a 4x4
// micro-tile in int64.  The overflow rule checked on the host (K * max|A| *
// max|B| < 2^63) makes every partial sum exact.
#include "ccm_internal.hpp"

namespace ccm {
namespace {

constexpr int kTM = 64, kTN = 64, kTK = 32, kThreads = 256;

template <typename ET, typename OT>
__global__ __launch_bounds__(kThreads) void k_gemm_generic(
    const uint32_t *__restrict__ aw, int abits, int asgn, const uint32_t *__restrict__ bw,
    int bbits, int bsgn, int64_t M, int64_t K, int64_t N, OT *__restrict__ C, RangeSlot *slot) {
  __shared__ ET As[kTK][kTM + 1];  // As[k][m]
  __shared__ ET Bs[kTK][kTN + 1];  // Bs[k][n]
  const int64_t m0 = (int64_t)blockIdx.y * kTM, n0 = (int64_t)blockIdx.x * kTN;
  const int tid = threadIdx.x;
  const int tm = (tid / 16) * 4, tn = (tid % 16) * 4;
  int64_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0;

  for (int64_t k0 = 0; k0 < K; k0 += kTK) {
    for (int q = tid; q < kTM * kTK; q += kThreads) {
      const int mm = q / kTK, kk = q % kTK;
      const int64_t m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < M && k < K) ? (ET)value_at(aw, (uint64_t)(m * K + k), abits, asgn) : ET(0);
    }
    for (int q = tid; q < kTK * kTN; q += kThreads) {
      const int kk = q / kTN, nn = q % kTN;
      const int64_t k = k0 + kk, n = n0 + nn;
      Bs[kk][nn] = (k < K && n < N) ? (ET)value_at(bw, (uint64_t)(k * N + n), bbits, bsgn) : ET(0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kTK; ++kk) {
      ET a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tm + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tn + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += (int64_t)a[i] * (int64_t)b[j];
    }
    __syncthreads();
  }

  int64_t lo = INT64_MAX, hi = INT64_MIN;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t m = m0 + tm + i;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t n = n0 + tn + j;
      if (m < M && n < N) {
        const int64_t v = acc[i][j];
        C[m * N + n] = (OT)v;
        lo = v < lo ? v : lo;
        hi = v > hi ? v : hi;
      }
    }
  }
  block_range_commit(lo, hi, 0, slot);
}

template <typename ET>
hipError_t launch_generic(const uint32_t *aw, int abits, int asgn, const uint32_t *bw,
                          int bbits, int bsgn, int64_t M, int64_t K, int64_t N, int out32,
                          void *scratch, RangeSlot *slot, hipStream_t s) {
  dim3 grid((unsigned)((N + kTN - 1) / kTN), (unsigned)((M + kTM - 1) / kTM));
  if (out32)
    k_gemm_generic<ET, int32_t><<<grid, kThreads, 0, s>>>(aw, abits, asgn, bw, bbits, bsgn, M,
                                                          K, N, (int32_t *)scratch, slot);
  else
    k_gemm_generic<ET, int64_t><<<grid, kThreads, 0, s>>>(aw, abits, asgn, bw, bbits, bsgn, M,
                                                          K, N, (int64_t *)scratch, slot);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_matmul(const uint32_t *aw, int abits, int asgn, const uint32_t *bw,
                         int bbits, int bsgn, int64_t M, int64_t K, int64_t N, int use_i8,
                         int out32, void *scratch, RangeSlot *slot, hipStream_t s) {
  (void)use_i8;
  // Operands that fit in 32 bits are staged as int32 (products stay exact in
  // int64); wider ones as int64.
  const bool narrow = (abits < 32 || (abits == 32 && asgn)) && (bbits < 32 || (bbits == 32 && bsgn));
  if (narrow)
    return launch_generic<int32_t>(aw, abits, asgn, bw, bbits, bsgn, M, K, N, out32, scratch,
                                   slot, s);
  return launch_generic<int64_t>(aw, abits, asgn, bw, bbits, bsgn, M, K, N, out32, scratch,
                                 slot, s);
}

}  // namespace ccm
