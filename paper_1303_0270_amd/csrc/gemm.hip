// C = A B on SM-packed operands, exact, written densely into scratch with the
// exact range of C (the max-reduction pass that fixes C's width).
//
// Generic path (any widths): 64x64 output tiles per 256-lane block, K in
// chunks of 32.  Each chunk of A (64x32) and B (32x64) is decoded from the
// packed streams straight into LDS; every lane then accumulates a 4x4
// micro-tile in int64.  The overflow rule checked on the host (K * max|A| *
// max|B| < 2^63) makes every partial sum exact.
#include "ccm_internal.hpp"
#include "group_codec.hpp"

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

// ---- int8 MFMA path --------------------------------------------------------
//
// B (K x N, row-major) is first re-packed column-major at the same width (the
// other unravel order the paper allows), so that both operands hold K
// contiguously: A as M rows of K, Bt as N rows of K.  Every K-chunk of a
// 128 x 128 output tile is then decoded from the packed fields straight into
// int8 LDS tiles and multiplied with v_mfma_i32_32x32x32_i8.  A and B operand
// lanes use the same assignment of the 32 K values of a step to (lane half,
// byte), so the products summed per output are exactly those of the dot
// product.  int32 accumulation is exact because the host only takes this
// path when K * max|A| * max|B| < 2^31.

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Bt[n][k] = B[k][n]: lane g builds output group g of the column-major stream
// (elements 32g..32g+31, walking k within column n and wrapping to n+1).
__global__ __launch_bounds__(256) void k_transpose_packed(const uint32_t *__restrict__ bw,
                                                          int bits, int sgn, int64_t K,
                                                          int64_t N, uint32_t *__restrict__ out,
                                                          uint64_t cap32, uint64_t ngroups_out) {
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups_out) return;
  const uint64_t n_elems = (uint64_t)K * (uint64_t)N;
  uint64_t e = g * kGroup;
  int64_t n = (int64_t)(e / (uint64_t)K), k = (int64_t)(e % (uint64_t)K);
  int64_t v[kGroup];
#pragma unroll
  for (int i = 0; i < kGroup; ++i) {
    v[i] = (e + i < n_elems) ? value_at(bw, (uint64_t)(k * N + n), bits, sgn) : 0;
    if (++k == K) {
      k = 0;
      ++n;
    }
  }
  const uint64_t w0 = g * (uint64_t)bits;
  codec::encode_rt(v, bits, out + w0, cap32 - w0);
}

constexpr int kMT = 128, kNT = 128, kKT = 64, kLdsPitch = kKT + 16;  // bytes per tile row

// Decodes row `row` (global index r of a rows x K stream), K-chunk [k0, k0+64)
// into 64 int8 values at dst.  Elements past K or rows past `rows` are zero.
template <int B>
__device__ __forceinline__ void decode_row_chunk(const uint32_t *__restrict__ w, int sgn,
                                                 int64_t r, int64_t rows, int64_t K, int64_t k0,
                                                 int8_t *dst) {
  uint32_t packed[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) packed[q] = 0;
  if (r < rows) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t kb = k0 + 32 * h;
      if (kb < K) {
        const uint64_t bit = ((uint64_t)r * (uint64_t)K + (uint64_t)kb) * (uint64_t)B;
        const uint32_t *p = w + (bit >> 5);
        const int s = (int)(bit & 31u);
        uint32_t ww[B + 1];
#pragma unroll
        for (int q = 0; q <= B; ++q) ww[q] = p[q];
        if (s != 0) {
#pragma unroll
          for (int q = 0; q < B; ++q) ww[q] = __builtin_amdgcn_alignbit(ww[q + 1], ww[q], s);
        }
        const int lim = K - kb < 32 ? (int)(K - kb) : 32;
#pragma unroll
        for (int i = 0; i < 32; ++i) {
          const uint64_t u = codec::field<B>(ww, i);
          int32_t v = sgn ? (int32_t)sext64(u, B) : (int32_t)u;
          if (i >= lim) v = 0;
          packed[8 * h + i / 4] |= ((uint32_t)v & 0xffu) << (8 * (i % 4));
        }
      }
    }
  }
  uint4 *d = reinterpret_cast<uint4 *>(dst);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    d[q] = make_uint4(packed[4 * q], packed[4 * q + 1], packed[4 * q + 2], packed[4 * q + 3]);
}

__device__ __forceinline__ void decode_row_chunk_rt(const uint32_t *w, int bits, int sgn,
                                                    int64_t r, int64_t rows, int64_t K,
                                                    int64_t k0, int8_t *dst) {
  switch (bits) {
    case 1: decode_row_chunk<1>(w, sgn, r, rows, K, k0, dst); break;
    case 2: decode_row_chunk<2>(w, sgn, r, rows, K, k0, dst); break;
    case 3: decode_row_chunk<3>(w, sgn, r, rows, K, k0, dst); break;
    case 4: decode_row_chunk<4>(w, sgn, r, rows, K, k0, dst); break;
    case 5: decode_row_chunk<5>(w, sgn, r, rows, K, k0, dst); break;
    case 6: decode_row_chunk<6>(w, sgn, r, rows, K, k0, dst); break;
    case 7: decode_row_chunk<7>(w, sgn, r, rows, K, k0, dst); break;
    default: decode_row_chunk<8>(w, sgn, r, rows, K, k0, dst); break;
  }
}

template <typename OT>
__global__ __launch_bounds__(256) void k_gemm_i8(const uint32_t *__restrict__ aw, int abits,
                                                 int asgn, const uint32_t *__restrict__ btw,
                                                 int bbits, int bsgn, int64_t M, int64_t K,
                                                 int64_t N, OT *__restrict__ C, RangeSlot *slot) {
  __shared__ __align__(16) int8_t As[kMT * kLdsPitch];
  __shared__ __align__(16) int8_t Bs[kNT * kLdsPitch];
  const int64_t m0 = (int64_t)blockIdx.y * kMT, n0 = (int64_t)blockIdx.x * kNT;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;  // 64 x 64 quadrant of the tile
  v16i acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0;

  for (int64_t k0 = 0; k0 < K; k0 += kKT) {
    // 256 lanes decode 128 A rows and 128 Bt rows, one 64-element chunk each
    if (tid < 128)
      decode_row_chunk_rt(aw, abits, asgn, m0 + tid, M, K, k0, As + tid * kLdsPitch);
    else
      decode_row_chunk_rt(btw, bbits, bsgn, n0 + (tid - 128), N, K, k0,
                          Bs + (tid - 128) * kLdsPitch);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKT; kk += 32) {
      const int koff = kk + 16 * (lane >> 5);
      v4i a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = *reinterpret_cast<const v4i *>(As + (wm * 64 + t * 32 + (lane & 31)) * kLdsPitch + koff);
        b[t] = *reinterpret_cast<const v4i *>(Bs + (wn * 64 + t * 32 + (lane & 31)) * kLdsPitch + koff);
      }
#pragma unroll
      for (int ta = 0; ta < 2; ++ta)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb)
          acc[ta][tb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[ta], b[tb], acc[ta][tb], 0, 0, 0);
    }
    __syncthreads();
  }

  // 32x32 accumulator layout: lane l, register r -> column l%32,
  // row 8*(r/4) + 4*(l/32) + r%4
  int64_t lo = INT64_MAX, hi = INT64_MIN;
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t i = m0 + wm * 64 + ta * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
        const int64_t j = n0 + wn * 64 + tb * 32 + (lane & 31);
        if (i < M && j < N) {
          const int64_t v = acc[ta][tb][r];
          C[i * N + j] = (OT)v;
          lo = v < lo ? v : lo;
          hi = v > hi ? v : hi;
        }
      }
  block_range_commit(lo, hi, 0, slot);
}

}  // namespace

uint64_t matmul_bt_words32(int64_t K, int64_t N, int bbits) {
  return cap_words32((uint64_t)K * (uint64_t)N, bbits);
}

hipError_t launch_matmul_i8(const uint32_t *aw, int abits, int asgn, const uint32_t *bw,
                            int bbits, int bsgn, int64_t M, int64_t K, int64_t N, int out32,
                            void *scratch_c, uint32_t *scratch_bt, RangeSlot *slot,
                            hipStream_t s) {
  const uint64_t cap = matmul_bt_words32(K, N, bbits);
  const uint64_t ngroups = (cap + bbits - 1) / bbits;
  k_transpose_packed<<<(unsigned)((ngroups + 255) / 256), 256, 0, s>>>(bw, bbits, bsgn, K, N,
                                                                       scratch_bt, cap, ngroups);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((N + kNT - 1) / kNT), (unsigned)((M + kMT - 1) / kMT));
  if (out32)
    k_gemm_i8<int32_t><<<grid, 256, 0, s>>>(aw, abits, asgn, scratch_bt, bbits, bsgn, M, K, N,
                                            (int32_t *)scratch_c, slot);
  else
    k_gemm_i8<int64_t><<<grid, 256, 0, s>>>(aw, abits, asgn, scratch_bt, bbits, bsgn, M, K, N,
                                            (int64_t *)scratch_c, slot);
  return hipGetLastError();
}

hipError_t launch_matmul(const uint32_t *aw, int abits, int asgn, const uint32_t *bw,
                         int bbits, int bsgn, int64_t M, int64_t K, int64_t N, int use_i8,
                         int out32, void *scratch, RangeSlot *slot, hipStream_t s) {
  if (use_i8) {
    // scratch = [dense C, rounded up to 256 bytes][column-major B payload]
    const uint64_t cbytes = ((out32 ? 4u : 8u) * (uint64_t)M * (uint64_t)N + 255u) / 256u * 256u;
    return launch_matmul_i8(aw, abits, asgn, bw, bbits, bsgn, M, K, N, out32, scratch,
                            (uint32_t *)((char *)scratch + cbytes), slot, s);
  }
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
