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
// Both operands are first decoded once into int8 scratch with K contiguous
// and zero-padded to a multiple of the K chunk: A as M rows, B transposed as N rows
// (B^T, the paper's other unravel order).  Decoding inside the GEMM's K loop
// would redo it for every output tile (N/256 times per A element) and read
// the packed rows one lane per row, which the memory pipeline serves one
// cache line per lane; decoded once, the tiles stream with coalesced 16-byte
// loads.  The GEMM then multiplies 256x256 output tiles per 1024-lane block
// (sixteen waves, each a 64x64 block of 2x2 32x32 accumulators) with
// v_mfma_i32_32x32x32_i8 over double-buffered LDS tiles, K in chunks of 128:
// the next chunk is loaded into registers before the current chunk's MFMAs
// and stored to the other buffer after them (tile shape, wave shape and chunk
// length measured against 128x64 waves and 64-byte chunks on the 8192^3
// product).  A and B operand lanes use the same assignment of
// the 32 K values of a step to (lane half, byte), so the products summed per
// output are exactly those of the dot product.  int32 accumulation is exact
// because the host only takes this path when K * max|A| * max|B| < 2^31.

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

constexpr int kBM = 256, kBN = 256, kBK = 128, kPitch8 = kBK + 16;  // LDS row pitch, bytes
constexpr int kWM = 64, kWN = 64;  // output rows and columns per wave
constexpr int kFM = kWM / 32, kFN = kWN / 32;  // 32x32 accumulator blocks per wave
constexpr int kGemmThreads = 64 * (kBM / kWM) * (kBN / kWN);
constexpr size_t kGemmLds = 2u * (kBM + kBN) * kPitch8;  // two buffers of A and B tiles

__host__ __device__ inline int64_t padded_k(int64_t K) { return (K + kBK - 1) / kBK * kBK; }

// Four int8 fields (values fit int8) into one word, byte i = field i.
__device__ __forceinline__ uint32_t bytes4(int32_t a, int32_t b, int32_t c, int32_t d) {
  return (uint32_t)(a & 0xff) | ((uint32_t)(b & 0xff) << 8) | ((uint32_t)(c & 0xff) << 16) |
         ((uint32_t)(d & 0xff) << 24);
}

// out[row][c .. c+32) = A[row][c .. c+32) as int8 (zero at or past K); one
// block per row, lane j takes columns 32j..32j+31 (one group's worth of fields,
// re-aligned with a funnel shift when the row starts inside a word).
template <int B>
__global__ __launch_bounds__(256) void k_decode_rows_i8(const uint32_t *__restrict__ w,
                                                        uint64_t cap, int sgn, int64_t K,
                                                        int64_t ldk, int8_t *__restrict__ out) {
  const int64_t row = blockIdx.x;
  for (int64_t c = 32 * (int64_t)threadIdx.x; c < ldk; c += 32 * 256) {
    uint32_t o[8];
    if (c < K) {
      const uint64_t bit = ((uint64_t)row * (uint64_t)K + (uint64_t)c) * B;
      const uint64_t w0 = bit >> 5;
      const int sh = (int)(bit & 31u);
      uint32_t ww[B + 1];
#pragma unroll
      for (int q = 0; q <= B; ++q) ww[q] = w[w0 + q < cap ? w0 + q : cap - 1];
#pragma unroll
      for (int q = 0; q < B; ++q) ww[q] = __builtin_amdgcn_alignbit(ww[q + 1], ww[q], sh);
      const int lim = K - c < 32 ? (int)(K - c) : 32;
      int32_t v[32];
#pragma unroll
      for (int i = 0; i < 32; ++i) {
        const uint64_t u = codec::field<B>(ww, i);
        v[i] = i < lim ? (sgn ? (int32_t)sext64(u, B) : (int32_t)u) : 0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) o[q] = bytes4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) o[q] = 0;
    }
    uint4 *d = reinterpret_cast<uint4 *>(out + row * ldk + c);
    d[0] = make_uint4(o[0], o[1], o[2], o[3]);
    d[1] = make_uint4(o[4], o[5], o[6], o[7]);
  }
}

// out[n][k] = B[k][n] as int8 (zero at or past K): lane l of a wave takes
// column n0 + l, so each step reads 64 neighbouring fields of one row of B;
// the wave's 32 consecutive k are packed into 32 bytes.
template <int B>
__global__ __launch_bounds__(256) void k_decode_cols_i8(const uint32_t *__restrict__ w,
                                                        uint64_t cap, int sgn, int64_t K,
                                                        int64_t N, int64_t ldk,
                                                        int8_t *__restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int64_t k0 = (int64_t)blockIdx.y * 128 + 32 * (threadIdx.x >> 6);
  if (n >= N || k0 >= ldk) return;
  int32_t v[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const int64_t k = k0 + i;
    v[i] = 0;
    if (k < K) {
      const uint64_t bit = ((uint64_t)k * (uint64_t)N + (uint64_t)n) * B;
      const uint64_t w0 = bit >> 5;
      uint32_t u;
      if constexpr (32 % B == 0) {  // fields never straddle a word
        u = (w[w0] >> (bit & 31u)) & ((1u << B) - 1u);
      } else {
        const uint32_t lo = w[w0], hi = w[w0 + 1 < cap ? w0 + 1 : cap - 1];
        u = __builtin_amdgcn_alignbit(hi, lo, (int)(bit & 31u)) & ((1u << B) - 1u);
      }
      v[i] = sgn ? ((int32_t)(u << (32 - B)) >> (32 - B)) : (int32_t)u;
    }
  }
  uint4 *d = reinterpret_cast<uint4 *>(out + n * ldk + k0);
#pragma unroll
  for (int q = 0; q < 2; ++q)
    d[q] = make_uint4(bytes4(v[16 * q], v[16 * q + 1], v[16 * q + 2], v[16 * q + 3]),
                      bytes4(v[16 * q + 4], v[16 * q + 5], v[16 * q + 6], v[16 * q + 7]),
                      bytes4(v[16 * q + 8], v[16 * q + 9], v[16 * q + 10], v[16 * q + 11]),
                      bytes4(v[16 * q + 12], v[16 * q + 13], v[16 * q + 14], v[16 * q + 15]));
}

template <typename OT>
__global__ __launch_bounds__(kGemmThreads) void k_gemm_i8(const int8_t *__restrict__ A,
                                                          const int8_t *__restrict__ Bt, int64_t M,
                                                          int64_t N, int64_t ldk,
                                                          OT *__restrict__ C, RangeSlot *slot) {
  extern __shared__ __align__(16) int8_t gemm_lds[];
  // buffer b: A tile at b * (kBM + kBN) * kPitch8, then the B tile
  auto tile = [&](int b, int opnd) {
    return gemm_lds + b * (kBM + kBN) * kPitch8 + opnd * kBM * kPitch8;
  };
  const int64_t m0 = (int64_t)blockIdx.y * kBM, n0 = (int64_t)blockIdx.x * kBN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave / (kBN / kWN), wn = wave % (kBN / kWN);  // the wave's kWM x kWN block

  // tile loads: 2 operands x 256 rows x kBK/16 pieces of 16 bytes, NP per
  // lane: lane t takes piece t % kPR of rows t / kPR + kRP * j; rows past the
  // end read the last row (their products land only in outputs not stored)
  constexpr int kPR = kBK / 16, kRP = kGemmThreads / kPR, kNP = 2 * kBM / kRP;
  const int prow = tid / kPR, pq = tid % kPR;
  const int lds0 = prow * kPitch8 + 16 * pq;
  v4u pre[kNP];  // native vectors: an array of uint4 structs is not kept in registers
#define CCM_GEMM_LOAD(k0)                                                               \
  _Pragma("unroll") for (int j = 0; j < kNP; ++j) {                                     \
    const int opnd = j / (kBM / kRP);                                                   \
    const int64_t r = (opnd ? n0 : m0) + prow + kRP * (j % (kBM / kRP));                \
    const int64_t lim = opnd ? N : M;                                                   \
    pre[j] = *reinterpret_cast<const v4u *>((opnd ? Bt : A) + (r < lim ? r : lim - 1) * ldk + \
                                              16 * pq + (k0));                          \
  }
#define CCM_GEMM_STORE(b)                                                               \
  _Pragma("unroll") for (int j = 0; j < kNP; ++j) {                                     \
    const int opnd = j / (kBM / kRP);                                                   \
    *reinterpret_cast<v4u *>(gemm_lds + (b) * (kBM + kBN) * kPitch8 + opnd * kBM * kPitch8 + \
                               lds0 + kRP * (j % (kBM / kRP)) * kPitch8) = pre[j];      \
  }

  v16i acc[kFM][kFN];
#pragma unroll
  for (int a = 0; a < kFM; ++a)
#pragma unroll
    for (int b = 0; b < kFN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0;

  const int64_t nk = ldk / kBK;
  CCM_GEMM_LOAD(0);
  CCM_GEMM_STORE(0);
  __syncthreads();
  for (int64_t kc = 0; kc < nk; ++kc) {
    const int cur = (int)(kc & 1);
    if (kc + 1 < nk) CCM_GEMM_LOAD((kc + 1) * kBK);  // in flight during the MFMAs
    const int8_t *as = tile(cur, 0), *bs = tile(cur, 1);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 32) {
      const int koff = kk + 16 * (lane >> 5);
      v4i a[kFM], b[kFN];
#pragma unroll
      for (int t = 0; t < kFM; ++t)
        a[t] = *reinterpret_cast<const v4i *>(as + (wm * kWM + t * 32 + (lane & 31)) * kPitch8 + koff);
#pragma unroll
      for (int t = 0; t < kFN; ++t)
        b[t] = *reinterpret_cast<const v4i *>(bs + (wn * kWN + t * 32 + (lane & 31)) * kPitch8 + koff);
#pragma unroll
      for (int ta = 0; ta < kFM; ++ta)
#pragma unroll
        for (int tb = 0; tb < kFN; ++tb)
          acc[ta][tb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[ta], b[tb], acc[ta][tb], 0, 0, 0);
    }
    if (kc + 1 < nk) CCM_GEMM_STORE(cur ^ 1);
    __syncthreads();  // the next buffer is written and this one is read
  }
#undef CCM_GEMM_LOAD
#undef CCM_GEMM_STORE

  // 32x32 accumulator layout: lane l, register r -> column l%32,
  // row 8*(r/4) + 4*(l/32) + r%4
  int64_t lo = INT64_MAX, hi = INT64_MIN;
#pragma unroll
  for (int ta = 0; ta < kFM; ++ta)
#pragma unroll
    for (int tb = 0; tb < kFN; ++tb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t i = m0 + wm * kWM + ta * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
        const int64_t j = n0 + wn * kWN + tb * 32 + (lane & 31);
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

uint64_t matmul_i8_bytes(int64_t M, int64_t K, int64_t N) {
  return ((uint64_t)(M + N) * (uint64_t)padded_k(K) + 255u) / 256u * 256u;
}

hipError_t launch_matmul_i8(const uint32_t *aw, int abits, int asgn, const uint32_t *bw,
                            int bbits, int bsgn, int64_t M, int64_t K, int64_t N, int out32,
                            void *scratch_c, int8_t *scratch_i8, RangeSlot *slot, hipStream_t s) {
  const int64_t ldk = padded_k(K);
  if (M > 0x7fffffffll || (N + 63) / 64 > 0x7fffffffll || ldk / 128 + 1 > 65535 ||
      (N + kBN - 1) / kBN > 0x7fffffffll || (M + kBM - 1) / kBM > 65535)
    return hipErrorInvalidValue;
  int8_t *ai8 = scratch_i8, *bti8 = scratch_i8 + M * ldk;
  const uint64_t acap = cap_words32((uint64_t)M * (uint64_t)K, abits);
  const uint64_t bcap = cap_words32((uint64_t)K * (uint64_t)N, bbits);
  const dim3 cgrid((unsigned)((N + 63) / 64), (unsigned)((ldk + 127) / 128));
  switch (abits) {
#define CCM_DEC_A(b)                                                                              \
  case b:                                                                                         \
    k_decode_rows_i8<b><<<(unsigned)M, 256, 0, s>>>(aw, acap, asgn, K, ldk, ai8);                 \
    break;
    CCM_DEC_A(1) CCM_DEC_A(2) CCM_DEC_A(3) CCM_DEC_A(4) CCM_DEC_A(5) CCM_DEC_A(6) CCM_DEC_A(7)
    CCM_DEC_A(8)
#undef CCM_DEC_A
    default: return hipErrorInvalidValue;
  }
  switch (bbits) {
#define CCM_DEC_B(b)                                                                            \
  case b:                                                                                       \
    k_decode_cols_i8<b><<<cgrid, 256, 0, s>>>(bw, bcap, bsgn, K, N, ldk, bti8);                 \
    break;
    CCM_DEC_B(1) CCM_DEC_B(2) CCM_DEC_B(3) CCM_DEC_B(4) CCM_DEC_B(5) CCM_DEC_B(6) CCM_DEC_B(7)
    CCM_DEC_B(8)
#undef CCM_DEC_B
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((N + kBN - 1) / kBN), (unsigned)((M + kBM - 1) / kBM));
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_gemm_i8<int32_t>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGemmLds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_gemm_i8<int64_t>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGemmLds);
    attr = true;
  }
  if (out32)
    k_gemm_i8<int32_t><<<grid, kGemmThreads, kGemmLds, s>>>(ai8, bti8, M, N, ldk,
                                                             (int32_t *)scratch_c, slot);
  else
    k_gemm_i8<int64_t><<<grid, kGemmThreads, kGemmLds, s>>>(ai8, bti8, M, N, ldk,
                                                             (int64_t *)scratch_c, slot);
  return hipGetLastError();
}

hipError_t launch_matmul(const uint32_t *aw, int abits, int asgn, const uint32_t *bw,
                         int bbits, int bsgn, int64_t M, int64_t K, int64_t N, int use_i8,
                         int out32, void *scratch, RangeSlot *slot, hipStream_t s) {
  if (use_i8) {
    // scratch = [dense C, rounded up to 256 bytes][A as int8][B^T as int8]
    const uint64_t cbytes = ((out32 ? 4u : 8u) * (uint64_t)M * (uint64_t)N + 255u) / 256u * 256u;
    return launch_matmul_i8(aw, abits, asgn, bw, bbits, bsgn, M, K, N, out32, scratch,
                            (int8_t *)scratch + cbytes, slot, s);
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
