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
// and zero-padded to a multiple of the K step: A as M rows, B transposed as N
// rows (B^T, the paper's other unravel order).  Decoding inside the GEMM's K
// loop would redo it for every output tile (N/256 times per A element) and
// read the packed rows one lane per row, which the memory pipeline serves one
// cache line per lane; decoded once, the tiles stream with coalesced 16-byte
// copies.  The GEMM (k_gemm_i8 below) multiplies 256x256 output tiles per
// 512-lane block, eight waves of 128x64 outputs, with v_mfma_i32_32x32x32_i8
// over two LDS buffers filled by memory-to-LDS copies, K in steps of 128.  A
// and B operand lanes use the same assignment of the 32 K values of a slice
// to (lane half, byte), so the products summed per output are exactly those
// of the dot product.  int32 accumulation is exact because the host only
// takes this path when K * max|A| * max|B| < 2^31.

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

constexpr int kBM = 256, kBN = 256, kBK = 128;  // block tile; K bytes per step (= LDS row)
constexpr int kKPad = kBK;                      // K padding of the int8 operands
constexpr int kWM = 128, kWN = 64;  // output rows and columns per wave
constexpr int kFM = kWM / 32, kFN = kWN / 32;  // 32x32 accumulator blocks per wave
constexpr int kGemmThreads = 64 * (kBM / kWM) * (kBN / kWN);
constexpr size_t kTileBytes = (size_t)(kBM + kBN) * kBK;  // A and B tiles of one K step
constexpr size_t kGemmLds = 2u * kTileBytes;              // two buffers
constexpr int kGroupM = 4;  // tile rows per group of the block order

__host__ __device__ inline int64_t padded_k(int64_t K) { return (K + kKPad - 1) / kKPad * kKPad; }

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

// out[n][k] = B[k][n] as int8 (zero at or past K), through an LDS tile of
// 128 k x 64 n per block: each lane first decodes one group (32 consecutive n
// of one row k of B, read as the group's words), then 4 lanes per n gather
// their 32 k each from the tile and write the 128 bytes of out's row n as
// 16-byte stores.
constexpr int kCtK = 128, kCtN = 64, kCtPitch = kCtN + 4;  // tile pitch in bytes

template <int B>
__global__ __launch_bounds__(256) void k_decode_cols_i8(const uint32_t *__restrict__ w,
                                                        uint64_t cap, int sgn, int64_t K,
                                                        int64_t N, int64_t ldk,
                                                        int8_t *__restrict__ out) {
  __shared__ __align__(16) uint8_t tile[kCtK * kCtPitch];
  const int64_t nb = (int64_t)blockIdx.x * kCtN, kb = (int64_t)blockIdx.y * kCtK;
  const int t = threadIdx.x;
  {
    const int kl = t >> 1, half = t & 1;
    const int64_t k = kb + kl, n0 = nb + 32 * half;
    int32_t v[32];
    if (k < K && n0 < N) {
      const uint64_t bit = ((uint64_t)k * (uint64_t)N + (uint64_t)n0) * B;
      const uint64_t w0 = bit >> 5;
      const int sh = (int)(bit & 31u);
      uint32_t ww[B + 1];
#pragma unroll
      for (int q = 0; q <= B; ++q) ww[q] = w[w0 + q < cap ? w0 + q : cap - 1];
#pragma unroll
      for (int q = 0; q < B; ++q) ww[q] = __builtin_amdgcn_alignbit(ww[q + 1], ww[q], sh);
      const int lim = N - n0 < 32 ? (int)(N - n0) : 32;
#pragma unroll
      for (int i = 0; i < 32; ++i) {
        const uint64_t u = codec::field<B>(ww, i);
        v[i] = i < lim ? (sgn ? (int32_t)sext64(u, B) : (int32_t)u) : 0;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 32; ++i) v[i] = 0;
    }
    uint32_t *row = reinterpret_cast<uint32_t *>(tile + kl * kCtPitch + 32 * half);
#pragma unroll
    for (int q = 0; q < 8; ++q) row[q] = bytes4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  }
  __syncthreads();
  const int nl = t >> 2, kq = t & 3;
  const int64_t n = nb + nl;
  if (n >= N || kb >= ldk) return;
  uint32_t o[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int k0 = 32 * kq + 4 * q;
    o[q] = (uint32_t)tile[k0 * kCtPitch + nl] | ((uint32_t)tile[(k0 + 1) * kCtPitch + nl] << 8) |
           ((uint32_t)tile[(k0 + 2) * kCtPitch + nl] << 16) |
           ((uint32_t)tile[(k0 + 3) * kCtPitch + nl] << 24);
  }
  uint4 *d = reinterpret_cast<uint4 *>(out + n * ldk + kb + 32 * kq);
  d[0] = make_uint4(o[0], o[1], o[2], o[3]);
  d[1] = make_uint4(o[4], o[5], o[6], o[7]);
}

// 16-byte chunk c of tile row r sits at chunk position c ^ swz(r) of its
// 128-byte LDS row, so the MFMA operand reads (lanes 0-31 rows r..r+31 at one
// chunk, lanes 32-63 at the next) are conflict-free whether the LDS serves 8
// lanes of 16 bytes per cycle from 32 banks (8 consecutive rows take
// distinct positions) or 16 lanes from 64 banks (rows of equal parity among
// 16 take distinct positions); the bank-conflict counter reads 0.
__device__ __forceinline__ int swz(int r) { return (r ^ (r >> 3)) & 7; }

// C = A B^T-layout int8 GEMM with exact int32 accumulation (MFMA
// v_mfma_i32_32x32x32_i8), C stored as int32 (the host takes this path only
// when every entry fits int32), and C's exact range.
//   * Block = 8 waves, 256 x 256 outputs; each wave owns 128 x 64 (4 x 2
//     MFMA blocks, 128 accumulator registers): 6 LDS reads of 16 bytes feed 8
//     MFMAs.
//   * K steps of 128: the A and B tiles (2 x 256 rows x 128 bytes) are copied
//     into LDS with memory-to-LDS loads (global_load_lds_dwordx4: each wave
//     instruction fills 8 rows, a lane's source chunk chosen so the row lands
//     swizzled), into the other of two buffers while the MFMAs consume this
//     one.  Rows past M or N copy the last row (their outputs are not stored).
//   * One barrier per step, at its end, once the lane's copies of the next
//     step have landed (its LDS reads of this step have returned by then:
//     the barrier also waits for them, as it must: the buffer just read is
//     refilled right after it).
//   * The operands of each 32-deep slice of K are read one slice ahead into
//     a second register set, one LDS read issued after each MFMA; slice 0 of
//     a step is read after the barrier that completes its buffer.
__device__ __forceinline__ void mfma_slice(const v4i (&a)[kFM], const v4i (&b)[kFN],
                                           v16i (&acc)[kFM][kFN]) {
#pragma unroll
  for (int ta = 0; ta < kFM; ++ta)
#pragma unroll
    for (int tb = 0; tb < kFN; ++tb)
      acc[ta][tb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[ta], b[tb], acc[ta][tb], 0, 0, 0);
}

__global__ __launch_bounds__(kGemmThreads) void k_gemm_i8(const int8_t *__restrict__ A,
                                                          const int8_t *__restrict__ Bt, int64_t M,
                                                          int64_t N, int64_t ldk,
                                                          int32_t *__restrict__ C, RangeSlot *slot) {
  extern __shared__ __align__(16) int8_t gemm_lds[];
  // Tile of this block.  Tiles are taken in groups of kGroupM tile rows
  // (consecutive tiles walk down the group, then across), and when the tile
  // count is a multiple of 8 each XCD (blocks are dealt to the 8 XCDs in
  // turn) gets one contiguous run of that order: the 32 blocks an XCD runs at
  // once then share 4 A panels and 8 B panels, whose K slices its L2 holds.
  const int64_t gx = (N + kBN - 1) / kBN, gy = (M + kBM - 1) / kBM, ntile = gx * gy;
  int64_t tix = blockIdx.x;
  if (ntile % 8 == 0) tix = (tix % 8) * (ntile / 8) + tix / 8;
  const int64_t gsz_full = (int64_t)kGroupM * gx;
  const int64_t first_m = tix / gsz_full * kGroupM;
  const int64_t gsz = gy - first_m < kGroupM ? gy - first_m : kGroupM;
  const int64_t tm = first_m + (tix % gsz_full) % gsz, tn = (tix % gsz_full) / gsz;
  const int64_t m0 = tm * kBM, n0 = tn * kBN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / (kBN / kWN), wn = wave % (kBN / kWN);  // the wave's kWM x kWN block

  // the copy of one K step: 2 x 256 rows of 128 bytes = 64 wave instructions
  // of 8 rows, kInstPerWave per wave; instruction I: operand I / 32, rows
  // 8 (I % 32) .. + 7
  constexpr int kRowsPerInst = 64 * 16 / kBK;
  constexpr int kInstPerWave = (2 * kBM / kRowsPerInst) / (kGemmThreads / 64);
  constexpr int kChunks = kBK / 16;
  const int lrow = lane / kChunks, lpos = lane % kChunks;
  auto stage = [&](int64_t k0, int buf) {
#pragma unroll
    for (int q = 0; q < kInstPerWave; ++q) {
      const int I = wave * kInstPerWave + q;
      const int opnd = I / (kBM / kRowsPerInst);
      const int rb = kRowsPerInst * (I % (kBM / kRowsPerInst));
      const int r = rb + lrow;
      const int64_t lim = opnd ? N : M;
      int64_t gr = (opnd ? n0 : m0) + r;
      gr = gr < lim ? gr : lim - 1;
      const int c = lpos ^ swz(r);
      const int8_t *src = (opnd ? Bt : A) + gr * ldk + k0 + 16 * c;
      int8_t *dst = gemm_lds + (size_t)buf * kTileBytes + (size_t)opnd * kBM * kBK + (size_t)rb * kBK;
      __builtin_amdgcn_global_load_lds((const void *)src,
                                       (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
    }
  };
  // LDS offsets of this lane's operand rows and their swizzle
  int aoff[kFM], boff[kFN], asw[kFM], bsw[kFN];
#pragma unroll
  for (int t = 0; t < kFM; ++t) {
    const int r = wm * kWM + t * 32 + (lane & 31);
    aoff[t] = r * kBK;
    asw[t] = swz(r);
  }
#pragma unroll
  for (int t = 0; t < kFN; ++t) {
    const int r = wn * kWN + t * 32 + (lane & 31);
    boff[t] = kBM * kBK + r * kBK;
    bsw[t] = swz(r);
  }
  // lanes 0-31 take bytes 0-15 of the slice's 32 K values, lanes 32-63 bytes
  // 16-31, for both operands
  auto fetch = [&](int buf, int kk, v4i(&a)[kFM], v4i(&b)[kFN]) {
    const int8_t *base = gemm_lds + (size_t)buf * kTileBytes;
    const int c = kk / 16 + (lane >> 5);
#pragma unroll
    for (int t = 0; t < kFM; ++t)
      a[t] = *reinterpret_cast<const v4i *>(base + aoff[t] + 16 * (c ^ asw[t]));
#pragma unroll
    for (int t = 0; t < kFN; ++t)
      b[t] = *reinterpret_cast<const v4i *>(base + boff[t] + 16 * (c ^ bsw[t]));
  };

  v16i acc[kFM][kFN];
#pragma unroll
  for (int a = 0; a < kFM; ++a)
#pragma unroll
    for (int b = 0; b < kFN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0;

  const int64_t nk = ldk / kBK;
  stage(0, 0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  // two operand sets: the reads of slice s + 1 are in flight during the
  // MFMAs of slice s (within a step; slice 0 of the next step is read after
  // the barrier, once its buffer is complete)
  v4i a0[kFM], b0[kFN], a1[kFM], b1[kFN];
  fetch(0, 0, a0, b0);
  for (int64_t kc = 0; kc < nk; ++kc) {
    const int cur = (int)(kc & 1);
    if (kc + 1 < nk) stage((kc + 1) * kBK, cur ^ 1);  // in flight during the MFMAs
#pragma unroll
    for (int s = 0; s < kBK / 32; ++s) {
      if (s % 2 == 0) {
        if (s + 1 < kBK / 32) fetch(cur, 32 * (s + 1), a1, b1);
        mfma_slice(a0, b0, acc);
      } else {
        if (s + 1 < kBK / 32) fetch(cur, 32 * (s + 1), a0, b0);
        mfma_slice(a1, b1, acc);
      }
      if (s + 1 < kBK / 32) {
        // one LDS read after each of the first six MFMAs, then the last two
#pragma unroll
        for (int q = 0; q < kFM + kFN; ++q) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // an MFMA
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // an LDS read
        }
        __builtin_amdgcn_sched_group_barrier(0x008, kFM * kFN - (kFM + kFN), 0);
      }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this lane's copies of the next step
    __syncthreads();  // everyone's copies have landed and this buffer is read
    if (kc + 1 < nk) fetch(cur ^ 1, 0, a0, b0);
  }

  // 32x32 accumulator layout: lane l, register r -> column l%32,
  // row 8*(r/4) + 4*(l/32) + r%4.  Row offsets are uniform multiples of N.
  int lo = 0x7fffffff, hi = -0x7fffffff - 1;
  const int64_t rbase = m0 + wm * kWM + 4 * (lane >> 5);
  const int64_t cbase = n0 + wn * kWN + (lane & 31);
  int32_t *cp = C + rbase * N + cbase;
#pragma unroll
  for (int ta = 0; ta < kFM; ++ta)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ro = ta * 32 + 8 * (r / 4) + (r % 4);
      int32_t *rowp = cp + (int64_t)ro * N;
      const bool rok = rbase + ro < M;
#pragma unroll
      for (int tb = 0; tb < kFN; ++tb) {
        const int v = acc[ta][tb][r];
        if (rok && cbase + tb * 32 < N) {
          rowp[tb * 32] = v;
          lo = v < lo ? v : lo;
          hi = v > hi ? v : hi;
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // one row at a time: no copies of all 128 accumulators
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
  if (!out32) return hipErrorInvalidValue;  // every entry fits int32 on this path
  if (M > 0x7fffffffll || (N + 63) / 64 > 0x7fffffffll || ldk / 128 + 1 > 65535 ||
      (N + kBN - 1) / kBN > 0x7fffffffll || (M + kBM - 1) / kBM > 65535)
    return hipErrorInvalidValue;
  int8_t *ai8 = scratch_i8, *bti8 = scratch_i8 + M * ldk;
  const uint64_t acap = cap_words32((uint64_t)M * (uint64_t)K, abits);
  const uint64_t bcap = cap_words32((uint64_t)K * (uint64_t)N, bbits);
  const dim3 cgrid((unsigned)((N + kCtN - 1) / kCtN), (unsigned)(ldk / kCtK));
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
  const int64_t ntile = ((N + kBN - 1) / kBN) * ((M + kBM - 1) / kBM);
  if (ntile > 0x7fffffffll) return hipErrorInvalidValue;
  const dim3 grid((unsigned)ntile);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_gemm_i8),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGemmLds);
    attr = true;
  }
  k_gemm_i8<<<grid, kGemmThreads, kGemmLds, s>>>(ai8, bti8, M, N, ldk, (int32_t *)scratch_c,
                                                 slot);
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
