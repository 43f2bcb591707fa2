// y = A^T x over a row-major packed stream (x: one value per row, y: one per
// column).  The same kernel serves y = A x for a matrix unravelled by column,
// whose stream is that of A^T unravelled by row.
//
//   * Block = 16 waves (b <= 8) or 8; a block owns a panel of 64 groups
//     (2048 columns) and a range of rows; lane l owns group 64 p + l, i.e.
//     columns 2048 p + 32 l .. + 31, and keeps their 32 sums in registers.
//   * Wave w walks rows r0 + w, r0 + w + W, ...  For each row it copies the
//     panel's stretch of the row (64 groups = 64 b words, contiguous) into its
//     own LDS ring of up to 8 (b <= 8) or 4 row buffers with 16-byte
//     memory-to-LDS loads (global_load_lds_dwordx4, a fixed count per lane so
//     the wait counts are constants): up to 7 or 3 rows are in flight while
//     it decodes one.  x of the wave's rows comes the same way, 64 rows at a
//     time, a chunk ahead.  No block barrier until the end: each wave reads
//     only what it copied.
//   * A lane reads its group's b words (plus one) from LDS; a row whose start
//     is not word-aligned (cols not a multiple of 32) shifts every group of
//     the row by the same bit offset, undone with one funnel shift per word.
//     The 32 fields decode at fixed offsets (width b is a template
//     parameter) and each adds field * x[r] to its column's sum.
//   * A wave whose rows all have x in [-2^15, 2^15) (checked up front) adds
//     field * x[r] with one v_mad_i32_i24 into 32-bit partial sums, which
//     cannot leave int32 within RUN rows (b <= 14).  8-wave blocks fold them
//     into the 64-bit sums every RUN rows; 16-wave blocks (128 registers a
//     lane) take this path only for waves of at most RUN rows, so no 64-bit
//     sums are live during their walk.  Other waves use 64-bit products.
//   * End: the waves' sums are added through LDS and each column's total
//     goes to y.  When the rows are split over several blocks (at most 32),
//     each split stores its column totals in caller scratch and a second
//     kernel adds them; without scratch the splits add into a zeroed y with
//     atomics (same-address atomics from 32 splits cost about 18 us on a
//     16384-column matrix, the second pass about 2).
//     Columns past the last (a ragged last group) are decoded but never
//     stored.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "ccm_internal.hpp"
#include "group_codec.hpp"

namespace ccm {
namespace mvt {

constexpr int kPanelGroups = 64;
constexpr size_t kMaxLds = 160 * 1024 - 64;

// Waves per block: 16 for narrow fields (short rows, so more waves share a
// panel's end-of-block reduction), 8 otherwise (the wide decode needs more
// registers).
template <int B>
constexpr int waves() {
  return B <= 8 ? 16 : 8;
}

// 16-byte vectors a lane copies per row: a stretch holds at most 64 b + 6
// words (64 groups, the alignment of its first word down to 16 bytes and a
// guard word), i.e. 16 b + 2 vectors.
template <int B>
constexpr int vec_per_lane() {
  return (16 * B + 2 + 63) / 64;
}

// x values per wave: two chunks of 64 rows, low and high words (2 KB).
template <int B>
constexpr size_t xlds_bytes() {
  return (size_t)waves<B>() * 2 * 2 * 64 * 4;
}

// Row buffers per wave (a ring: NB - 1 rows in flight while one is decoded),
// as many as fit, at most 8 (short rows) or 4.
template <int B>
constexpr int nbuf() {
  int n = B <= 8 ? 8 : 4;
  while (n > 1 && xlds_bytes<B>() + (size_t)waves<B>() * n * vec_per_lane<B>() * 64 * 16 > kMaxLds)
    --n;
  return n;
}

template <int B>
constexpr size_t lds_bytes() {
  const size_t stage = xlds_bytes<B>() + (size_t)waves<B>() * nbuf<B>() * vec_per_lane<B>() * 64 * 16;
  const size_t red = (size_t)waves<B>() * 64 * 4 * 8;  // 4 columns per round
  return stage > red ? stage : red;
}

// Rows of int16-range x whose products fit one int32 partial sum: |a| is at
// most 2^b - 1 (unsigned) or 2^(b-1) (signed) and |x| at most 2^15, so RUN
// rows add at most RUN * |a|max * 2^15 <= 2^31 - 1 in magnitude.  0: no
// 32-bit path (fewer than 4 rows per fold).
template <int B, bool SGN>
constexpr int run_rows() {
  if (B > 16) return 0;
  const long long amax = SGN ? (1ll << (B - 1)) : (1ll << B) - 1;
  const long long run = 2147483647ll / (amax << 15);
  return run >= 4 ? (int)(run < 65536 ? run : 65536) : 0;
}

// d = a * b + c on the low 24 bits of a and b (v_mad_i32_i24), one
// instruction per element (the compiler would otherwise split such chains).
__device__ __forceinline__ int32_t mad24_t(int32_t a, int32_t b, int32_t c) {
  int32_t d;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

template <int N>
__device__ __forceinline__ void wait_vm() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Waits until at most m * NL copies are outstanding (m < NB, wave-uniform;
// the count is an immediate, so one case per m).
template <int NL, int NB, int M = NB - 1>
__device__ __forceinline__ void wait_rows(int m) {
  if constexpr (M == 0) {
    wait_vm<0>();
  } else {
    static_assert(M * NL <= 63, "vmcnt holds at most 63");
    if (m >= M)
      wait_vm<M * NL>();
    else
      wait_rows<NL, NB, M - 1>(m);
  }
}

template <int B, bool SGN, typename XT>
__global__ __launch_bounds__(64 * waves<B>()) void k_matvec_t(const uint32_t *__restrict__ w,
                                                       int64_t rows, int64_t cols,
                                                       int64_t rows_per_block,
                                                       const XT *__restrict__ x,
                                                       int64_t *__restrict__ y,
                                                       int64_t *__restrict__ part,
                                                       int atomic_out) {
  constexpr int NL = vec_per_lane<B>();
  constexpr int NB = nbuf<B>();
  constexpr int kWaves = waves<B>();
  extern __shared__ uint4 lds4[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ngr = (cols + kGroup - 1) / kGroup;
  const int64_t g0 = (int64_t)blockIdx.x * kPanelGroups;
  const int64_t gend = g0 + kPanelGroups < ngr ? g0 + kPanelGroups : ngr;
  const int64_t cend = gend * kGroup < cols ? gend * kGroup : cols;
  const int64_t rb = (int64_t)blockIdx.y * rows_per_block;
  const int64_t re = rb + rows_per_block < rows ? rb + rows_per_block : rows;
  uint32_t *xl = reinterpret_cast<uint32_t *>(lds4) + (size_t)wave * 256;  // [chunk slot][lo, hi][64]
  uint4 *mybuf = lds4 + xlds_bytes<B>() / 16 + (size_t)wave * NB * NL * 64;

  // Row r's stretch starts at stream bit (r cols + 32 g0) b and spans `span`
  // bits; the rows of a wave are kWaves apart, `dbit` bits.
  const uint64_t span = ((uint64_t)cend - (uint64_t)g0 * kGroup) * B;
  const uint64_t dbit = (uint64_t)kWaves * (uint64_t)cols * B;
  // Copies the stretch starting at stream bit `bit` (from the 16-byte
  // boundary at or below it) into buffer `buf`.  The wave's earlier LDS reads
  // complete first (and the compiler may not move them past this point): the
  // copy overwrites the words read NB - 1 rows ago.
  auto stage = [&](uint64_t bit, int buf) {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    const uint64_t ws = (bit >> 5) & ~3ull;
    const uint64_t we = ((bit + span) >> 5) + 2u;
    const int nvec = (int)((we - ws + 3u) >> 2);
    const uint4 *src = (const uint4 *)(w + ws);
    uint4 *dst = mybuf + (size_t)buf * NL * 64;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      int v = i * 64 + lane;
      v = v < nvec ? v : nvec - 1;  // a fixed count per lane; extra copies repeat the last
      __builtin_amdgcn_global_load_lds((const void *)(src + v),
                                       (__attribute__((address_space(3))) void *)(dst + i * 64),
                                       16, 0, 0);
    }
  };

  constexpr int RUN = run_rows<B, SGN>();
  // 16-wave blocks (b <= 8) have 128 registers a lane: their 32-bit path
  // keeps no 64-bit sums during the walk, so it takes waves with at most RUN
  // rows; 8-wave blocks fold every RUN rows.
  constexpr bool kFoldInLoop = kWaves == 8;
  int64_t acc[kGroup];
#pragma unroll
  for (int j = 0; j < kGroup; ++j) acc[j] = 0;

  const int64_t r0 = rb + wave;
  // this wave's rows: r0, r0 + kWaves, ... < re
  const int64_t nrows = r0 < re ? (re - r0 + kWaves - 1) / kWaves : 0;

  // Copies x of rows 64 c .. 64 c + 63 of this wave (clamped to its last
  // row; nrows > 0) into chunk slot c % 2, low and high words, memory to LDS
  // like the row copies: every wait that covers a later row copy covers it.
  auto stage_x = [&](int64_t c) {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // earlier reads of the slot
    int64_t i = c * 64 + lane;
    i = i < nrows ? i : nrows - 1;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(x + r0 + i * kWaves);
    uint32_t *dst = xl + (c & 1) * 128;
    __builtin_amdgcn_global_load_lds((const void *)src,
                                     (__attribute__((address_space(3))) void *)dst, 4, 0, 0);
    if constexpr (sizeof(XT) == 8)
      __builtin_amdgcn_global_load_lds((const void *)(src + 1),
                                       (__attribute__((address_space(3))) void *)(dst + 64), 4,
                                       0, 0);
  };

  // 32-bit path for this wave: every x of its rows in [-2^15, 2^15)
  bool narrow = false;
  if constexpr (RUN > 0) {
    if (kFoldInLoop || nrows <= RUN) {
      int bad = 0;
      for (int64_t i = lane; i < nrows; i += 64) {
        const int64_t xv = (int64_t)x[r0 + i * kWaves];
        bad |= ((uint64_t)xv + 32768u) >= 65536u;
      }
      narrow = !__any(bad);
    }
  }

  // The row walk; NARROW: products into 32-bit partial sums.
  auto walk = [&](auto narrow_tag) {
    constexpr bool NARROW = decltype(narrow_tag)::value;
    int32_t psum[NARROW ? kGroup : 1];
#pragma unroll
    for (int j = 0; j < (NARROW ? kGroup : 1); ++j) psum[j] = 0;
    int nrun = 0;  // rows in psum (wave-uniform)
    auto fold = [&]() {
      if constexpr (NARROW) {
#pragma unroll
        for (int j = 0; j < kGroup; ++j) {
          acc[j] += (int64_t)psum[j];
          psum[j] = 0;
        }
      }
      nrun = 0;
    };
    // x of the wave's rows, 64 at a time through LDS, the next 64 requested
    // a chunk ahead.  (A scalar load per row would be waited for at once by
    // the next copy's LDS wait, which shares its counter; a register chunk
    // would make the compiler wait for the whole queue at every row.)
    if (nrows > 0) stage_x(0);
    if (nrows > 64) stage_x(1);
    uint64_t bit = ((uint64_t)r0 * (uint64_t)cols + (uint64_t)g0 * kGroup) * B;  // row i
#pragma unroll
    for (int q = 0; q < NB - 1; ++q)
      if (q < nrows) stage(bit + (uint64_t)q * dbit, q);
    uint64_t abit = bit + (uint64_t)(NB - 1) * dbit;  // row i + NB - 1
    for (int64_t i = 0; i < nrows; ++i, bit += dbit, abit += dbit) {
      const int cur = (int)(i % NB);
      if (i > 0 && (i & 63) == 0 && i + 64 < nrows) stage_x((i >> 6) + 1);
      const int64_t ia = i + NB - 1;  // the row copied ahead now
      if (ia < nrows) stage(abit, (int)(ia % NB));
      // copies issued after row r's: rows i+1 .. min(ia, nrows-1)
      const int64_t later = (ia < nrows ? ia : nrows - 1) - i;
      wait_rows<NL, NB>((int)later);
      const uint32_t *xw = xl + ((i >> 6) & 1) * 128 + (i & 63);
      XT xr;
      if constexpr (sizeof(XT) == 8)
        xr = (XT)(((uint64_t)xw[64] << 32) | xw[0]);
      else
        xr = (XT)xw[0];
      // group g0 + lane starts 32 b lane bits after the row's first: word
      // (bit / 32) % 4 + b lane of the copy, at the row's bit offset
      const uint32_t *buf = (const uint32_t *)(mybuf + (size_t)cur * NL * 64);
      const uint32_t off = (uint32_t)bit & 31u;
      const uint32_t *gw = buf + (((uint32_t)(bit >> 5)) & 3u) + lane * B;
      uint32_t wd[B + 1];
#pragma unroll
      for (int k = 0; k <= B; ++k) wd[k] = gw[k];
      uint32_t al[B];
#pragma unroll
      for (int k = 0; k < B; ++k) al[k] = __builtin_amdgcn_alignbit(wd[k + 1], wd[k], off);
      if constexpr (NARROW) {
        const int32_t xs = (int32_t)xr;
#pragma unroll
        for (int j = 0; j < kGroup; ++j) {
          const int p = j * B, k = p >> 5, o = p & 31;
          const uint32_t src =
              o + B <= 32 ? al[k] : __builtin_amdgcn_alignbit(al[k + 1], al[k], o);
          const int sh = o + B <= 32 ? o : 0;
          const int32_t f = SGN ? __builtin_amdgcn_sbfe((int32_t)src, sh, B)
                                : (int32_t)__builtin_amdgcn_ubfe(src, sh, B);
          psum[j] = mad24_t(f, xs, psum[j]);
        }
        if constexpr (kFoldInLoop)
          if (++nrun == RUN) fold();
      } else if constexpr (B <= 32) {
        uint32_t v[kGroup];
        codec::decode32<B>(al, SGN ? 1 : 0, v);
#pragma unroll
        for (int j = 0; j < kGroup; ++j) {
          if constexpr (SGN || B < 32)
            acc[j] += (int64_t)opaque_i32((int32_t)v[j]) * (int64_t)xr;
          else
            acc[j] += (int64_t)((uint64_t)v[j] * (uint64_t)(int64_t)xr);
        }
      } else {
        int64_t v[kGroup];
        codec::decode<B>(al, SGN ? 1 : 0, v);
#pragma unroll
        for (int j = 0; j < kGroup; ++j)
          acc[j] += (int64_t)((uint64_t)v[j] * (uint64_t)(int64_t)xr);
      }
    }
    fold();
  };
  if constexpr (RUN > 0) {
    if (narrow)
      walk(std::true_type{});
    else
      walk(std::false_type{});
  } else {
    walk(std::false_type{});
  }

  // sum the waves' column sums, 4 columns of every lane per round
  __syncthreads();
  int64_t *red = (int64_t *)lds4;
  const int t = threadIdx.x;
  const int tl = t & 63, tj = (t >> 6) & 3;
  const int64_t gt = g0 + tl;
#pragma unroll
  for (int j0 = 0; j0 < kGroup; j0 += 4) {
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) red[((wave * 4) + jj) * 64 + lane] = acc[j0 + jj];
    __syncthreads();
    if (t < 256) {  // 64 lanes x 4 columns
      uint64_t sum = 0;
#pragma unroll
      for (int v = 0; v < kWaves; ++v) sum += (uint64_t)red[((v * 4) + tj) * 64 + tl];
      const int64_t col = gt * kGroup + j0 + tj;
      if (gt < gend && col < cols) {
        if (part)
          part[(uint64_t)blockIdx.y * (uint64_t)cols + (uint64_t)col] = (int64_t)sum;
        else if (atomic_out)
          atomicAdd((unsigned long long *)&y[col], (unsigned long long)sum);
        else
          y[col] = (int64_t)sum;
      }
    }
    __syncthreads();
  }
}

int compute_units_t();

template <int B, bool SGN, typename XT>
hipError_t launch_t(const uint32_t *w, int64_t rows, int64_t cols, const XT *x, int64_t *y,
                    int64_t *part, uint64_t part_words, hipStream_t s) {
  const int64_t ngr = (cols + kGroup - 1) / kGroup;
  const int64_t npanels = (ngr + kPanelGroups - 1) / kPanelGroups;
  if (npanels > 0x7fffffffll) return hipErrorInvalidValue;
  constexpr size_t lds = lds_bytes<B>();
  static int occ = 0;
  if (occ == 0) {
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void *)k_matvec_t<B, SGN, XT>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k_matvec_t<B, SGN, XT>, 64 * waves<B>(),
                                                     lds) !=
            hipSuccess ||
        o < 1)
      o = 1;
    occ = o;
  }
  // Rows split so the resident blocks cover the grid once; at most
  // kMaxSplitsT splits (each adds one partial sum per column), at least 8
  // rows per wave.
  int64_t splits = ((int64_t)occ * compute_units_t() + npanels - 1) / npanels;
  const int64_t max_splits = (rows + 8 * waves<B>() - 1) / (8 * waves<B>());
  splits = splits > kMaxSplitsT ? kMaxSplitsT : splits;
  splits = splits < 1 ? 1 : (splits > max_splits ? max_splits : splits);
  if (splits < 1) splits = 1;
  const int64_t rpb = (rows + splits - 1) / splits;
  splits = (rows + rpb - 1) / rpb;
  if (splits > 65535) return hipErrorInvalidValue;
  // Several splits: partial sums through part when it holds them all (plain
  // stores, then one summing pass), else atomics into a zeroed y (same-address
  // atomics from every split cost more than the second pass).
  const bool staged = splits > 1 && part && (uint64_t)splits * (uint64_t)cols <= part_words;
  if (splits > 1 && !staged) {
    hipError_t e = launch_fill_i64(y, (uint64_t)cols, 0, s);
    if (e != hipSuccess) return e;
  }
  dim3 grid((unsigned)npanels, (unsigned)splits);
  k_matvec_t<B, SGN, XT><<<grid, 64 * waves<B>(), lds, s>>>(
      w, rows, cols, rpb, x, y, staged ? part : nullptr, splits > 1 ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !staged) return e;
  return launch_sum_splits(part, splits, cols, y, s);
}

template <int B>
hipError_t launch_width_t(const uint32_t *w, int64_t rows, int64_t cols, int sgn, const void *x,
                          int xdtype, int64_t *y, int64_t *part, uint64_t part_words,
                          hipStream_t s) {
  if (xdtype == CCM_I64)
    return sgn ? launch_t<B, true, int64_t>(w, rows, cols, (const int64_t *)x, y, part,
                                            part_words, s)
               : launch_t<B, false, int64_t>(w, rows, cols, (const int64_t *)x, y, part,
                                             part_words, s);
  return sgn ? launch_t<B, true, int32_t>(w, rows, cols, (const int32_t *)x, y, part, part_words,
                                          s)
             : launch_t<B, false, int32_t>(w, rows, cols, (const int32_t *)x, y, part,
                                           part_words, s);
}

}  // namespace mvt
}  // namespace ccm
