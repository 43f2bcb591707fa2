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
//     it decodes one.  No block
//     barrier until the end: each wave reads only what it copied.
//   * A lane reads its group's b words (plus one) from LDS; a row whose start
//     is not word-aligned (cols not a multiple of 32) shifts every group of
//     the row by the same bit offset, undone with one funnel shift per word.
//     The 32 fields decode at fixed offsets (width b is a template
//     parameter) and each adds field * x[r] to its column's sum.
//   * End: the waves' sums are added through LDS and each column's total
//     goes to y, atomically when the rows are split over several blocks (y
//     zeroed first; at most 32 splits, since same-address atomics are slow).
//     Columns past the last (a ragged last group) are decoded but never
//     stored.
#pragma once

#include <hip/hip_runtime.h>

#include "ccm_internal.hpp"
#include "group_codec.hpp"

namespace ccm {
namespace mvt {

constexpr int kPanelGroups = 64;
constexpr size_t kMaxLds = 160 * 1024 - 64;

// Waves per block: 16 for narrow fields (short rows, so more waves share a
// panel's atomics), 8 otherwise (the wide decode needs more registers).
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

// Row buffers per wave (a ring: NB - 1 rows in flight while one is decoded),
// as many as fit, at most 8 (short rows) or 4.
template <int B>
constexpr int nbuf() {
  int n = B <= 8 ? 8 : 4;
  while (n > 1 && (size_t)waves<B>() * n * vec_per_lane<B>() * 64 * 16 > kMaxLds) --n;
  return n;
}

template <int B>
constexpr size_t lds_bytes() {
  const size_t stage = (size_t)waves<B>() * nbuf<B>() * vec_per_lane<B>() * 64 * 16;
  const size_t red = (size_t)waves<B>() * 64 * 4 * 8;  // 4 columns per round
  return stage > red ? stage : red;
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
                                                       int64_t *__restrict__ y, int atomic_out) {
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
  uint4 *mybuf = lds4 + (size_t)wave * NB * NL * 64;

  // Copies row r's stretch into buffer `buf`; returns its first word.  The
  // wave's earlier LDS reads complete first (and the compiler may not move
  // them past this point): the copy overwrites the words read NB - 1 rows
  // ago.
  auto stage = [&](int64_t r, int buf) -> uint64_t {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    const uint64_t s = ((uint64_t)r * (uint64_t)cols + (uint64_t)g0 * kGroup) * B;
    const uint64_t e = ((uint64_t)r * (uint64_t)cols + (uint64_t)cend) * B;
    const uint64_t ws = (s >> 5) & ~3ull;
    const uint64_t we = (e >> 5) + 2u;
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
    return ws;
  };

  int64_t acc[kGroup];
#pragma unroll
  for (int j = 0; j < kGroup; ++j) acc[j] = 0;

  const int64_t g = g0 + lane;
  const int64_t r0 = rb + wave;
  // this wave's rows: r0, r0 + kWaves, ... < re
  const int64_t nrows = r0 < re ? (re - r0 + kWaves - 1) / kWaves : 0;
  uint64_t wsr[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) wsr[q] = 0;
#pragma unroll
  for (int q = 0; q < NB - 1; ++q)
    if (q < nrows) wsr[q] = stage(r0 + (int64_t)q * kWaves, q);
  for (int64_t i = 0; i < nrows; ++i) {
    const int64_t r = r0 + i * kWaves;
    const int cur = (int)(i % NB);
    const XT xr = x[r];  // issued before the next copy, so the waits below cover it
    const int64_t ia = i + NB - 1;  // the row copied ahead now
    if (ia < nrows) wsr[(int)(ia % NB)] = stage(r0 + ia * kWaves, (int)(ia % NB));
    // copies issued after row r's: rows i+1 .. min(ia, nrows-1)
    const int64_t later = (ia < nrows ? ia : nrows - 1) - i;
    wait_rows<NL, NB>((int)later);
    uint64_t ws = 0;
#pragma unroll
    for (int q = 0; q < NB; ++q) ws = q == cur ? wsr[q] : ws;
    const uint32_t *buf = (const uint32_t *)(mybuf + (size_t)cur * NL * 64);
    const uint64_t gs = ((uint64_t)r * (uint64_t)cols + (uint64_t)g * kGroup) * B;
    const uint32_t off = (uint32_t)(gs & 31u);  // the same for every group of the row
    const uint32_t *gw = buf + ((gs >> 5) - ws);
    uint32_t wd[B + 1];
#pragma unroll
    for (int k = 0; k <= B; ++k) wd[k] = gw[k];
    uint32_t al[B];
#pragma unroll
    for (int k = 0; k < B; ++k) al[k] = __builtin_amdgcn_alignbit(wd[k + 1], wd[k], off);
    if constexpr (B <= 32) {
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
        if (atomic_out)
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
                    hipStream_t s) {
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
  // Rows split so the resident blocks cover the grid once; at most 32 splits
  // (each split adds one atomic per column), at least 8 rows per wave.
  int64_t splits = ((int64_t)occ * compute_units_t() + npanels - 1) / npanels;
  const int64_t max_splits = (rows + 8 * waves<B>() - 1) / (8 * waves<B>());
  splits = splits > 32 ? 32 : splits;
  splits = splits < 1 ? 1 : (splits > max_splits ? max_splits : splits);
  if (splits < 1) splits = 1;
  const int64_t rpb = (rows + splits - 1) / splits;
  splits = (rows + rpb - 1) / rpb;
  if (splits > 65535) return hipErrorInvalidValue;
  if (splits > 1) {
    hipError_t e = launch_fill_i64(y, (uint64_t)cols, 0, s);
    if (e != hipSuccess) return e;
  }
  dim3 grid((unsigned)npanels, (unsigned)splits);
  k_matvec_t<B, SGN, XT><<<grid, 64 * waves<B>(), lds, s>>>(w, rows, cols, rpb, x, y,
                                                             splits > 1 ? 1 : 0);
  return hipGetLastError();
}

template <int B>
hipError_t launch_width_t(const uint32_t *w, int64_t rows, int64_t cols, int sgn, const void *x,
                          int xdtype, int64_t *y, hipStream_t s) {
  if (xdtype == CCM_I64)
    return sgn ? launch_t<B, true, int64_t>(w, rows, cols, (const int64_t *)x, y, s)
               : launch_t<B, false, int64_t>(w, rows, cols, (const int64_t *)x, y, s);
  return sgn ? launch_t<B, true, int32_t>(w, rows, cols, (const int32_t *)x, y, s)
             : launch_t<B, false, int32_t>(w, rows, cols, (const int32_t *)x, y, s);
}

}  // namespace mvt
}  // namespace ccm
