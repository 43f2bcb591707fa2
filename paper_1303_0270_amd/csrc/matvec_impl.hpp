// y = A x on an SM-packed matrix, one kernel instantiation per field width.
//
// Work layout (gfx950, 64-lane waves, 256-lane blocks):
//   * A block owns a column panel of x, staged once into LDS (zero-padded to
//     whole groups, with a 4-dword skew per group so 16-byte LDS reads of
//     consecutive groups hit distinct banks), and loops over row blocks.
//   * Each wave owns R rows at a time.  Lane l walks groups l, l+64, ... of
//     those rows: for every group it reads 32 x values from LDS once and
//     reuses them for all R rows (x traffic per element falls as 1/R).
//   * A row's group j starts at stream bit (r*cols + c0 + 32j)*b.  The word
//     offset differs per row but the bit shift s = (r*cols + c0)*b mod 32 is
//     the same for every group of the row (wave-uniform), so one funnel shift
//     (v_alignbit_b32) per word re-aligns the group and every field is then
//     extracted at a compile-time offset with one v_bfe (two when it
//     straddles a word).
//   * Products accumulate exactly in int64 (mod 2^64).  When the block finds
//     every x of its panel in int16 range and b <= 10, 32 products of a group
//     are summed in int32 with 24-bit multiply-adds first: |sum| < 32 * 2^10
//     * 2^15 = 2^30, so the int32 partial is exact.
//   * Row results are reduced across the wave with shuffles; with several
//     column panels the partial row sums are combined with int64 atomics.
#pragma once

#include "ccm_internal.hpp"

namespace ccm {
namespace mv {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <typename XT>
struct XLayout;
template <>
struct XLayout<int32_t> {
  static constexpr int kPitch = kGroup + 4;  // int32 elements per staged group
  static constexpr int kPanel = 8192;        // columns per block
};
template <>
struct XLayout<int64_t> {
  static constexpr int kPitch = kGroup + 2;  // int64 elements (68 dwords)
  static constexpr int kPanel = 4096;
};

constexpr int rows_per_wave(int b) { return b <= 4 ? 16 : b <= 8 ? 8 : b <= 16 ? 4 : b <= 32 ? 2 : 1; }

// Field i (compile-time after unrolling) of a re-aligned group of b-bit
// fields held in w[0..b].  b <= 32: the value as int64.
template <int B, bool SGN>
__device__ __forceinline__ int64_t group_field(const uint32_t *w, int i) {
  const int p = i * B;
  const int k = p >> 5;
  const int off = p & 31;
  if constexpr (B < 32) {
    uint32_t src;
    int o2;
    if (off + B <= 32) {
      src = w[k];
      o2 = off;
    } else {
      src = __builtin_amdgcn_alignbit(w[k + 1], w[k], off);
      o2 = 0;
    }
    if constexpr (SGN)
      return (int64_t)opaque_i32(__builtin_amdgcn_sbfe((int32_t)src, o2, B));
    else
      return (int64_t)__builtin_amdgcn_ubfe(src, o2, B);
  } else if constexpr (B == 32) {
    const uint32_t src = w[k];
    if constexpr (SGN)
      return (int64_t)(int32_t)src;
    else
      return (int64_t)src;
  } else {
    const uint32_t lo = off ? __builtin_amdgcn_alignbit(w[k + 1], w[k], off) : w[k];
    uint32_t hi;
    if (off + B > 64)
      hi = __builtin_amdgcn_alignbit(w[k + 2], w[k + 1], off);
    else
      hi = w[k + 1] >> off;
    int64_t h;
    if constexpr (B == 64)
      h = (int64_t)(int32_t)hi;
    else if constexpr (SGN)
      h = (int64_t)opaque_i32(__builtin_amdgcn_sbfe((int32_t)hi, 0, B - 32));
    else
      h = (int64_t)__builtin_amdgcn_ubfe(hi, 0, B - 32);
    return (int64_t)(((uint64_t)h << 32) | (uint64_t)lo);
  }
}

// 24-bit signed field for the int32 fast path (b <= 10).
template <int B, bool SGN>
__device__ __forceinline__ int32_t group_field24(const uint32_t *w, int i) {
  return (int32_t)group_field<B, SGN>(w, i);
}

// a * x modulo 2^64.  With b <= 32 and int32 x the product is exact in int64
// (|a x| < 2^63), which lets the compiler use one v_mad_i64_i32 per element.
template <int B, typename XT>
__device__ __forceinline__ uint64_t mul_mod64(int64_t a, XT x) {
  if constexpr (sizeof(XT) == 4 && B <= 32)
    return (uint64_t)(a * (int64_t)x);
  else
    return (uint64_t)a * (uint64_t)(int64_t)x;
}

template <int B, bool SGN, typename XT>
__global__ __launch_bounds__(kThreads, 2) void k_matvec(const uint32_t *__restrict__ A,
                                                        int64_t rows, int64_t cols,
                                                        const XT *__restrict__ x,
                                                        int64_t *__restrict__ y,
                                                        int atomic_out) {
  constexpr int R = rows_per_wave(B);
  constexpr int P = XLayout<XT>::kPitch;
  constexpr int NW = B + 1;  // words fetched per group (one extra for the funnel shift)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  XT *xs = reinterpret_cast<XT *>(smem_raw);

  const int64_t c0 = (int64_t)blockIdx.y * XLayout<XT>::kPanel;
  const int64_t pc = cols - c0 < XLayout<XT>::kPanel ? cols - c0 : XLayout<XT>::kPanel;
  const int ng = (int)((pc + kGroup - 1) / kGroup);

  // stage the x panel, zero-padded to whole groups
  int small = 1;
  for (int q = threadIdx.x; q < ng * kGroup; q += kThreads) {
    const XT v = q < pc ? x[c0 + q] : XT(0);
    xs[(q >> 5) * P + (q & 31)] = v;
    small &= (v >= -32768 && v <= 32767);
  }
  const bool fast = (B <= 10) && (sizeof(XT) == 4) && __syncthreads_and(small);
  if (!(B <= 10 && sizeof(XT) == 4)) __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nrb = (rows + kWaves * R - 1) / (kWaves * R);

  for (int64_t rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
    const int64_t r0 = rb * (kWaves * R) + (int64_t)wave * R;
    const int nv = rows - r0 >= R ? R : (rows - r0 > 0 ? (int)(rows - r0) : 0);
    if (nv == 0) continue;  // wave-uniform

    const uint32_t *rowp[R];
    int shift[R];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int64_t r = r0 + (rr < nv ? rr : 0);
      const uint64_t bit = ((uint64_t)r * (uint64_t)cols + (uint64_t)c0) * (uint64_t)B;
      rowp[rr] = A + (bit >> 5);
      shift[rr] = (int)(bit & 31u);
    }
    uint64_t acc[R];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) acc[rr] = 0;

    for (int j = lane; j < ng; j += 64) {
      XT xv[kGroup];
      const XT *xg = xs + j * P;
#pragma unroll
      for (int i = 0; i < kGroup; ++i) xv[i] = xg[i];

      uint32_t w[R][NW];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        if (rr < nv) {
          const uint32_t *gp = rowp[rr] + (uint64_t)j * B;
#pragma unroll
          for (int k = 0; k < NW; ++k) w[rr][k] = gp[k];
        }
      }
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        if (rr < nv) {
          const int s = shift[rr];
          if (s != 0) {
#pragma unroll
            for (int k = 0; k < B; ++k) w[rr][k] = __builtin_amdgcn_alignbit(w[rr][k + 1], w[rr][k], s);
          }
          if constexpr (B <= 10 && sizeof(XT) == 4) {
            if (fast) {
              int32_t part = 0;
#pragma unroll
              for (int i = 0; i < kGroup; ++i)
                part = __mul24(group_field24<B, SGN>(w[rr], i), (int32_t)xv[i]) + part;
              acc[rr] += (uint64_t)(int64_t)part;
              continue;
            }
          }
          uint64_t a64 = 0;
#pragma unroll
          for (int i = 0; i < kGroup; ++i)
            a64 += mul_mod64<B, XT>(group_field<B, SGN>(w[rr], i), xv[i]);
          acc[rr] += a64;
        }
      }
    }

#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      if (rr < nv) {
        const int64_t v = wave_sum((int64_t)acc[rr]);
        if (lane == 0) {
          if (atomic_out)
            atomicAdd((unsigned long long *)&y[r0 + rr], (unsigned long long)v);
          else
            y[r0 + rr] = v;
        }
      }
    }
  }
}

template <int B, bool SGN, typename XT>
hipError_t launch_one(const uint32_t *w, int64_t rows, int64_t cols, const XT *x, int64_t *y,
                      hipStream_t s) {
  constexpr int R = rows_per_wave(B);
  const int64_t npanels = (cols + XLayout<XT>::kPanel - 1) / XLayout<XT>::kPanel;
  const int64_t nrb = (rows + kWaves * R - 1) / (kWaves * R);
  int64_t gx = nrb < 1024 ? nrb : 1024;
  if (npanels > 1) {
    const int64_t cap = 2048 / npanels > 1 ? 2048 / npanels : 1;
    gx = gx < cap ? gx : cap;
    hipError_t e = launch_fill_i64(y, (uint64_t)rows, 0, s);
    if (e != hipSuccess) return e;
  }
  const int64_t pcols = cols < XLayout<XT>::kPanel ? cols : XLayout<XT>::kPanel;
  const size_t lds = (size_t)((pcols + kGroup - 1) / kGroup) * XLayout<XT>::kPitch * sizeof(XT);
  dim3 grid((unsigned)gx, (unsigned)npanels);
  k_matvec<B, SGN, XT><<<grid, kThreads, lds, s>>>(w, rows, cols, x, y, npanels > 1 ? 1 : 0);
  return hipGetLastError();
}

template <int B>
hipError_t launch_width(const uint32_t *w, int64_t rows, int64_t cols, int sgn, const void *x,
                        int xdtype, int64_t *y, hipStream_t s) {
  if (xdtype == CCM_I32) {
    return sgn ? launch_one<B, true, int32_t>(w, rows, cols, (const int32_t *)x, y, s)
               : launch_one<B, false, int32_t>(w, rows, cols, (const int32_t *)x, y, s);
  }
  return sgn ? launch_one<B, true, int64_t>(w, rows, cols, (const int64_t *)x, y, s)
             : launch_one<B, false, int64_t>(w, rows, cols, (const int64_t *)x, y, s);
}

using LaunchFn = hipError_t (*)(const uint32_t *, int64_t, int64_t, int, const void *, int,
                                int64_t *, hipStream_t);

}  // namespace mv
}  // namespace ccm
