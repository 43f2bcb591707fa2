// y = A x on an SM-packed matrix, one kernel instantiation per field width.
//
// Work layout (gfx950, 64-lane waves, 256-lane blocks):
//   * A block owns a column panel of x, staged once into LDS (zero-padded to
//     whole groups, with a 4-dword skew per group so 16-byte LDS reads of
//     consecutive groups hit distinct banks), and one block of 4*R rows.
//   * Each wave owns R rows.  Lane l walks groups l, l+64, ... of those rows:
//     for every group it reads its 32 x values from LDS once and reuses them
//     for all R rows.  The next group's words are fetched before the current
//     group is decoded.
//   * A row's group j starts at stream bit (r*cols + c0 + 32j)*b.  The word
//     offset differs per row but the bit shift s = (r*cols + c0)*b mod 32 is
//     the same for every group of the row (wave-uniform), so one funnel shift
//     (v_alignbit_b32) per word re-aligns the group and every field is then
//     extracted at a compile-time offset with one v_bfe (two instructions when
//     it straddles a word).
//   * Exact arithmetic.  When the block finds its whole x panel in int16
//     range, products are summed in int32 over runs short enough that the
//     partial sum cannot overflow (fixed per width at compile time: max|a| *
//     2^15 * run < 2^31) with 24-bit multiply-adds, then widened to int64.
//     Otherwise products are formed in 64 bits, accumulated in four
//     independent chains, modulo 2^64.
//   * b = 1 with int16-range x uses nibble dot products: x' = x + 2^15 is
//     split into four 4-bit digits, arranged per group so that
//     v_dot8_u32_u4 multiplies eight 1-bit fields (spread to nibbles with a
//     shift and a mask) by eight digits at once; the row result is
//     sum_d 16^d acc_d - 2^15 * popcount, negated for signed fields.
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

// Digit words of the b = 1 path: 16 per group (+4 skew).
constexpr int kDigitPitch = 20;

constexpr int rows_per_wave(int b) { return b <= 10 ? 4 : b <= 16 ? 2 : 1; }

// Elements per exact int32 partial sum on the int16-x path (0: use int64).
constexpr int run_len(int b, bool sgn) {
  if (b > 16) return 0;
  const long long maxa = sgn ? (1ll << (b - 1)) : ((1ll << b) - 1);
  const long long t = ((1ll << 31) - 1) / (maxa * 32768ll);
  return t >= 32 ? 32 : (t >= 16 ? 16 : (t >= 8 ? 8 : (t >= 4 ? 4 : (t >= 2 ? 2 : (t >= 1 ? 1 : 0)))));
}

// Field i (compile-time after unrolling) of a re-aligned group held in w[].
// OPQ hides signed extracts from the optimizer; only the 64-bit product
// chains need it (see opaque_i32).
template <int B, bool SGN, bool OPQ = true>
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
    if constexpr (SGN) {
      const int32_t v = __builtin_amdgcn_sbfe((int32_t)src, o2, B);
      return (int64_t)(OPQ ? opaque_i32(v) : v);
    } else {
      return (int64_t)__builtin_amdgcn_ubfe(src, o2, B);
    }
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

// a * x modulo 2^64.  With b <= 32 and int32 x the product is exact in int64
// (|a x| < 2^63), so the compiler can use one v_mad_i64_i32 per element.
template <int B, typename XT>
__device__ __forceinline__ uint64_t mul_mod64(int64_t a, XT x) {
  if constexpr (sizeof(XT) == 4 && B <= 32)
    return (uint64_t)(a * (int64_t)x);
  else
    return (uint64_t)a * (uint64_t)(int64_t)x;
}

// d = a * b + c on the low 24 bits of a and b (v_mad_i32_i24).  Written as one
// instruction: left to itself the compiler re-associates such chains into a
// 24-bit multiply plus a three-input add per element pair (1.5 instructions
// per element instead of 1).
__device__ __forceinline__ int32_t mad24(int32_t a, int32_t b, int32_t c) {
  int32_t d;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

// Dot product of one group with int16-range x (exact; int32 runs).
template <int B, bool SGN>
__device__ __forceinline__ uint64_t group_dot_small(const uint32_t *w, const int32_t *xv) {
  constexpr int T = run_len(B, SGN);
  uint64_t acc = 0;
#pragma unroll
  for (int r0 = 0; r0 < kGroup; r0 += T) {
    int32_t part = 0;
#pragma unroll
    for (int i = r0; i < r0 + T; ++i)
      part = mad24((int32_t)group_field<B, SGN, false>(w, i), xv[i], part);
    acc += (uint64_t)(int64_t)part;
  }
  return acc;
}

// Dot product of one group, general x (64-bit products, four chains).
// Scheduling barriers every 8 elements bound the live ranges (the 64-bit
// products otherwise get hoisted together and cost occupancy).
template <int B, bool SGN, typename XT>
__device__ __forceinline__ uint64_t group_dot_wide(const uint32_t *w, const XT *xv) {
  uint64_t c[4] = {0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < kGroup; ++i) {
    c[i & 3] += mul_mod64<B, XT>(group_field<B, SGN>(w, i), xv[i]);
    if ((i & 7) == 7) __builtin_amdgcn_sched_barrier(0);
  }
  return (c[0] + c[1]) + (c[2] + c[3]);
}

// Row-block loop of the general kernel for one arithmetic mode (0: 64-bit
// products; 1: int16-range x, exact int32 runs; 2: b = 1 digit dot
// products).  Instantiated per mode so each loop gets its own registers.
template <int B, bool SGN, typename XT, int MODE>
__device__ __forceinline__ void mv_rows(const uint32_t *__restrict__ A, int64_t rows,
                                        int64_t cols, int64_t c0, int ng, const XT *xs,
                                        const uint32_t *xd, int64_t *__restrict__ y,
                                        int atomic_out) {
  constexpr int R = rows_per_wave(B);
  constexpr int P = XLayout<XT>::kPitch;
  constexpr int NW = B + 1;  // words fetched per group (one extra for the funnel shift)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nrb = (rows + kWaves * R - 1) / (kWaves * R);
  for (int64_t rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
    const int64_t r0 = rb * (kWaves * R) + (int64_t)wave * R;
    const int nv = rows - r0 >= R ? R : (rows - r0 > 0 ? (int)(rows - r0) : 0);
    if (nv == 0) continue;  // wave-uniform; no block barrier inside this loop

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
    uint32_t dacc[R][5];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      acc[rr] = 0;
#pragma unroll
      for (int d = 0; d < 5; ++d) dacc[rr][d] = 0;
    }

    uint32_t wn[R][NW];
    auto fetch = [&](int j) {
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        if (rr < nv) {
          const uint32_t *gp = rowp[rr] + (uint64_t)j * B;
#pragma unroll
          for (int k = 0; k < NW; ++k) wn[rr][k] = gp[k];
        }
      }
    };
    if (lane < ng) fetch(lane);

    for (int j = lane; j < ng; j += 64) {
      uint32_t w[R][NW];
#pragma unroll
      for (int rr = 0; rr < R; ++rr)
#pragma unroll
        for (int k = 0; k < NW; ++k) w[rr][k] = wn[rr][k];
      if (j + 64 < ng) fetch(j + 64);

#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        if (rr < nv) {
          const int s = shift[rr];
          if (s != 0) {
#pragma unroll
            for (int k = 0; k < B; ++k)
              w[rr][k] = __builtin_amdgcn_alignbit(w[rr][k + 1], w[rr][k], s);
          }
        }
      }

      if constexpr (MODE == 2) {
        const uint4 *dg = reinterpret_cast<const uint4 *>(xd + j * kDigitPitch);
        const uint4 d0 = dg[0], d1 = dg[1], d2 = dg[2], d3 = dg[3];
        const uint32_t X[16] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w,
                                d2.x, d2.y, d2.z, d2.w, d3.x, d3.y, d3.z, d3.w};
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          if (rr < nv) {
            const uint32_t a = w[rr][0];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
              const uint32_t an = (a >> s4) & 0x11111111u;
#pragma unroll
              for (int d = 0; d < 4; ++d)
                dacc[rr][d] = __builtin_amdgcn_udot8(an, X[d * 4 + s4], dacc[rr][d], false);
            }
            dacc[rr][4] += (uint32_t)__builtin_popcount(a);
          }
        }
      } else {
        XT xv[kGroup];
        const XT *xg = xs + j * P;
#pragma unroll
        for (int i = 0; i < kGroup; ++i) xv[i] = xg[i];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          if (rr < nv) {
            if constexpr (MODE == 1)
              acc[rr] += group_dot_small<B, SGN>(w[rr], reinterpret_cast<const int32_t *>(xv));
            else
              acc[rr] += group_dot_wide<B, SGN, XT>(w[rr], xv);
          }
        }
      }
    }

#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      if (rr < nv) {
        uint64_t v = acc[rr];
        if constexpr (MODE == 2) {
          const int64_t t = (int64_t)dacc[rr][0] + ((int64_t)dacc[rr][1] << 4) +
                            ((int64_t)dacc[rr][2] << 8) + ((int64_t)dacc[rr][3] << 12) -
                            ((int64_t)dacc[rr][4] << 15);
          v = (uint64_t)(SGN ? -t : t);
        }
        const int64_t sum = wave_sum((int64_t)v);
        if (lane == 0) {
          if (atomic_out)
            atomicAdd((unsigned long long *)&y[r0 + rr], (unsigned long long)sum);
          else
            y[r0 + rr] = sum;
        }
      }
    }
  }
}

template <int B, bool SGN, typename XT>
__global__ __launch_bounds__(kThreads) void k_matvec(const uint32_t *__restrict__ A,
                                                     int64_t rows, int64_t cols,
                                                     const XT *__restrict__ x,
                                                     int64_t *__restrict__ y, int atomic_out,
                                                     int x_aligned16) {
  constexpr int P = XLayout<XT>::kPitch;
  constexpr bool kSmallPath = (B <= 16) && (sizeof(XT) == 4);
  constexpr bool kDigits = (B == 1) && (sizeof(XT) == 4);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  XT *xs = reinterpret_cast<XT *>(smem_raw);

  const int64_t c0 = (int64_t)blockIdx.y * XLayout<XT>::kPanel;
  const int64_t pc = cols - c0 < XLayout<XT>::kPanel ? cols - c0 : XLayout<XT>::kPanel;
  const int ng = (int)((pc + kGroup - 1) / kGroup);

  // stage the x panel, zero-padded to whole groups: 16-byte chunks, eight
  // independent loads in flight per lane
  int small = 1;
  {
    constexpr int PER = 16 / sizeof(XT);
    constexpr int UNR = 8;
    const int nchunk = ng * kGroup / PER;
    for (int q0 = threadIdx.x; q0 < nchunk; q0 += kThreads * UNR) {
      XT v[UNR][PER];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * kThreads;
        const int e = q * PER;
        if (q < nchunk && x_aligned16 && e + PER <= pc) {
          const uint4 t = *reinterpret_cast<const uint4 *>(x + c0 + e);
          const XT *tv = reinterpret_cast<const XT *>(&t);
#pragma unroll
          for (int k = 0; k < PER; ++k) v[u][k] = tv[k];
        } else {
#pragma unroll
          for (int k = 0; k < PER; ++k) v[u][k] = (q < nchunk && e + k < pc) ? x[c0 + e + k] : XT(0);
        }
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * kThreads;
        if (q < nchunk) {
          const int e = q * PER;
          XT *dst = xs + (e >> 5) * P + (e & 31);
#pragma unroll
          for (int k = 0; k < PER; ++k) {
            dst[k] = v[u][k];
            small &= (v[u][k] >= -32768 && v[u][k] <= 32767);
          }
        }
      }
    }
  }
  bool fast = false;
  if constexpr (kSmallPath)
    fast = __syncthreads_and(small);
  else
    __syncthreads();

  uint32_t *xd = nullptr;
  if constexpr (kDigits) {
    // digit words: X[d][s] nibble q = digit d of x'_{4q+s}, x' = x + 2^15
    xd = reinterpret_cast<uint32_t *>(xs + ng * P);
    if (fast) {
      for (int j = threadIdx.x; j < ng; j += kThreads) {
        const int32_t *xg = reinterpret_cast<const int32_t *>(xs) + j * P;
        uint32_t dw[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) dw[t] = 0;
#pragma unroll
        for (int i = 0; i < kGroup; ++i) {
          const uint32_t u = (uint32_t)(xg[i] + 32768);
          const int s = i & 3, q = i >> 2;
#pragma unroll
          for (int d = 0; d < 4; ++d) dw[d * 4 + s] |= ((u >> (4 * d)) & 15u) << (4 * q);
        }
#pragma unroll
        for (int t = 0; t < 16; ++t) xd[j * kDigitPitch + t] = dw[t];
      }
      __syncthreads();
    }
  }

  if constexpr (kSmallPath) {
    if (fast) {
      if constexpr (kDigits)
        mv_rows<B, SGN, XT, 2>(A, rows, cols, c0, ng, xs, xd, y, atomic_out);
      else
        mv_rows<B, SGN, XT, 1>(A, rows, cols, c0, ng, xs, xd, y, atomic_out);
      return;
    }
  }
  mv_rows<B, SGN, XT, 0>(A, rows, cols, c0, ng, xs, xd, y, atomic_out);
}

// Blocks per CU that fit at once (from the occupancy API), cached per
// instantiation.
template <int B, bool SGN, typename XT>
int resident_blocks(size_t lds) {
  static int cached = 0;
  if (cached == 0) {
    int occ = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_matvec<B, SGN, XT>, kThreads, lds) !=
            hipSuccess ||
        occ < 1)
      occ = 1;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    cached = occ * cus;
  }
  return cached;
}

template <int B, bool SGN, typename XT>
hipError_t launch_one(const uint32_t *w, int64_t rows, int64_t cols, const XT *x, int64_t *y,
                      hipStream_t s) {
  constexpr int R = rows_per_wave(B);
  const int64_t npanels = (cols + XLayout<XT>::kPanel - 1) / XLayout<XT>::kPanel;
  const int64_t nrb = (rows + kWaves * R - 1) / (kWaves * R);
  if (nrb > 0x7fffffffll || npanels > 65535) return hipErrorInvalidValue;
  if (npanels > 1) {
    hipError_t e = launch_fill_i64(y, (uint64_t)rows, 0, s);
    if (e != hipSuccess) return e;
  }
  const int64_t pcols = cols < XLayout<XT>::kPanel ? cols : XLayout<XT>::kPanel;
  const int64_t ngp = (pcols + kGroup - 1) / kGroup;
  size_t lds = (size_t)ngp * XLayout<XT>::kPitch * sizeof(XT);
  if (B == 1 && sizeof(XT) == 4) lds += (size_t)ngp * kDigitPitch * sizeof(uint32_t);
  // persistent blocks: as many as are resident at once, split over the panels
  int64_t gx = resident_blocks<B, SGN, XT>(lds) / npanels;
  gx = gx < 1 ? 1 : (gx > nrb ? nrb : gx);
  dim3 grid((unsigned)gx, (unsigned)npanels);
  const int al = ((uintptr_t)x % 16) == 0;
  k_matvec<B, SGN, XT><<<grid, kThreads, lds, s>>>(w, rows, cols, x, y, npanels > 1 ? 1 : 0, al);
  return hipGetLastError();
}

// Aligned variant for b <= 15, int32 x on a 16-byte boundary: rows start on
// 16-byte boundaries (cols % 128 == 0, so r*cols*b/32 is a multiple of 4
// words) and every panel holds whole quads of groups.  Quad q of a row panel
// is the four groups 4q..4q+3, i.e. 4b contiguous words fetched with b
// 16-byte loads.
//   * 512- or 1024-lane blocks (AlCfg), 16384-column panels (67.6 KB of LDS:
//     two or one blocks per CU, 16 waves), so a matrix up to 16384 columns
//     wide is one panel: each row sum is stored once, with no zero-fill pass
//     and no atomics.
//   * A wave owns R rows of a row block; lane l owns quads l and l+64 of the
//     panel.  One "unit" is (row block, quad slot): R*b 16-byte loads per lane.
//   * With PF the next unit's words are requested before the current one is
//     decoded (two register sets, used alternately).  Every unit issues the
//     same loads -- addresses past the last row or quad are clamped to valid
//     ones, and past the last unit the current one is fetched again (a cache
//     hit) -- so the compiler can wait for exactly the older unit's loads
//     (the load counter is in order) instead of draining the queue.  The x
//     panel is requested first, then the first unit, so the unit's latency
//     overlaps the LDS staging.
//   * LDS keeps each quad's x values (128 int32) or digit words (64)
//     contiguous plus a 4-dword skew, so the 16-byte LDS reads of neighbouring
//     lanes fall in distinct banks.
//   * b = 1: lane g builds the digit words of group g straight from its 32 x
//     values (byte permutes and nibble masks), with no int32 copy of x.
//   * b = 2..4 with int16-range x: nibble dot products as well.  The fields
//     of eight consecutive columns are moved to the eight nibbles of a word
//     (nib_spread: two bit-selects and a masked shift for b = 2 and 3,
//     nothing for b = 4) and v_dot8 multiplies them by the matching base-16
//     digits of x + 2^15, one product per digit, so a field costs about 1.4
//     instructions instead of an extract and a 24-bit multiply-add.
constexpr int kPanelAl = 16384;
constexpr int kQuadX = 4 * kGroup + 4;  // int32 per quad of groups
constexpr int kQuadD = 4 * 16 + 4;      // digit words per quad of groups

// PF: the next unit is loaded into a second register set while the current
// one is decoded.  Measured on the 16384^2 sweep, it pays for b <= 4 only;
// wider fields issue enough bytes per unit for the other waves to hide the
// latency.
// NT: lanes per block.  1024 (one block per CU) stages x once per CU instead of
// twice; measured on the sweep it pays for b <= 4 (about 0.5 us of 15-28 us)
// and loses 1-2 us at b = 7 and 12.
// R: rows per wave and unit.  b = 2..4 (nibble products) take one row per
// unit: measured at b = 3 on the sweep, 22.8 us against 23.9 us with two rows
// (the smaller last unit leaves less decode after the last load lands).
template <int B>
struct AlCfg {
  static constexpr int R = B == 1 ? 4 : 1;
  static constexpr bool PF = B <= 4;
  static constexpr int NT = B <= 4 ? 1024 : 512;
};

// Stages x[c0, c0+pc) (pc a multiple of 128) into xs (quad-skewed), general
// loop for the slow path; returns whether this thread saw only int16-range
// values.
template <int NT>
__device__ __forceinline__ int stage_x_al(const int32_t *__restrict__ x, int64_t c0, int pc,
                                          int32_t *xs) {
  uint32_t m = 0;
  const int nchunk = pc / 4;
  for (int q = threadIdx.x; q < nchunk; q += NT) {
    const int4 v = *reinterpret_cast<const int4 *>(x + c0 + 4 * q);
    const int e = 4 * q;
    *reinterpret_cast<int4 *>(xs + e + 4 * (e >> 7)) = v;
    m |= ((uint32_t)v.x + 32768u) | ((uint32_t)v.y + 32768u) | ((uint32_t)v.z + 32768u) |
         ((uint32_t)v.w + 32768u);
  }
  return (m >> 16) == 0;
}

// b = 1: digit words of group g from its 32 x values v[] (already offset by
// 2^15).  Word xd[(g/4)*kQuadD + (g%4)*16 + 4d + s] holds in nibble q digit d
// of x'_{32g + 4q + s}, x' = x + 2^15.
__device__ __forceinline__ void store_digits_al(const uint32_t *v, int g, uint32_t *xd) {
  uint32_t D[4][4];  // [digit][s]
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    // values u_q = x'_{4q+s}, q = 0..7; byte 0 holds digits 0,1, byte 1 digits 2,3
    const uint32_t *u = v + s;
    // v_perm_b32: selector bytes 0-3 pick the second operand's bytes, 4-7 the
    // first's; t02 = [u0.b0, u2.b0, u0.b1, u2.b1] and the like
    const uint32_t t02 = __builtin_amdgcn_perm(u[8], u[0], 0x05010400u);
    const uint32_t t46 = __builtin_amdgcn_perm(u[24], u[16], 0x05010400u);
    const uint32_t t13 = __builtin_amdgcn_perm(u[12], u[4], 0x05010400u);
    const uint32_t t57 = __builtin_amdgcn_perm(u[28], u[20], 0x05010400u);
    const uint32_t le = __builtin_amdgcn_perm(t46, t02, 0x05040100u);  // byte 0 of u0,u2,u4,u6
    const uint32_t he = __builtin_amdgcn_perm(t46, t02, 0x07060302u);  // byte 1
    const uint32_t lo = __builtin_amdgcn_perm(t57, t13, 0x05040100u);  // byte 0 of u1,u3,u5,u7
    const uint32_t ho = __builtin_amdgcn_perm(t57, t13, 0x07060302u);
    // byte k of digit word d: low nibble from u_{2k}, high nibble from u_{2k+1}
    D[0][s] = (le & 0x0F0F0F0Fu) | ((lo & 0x0F0F0F0Fu) << 4);
    D[1][s] = ((le >> 4) & 0x0F0F0F0Fu) | (lo & 0xF0F0F0F0u);
    D[2][s] = (he & 0x0F0F0F0Fu) | ((ho & 0x0F0F0F0Fu) << 4);
    D[3][s] = ((he >> 4) & 0x0F0F0F0Fu) | (ho & 0xF0F0F0F0u);
  }
  uint32_t *dst = xd + (g >> 2) * kQuadD + (g & 3) * 16;
#pragma unroll
  for (int d = 0; d < 4; ++d)
    *reinterpret_cast<uint4 *>(dst + 4 * d) = make_uint4(D[d][0], D[d][1], D[d][2], D[d][3]);
}


// ---- b = 2..4: nibble dot products -------------------------------------
// Digit words of one group: chunk c (columns 32g + 8c .. 32g + 8c + 7) at
// words 4c .. 4c + 3 of the group's 16; word 4c + d holds in nibble i digit d
// of u = x_{32g+8c+i} + 2^15.  For b <= 3 the top digit is stored as d - 8 (a
// signed nibble): x = d0 + 16 d1 + 256 d2 + 4096 (d3 - 8), so the products
// with non-negative fields need no offset term.  Fields of b = 4 reach 15,
// which is no signed nibble, so there the top digit stays unsigned and the
// offset 2^15 * sum(fields) is taken off.  Word 64 of each quad (in the skew)
// holds the quad's sum of x, for signed fields (below).
// Two threads per group: thread half h builds chunks 2h and 2h + 1 from its
// 16 values v[] (already offset by 2^15); st: whether group g exists.
template <int B>
__device__ __forceinline__ void nib_store_digits(const uint32_t *v, int g, int h, bool st,
                                                 uint32_t *xd) {
  uint32_t *dst = xd + (g >> 2) * kQuadD + (g & 3) * 16 + 8 * h;
  int32_t gs = 0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    uint32_t D[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t u = v[8 * c + i];
      gs += (int32_t)u - 32768;
#pragma unroll
      for (int d = 0; d < 4; ++d) D[d] |= ((u >> (4 * d)) & 15u) << (4 * i);
    }
    if constexpr (B < 4) D[3] ^= 0x88888888u;
    if (st) *reinterpret_cast<uint4 *>(dst + 4 * c) = make_uint4(D[0], D[1], D[2], D[3]);
  }
  // the quad's four groups are the eight lanes 8k .. 8k + 7
  gs += __shfl_xor(gs, 1);
  gs += __shfl_xor(gs, 2);
  gs += __shfl_xor(gs, 4);
  if (st && (g & 3) == 0 && h == 0) xd[(g >> 2) * kQuadD + 64] = (uint32_t)gs;
}

// Signed fields: flipping a field's top bit turns its two's complement value a
// into p = a + 2^(b-1) in [0, 2^b), so sum a x = sum p x - 2^(b-1) sum x.
// The bits to flip in word k of a group (top bit of field i at 32-bit stream
// position b i + b - 1).
template <int B>
__device__ __forceinline__ constexpr uint32_t nib_top_bits(int k) {
  if constexpr (B == 2) return 0xAAAAAAAAu;
  else if constexpr (B == 4) return 0x88888888u;
  else return k == 0 ? 0x24924924u : (k == 1 ? 0x49249249u : 0x92492492u);
}

// The four chunks of eight fields of one group's b words, each in the low 8b
// bits (higher bits are ignored by nib_spread).
template <int B>
__device__ __forceinline__ void nib_chunks(const uint32_t *w, uint32_t (&ch)[4]) {
  if constexpr (B == 2) {
    ch[0] = w[0];
    ch[1] = w[0] >> 16;
    ch[2] = w[1];
    ch[3] = w[1] >> 16;
  } else if constexpr (B == 3) {
    ch[0] = w[0];
    ch[1] = __builtin_amdgcn_alignbit(w[1], w[0], 24);
    ch[2] = __builtin_amdgcn_alignbit(w[2], w[1], 16);
    ch[3] = w[2] >> 8;
  } else {
    ch[0] = w[0];
    ch[1] = w[1];
    ch[2] = w[2];
    ch[3] = w[3];
  }
}

// Field i (bits i b .. i b + b - 1 of c) to nibble i, zero-extended.  Three
// halving steps move the upper half of every block by the block's slack;
// v_bitop3_b32 with table 0xE4 selects bit by bit (third operand ? first :
// second), written as the builtin so the compiler does not re-associate the
// masks of consecutive steps.
template <int B>
__device__ __forceinline__ uint32_t nib_spread(uint32_t c) {
  if constexpr (B == 2) {
    const uint32_t t1 = __builtin_amdgcn_bitop3_b32(c, c << 8, 0x000000FFu, 0xE4);
    const uint32_t t2 = __builtin_amdgcn_bitop3_b32(t1, t1 << 4, 0x000F000Fu, 0xE4);
    return ((t2 << 2) & 0x30303030u) | (t2 & 0x03030303u);
  } else if constexpr (B == 3) {
    const uint32_t t1 = __builtin_amdgcn_bitop3_b32(c, c << 4, 0x00000FFFu, 0xE4);
    const uint32_t t2 = __builtin_amdgcn_bitop3_b32(t1, t1 << 2, 0x003F003Fu, 0xE4);
    return ((t2 << 1) & 0x70707070u) | (t2 & 0x07070707u);
  } else {
    return c;
  }
}

// RG (ragged): any number of columns.  Rows then start at any bit, so a unit
// fetches the 16-byte-aligned superset of each quad (b + 1 vectors, clamped to
// the payload capacity) and shifts it into place when it is decoded: the
// offset o = (r cols + c0) b mod 128 is the same for every quad of a row and
// uniform across the wave, so the word part of the shift is a uniform branch
// and the bit part one funnel shift per word.  x is staged zero-padded to
// whole quads (the fields past the row's end, which belong to the next row,
// meet x = 0).
template <int B, bool SGN, int NT = AlCfg<B>::NT, bool RG = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void
k_matvec_al(const uint32_t *__restrict__ A, int64_t rows, int64_t cols,
            const int32_t *__restrict__ x, int64_t *__restrict__ y, int atomic_out, int g_full) {
  static_assert(NT >= 512 && NT % 64 == 0, "a lane per b = 1 group of a 16384-column panel");
  constexpr int R = AlCfg<B>::R;
  constexpr bool PF = AlCfg<B>::PF;
  constexpr int NWD = 4 * B;  // words per (row, quad)
  constexpr int NWR = RG ? NWD + 4 : NWD;  // words a unit holds per row
  constexpr bool kNib = B >= 2 && B <= 4;
  static_assert(!kNib || NT == 1024, "two lanes per group of a 16384-column panel");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int32_t *xs = reinterpret_cast<int32_t *>(smem_raw);
  uint32_t *xd = reinterpret_cast<uint32_t *>(smem_raw);  // b <= 4 fast path only

  // A 1-D grid over the column panels: g_full blocks for each full panel,
  // the rest for the last one (the host sizes the shares by the panels'
  // quads), each share striding over the row blocks.
  const int npan = (int)((cols + kPanelAl - 1) / kPanelAl);
  const int nfb = (npan - 1) * g_full;
  const bool in_full = (int)blockIdx.x < nfb;
  const int pan = in_full ? (int)blockIdx.x / g_full : npan - 1;
  const int bj = in_full ? (int)blockIdx.x % g_full : (int)blockIdx.x - nfb;
  const int gstr = in_full ? g_full : (int)gridDim.x - nfb;
  const int64_t c0 = (int64_t)pan * kPanelAl;
  // a multiple of 128 unless RG
  const int pc = (int)(cols - c0 < kPanelAl ? cols - c0 : kPanelAl);
  const int nq = (pc + 4 * kGroup - 1) / (4 * kGroup);
  const int nslot = (nq + 63) / 64;  // quad slots per lane: 1 or 2 (wave-uniform)

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nrb = (rows + (NT / 64) * R - 1) / ((NT / 64) * R);  // > bj
  const uint64_t row_words = (uint64_t)cols * B / 32;  // a multiple of 4
  const uint64_t panel_word = (uint64_t)c0 * B / 32;

  // rows r0 .. r0+nv-1 of row block rb belong to this wave
  auto rows_of = [&](int64_t rb, int64_t &r0) -> int {
    r0 = rb * ((NT / 64) * R) + (int64_t)wave * R;
    const int64_t left = rows - r0;
    return left >= R ? R : (left > 0 ? (int)left : 0);
  };
  // RG: last 16-byte vector inside the payload capacity
  const uint64_t vmax = RG ? cap_words32((uint64_t)rows * (uint64_t)cols, B) / 4 - 1 : 0;
  // the unit's words; rows and quads past the end are clamped to the last one
  auto load_unit = [&](uint32_t (&w)[R][NWR], int64_t rb, int h) {
    const int64_t r0 = rb * ((NT / 64) * R) + (int64_t)wave * R;
    const int qq = lane + 64 * h;
    const int q = qq < nq ? qq : nq - 1;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int64_t r = r0 + rr < rows ? r0 + rr : rows - 1;
      if constexpr (RG) {
        const uint64_t v0 = (((uint64_t)r * (uint64_t)cols + (uint64_t)c0) * B >> 7) +
                            (uint64_t)q * B;
        const uint4 *src = reinterpret_cast<const uint4 *>(A);
#pragma unroll
        for (int u = 0; u <= B; ++u) {
          const uint4 t = src[v0 + u < vmax ? v0 + u : vmax];
          w[rr][4 * u] = t.x;
          w[rr][4 * u + 1] = t.y;
          w[rr][4 * u + 2] = t.z;
          w[rr][4 * u + 3] = t.w;
        }
        continue;
      }
      const uint4 *src = reinterpret_cast<const uint4 *>(A + (uint64_t)r * row_words + panel_word +
                                                         (uint64_t)q * NWD);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const uint4 t = src[u];
        w[rr][4 * u] = t.x;
        w[rr][4 * u + 1] = t.y;
        w[rr][4 * u + 2] = t.z;
        w[rr][4 * u + 3] = t.w;
      }
    }
  };
  // request x (clamped, fixed count), then the first unit, then consume x
  const int4 *x4 = reinterpret_cast<const int4 *>(x + c0);
  int4 xv[8];
  // RG: the 16-byte chunk of x at panel offset e (4 | e), zero past the end
  auto x_chunk = [&](int e) -> int4 {
    if (e + 4 <= pc) return x4[e >> 2];
    int4 v = {0, 0, 0, 0};
    if (e < pc) v.x = x[c0 + e];
    if (e + 1 < pc) v.y = x[c0 + e + 1];
    if (e + 2 < pc) v.z = x[c0 + e + 2];
    return v;
  };
  if constexpr (RG && (kNib || B == 1)) {
    // as below, groups past the end of x read as zeros
    constexpr int NV = kNib ? 4 : 8;
    const int e0 = kNib ? 32 * ((int)threadIdx.x >> 1) + 16 * ((int)threadIdx.x & 1)
                        : 32 * (int)threadIdx.x;
#pragma unroll
    for (int i = 0; i < NV; ++i) xv[i] = x_chunk(e0 + 4 * i);
  } else if constexpr (RG) {
#pragma unroll
    for (int u = 0; u < kPanelAl / 4 / NT; ++u) xv[u] = x_chunk(4 * ((int)threadIdx.x + NT * u));
  } else if constexpr (kNib) {
    // lane t: half t % 2 of group t / 2 (16 values)
    const int ng = pc / kGroup;
    const int g0 = (int)threadIdx.x >> 1;
    const int g = g0 < ng ? g0 : ng - 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) xv[i] = x4[8 * g + 4 * ((int)threadIdx.x & 1) + i];
  } else if constexpr (B == 1) {
    // lane g: the 32 values of group g (pc <= 16384: one group per lane)
    const int ng = pc / kGroup;
    const int g = (int)threadIdx.x < ng ? (int)threadIdx.x : ng - 1;
#pragma unroll
    for (int i = 0; i < 8; ++i) xv[i] = x4[8 * g + i];
  } else {
    // lane t: 16-byte chunks t, t+NT, ... (pc/4 <= 4096 chunks: one round)
    const int nchunk = pc / 4;
#pragma unroll
    for (int u = 0; u < kPanelAl / 4 / NT; ++u) {
      const int q = (int)threadIdx.x + NT * u;
      xv[u] = x4[q < nchunk ? q : nchunk - 1];
    }
  }
  uint32_t w0[R][NWR], w1[R][NWR];
  int64_t rb = bj;
  __builtin_amdgcn_sched_barrier(0);  // x requests first
  // the first unit overlaps the staging (measured: a loss for b > 8)
  constexpr bool kEarly = PF || B <= 8;
  if constexpr (kEarly) load_unit(w0, rb, 0);

  uint32_t m = 0;
  if constexpr (B == 1) {
    uint32_t v[kGroup];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      v[4 * i] = (uint32_t)xv[i].x + 32768u;
      v[4 * i + 1] = (uint32_t)xv[i].y + 32768u;
      v[4 * i + 2] = (uint32_t)xv[i].z + 32768u;
      v[4 * i + 3] = (uint32_t)xv[i].w + 32768u;
    }
#pragma unroll
    for (int i = 0; i < kGroup; i += 2) m |= v[i] | v[i + 1];
    if ((int)threadIdx.x < (RG ? 4 * nq : pc / kGroup)) store_digits_al(v, threadIdx.x, xd);
  } else if constexpr (kNib) {
    uint32_t v[16];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[4 * i] = (uint32_t)xv[i].x + 32768u;
      v[4 * i + 1] = (uint32_t)xv[i].y + 32768u;
      v[4 * i + 2] = (uint32_t)xv[i].z + 32768u;
      v[4 * i + 3] = (uint32_t)xv[i].w + 32768u;
    }
#pragma unroll
    for (int i = 0; i < 16; i += 2) m |= v[i] | v[i + 1];
    const int g = (int)threadIdx.x >> 1;
    nib_store_digits<B>(v, g, (int)threadIdx.x & 1, g < (RG ? 4 * nq : pc / kGroup), xd);
  } else {
    const int nchunk = RG ? 32 * nq : pc / 4;  // RG: the zero padding too
#pragma unroll
    for (int u = 0; u < kPanelAl / 4 / NT; ++u) {
      const int q = (int)threadIdx.x + NT * u;
      if (q < nchunk) {
        const int e = 4 * q;
        *reinterpret_cast<int4 *>(xs + e + 4 * (e >> 7)) = xv[u];
      }
      // x in [-2^15, 2^15) iff x + 2^15 < 2^16 as unsigned (clamped chunks repeat valid ones)
      m |= ((uint32_t)xv[u].x + 32768u) | ((uint32_t)xv[u].y + 32768u) |
           ((uint32_t)xv[u].z + 32768u) | ((uint32_t)xv[u].w + 32768u);
    }
  }
  const bool fast = __syncthreads_and((m >> 16) == 0);

  if (!fast) {
    // general x: 64-bit products, one row and one group at a time
    if constexpr (RG) {
      if constexpr (B == 1 || kNib) {
        for (int q = threadIdx.x; q < 32 * nq; q += NT) {
          const int e = 4 * q;
          *reinterpret_cast<int4 *>(xs + e + 4 * (e >> 7)) = x_chunk(e);
        }
        __syncthreads();
      }
      for (; rb < nrb; rb += gstr) {
        int64_t r0;
        const int nv = rows_of(rb, r0);
#pragma unroll 1
        for (int rr = 0; rr < nv; ++rr) {
          uint64_t a = 0;
#pragma unroll 1
          for (int gi = lane; 32 * gi < pc; gi += 64) {
            // b + 1 words from the group's first (inside the capacity's
            // guard words), shifted into place
            const uint64_t pb = ((uint64_t)(r0 + rr) * (uint64_t)cols + (uint64_t)c0 +
                                 32u * (uint64_t)gi) * B;
            const uint32_t *src = A + (pb >> 5);
            const int sh = (int)(pb & 31u);
            uint32_t w[B + 1];
#pragma unroll
            for (int k = 0; k <= B; ++k) w[k] = src[k];
#pragma unroll
            for (int k = 0; k < B; ++k) w[k] = __builtin_amdgcn_alignbit(w[k + 1], w[k], sh);
            a += group_dot_wide<B, SGN, int32_t>(w, xs + (gi >> 2) * kQuadX + (gi & 3) * kGroup);
          }
          const int64_t sum = wave_sum((int64_t)a);
          if (lane == 0) {
            if (atomic_out)
              atomicAdd((unsigned long long *)&y[r0 + rr], (unsigned long long)sum);
            else
              y[r0 + rr] = sum;
          }
        }
      }
      return;
    }
    if constexpr (B == 1 || kNib) {
      (void)stage_x_al<NT>(x, c0, pc, xs);
      __syncthreads();
    }
    for (; rb < nrb; rb += gstr) {
      int64_t r0;
      const int nv = rows_of(rb, r0);
#pragma unroll 1
      for (int rr = 0; rr < nv; ++rr) {
        uint64_t a = 0;
#pragma unroll 1
        for (int q = lane; q < nq; q += 64) {
          const uint32_t *src = A + (uint64_t)(r0 + rr) * row_words + panel_word + (uint64_t)q * NWD;
#pragma unroll 1
          for (int t = 0; t < 4; ++t) {
            uint32_t w[B];
#pragma unroll
            for (int k = 0; k < B; ++k) w[k] = src[t * B + k];
            a += group_dot_wide<B, SGN, int32_t>(w, xs + q * kQuadX + t * kGroup);
          }
        }
        const int64_t sum = wave_sum((int64_t)a);
        if (lane == 0) {
          if (atomic_out)
            atomicAdd((unsigned long long *)&y[r0 + rr], (unsigned long long)sum);
          else
            y[r0 + rr] = sum;
        }
      }
    }
    return;
  }

  uint64_t acc[R];
#pragma unroll
  for (int rr = 0; rr < R; ++rr) acc[rr] = 0;
  // b = 1: a lane's share of a row within one panel (at most 256 fields, each
  // adding x + 2^15 < 2^16 less 2^15 per set field) and the wave's total (at
  // most 16384 fields) both fit int32, so the digit sums, the lane sums and
  // the reduction across the wave stay 32-bit (about 1 us less per launch
  // on the 16384^2 sweep)
  int32_t acc32[R];
#pragma unroll
  for (int rr = 0; rr < R; ++rr) acc32[rr] = 0;

  // decode one unit (quad slot h of the wave's R rows) held in w into acc.
  // Branch-free: lanes past the last quad decode the clamped copy and add
  // nothing, rows past the end are decoded and never stored -- so every path
  // waits for the unit's loads at the same point.
  auto decode_unit = [&](const uint32_t (&w)[R][NWD], int h) {
    const int qq = lane + 64 * h;
    const bool live = qq < nq;
    const int q = live ? qq : nq - 1;
    if constexpr (B == 1) {
      uint32_t dacc[R][5];
#pragma unroll
      for (int rr = 0; rr < R; ++rr)
#pragma unroll
        for (int d = 0; d < 5; ++d) dacc[rr][d] = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint4 *dg = reinterpret_cast<const uint4 *>(xd + q * kQuadD + t * 16);
        const uint4 d0 = dg[0], d1 = dg[1], d2 = dg[2], d3 = dg[3];
        const uint32_t X[16] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w,
                                d2.x, d2.y, d2.z, d2.w, d3.x, d3.y, d3.z, d3.w};
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          const uint32_t a = w[rr][t];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const uint32_t an = (a >> s) & 0x11111111u;
#pragma unroll
            for (int d = 0; d < 4; ++d)
              dacc[rr][d] = __builtin_amdgcn_udot8(an, X[d * 4 + s], dacc[rr][d], false);
          }
          dacc[rr][4] += (uint32_t)__builtin_popcount(a);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int32_t tt = (int32_t)(dacc[rr][0] + (dacc[rr][1] << 4) + (dacc[rr][2] << 8) +
                                     (dacc[rr][3] << 12) - (dacc[rr][4] << 15));
        acc32[rr] += live ? (SGN ? -tt : tt) : 0;
      }
    } else if constexpr (kNib) {
      // per row: a[0..3] digit sums (a[3] signed for b <= 3), a[4] the sum
      // of the fields (b = 4)
      uint32_t a[R][5];
#pragma unroll
      for (int rr = 0; rr < R; ++rr)
#pragma unroll
        for (int d = 0; d < 5; ++d) a[rr][d] = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint4 *dg = reinterpret_cast<const uint4 *>(xd + q * kQuadD + t * 16);
        uint4 D[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) D[c] = dg[c];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          uint32_t wv[B];
#pragma unroll
          for (int k = 0; k < B; ++k) wv[k] = w[rr][t * B + k] ^ (SGN ? nib_top_bits<B>(k) : 0u);
          uint32_t ch[4];
          nib_chunks<B>(wv, ch);
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const uint32_t n = nib_spread<B>(ch[c]);
            a[rr][0] = __builtin_amdgcn_udot8(n, D[c].x, a[rr][0], false);
            a[rr][1] = __builtin_amdgcn_udot8(n, D[c].y, a[rr][1], false);
            a[rr][2] = __builtin_amdgcn_udot8(n, D[c].z, a[rr][2], false);
            if constexpr (B < 4) {
              a[rr][3] = (uint32_t)__builtin_amdgcn_sdot8((int)n, (int)D[c].w, (int)a[rr][3], false);
            } else {
              a[rr][3] = __builtin_amdgcn_udot8(n, D[c].w, a[rr][3], false);
              a[rr][4] = __builtin_amdgcn_udot8(n, 0x11111111u, a[rr][4], false);
            }
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      // a unit's share of a row (128 fields) fits int32: |sum| <= 128 * 15 *
      // 2^16; the quad's sum of x times 2^(b-1) for signed fields
      const uint32_t corr = SGN ? xd[q * kQuadD + 64] << (B - 1) : 0u;
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int32_t tt = (int32_t)(a[rr][0] + (a[rr][1] << 4) + (a[rr][2] << 8) +
                                     (a[rr][3] << 12) - (a[rr][4] << 15) - corr);
        acc[rr] += live ? (uint64_t)(int64_t)tt : 0u;
      }
    } else {
      uint64_t part[R];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) part[rr] = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        int32_t xg[kGroup];
        const int32_t *xp = xs + q * kQuadX + t * kGroup;
#pragma unroll
        for (int i = 0; i < kGroup; ++i) xg[i] = xp[i];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) part[rr] += group_dot_small<B, SGN>(&w[rr][t * B], xg);
        // keep each group's x values live for that group only
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int rr = 0; rr < R; ++rr) acc[rr] += live ? part[rr] : 0u;
    }
  };

  // RG: each row's words shifted into place first (see the kernel's header)
  auto compute_unit = [&](const uint32_t (&w)[R][NWR], int h) {
    if constexpr (RG) {
      const int64_t r0 = rb * ((NT / 64) * R) + (int64_t)wave * R;
      uint32_t wa[R][NWD];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int64_t r = r0 + rr < rows ? r0 + rr : rows - 1;
        const uint32_t o = (uint32_t)((((uint64_t)r * (uint64_t)cols + (uint64_t)c0) * B) & 127u);
        const int sh = (int)(o & 31u);
        switch (o >> 5) {
#define CCM_REALIGN(hw)                                                                     \
  case hw:                                                                                  \
    _Pragma("unroll") for (int k = 0; k < NWD; ++k) wa[rr][k] =                              \
        __builtin_amdgcn_alignbit(w[rr][k + hw + 1], w[rr][k + hw], sh);                     \
    break;
          CCM_REALIGN(0)
          CCM_REALIGN(1)
          CCM_REALIGN(2)
          CCM_REALIGN(3)
#undef CCM_REALIGN
        }
      }
      decode_unit(wa, h);
    } else {
      decode_unit(w, h);
    }
  };

  // Row sums of the fast path wait in a register: lane j holds entry j of the
  // wave's current batch (row j % R of the wave's rows in row block first_rb +
  // (j / R) * gstr), written with one store per 64 entries.  A store's
  // address and data registers may only be reused once it has completed, and
  // the load counter is in order, so a store issued after a unit's loads
  // would make the next reuse wait for those loads as well: the batch store is
  // therefore issued at the start of a step, before that step's loads, and
  // its address register stays reserved (ydst) until the next batch.
  uint64_t ybuf = 0;
  int nst = 0;
  int64_t first_rb = rb;
  int64_t *ydst = y;
  auto flush = [&]() {
    const int64_t rbj = first_rb + (int64_t)(lane / R) * gstr;
    const int64_t row = rbj * ((NT / 64) * R) + (int64_t)wave * R + lane % R;
    const bool ok = lane < nst && row < rows;
    ydst = y + (ok ? row : 0);
    if (ok) {
      if (atomic_out)
        atomicAdd((unsigned long long *)ydst, (unsigned long long)ybuf);
      else
        *ydst = (int64_t)ybuf;
    }
    nst = 0;
  };
  auto collect = [&](int64_t rb_) {
    if (nst == 0) first_rb = rb_;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      uint64_t sum;
      if constexpr (B == 1) {
        sum = (uint64_t)(int64_t)wave_sum32(acc32[rr]);
        acc32[rr] = 0;
      } else {
        sum = (uint64_t)wave_sum((int64_t)acc[rr]);
        acc[rr] = 0;
      }
      ybuf = lane == nst + rr ? sum : ybuf;
    }
    nst += R;
  };

  // units in order (rb, 0), (rb, 1), ..., (rb + gstr, 0), ...
  int h = 0;
  if constexpr (PF) {
    auto step = [&](uint32_t (&cur)[R][NWR], uint32_t (&nxt)[R][NWR]) -> bool {
      if (nst == 64) flush();
      int64_t rb2 = rb;
      int h2 = h + 1;
      if (h2 == nslot) {
        h2 = 0;
        rb2 += gstr;
      }
      const bool more = rb2 < nrb;
      load_unit(nxt, more ? rb2 : rb, more ? h2 : h);
      compute_unit(cur, h);
      if (h == nslot - 1) collect(rb);
      rb = rb2;
      h = h2;
      asm volatile("" ::"v"(ydst));
      return more;
    };
    while (step(w0, w1) && step(w1, w0)) {
    }
  } else {
    // one unit at a time: row sums are stored as they complete
    for (; rb < nrb; rb += gstr) {
      for (h = 0; h < nslot; ++h) {
        if (!kEarly || h > 0 || rb != (int64_t)bj) load_unit(w0, rb, h);
        compute_unit(w0, h);
      }
      int64_t r0;
      const int nv = rows_of(rb, r0);
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int64_t sum = wave_sum((int64_t)acc[rr]);
        acc[rr] = 0;
        if (lane == 0 && rr < nv) {
          if (atomic_out)
            atomicAdd((unsigned long long *)&y[r0 + rr], (unsigned long long)sum);
          else
            y[r0 + rr] = sum;
        }
      }
    }
  }
  if (nst > 0) flush();
}

template <int B, bool SGN, int NT = AlCfg<B>::NT, bool RG = false>
int resident_blocks_al(size_t lds) {
  static int cached = 0;
  if (cached == 0) {
    int occ = 0, dev = 0, cus = 0;
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_matvec_al<B, SGN, NT, RG>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_matvec_al<B, SGN, NT, RG>, NT,
                                                     lds) != hipSuccess ||
        occ < 1)
      occ = 1;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    cached = occ * cus;
  }
  return cached;
}

template <int B, bool SGN, bool RG = false, int NT = AlCfg<B>::NT>
hipError_t launch_aligned(const uint32_t *w, int64_t rows, int64_t cols, const int32_t *x,
                          int64_t *y, hipStream_t s) {
  constexpr int R = AlCfg<B>::R;
  const int64_t npanels = (cols + kPanelAl - 1) / kPanelAl;
  const int64_t nrb = (rows + (NT / 64) * R - 1) / ((NT / 64) * R);
  if (nrb > 0x7fffffffll || npanels > 65535) return hipErrorInvalidValue;
  if (npanels > 1) {
    hipError_t e = launch_fill_i64(y, (uint64_t)rows, 0, s);
    if (e != hipSuccess) return e;
  }
  const int64_t nqp = ((cols < kPanelAl ? cols : kPanelAl) + 4 * kGroup - 1) / (4 * kGroup);
  const size_t lds = (size_t)nqp * kQuadX * sizeof(int32_t);  // >= the digit words
  const int64_t res =
      resident_blocks_al<B, SGN, NT, RG>((size_t)(kPanelAl / (4 * kGroup)) * kQuadX * 4);
  auto clampg = [&](int64_t g) { return g < 1 ? 1 : (g > nrb ? nrb : g); };
  // resident blocks shared by the panels in proportion to their units per
  // row block (quad slots: 2 for a full panel, 1 for a last panel of at most
  // 64 quads, whose units cost as much however few of their lanes are live),
  // so that a narrow last panel does not hold blocks the full panels need;
  // every block owns at least one row block
  const int64_t nq_last = (cols - (npanels - 1) * kPanelAl + 4 * kGroup - 1) / (4 * kGroup);
  const int64_t ns_last = (nq_last + 63) / 64;
  const int64_t g_full =
      npanels == 1 ? clampg(res) : clampg(res * 2 / ((npanels - 1) * 2 + ns_last));
  const int64_t g_last = npanels == 1 ? g_full : clampg(g_full * ns_last / 2);
  const int64_t grid = (npanels - 1) * g_full + g_last;
  if (grid > 0x7fffffffll) return hipErrorInvalidValue;
  k_matvec_al<B, SGN, NT, RG><<<dim3((unsigned)grid), NT, lds, s>>>(
      w, rows, cols, x, y, npanels > 1 ? 1 : 0, (int)g_full);
  return hipGetLastError();
}

// Wide-field variant for b >= 16 and int32 x, any row alignment.  Same
// pipeline as the aligned kernel: 1024-lane blocks over 16384-column panels
// (a 73.7 KB x panel, one block per CU), one row per wave, lane l owns
// groups l, l+64, ... of the panel; a unit is (row, group slot), b+1 words per
// lane (the extra word feeds the funnel shift of rows that start inside a
// word).  With PF the next unit's words are in flight while the current one
// is decoded; loads are issued in fixed count (clamped addresses) so the
// compiler waits only for the older unit.  Products are 64-bit (int16-range
// runs would be one element long at these widths).
constexpr int kPanelW = 16384;
constexpr int kPitchW = kGroup + 4;  // int32 per staged group

template <int B>
struct WCfg {
  static constexpr bool PF = B <= 24;  // measured: larger widths run faster without
  // one 1024-lane block per CU (x staged once per CU): 1-2.5 us faster than two
  // 512-lane blocks at b = 17 and 31 on the sweep
  static constexpr int NT = 1024;
};

template <int B, bool SGN, int NT = WCfg<B>::NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void
k_matvec_w(const uint32_t *__restrict__ A, int64_t rows, int64_t cols,
           const int32_t *__restrict__ x, int64_t *__restrict__ y, int atomic_out,
           int x_aligned16, int g_full) {
  constexpr bool PF = WCfg<B>::PF;
  constexpr int NWG = B + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int32_t *xs = reinterpret_cast<int32_t *>(smem_raw);

  // a 1-D grid over the column panels, as in the aligned kernel
  const int npan = (int)((cols + kPanelW - 1) / kPanelW);
  const int nfb = (npan - 1) * g_full;
  const bool in_full = (int)blockIdx.x < nfb;
  const int pan = in_full ? (int)blockIdx.x / g_full : npan - 1;
  const int bj = in_full ? (int)blockIdx.x % g_full : (int)blockIdx.x - nfb;
  const int gstr = in_full ? g_full : (int)gridDim.x - nfb;
  const int64_t c0 = (int64_t)pan * kPanelW;
  const int pc = (int)(cols - c0 < kPanelW ? cols - c0 : kPanelW);
  const int ng = (pc + kGroup - 1) / kGroup;
  const int nslot = (ng + 63) / 64;  // wave-uniform
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nrb = (rows + (NT / 64) - 1) / (NT / 64);  // > bj

  // the unit's words and the row's funnel shift (the same for every group of
  // a row); rows past the end and groups past the last are clamped
  auto load_unit = [&](uint32_t (&w)[NWG], int64_t rb, int h, int &shift) {
    const int64_t r0 = rb * (NT / 64) + wave;
    const int64_t r = r0 < rows ? r0 : rows - 1;
    const int jj = lane + 64 * h;
    const int j = jj < ng ? jj : ng - 1;
    const uint64_t bit = ((uint64_t)r * (uint64_t)cols + (uint64_t)c0) * (uint64_t)B;
    shift = (int)(bit & 31u);
    const uint32_t *gp = A + (bit >> 5) + (uint64_t)j * B;
#pragma unroll
    for (int k = 0; k < NWG; ++k) w[k] = gp[k];
  };

  uint32_t w0[NWG], w1[NWG];
  int s0 = 0, s1 = 0;
  int64_t rb = bj;

  // stage the x panel, zero-padded to whole groups
  const int nchunk = ng * kGroup / 4;
  if (x_aligned16 && pc == ng * kGroup) {
    // whole groups, aligned x: every chunk requested at once (a fixed count,
    // clamped), then the first unit, then the chunks stored -- the wait for
    // the chunks leaves the unit's loads in flight (the counter is in order)
    constexpr int kXPer = kPanelW / 4 / NT;
    const int4 *x4 = reinterpret_cast<const int4 *>(x + c0);
    int4 xv[kXPer];
#pragma unroll
    for (int u = 0; u < kXPer; ++u) {
      const int q = (int)threadIdx.x + NT * u;
      xv[u] = x4[q < nchunk ? q : nchunk - 1];
    }
    if constexpr (PF) load_unit(w0, rb, 0, s0);  // in flight across the barrier
#pragma unroll
    for (int u = 0; u < kXPer; ++u) {
      const int e = 4 * ((int)threadIdx.x + NT * u);
      if (e < 4 * nchunk) *reinterpret_cast<int4 *>(xs + (e >> 5) * kPitchW + (e & 31)) = xv[u];
    }
  } else {
    for (int q = threadIdx.x; q < nchunk; q += NT) {
      const int e = 4 * q;
      int4 v;
      if (x_aligned16 && e + 4 <= pc)
        v = *reinterpret_cast<const int4 *>(x + c0 + e);
      else
        v = make_int4(e < pc ? x[c0 + e] : 0, e + 1 < pc ? x[c0 + e + 1] : 0,
                      e + 2 < pc ? x[c0 + e + 2] : 0, e + 3 < pc ? x[c0 + e + 3] : 0);
      *reinterpret_cast<int4 *>(xs + (e >> 5) * kPitchW + (e & 31)) = v;
    }
    if constexpr (PF) load_unit(w0, rb, 0, s0);  // in flight across the barrier
  }
  __syncthreads();

  uint64_t acc = 0;
  auto compute_unit = [&](uint32_t (&w)[NWG], int shift, int h) {
    const int jj = lane + 64 * h;
    const bool live = jj < ng;
    const int j = live ? jj : ng - 1;
    // consume every word before the (wave-uniform) shift test, so that all
    // paths wait for the unit's loads at the same point
#pragma unroll
    for (int k = 0; k < NWG; ++k) asm volatile("" ::"v"(w[k]));
    if (shift != 0) {
#pragma unroll
      for (int k = 0; k < B; ++k) w[k] = __builtin_amdgcn_alignbit(w[k + 1], w[k], shift);
    }
    const uint64_t d = group_dot_wide<B, SGN, int32_t>(w, xs + j * kPitchW);
    acc += live ? d : 0u;
  };

  if constexpr (PF) {
    // row sums wait in a register (lane j: entry j of the batch, row
    // first_rb + j * gstr of this wave) and are stored once per 64 rows,
    // before a step's loads (see the aligned kernel)
    uint64_t ybuf = 0;
    int nst = 0;
    int64_t first_rb = rb;
    int64_t *ydst = y;
    auto flush = [&]() {
      const int64_t row = (first_rb + (int64_t)lane * gstr) * (NT / 64) + wave;
      const bool ok = lane < nst && row < rows;
      ydst = y + (ok ? row : 0);
      if (ok) {
        if (atomic_out)
          atomicAdd((unsigned long long *)ydst, (unsigned long long)ybuf);
        else
          *ydst = (int64_t)ybuf;
      }
      nst = 0;
    };
    int h = 0;
    auto step = [&](uint32_t (&cur)[NWG], int &scur, uint32_t (&nxt)[NWG], int &snxt) -> bool {
      if (nst == 64) flush();
      int64_t rb2 = rb;
      int h2 = h + 1;
      if (h2 == nslot) {
        h2 = 0;
        rb2 += gstr;
      }
      const bool more = rb2 < nrb;
      load_unit(nxt, more ? rb2 : rb, more ? h2 : h, snxt);
      compute_unit(cur, scur, h);
      if (h == nslot - 1) {
        if (nst == 0) first_rb = rb;
        const uint64_t sum = (uint64_t)wave_sum((int64_t)acc);
        ybuf = lane == nst ? sum : ybuf;
        acc = 0;
        ++nst;
      }
      rb = rb2;
      h = h2;
      asm volatile("" ::"v"(ydst));
      return more;
    };
    while (step(w0, s0, w1, s1) && step(w1, s1, w0, s0)) {
    }
    if (nst > 0) flush();
  } else {
    for (; rb < nrb; rb += gstr) {
      for (int h = 0; h < nslot; ++h) {
        load_unit(w0, rb, h, s0);
        compute_unit(w0, s0, h);
      }
      const int64_t sum = wave_sum((int64_t)acc);
      acc = 0;
      const int64_t r = rb * (NT / 64) + wave;
      if (lane == 0 && r < rows) {
        if (atomic_out)
          atomicAdd((unsigned long long *)&y[r], (unsigned long long)sum);
        else
          y[r] = sum;
      }
    }
  }
}

template <int B, bool SGN, int NT = WCfg<B>::NT>
int resident_blocks_w(size_t lds) {
  static int cached = 0;
  if (cached == 0) {
    int occ = 0, dev = 0, cus = 0;
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_matvec_w<B, SGN, NT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_matvec_w<B, SGN, NT>, NT, lds) !=
            hipSuccess ||
        occ < 1)
      occ = 1;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    cached = occ * cus;
  }
  return cached;
}

template <int B, bool SGN, int NT = WCfg<B>::NT>
hipError_t launch_wide(const uint32_t *w, int64_t rows, int64_t cols, const int32_t *x,
                       int64_t *y, hipStream_t s) {
  const int64_t npanels = (cols + kPanelW - 1) / kPanelW;
  const int64_t nrb = (rows + (NT / 64) - 1) / (NT / 64);
  if (nrb > 0x7fffffffll || npanels > 65535) return hipErrorInvalidValue;
  if (npanels > 1) {
    hipError_t e = launch_fill_i64(y, (uint64_t)rows, 0, s);
    if (e != hipSuccess) return e;
  }
  const int64_t ngp = ((cols < kPanelW ? cols : kPanelW) + kGroup - 1) / kGroup;
  const size_t lds = (size_t)ngp * kPitchW * sizeof(int32_t);
  const int64_t res = resident_blocks_w<B, SGN, NT>((size_t)(kPanelW / kGroup) * kPitchW * 4);
  auto clampg = [&](int64_t g) { return g < 1 ? 1 : (g > nrb ? nrb : g); };
  // blocks shared by the panels in proportion to their group slots per row
  // (8 for a full panel), as in the aligned kernel; every block owns at least
  // one row
  const int64_t ng_last = (cols - (npanels - 1) * kPanelW + kGroup - 1) / kGroup;
  const int64_t ns_last = (ng_last + 63) / 64;
  const int64_t ns_full = kPanelW / kGroup / 64;
  const int64_t g_full = npanels == 1 ? clampg(res)
                                      : clampg(res * ns_full / ((npanels - 1) * ns_full + ns_last));
  const int64_t g_last = npanels == 1 ? g_full : clampg(g_full * ns_last / ns_full);
  const int64_t grid = (npanels - 1) * g_full + g_last;
  if (grid > 0x7fffffffll) return hipErrorInvalidValue;
  const int al = ((uintptr_t)x % 16) == 0;
  k_matvec_w<B, SGN, NT><<<dim3((unsigned)grid), NT, lds, s>>>(
      w, rows, cols, x, y, npanels > 1 ? 1 : 0, al, (int)g_full);
  return hipGetLastError();
}

template <int B>
hipError_t launch_width(const uint32_t *w, int64_t rows, int64_t cols, int sgn, const void *x,
                        int xdtype, int64_t *y, hipStream_t s) {
  // b = 16 needs 64-bit products even for int16 x (no room for int32 runs)
  // and more registers than the aligned kernel's occupancy target allows
  if constexpr (B <= 15) {
    if (xdtype == CCM_I32 && cols % 128 == 0 && ((uintptr_t)w % 16) == 0 &&
        ((uintptr_t)x % 16) == 0)
      return sgn ? launch_aligned<B, true>(w, rows, cols, (const int32_t *)x, y, s)
                 : launch_aligned<B, false>(w, rows, cols, (const int32_t *)x, y, s);
  }
  // any other column count at b <= 4: measured on 16384 x 16383 and
  // 16384 x 12345 against the general kernel, b = 1 19.1 / 18.1 us against
  // 24.1 / 21.9, b = 3 28.1 / 26.2 against 37.0 / 31.8; at b = 7 it lost
  // (58.7 / 49.1 against 51.9 / 44.1), so wider fields keep the general kernel
  if constexpr (B <= 4) {
    if (xdtype == CCM_I32 && ((uintptr_t)w % 16) == 0 && ((uintptr_t)x % 16) == 0)
      return sgn ? launch_aligned<B, true, true>(w, rows, cols, (const int32_t *)x, y, s)
                 : launch_aligned<B, false, true>(w, rows, cols, (const int32_t *)x, y, s);
  }
  if constexpr (B >= 16) {
    if (xdtype == CCM_I32)
      return sgn ? launch_wide<B, true>(w, rows, cols, (const int32_t *)x, y, s)
                 : launch_wide<B, false>(w, rows, cols, (const int32_t *)x, y, s);
  }
  if (xdtype == CCM_I32) {
    return sgn ? launch_one<B, true, int32_t>(w, rows, cols, (const int32_t *)x, y, s)
               : launch_one<B, false, int32_t>(w, rows, cols, (const int32_t *)x, y, s);
  }
  return sgn ? launch_one<B, true, int64_t>(w, rows, cols, (const int64_t *)x, y, s)
             : launch_one<B, false, int64_t>(w, rows, cols, (const int64_t *)x, y, s);
}

}  // namespace mv
}  // namespace ccm
