// Range reduction, SM packing / unpacking, element access and elementwise
// operations on packed matrices (gfx950).
//
// Packing follows Method 1 (Eq. 3 and the straddle step): element e's b-bit
// field goes to stream bits [e*b, e*b+b), least significant bit first.  Every
// packing kernel works group-per-lane: a lane turns 32 consecutive elements
// into exactly b 32-bit words, so no two lanes ever write the same word and no
// atomics are needed; lanes of a wave share one bit phase, which keeps the
// runtime-width reader/writer branch-uniform.  Dense operands are staged
// through LDS so that HBM reads and writes stay coalesced.
#include "ccm_internal.hpp"
#include "group_codec.hpp"

#include <limits>

namespace ccm {
namespace {

constexpr int kTileThreads = 128;           // lanes per block in the tile kernels
constexpr int kTileElems = kTileThreads * kGroup;
constexpr int kPad = kGroup + 1;            // LDS row pitch (elements) of a lane's group

__global__ void k_range_init(RangeSlot *slot) {
  if (threadIdx.x < kRangeSpread) {
    RangeSlot *r = slot + kRangeStride * threadIdx.x;
    r->vmin = INT64_MAX;
    r->vmax = INT64_MIN;
    r->flag = 0;
    r->pad = 0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_range_dense(const T *__restrict__ d, uint64_t n,
                                                     RangeSlot *slot, int aligned16) {
  constexpr int PER = 16 / sizeof(T);  // elements per 16-byte load
  constexpr int UNR = 4;
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t done = 0;
  if (aligned16) {
    const uint64_t n16 = n / PER;
    const uint4 *v = reinterpret_cast<const uint4 *>(d);
    uint64_t i = tid;
    for (; i + (UNR - 1) * stride < n16; i += UNR * stride) {
      uint4 r[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) r[u] = v[i + u * stride];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const T *t = reinterpret_cast<const T *>(&r[u]);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          const int64_t x = (int64_t)t[q];
          lo = x < lo ? x : lo;
          hi = x > hi ? x : hi;
        }
      }
    }
    for (; i < n16; i += stride) {
      const uint4 r = v[i];
      const T *t = reinterpret_cast<const T *>(&r);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int64_t x = (int64_t)t[q];
        lo = x < lo ? x : lo;
        hi = x > hi ? x : hi;
      }
    }
    done = n16 * PER;
  }
  for (uint64_t e = done + tid; e < n; e += stride) {
    const int64_t x = (int64_t)d[e];
    lo = x < lo ? x : lo;
    hi = x > hi ? x : hi;
  }
  block_range_commit(lo, hi, 0, slot);
}

// dense (n values) -> packed words [0, cap32): lane g writes words [g*b, g*b+b).
// The block's 32*128 elements are first staged through LDS with 16-byte
// loads, all issued before any is consumed.
// With DEVW the width comes from res (a result whose range was reduced on the
// device): the block exits when res reports an error, and the capacity and
// group count follow that width; the grid covers any width up to the launch's
// maximum.
template <typename T, bool DEVW = false>
__global__ __launch_bounds__(kTileThreads) void k_compress(const T *__restrict__ d, uint64_t n,
                                                           int bits, uint32_t *__restrict__ out,
                                                           uint64_t cap32, uint64_t ngroups,
                                                           int aligned16,
                                                           const ccm_result *res = nullptr) {
  if constexpr (DEVW) {
    if (res->status != CCM_OK) return;
    bits = res->bits;
    cap32 = cap_words32(n, bits);
    ngroups = (cap32 + bits - 1) / bits;
  }
  constexpr int PER = 16 / sizeof(T);
  constexpr int NLOAD = kTileElems / (kTileThreads * PER);
  // the input tile, reused for the block's packed words (at most 32 words a
  // group for int32 input, 64 for int64)
  constexpr int kOutWords = kTileThreads * (sizeof(T) == 4 ? 32 : 64);
  constexpr size_t kBytes = sizeof(T) * kTileThreads * kPad > 4 * (size_t)kOutWords
                                ? sizeof(T) * kTileThreads * kPad
                                : 4 * (size_t)kOutWords;
  __shared__ __align__(16) unsigned char lds[kBytes];
  T *tile = reinterpret_cast<T *>(lds);
  const uint64_t g0 = (uint64_t)blockIdx.x * kTileThreads;
  const uint64_t e0 = g0 * kGroup;
  if (aligned16 && e0 + kTileElems <= n) {
    const uint4 *src = reinterpret_cast<const uint4 *>(d + e0);
    uint4 r[NLOAD];
#pragma unroll
    for (int j = 0; j < NLOAD; ++j) r[j] = src[threadIdx.x + j * kTileThreads];
#pragma unroll
    for (int j = 0; j < NLOAD; ++j) {
      const int q = (threadIdx.x + j * kTileThreads) * PER;
      const T *t = reinterpret_cast<const T *>(&r[j]);
#pragma unroll
      for (int u = 0; u < PER; ++u) tile[q + u + (q >> 5)] = t[u];
    }
  } else {
    for (int q = threadIdx.x; q < kTileElems; q += kTileThreads) {
      const uint64_t e = e0 + q;
      tile[q + (q >> 5)] = e < n ? d[e] : T(0);
    }
  }
  __syncthreads();
  int64_t v[kGroup];
  const T *row = tile + threadIdx.x * kPad;
#pragma unroll
  for (int i = 0; i < kGroup; ++i) v[i] = (int64_t)row[i];
  // lane g encodes group g into LDS; the block's contiguous run of words then
  // leaves with 16-byte stores (past the last group: zeros, never stored)
  __syncthreads();
  uint32_t *s_out = reinterpret_cast<uint32_t *>(lds);
  codec::encode_rt(v, bits, s_out + threadIdx.x * bits, (uint64_t)bits);
  __syncthreads();
  store_block_run(s_out, bits, out, cap32);
  (void)ngroups;
}

// packed -> dense int64 (n values)
__global__ __launch_bounds__(kTileThreads) void k_decompress(const uint32_t *__restrict__ wds,
                                                             uint64_t n, int bits, int sgn,
                                                             int64_t *__restrict__ out) {
  __shared__ int64_t tile[kTileThreads * kPad];
  const uint64_t g0 = (uint64_t)blockIdx.x * kTileThreads;
  const uint64_t g = g0 + threadIdx.x;
  const uint64_t ngroups = (n + kGroup - 1) / kGroup;
  if (g < ngroups) {
    int64_t v[kGroup];
    codec::decode_rt(wds + g * (uint64_t)bits, bits, sgn, v);
    int64_t *dst = tile + threadIdx.x * kPad;
#pragma unroll
    for (int i = 0; i < kGroup; ++i) dst[i] = v[i];
  }
  __syncthreads();
  const uint64_t e0 = g0 * kGroup;
  for (int q = threadIdx.x; q < kTileElems; q += kTileThreads) {
    const uint64_t e = e0 + q;
    if (e < n) st_nt(out + e, tile[q + (q >> 5)]);
  }
}

__global__ void k_gather(const uint32_t *__restrict__ wds, int64_t rows, int64_t cols, int bits,
                         int sgn, const int64_t *__restrict__ ii, const int64_t *__restrict__ jj,
                         int64_t n, int64_t *__restrict__ out, int32_t *bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t i = ii[t], j = jj[t];
  if (i < 0 || i >= rows || j < 0 || j >= cols) {
    out[t] = 0;
    if (bad) atomicOr(bad, 1);
    return;
  }
  out[t] = value_at(wds, (uint64_t)(i * cols + j), bits, sgn);
}

__global__ void k_get_one(const uint32_t *__restrict__ wds, uint64_t e, int bits, int sgn,
                          int64_t *out) {
  *out = value_at(wds, e, bits, sgn);
}

// One elementwise result value; returns overflow in *ovf.
__device__ __forceinline__ int64_t ewise_value(int op, int64_t a, int64_t b, int64_t scalar,
                                               int *ovf) {
  if (op == EW_ADD) {
    const int64_t s = (int64_t)((uint64_t)a + (uint64_t)b);
    *ovf |= ((a ^ s) & (b ^ s)) < 0;
    return s;
  }
  int64_t p;
  *ovf |= __builtin_mul_overflow(a, scalar, &p);
  return p;
}

// Range pass of an elementwise result: one group of 32 elements per lane and
// step, grid-stride over the groups (a bounded grid keeps the per-block
// atomics on the one result slot few).
__global__ __launch_bounds__(256) void k_ewise_range(int op, PackedOperand a, PackedOperand b,
                                                     int64_t scalar, uint64_t n,
                                                     RangeSlot *slot) {
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  int ovf = 0;
  const uint64_t ngroups = (n + kGroup - 1) / kGroup;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups;
       g += (uint64_t)gridDim.x * blockDim.x) {
    int64_t va[kGroup], vb[kGroup];
    codec::decode_rt(a.w + g * (uint64_t)a.bits, a.bits, a.sgn, va);
    if (op == EW_ADD) codec::decode_rt(b.w + g * (uint64_t)b.bits, b.bits, b.sgn, vb);
    const uint64_t e0 = g * kGroup;
#pragma unroll
    for (int i = 0; i < kGroup; ++i) {
      if (e0 + i < n) {
        const int64_t c = ewise_value(op, va[i], op == EW_ADD ? vb[i] : 0, scalar, &ovf);
        lo = c < lo ? c : lo;
        hi = c > hi ? c : hi;
      }
    }
  }
  block_range_commit(lo, hi, ovf, slot);
}

// The range commit for packing grids (one block per 256 groups, so tens of
// thousands of blocks): as block_range_commit, but a block's extreme goes to
// its slot only if it beats the value read there.  A slot only narrows
// (min falls, max rises), so any value read from it is at least as narrow as
// what it holds now, and a block whose extreme does not beat it cannot change
// the result.  With values in random order a slot sees about ln(blocks)
// improvements instead of one atomic per block.
__device__ inline void block_range_fold(int64_t lo, int64_t hi, RangeSlot *slot) {
  __shared__ int64_t s_lo[4], s_hi[4];  // 256 threads: four waves
  lo = wave_min(lo);
  hi = wave_max(hi);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      lo = s_lo[w] < lo ? s_lo[w] : lo;
      hi = s_hi[w] > hi ? s_hi[w] : hi;
    }
    RangeSlot *r = slot + kRangeStride * (blockIdx.x % kRangeSpread);
    const int64_t seen_lo = __hip_atomic_load(&r->vmin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t seen_hi = __hip_atomic_load(&r->vmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (lo < seen_lo) atomicMin((long long *)&r->vmin, (long long)lo);
    if (hi > seen_hi) atomicMax((long long *)&r->vmax, (long long)hi);
  }
}


// Packing pass of an elementwise result: thread t of block x packs the 32
// results of group 256 x + t (zeros past n) at out_bits, through LDS.  With
// RANGE (only for results known to fit int64) it also folds the exact
// extremes of the results below n into slot.
// With DEVW the width comes from res: the block exits when res reports an
// error or when res->bits == skip_bits (the payload already holds the result
// at that width), otherwise it packs at res->bits (at most the launch's width).
template <bool RANGE, bool DEVW = false>
__global__ __launch_bounds__(256) void k_ewise_pack(int op, PackedOperand a, PackedOperand b,
                                                    int64_t scalar, uint64_t n, int out_bits,
                                                    uint32_t *__restrict__ out, uint64_t cap32,
                                                    RangeSlot *slot,
                                                    const ccm_result *res = nullptr,
                                                    int skip_bits = 0) {
  if constexpr (DEVW) {
    if (res->status != CCM_OK || res->bits == skip_bits) return;
    out_bits = res->bits;
    cap32 = cap_words32(n, out_bits);
  }
  extern __shared__ __align__(16) uint32_t s_out[];  // 256 out_bits words
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t ngroups_in = (n + kGroup - 1) / kGroup;
  int64_t vc[kGroup];
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  if (g >= ngroups_in) {
#pragma unroll
    for (int i = 0; i < kGroup; ++i) vc[i] = 0;
  } else {
    int64_t va[kGroup], vb[kGroup];
    codec::decode_rt(a.w + g * (uint64_t)a.bits, a.bits, a.sgn, va);
    if (op == EW_ADD) codec::decode_rt(b.w + g * (uint64_t)b.bits, b.bits, b.sgn, vb);
    const uint64_t e0 = g * kGroup;
    int ovf = 0;
#pragma unroll
    for (int i = 0; i < kGroup; ++i) {
      vc[i] = e0 + i < n ? ewise_value(op, va[i], op == EW_ADD ? vb[i] : 0, scalar, &ovf) : 0;
      if (RANGE && e0 + i < n) {
        lo = vc[i] < lo ? vc[i] : lo;
        hi = vc[i] > hi ? vc[i] : hi;
      }
    }
  }
  // every thread of the block reaches the commit's barriers (no early exit)
  if constexpr (RANGE) block_range_fold(lo, hi, slot);
  codec::encode_rt(vc, out_bits, s_out + threadIdx.x * out_bits, (uint64_t)out_bits);
  __syncthreads();
  store_block_run(s_out, out_bits, out, cap32);
}

// 32-bit variants, taken when the operands' and the result's exact ranges
// (from the headers) all fit the value type VT (int32_t or uint32_t): the sum
// or product is then exact in VT and cannot overflow, so every element costs
// a few 32-bit instructions instead of 64-bit arithmetic with overflow tests.
template <int OP, typename VT>
__device__ __forceinline__ VT ewise_value32(VT a, VT b, VT scalar) {
  return OP == EW_ADD ? (VT)(a + b) : (VT)(a * scalar);
}

// The 32 results of group g (every element below n, or zero past it when
// CHECK: only the last group of a ragged matrix needs the test).
template <int OP, typename VT, bool CHECK>
__device__ __forceinline__ void ewise_group32(const PackedOperand &a, const PackedOperand &b,
                                              VT sc, uint64_t g, uint64_t n, uint32_t *vc) {
  codec::decode32_rt(a.w + g * (uint64_t)a.bits, a.bits, a.sgn, vc);
  if constexpr (OP == EW_ADD) {
    uint32_t vb[kGroup];
    codec::decode32_rt(b.w + g * (uint64_t)b.bits, b.bits, b.sgn, vb);
#pragma unroll
    for (int i = 0; i < kGroup; ++i)
      vc[i] = (uint32_t)ewise_value32<OP, VT>((VT)vc[i], (VT)vb[i], sc);
  } else {
#pragma unroll
    for (int i = 0; i < kGroup; ++i) vc[i] = (uint32_t)ewise_value32<OP, VT>((VT)vc[i], (VT)0, sc);
  }
  if constexpr (CHECK) {
    const uint64_t left = n - g * kGroup;  // < 32 here
#pragma unroll
    for (int i = 0; i < kGroup; ++i) vc[i] = (uint64_t)i < left ? vc[i] : 0u;
  }
}

template <int OP, typename VT>
__global__ __launch_bounds__(256) void k_ewise_range32(PackedOperand a, PackedOperand b,
                                                       int64_t scalar, uint64_t n,
                                                       RangeSlot *slot) {
  VT lo = std::numeric_limits<VT>::max(), hi = std::numeric_limits<VT>::min();
  const VT sc = (VT)scalar;
  const uint64_t nfull = n / kGroup;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (uint64_t g = tid; g < nfull; g += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t vc[kGroup];
    ewise_group32<OP, VT, false>(a, b, sc, g, n, vc);
#pragma unroll
    for (int i = 0; i < kGroup; ++i) {
      lo = (VT)vc[i] < lo ? (VT)vc[i] : lo;
      hi = (VT)vc[i] > hi ? (VT)vc[i] : hi;
    }
  }
  if (tid == 0 && nfull * kGroup < n) {  // the ragged last group
    uint32_t vc[kGroup];
    ewise_group32<OP, VT, true>(a, b, sc, nfull, n, vc);
    for (uint64_t i = 0; i < n - nfull * kGroup; ++i) {
      lo = (VT)vc[i] < lo ? (VT)vc[i] : lo;
      hi = (VT)vc[i] > hi ? (VT)vc[i] : hi;
    }
  }
  block_range_commit((int64_t)lo, (int64_t)hi, 0, slot);
}

// Packing pass, 32-bit results: thread t of block x packs group 256 x + t
// (zeros past n) at out_bits, through LDS (store_block_run).  With RANGE it
// also folds the exact extremes of the results below n into slot, so a
// result packed at a width bounded from the operands' headers learns its
// exact range in the same pass over the operands.
template <int OP, typename VT, bool RANGE, bool DEVW = false>
__global__ __launch_bounds__(256) void k_ewise_pack32(PackedOperand a, PackedOperand b,
                                                      int64_t scalar, uint64_t n, int out_bits,
                                                      uint32_t *__restrict__ out, uint64_t cap32,
                                                      RangeSlot *slot,
                                                      const ccm_result *res = nullptr,
                                                      int skip_bits = 0) {
  if constexpr (DEVW) {  // as in k_ewise_pack
    if (res->status != CCM_OK || res->bits == skip_bits) return;
    out_bits = res->bits;
    cap32 = cap_words32(n, out_bits);
  }
  extern __shared__ __align__(16) uint32_t s_out[];  // 256 out_bits words
  const uint64_t nfull = n / kGroup;
  VT lo = std::numeric_limits<VT>::max(), hi = std::numeric_limits<VT>::min();
  {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t vc[kGroup];
    if (g < nfull) {
      ewise_group32<OP, VT, false>(a, b, (VT)scalar, g, n, vc);
      if constexpr (RANGE) {
        // a whole group: every result counts (no per-element test)
#pragma unroll
        for (int i = 0; i < kGroup; ++i) {
          lo = (VT)vc[i] < lo ? (VT)vc[i] : lo;
          hi = (VT)vc[i] > hi ? (VT)vc[i] : hi;
        }
      }
    } else if (g * kGroup < n) {
      ewise_group32<OP, VT, true>(a, b, (VT)scalar, g, n, vc);
      if constexpr (RANGE) {
        const int left = (int)(n - g * kGroup);
#pragma unroll
        for (int i = 0; i < kGroup; ++i) {
          if (i < left) {
            lo = (VT)vc[i] < lo ? (VT)vc[i] : lo;
            hi = (VT)vc[i] > hi ? (VT)vc[i] : hi;
          }
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < kGroup; ++i) vc[i] = 0;
    }
    codec::encode32_rt(vc, out_bits, s_out + threadIdx.x * out_bits, (uint64_t)out_bits);
  }
  // every thread of the block reaches the commit's barriers (no early exit)
  if constexpr (RANGE) block_range_fold((int64_t)lo, (int64_t)hi, slot);
  __syncthreads();
  store_block_run(s_out, out_bits, out, cap32);
}

// One-pass add of two operands of one width b and one signedness into a
// result of b + 1 bits, the usual case (random operands of one width): the
// same work as k_ewise_pack32<add, int32_t, RANGE> with every width known at
// compile time, so no per-group dispatch on the widths (b <= 15: the sums
// fit int32).
template <int B, bool SGN>
__global__ __launch_bounds__(256) void k_add_same(const uint32_t *__restrict__ aw,
                                                  const uint32_t *__restrict__ bw, uint64_t n,
                                                  uint32_t *__restrict__ out, uint64_t cap32,
                                                  RangeSlot *slot) {
  constexpr int OB = B + 1;
  __shared__ __align__(16) uint32_t s_out[256 * OB];
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nfull = n / kGroup;
  int32_t lo = INT32_MAX, hi = INT32_MIN;
  uint32_t vc[kGroup];
  if (g * kGroup < n) {
    uint32_t wa[B], wb[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      wa[q] = aw[g * B + q];
      wb[q] = bw[g * B + q];
    }
#pragma unroll
    for (int i = 0; i < kGroup; ++i)
      vc[i] = codec::field32<B, SGN>(wa, i) + codec::field32<B, SGN>(wb, i);
    if (g < nfull) {
#pragma unroll
      for (int i = 0; i < kGroup; ++i) {
        lo = (int32_t)vc[i] < lo ? (int32_t)vc[i] : lo;
        hi = (int32_t)vc[i] > hi ? (int32_t)vc[i] : hi;
      }
    } else {
      const int left = (int)(n - g * kGroup);
#pragma unroll
      for (int i = 0; i < kGroup; ++i) {
        vc[i] = i < left ? vc[i] : 0u;
        if (i < left) {
          lo = (int32_t)vc[i] < lo ? (int32_t)vc[i] : lo;
          hi = (int32_t)vc[i] > hi ? (int32_t)vc[i] : hi;
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < kGroup; ++i) vc[i] = 0;
  }
  // every thread of the block reaches the commit's barriers (no early exit)
  block_range_fold((int64_t)lo, (int64_t)hi, slot);
  codec::encode32<OB>(vc, s_out + threadIdx.x * OB, (uint64_t)OB);
  __syncthreads();
  store_block_run(s_out, OB, out, cap32);
}

// One wave folds the spread range slots into a ccm_result.
__global__ __launch_bounds__(64) void k_result_finalize(const RangeSlot *slot, int64_t rows,
                                                        int64_t cols, int check_flag,
                                                        ccm_result *res) {
  const RangeSlot r = slot[kRangeStride * threadIdx.x];  // 64 lanes, 64 slots
  const int64_t lo = wave_min(r.vmin), hi = wave_max(r.vmax);
  const int flag = __any(r.flag) ? 1 : 0;
  if (threadIdx.x == 0) {
    ccm_result o = {};
    o.rows = rows;
    o.cols = cols;
    o.vmin = lo;
    o.vmax = hi;
    if (check_flag && flag) {
      o.status = CCM_E_OVERFLOW;
    } else {
      int b = 0, sg = 0;
      width_of(lo, hi, &b, &sg);
      o.bits = b;
      o.is_signed = sg;
      o.words = (uint64_t)rows * (uint64_t)cols * (uint64_t)b / 64u + 1u;
      o.status = CCM_OK;
    }
    *res = o;
  }
}

__global__ void k_fill_i64(int64_t *p, uint64_t n, int64_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) p[e] = v;
}

// ---- synthetic data -------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_fill_uniform(T *d, uint64_t n, int64_t lo, uint64_t span,
                                                      uint64_t seed, uint64_t sid,
                                                      uint64_t start) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
    d[e] = (T)uniform_at(seed, sid, start + e, lo, span);
}

__global__ __launch_bounds__(256) void k_gen_range(uint64_t n, int64_t lo, uint64_t span,
                                                   uint64_t seed, uint64_t sid,
                                                   RangeSlot *slot) {
  int64_t mn = INT64_MAX, mx = INT64_MIN;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const int64_t v = uniform_at(seed, sid, e, lo, span);
    mn = v < mn ? v : mn;
    mx = v > mx ? v : mx;
  }
  block_range_commit(mn, mx, 0, slot);
}

__global__ __launch_bounds__(256) void k_gen_pack(uint64_t n, int64_t lo, uint64_t span,
                                                  uint64_t seed, uint64_t sid, int bits,
                                                  uint32_t *__restrict__ out, uint64_t cap32,
                                                  uint64_t ngroups_out) {
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups_out) return;
  const uint64_t e0 = g * kGroup;
  int64_t v[kGroup];
#pragma unroll
  for (int i = 0; i < kGroup; ++i) {
    const uint64_t e = e0 + i;
    v[i] = e < n ? uniform_at(seed, sid, e, lo, span) : 0;
  }
  const uint64_t w0 = g * (uint64_t)bits;
  codec::encode_rt(v, bits, out + w0, cap32 - w0);
}

inline unsigned grid_for(uint64_t work, unsigned per_block, unsigned cap = 1u << 20) {
  uint64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_range_init(RangeSlot *slot, hipStream_t s) {
  k_range_init<<<1, kRangeSpread, 0, s>>>(slot);
  return hipGetLastError();
}

hipError_t launch_range_dense(const void *dense, int dtype, uint64_t n, RangeSlot *slot,
                              hipStream_t s) {
  const unsigned grid = grid_for(n, 256 * 16, 4096);
  const int al = ((uintptr_t)dense % 16) == 0;
  if (dtype == CCM_I64)
    k_range_dense<int64_t><<<grid, 256, 0, s>>>((const int64_t *)dense, n, slot, al);
  else
    k_range_dense<int32_t><<<grid, 256, 0, s>>>((const int32_t *)dense, n, slot, al);
  return hipGetLastError();
}

hipError_t launch_compress(const void *dense, int dtype, uint64_t n, int bits, uint32_t *out,
                           uint64_t cap32, hipStream_t s) {
  const uint64_t ngroups = (cap32 + bits - 1) / bits;
  const unsigned grid = grid_for(ngroups, kTileThreads, 0x7fffffffu);
  const int al = ((uintptr_t)dense % 16) == 0;
  if (dtype == CCM_I64)
    k_compress<int64_t><<<grid, kTileThreads, 0, s>>>((const int64_t *)dense, n, bits, out,
                                                       cap32, ngroups, al);
  else
    k_compress<int32_t><<<grid, kTileThreads, 0, s>>>((const int32_t *)dense, n, bits, out,
                                                       cap32, ngroups, al);
  return hipGetLastError();
}

hipError_t launch_decompress(const uint32_t *w, uint64_t n, int bits, int sgn, int64_t *out,
                             hipStream_t s) {
  const uint64_t ngroups = (n + kGroup - 1) / kGroup;
  k_decompress<<<grid_for(ngroups, kTileThreads, 0x7fffffffu), kTileThreads, 0, s>>>(
      w, n, bits, sgn, out);
  return hipGetLastError();
}

hipError_t launch_gather(const uint32_t *w, int64_t rows, int64_t cols, int bits, int sgn,
                         const int64_t *ii, const int64_t *jj, int64_t n, int64_t *out,
                         int32_t *bad, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_gather<<<grid_for((uint64_t)n, 256, 0x7fffffffu), 256, 0, s>>>(w, rows, cols, bits, sgn, ii,
                                                                   jj, n, out, bad);
  return hipGetLastError();
}

hipError_t launch_get_one(const uint32_t *w, uint64_t e, int bits, int sgn, int64_t *out,
                          hipStream_t s) {
  k_get_one<<<1, 1, 0, s>>>(w, e, bits, sgn, out);
  return hipGetLastError();
}

hipError_t launch_ewise_range(int op, PackedOperand a, PackedOperand b, int64_t scalar,
                              uint64_t n, int vclass, RangeSlot *slot, hipStream_t s) {
  const uint64_t ngroups = (n + kGroup - 1) / kGroup;
  const unsigned grid = grid_for(ngroups, 256, 2048);
  if (vclass == EW_I32 && op == EW_ADD)
    k_ewise_range32<EW_ADD, int32_t><<<grid, 256, 0, s>>>(a, b, scalar, n, slot);
  else if (vclass == EW_I32)
    k_ewise_range32<EW_SCALE, int32_t><<<grid, 256, 0, s>>>(a, b, scalar, n, slot);
  else if (vclass == EW_U32 && op == EW_ADD)
    k_ewise_range32<EW_ADD, uint32_t><<<grid, 256, 0, s>>>(a, b, scalar, n, slot);
  else if (vclass == EW_U32)
    k_ewise_range32<EW_SCALE, uint32_t><<<grid, 256, 0, s>>>(a, b, scalar, n, slot);
  else
    k_ewise_range<<<grid, 256, 0, s>>>(op, a, b, scalar, n, slot);
  return hipGetLastError();
}

hipError_t launch_ewise_pack(int op, PackedOperand a, PackedOperand b, int64_t scalar,
                             uint64_t n, int vclass, int out_bits, uint32_t *out, uint64_t cap32,
                             hipStream_t s) {
  const uint64_t ngroups_out = (cap32 + out_bits - 1) / out_bits;
  const unsigned grid = grid_for(ngroups_out, 256, 0x7fffffffu);
  const size_t lds32 = (size_t)256 * (size_t)(out_bits <= 32 ? out_bits : 32) * 4u;
  if (vclass == EW_I32 && out_bits <= 32 && op == EW_ADD)
    k_ewise_pack32<EW_ADD, int32_t, false>
        <<<grid, 256, lds32, s>>>(a, b, scalar, n, out_bits, out, cap32, nullptr);
  else if (vclass == EW_I32 && out_bits <= 32)
    k_ewise_pack32<EW_SCALE, int32_t, false>
        <<<grid, 256, lds32, s>>>(a, b, scalar, n, out_bits, out, cap32, nullptr);
  else if (vclass == EW_U32 && out_bits <= 32 && op == EW_ADD)
    k_ewise_pack32<EW_ADD, uint32_t, false>
        <<<grid, 256, lds32, s>>>(a, b, scalar, n, out_bits, out, cap32, nullptr);
  else if (vclass == EW_U32 && out_bits <= 32)
    k_ewise_pack32<EW_SCALE, uint32_t, false>
        <<<grid, 256, lds32, s>>>(a, b, scalar, n, out_bits, out, cap32, nullptr);
  else
    k_ewise_pack<false><<<grid, 256, (size_t)256 * (size_t)out_bits * 4u, s>>>(
        op, a, b, scalar, n, out_bits, out, cap32, nullptr);
  return hipGetLastError();
}

hipError_t launch_add_pack_range(PackedOperand a, PackedOperand b, uint64_t n, int vclass,
                                 int out_bits, uint32_t *out, uint64_t cap32, RangeSlot *slot,
                                 hipStream_t s) {
  if (out_bits < 1 || out_bits > 64 || (vclass != EW_I64 && out_bits > 32))
    return hipErrorInvalidValue;
  const uint64_t ngroups_out = (cap32 + out_bits - 1) / out_bits;
  const unsigned grid = grid_for(ngroups_out, 256, 0x7fffffffu);
  const size_t lds = (size_t)256 * (size_t)out_bits * 4u;
  if (a.bits == b.bits && a.sgn == b.sgn && out_bits == a.bits + 1 && a.bits <= 15) {
    switch (a.bits * 2 + (a.sgn ? 1 : 0)) {
#define CCM_ADD_SAME(bb)                                                                       \
  case 2 * bb:                                                                                 \
    k_add_same<bb, false><<<grid, 256, 0, s>>>(a.w, b.w, n, out, cap32, slot);                 \
    break;                                                                                     \
  case 2 * bb + 1:                                                                             \
    k_add_same<bb, true><<<grid, 256, 0, s>>>(a.w, b.w, n, out, cap32, slot);                  \
    break;
      CCM_ADD_SAME(1) CCM_ADD_SAME(2) CCM_ADD_SAME(3) CCM_ADD_SAME(4) CCM_ADD_SAME(5)
      CCM_ADD_SAME(6) CCM_ADD_SAME(7) CCM_ADD_SAME(8) CCM_ADD_SAME(9) CCM_ADD_SAME(10)
      CCM_ADD_SAME(11) CCM_ADD_SAME(12) CCM_ADD_SAME(13) CCM_ADD_SAME(14) CCM_ADD_SAME(15)
#undef CCM_ADD_SAME
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (vclass == EW_I32)
    k_ewise_pack32<EW_ADD, int32_t, true>
        <<<grid, 256, lds, s>>>(a, b, 0, n, out_bits, out, cap32, slot);
  else if (vclass == EW_U32)
    k_ewise_pack32<EW_ADD, uint32_t, true>
        <<<grid, 256, lds, s>>>(a, b, 0, n, out_bits, out, cap32, slot);
  else {
    // 64 KB of output staging at 64 bits, next to the range commit's static LDS
    static const bool lds_set =
        hipFuncSetAttribute(reinterpret_cast<const void *>(k_ewise_pack<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 256 * 64 * 4) ==
        hipSuccess;
    (void)lds_set;
    k_ewise_pack<true><<<grid, 256, lds, s>>>(EW_ADD, a, b, 0, n, out_bits, out, cap32, slot);
  }
  return hipGetLastError();
}

// Groups a packing grid must cover for every width up to max_bits (the
// capacity's guard words make narrow widths need the most groups).
static uint64_t groups_upto(uint64_t n, int max_bits) {
  uint64_t g = 0;
  for (int b = 1; b <= max_bits; ++b) {
    const uint64_t c = (cap_words32(n, b) + b - 1) / b;
    g = c > g ? c : g;
  }
  return g;
}

hipError_t launch_result_finalize(const RangeSlot *slot, int64_t rows, int64_t cols,
                                  int check_flag, ccm_result *res, hipStream_t s) {
  k_result_finalize<<<1, kRangeSpread, 0, s>>>(slot, rows, cols, check_flag, res);
  return hipGetLastError();
}

hipError_t launch_compress_dev(const void *dense, int dtype, uint64_t n, int max_bits,
                               uint32_t *out, const ccm_result *res, hipStream_t s) {
  if (max_bits < 1 || max_bits > 64) return hipErrorInvalidValue;
  const uint64_t ngroups = groups_upto(n, max_bits);
  const unsigned grid = grid_for(ngroups, kTileThreads, 0x7fffffffu);
  const int al = ((uintptr_t)dense % 16) == 0;
  if (dtype == CCM_I64)
    k_compress<int64_t, true><<<grid, kTileThreads, 0, s>>>((const int64_t *)dense, n, 0, out, 0,
                                                             0, al, res);
  else
    k_compress<int32_t, true><<<grid, kTileThreads, 0, s>>>((const int32_t *)dense, n, 0, out, 0,
                                                             0, al, res);
  return hipGetLastError();
}

hipError_t launch_ewise_pack_dev(int op, PackedOperand a, PackedOperand b, int64_t scalar,
                                 uint64_t n, int vclass, int max_bits, int skip_bits,
                                 uint32_t *out, const ccm_result *res, hipStream_t s) {
  if (max_bits < 1 || max_bits > 64 || (vclass != EW_I64 && max_bits > 32))
    return hipErrorInvalidValue;
  const unsigned grid = grid_for(groups_upto(n, max_bits), 256, 0x7fffffffu);
  const size_t lds = (size_t)256 * (size_t)max_bits * 4u;
  if (vclass == EW_I32 && op == EW_ADD)
    k_ewise_pack32<EW_ADD, int32_t, false, true>
        <<<grid, 256, lds, s>>>(a, b, scalar, n, 0, out, 0, nullptr, res, skip_bits);
  else if (vclass == EW_I32)
    k_ewise_pack32<EW_SCALE, int32_t, false, true>
        <<<grid, 256, lds, s>>>(a, b, scalar, n, 0, out, 0, nullptr, res, skip_bits);
  else if (vclass == EW_U32 && op == EW_ADD)
    k_ewise_pack32<EW_ADD, uint32_t, false, true>
        <<<grid, 256, lds, s>>>(a, b, scalar, n, 0, out, 0, nullptr, res, skip_bits);
  else if (vclass == EW_U32)
    k_ewise_pack32<EW_SCALE, uint32_t, false, true>
        <<<grid, 256, lds, s>>>(a, b, scalar, n, 0, out, 0, nullptr, res, skip_bits);
  else {
    static const bool lds_set =
        hipFuncSetAttribute(reinterpret_cast<const void *>(k_ewise_pack<false, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 256 * 64 * 4) ==
        hipSuccess;
    (void)lds_set;
    k_ewise_pack<false, true><<<grid, 256, lds, s>>>(op, a, b, scalar, n, 0, out, 0, nullptr, res,
                                                     skip_bits);
  }
  return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t *p, uint64_t n, int64_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_fill_i64<<<grid_for(n, 256, 4096), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_uniform(void *dense, int dtype, uint64_t n, int64_t lo, uint64_t span,
                               uint64_t seed, uint64_t stream_id, uint64_t start,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned grid = grid_for(n, 256 * 8, 16384);
  if (dtype == CCM_I64)
    k_fill_uniform<int64_t><<<grid, 256, 0, s>>>((int64_t *)dense, n, lo, span, seed, stream_id,
                                                  start);
  else
    k_fill_uniform<int32_t><<<grid, 256, 0, s>>>((int32_t *)dense, n, lo, span, seed, stream_id,
                                                  start);
  return hipGetLastError();
}

hipError_t launch_gen_range(uint64_t n, int64_t lo, uint64_t span, uint64_t seed,
                            uint64_t stream_id, RangeSlot *slot, hipStream_t s) {
  k_gen_range<<<grid_for(n, 256 * 16, 2048), 256, 0, s>>>(n, lo, span, seed, stream_id, slot);
  return hipGetLastError();
}

hipError_t launch_gen_pack(uint64_t n, int64_t lo, uint64_t span, uint64_t seed,
                           uint64_t stream_id, int bits, uint32_t *out, uint64_t cap32,
                           hipStream_t s) {
  const uint64_t ngroups_out = (cap32 + bits - 1) / bits;
  k_gen_pack<<<grid_for(ngroups_out, 256, 0x7fffffffu), 256, 0, s>>>(
      n, lo, span, seed, stream_id, bits, out, cap32, ngroups_out);
  return hipGetLastError();
}

}  // namespace ccm
