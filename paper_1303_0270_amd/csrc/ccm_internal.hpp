// Internal declarations of libccm: device helpers shared by the kernels and
// the launchers the C ABI layer (api.cpp) calls.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ccm.h"

namespace ccm {

// ---------------------------------------------------------------------------
// Layout constants
// ---------------------------------------------------------------------------

// A "group" is 32 consecutive elements of the row-major stream.  Group g
// occupies stream bits [32*g*b, 32*(g+1)*b), i.e. exactly 32-bit words
// [g*b, (g+1)*b): every group starts on a word boundary whatever b is, so a
// lane that owns a group decodes it with fixed (compile-time) bit offsets.
constexpr int kGroup = 32;

// Payload capacity in 32-bit words: every group that holds an element (so a
// writer may write whole groups), plus b + 4 guard words (a reader may fetch
// one group-length past a field that starts in the last group, and three
// words around any field), rounded up to 256 bytes.
__host__ __device__ inline uint64_t cap_words32(uint64_t n, int bits) {
  uint64_t full = (n * (uint64_t)bits + 31u) / 32u;
  uint64_t need = full + (uint64_t)bits + 4u;
  return (need + 63u) / 64u * 64u;
}

__host__ __device__ inline uint64_t mask64(int bits) {
  return bits >= 64 ? ~0ull : ((1ull << bits) - 1ull);
}

__host__ __device__ inline uint32_t mask32(int bits) {
  return bits >= 32 ? ~0u : ((1u << bits) - 1u);
}

// Returns v unchanged (no instruction) but hides how it was computed from the
// optimizer.  Used on sign-extended bit-field extracts (v_bfe_i32): when such a
// value feeds a 64-bit multiply-accumulate chain, the compiler has been seen
// to drop the sign(a)*x correction term of the 64-bit product, as if the
// extract were non-negative.
__device__ __forceinline__ int32_t opaque_i32(int32_t v) {
  asm("" : "+v"(v));
  return v;
}

// The width rule (Eq. 1 for a non-negative range; otherwise the smallest
// two's complement width holding [vmin, vmax]), for device code that decides
// a result's width from a range it has just reduced.  vmin <= vmax.
__host__ __device__ inline int bitlen_u64(uint64_t u) {
  int L = 0;
  while (L < 64 && (u >> L) != 0) ++L;
  return L;
}
__host__ __device__ inline void width_of(int64_t vmin, int64_t vmax, int *bits, int *sgn) {
  if (vmin >= 0) {
    *sgn = 0;
    *bits = vmax <= 1 ? 1 : bitlen_u64((uint64_t)vmax);
  } else {
    const int lo = bitlen_u64(~(uint64_t)vmin);
    const int hi = vmax > 0 ? bitlen_u64((uint64_t)vmax) : 0;
    *sgn = 1;
    *bits = 1 + (lo > hi ? lo : hi);
  }
}

// Two's-complement sign extension of the low `bits` bits.
__host__ __device__ inline int64_t sext64(uint64_t u, int bits) {
  const int s = 64 - bits;
  return (int64_t)(u << s) >> s;
}

// ---------------------------------------------------------------------------
// Runtime-width bit reader / writer for one lane's group.  All lanes of a wave
// process groups with the same bit phase, so `avail` / `used` and every branch
// on them are wave-uniform: the refill and flush points cost no divergence.
// ---------------------------------------------------------------------------

struct BitReader {
  const uint32_t *p;
  uint64_t buf;
  int avail;

  __device__ explicit BitReader(const uint32_t *ptr) : p(ptr), buf(0), avail(0) {}

  // next nb bits (1 <= nb <= 32)
  __device__ __forceinline__ uint32_t take(int nb) {
    if (avail < nb) {
      buf |= (uint64_t)(*p) << avail;
      ++p;
      avail += 32;
    }
    const uint32_t v = (uint32_t)buf & mask32(nb);
    buf >>= nb;
    avail -= nb;
    return v;
  }

  // next field of `bits` bits (1..64), zero-extended
  __device__ __forceinline__ uint64_t field(int bits) {
    if (bits <= 32) return take(bits);
    const uint64_t lo = take(32);
    return lo | ((uint64_t)take(bits - 32) << 32);
  }
};

struct BitWriter {
  uint32_t *p;
  uint64_t idx, cap;  // next word index, capacity in words (stores past it are dropped)
  uint64_t buf;
  int used;

  __device__ BitWriter(uint32_t *base, uint64_t first_word, uint64_t cap_words)
      : p(base), idx(first_word), cap(cap_words), buf(0), used(0) {}

  __device__ __forceinline__ void put(uint32_t v, int nb) {
    buf |= (uint64_t)(v & mask32(nb)) << used;
    used += nb;
    if (used >= 32) {
      if (idx < cap) p[idx] = (uint32_t)buf;
      ++idx;
      buf >>= 32;
      used -= 32;
    }
  }

  __device__ __forceinline__ void field(uint64_t u, int bits) {
    if (bits <= 32) {
      put((uint32_t)u, bits);
    } else {
      put((uint32_t)u, 32);
      put((uint32_t)(u >> 32), bits - 32);
    }
  }
};

// Field e of a stream of `bits`-bit fields (random access; reads words
// e*bits/32 .. +2, all inside the payload capacity).
__device__ __forceinline__ uint64_t field_at(const uint32_t *w, uint64_t e, int bits) {
  const uint64_t p = e * (uint64_t)bits;
  const uint64_t k = p >> 5;
  const int off = (int)(p & 31u);
  uint64_t v = ((uint64_t)w[k] | ((uint64_t)w[k + 1] << 32)) >> off;
  if (off + bits > 64) v |= (uint64_t)w[k + 2] << (64 - off);
  return v & mask64(bits);
}

__device__ __forceinline__ int64_t value_at(const uint32_t *w, uint64_t e, int bits, int sgn) {
  const uint64_t u = field_at(w, e, bits);
  return sgn ? sext64(u, bits) : (int64_t)u;
}

// ---------------------------------------------------------------------------
// Wave and block reductions (64-lane wavefronts)
// ---------------------------------------------------------------------------

// Sum over the wave modulo 2^64.
// One 64-bit add of a DPP-permuted copy (CTRL: a GFX9 DPP control word).
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_add64(uint64_t v) {
  const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  const uint32_t lo2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, CTRL, 0xf, 0xf, true);
  const uint32_t hi2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi, CTRL, 0xf, 0xf, true);
  const uint32_t s = lo + lo2;
  return ((uint64_t)(hi + hi2 + (s < lo ? 1u : 0u)) << 32) | s;
}

// Sum over the 64 lanes of a wave, mod 2^64; every lane must be active.  Four
// DPP steps leave each 16-lane row's sum in all of its lanes (quad swaps, then
// the half-row and row mirrors); the four row sums are read out as scalars.
// Stores of large outputs that no kernel reads again soon (packed payloads,
// decompressed matrices): marked nontemporal, so the caches do not keep them
// dirty.  Dirty lines left by one kernel are written back while the next one
// reads, at its expense (measured: a k = 3 matvec right after a plain 1 GiB
// write takes 50 us, after the same write made nontemporal 28 us, as after a
// read).
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_nt(uint32_t *p, uint32_t v) {
  __builtin_nontemporal_store(v, p);
}
__device__ __forceinline__ void st_nt(int64_t *p, int64_t v) {
  __builtin_nontemporal_store(v, p);
}
__device__ __forceinline__ void st_nt4(uint32_t *p, uint32_t a, uint32_t b, uint32_t c,
                                       uint32_t d) {
  const u32x4_t t = {a, b, c, d};
  __builtin_nontemporal_store(t, reinterpret_cast<u32x4_t *>(p));
}

// Writes a block's output run: thread t of block x encoded group
// blockDim.x x + t into s_out[t out_bits ..), and the block's groups are
// consecutive, so its words are out[blockDim.x x out_bits ..) contiguous:
// 16-byte nontemporal stores, words at or past cap32 dropped.  (A thread
// storing its own group directly issues out_bits stores of 64 lanes each at
// a stride of out_bits words, which nontemporal stores turn into partial-line
// writes: compress took 1.48 ms per 16384^2 matrix that way against 0.87 ms
// with plain stores.)
__device__ __forceinline__ void store_block_run(const uint32_t *s_out, int out_bits,
                                                uint32_t *__restrict__ out, uint64_t cap32) {
  const uint64_t base = (uint64_t)blockIdx.x * blockDim.x * (uint64_t)out_bits;  // a word index
  if (base >= cap32) return;
  const uint64_t left = cap32 - base;
  const uint64_t run = (uint64_t)blockDim.x * (uint64_t)out_bits;
  const uint32_t nw = (uint32_t)(left < run ? left : run);
  uint4 *o4 = reinterpret_cast<uint4 *>(out + base);  // 1024 out_bits bytes per block: aligned
  const uint4 *l4 = reinterpret_cast<const uint4 *>(s_out);
  for (uint32_t q = threadIdx.x; q < nw / 4; q += blockDim.x) {
    const uint4 t = l4[q];
    st_nt4(reinterpret_cast<uint32_t *>(o4 + q), t.x, t.y, t.z, t.w);
  }
  for (uint32_t q = (nw & ~3u) + threadIdx.x; q < nw; q += blockDim.x)
    st_nt(out + base + q, s_out[q]);
}

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
  uint64_t u = (uint64_t)v;
  u = dpp_add64<0xB1>(u);   // quad_perm [1,0,3,2]
  u = dpp_add64<0x4E>(u);   // quad_perm [2,3,0,1]
  u = dpp_add64<0x141>(u);  // row_half_mirror
  u = dpp_add64<0x140>(u);  // row_mirror
  const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
  uint64_t t = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    t += ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(hi, 16 * r) << 32) |
         (uint32_t)__builtin_amdgcn_readlane(lo, 16 * r);
  return (int64_t)t;
}

// int32 sum over the 64 lanes of a wave (same steps as wave_sum); the caller
// guarantees the total fits int32.
__device__ __forceinline__ int32_t wave_sum32(int32_t v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);  // row_mirror
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
         __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

__device__ __forceinline__ int64_t wave_min(int64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const int64_t o = __shfl_xor(v, m, 64);
    v = o < v ? o : v;
  }
  return v;
}

__device__ __forceinline__ int64_t wave_max(int64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const int64_t o = __shfl_xor(v, m, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Reduction target of the range passes: exact min, max and an error flag
// (32 bytes, so kRangeStride of them make one 128-byte line).
struct alignas(32) RangeSlot {
  int64_t vmin;
  int64_t vmax;
  int32_t flag;
  int32_t pad;
};

// A range result lives in kRangeSpread slots, one 128-byte line apart: block
// i folds into slot i % kRangeSpread, so a few thousand blocks do not
// serialize on one address (same-address device atomics cost tens of ns
// each); the host folds the slots after the copy back.
constexpr int kRangeSpread = 64;
constexpr int kRangeStride = 4;  // RangeSlot units per slot (128 bytes)
constexpr size_t kRangeBytes = sizeof(RangeSlot) * kRangeStride * kRangeSpread;
static_assert(sizeof(RangeSlot) * kRangeStride == 128, "one range slot per 128-byte line");

// Spread 64-bit sums (pairs), laid out like the range slots: pair i at
// uint64 offset 2 * kSumStride * i (128 bytes apart).
constexpr int kSumStride = 8;
constexpr size_t kSumBytes = sizeof(uint64_t) * 2 * kSumStride * kRangeSpread;

// Block-wide (min, max, flag) folded into the block's slot of a spread range
// result with one atomic each per block.  Every thread of the block must call
// it.
__device__ inline void block_range_commit(int64_t lo, int64_t hi, int flag, RangeSlot *slot) {
  __shared__ int64_t s_lo[16], s_hi[16];
  __shared__ int s_flag[16];
  lo = wave_min(lo);
  hi = wave_max(hi);
  const int wf = __any(flag) ? 1 : 0;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
    s_flag[wave] = wf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    slot += kRangeStride * ((blockIdx.x + blockIdx.y * gridDim.x) % kRangeSpread);
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 1; w < nw; ++w) {
      lo = s_lo[w] < lo ? s_lo[w] : lo;
      hi = s_hi[w] > hi ? s_hi[w] : hi;
    }
    int f = 0;
    for (int w = 0; w < nw; ++w) f |= s_flag[w];
    atomicMin((long long *)&slot->vmin, (long long)lo);
    atomicMax((long long *)&slot->vmax, (long long)hi);
    if (f) atomicOr(&slot->flag, 1);
  }
}

// ---------------------------------------------------------------------------
// Launchers (each returns the launch's hipError_t)
// ---------------------------------------------------------------------------

hipError_t launch_range_init(RangeSlot *slot, hipStream_t s);
hipError_t launch_range_dense(const void *dense, int dtype, uint64_t n, RangeSlot *slot,
                              hipStream_t s);
hipError_t launch_compress(const void *dense, int dtype, uint64_t n, int bits, uint32_t *out,
                           uint64_t cap32, hipStream_t s);
hipError_t launch_decompress(const uint32_t *w, uint64_t n, int bits, int sgn, int64_t *out,
                             hipStream_t s);
hipError_t launch_get_one(const uint32_t *w, uint64_t e, int bits, int sgn, int64_t *out,
                          hipStream_t s);
hipError_t launch_gather(const uint32_t *w, int64_t rows, int64_t cols, int bits, int sgn,
                         const int64_t *ii, const int64_t *jj, int64_t n, int64_t *out,
                         int32_t *bad, hipStream_t s);

// Elementwise ops on two packed operands (b may be null for unary ops).
enum EwiseOp { EW_ADD = 0, EW_SCALE = 1 };
// Value class of an elementwise pass: every operand value and every result
// fits int32 / uint32 (exact 32-bit arithmetic), or general int64 with
// overflow detection.
enum EwiseClass { EW_I64 = 0, EW_I32 = 1, EW_U32 = 2 };
struct PackedOperand {
  const uint32_t *w;
  int bits;
  int sgn;
};
hipError_t launch_ewise_range(int op, PackedOperand a, PackedOperand b, int64_t scalar,
                              uint64_t n, int vclass, RangeSlot *slot, hipStream_t s);
hipError_t launch_ewise_pack(int op, PackedOperand a, PackedOperand b, int64_t scalar,
                             uint64_t n, int vclass, int out_bits, uint32_t *out, uint64_t cap32,
                             hipStream_t s);
// A + B packed at out_bits (at most 32 for the 32-bit classes) while the
// exact extremes of the sums fold into slot, which the caller initialised.
// The caller guarantees that no sum leaves int64 (the headers bound them).
hipError_t launch_add_pack_range(PackedOperand a, PackedOperand b, uint64_t n, int vclass,
                                 int out_bits, uint32_t *out, uint64_t cap32, RangeSlot *slot,
                                 hipStream_t s);

hipError_t launch_fill_i64(int64_t *p, uint64_t n, int64_t v, hipStream_t s);
// floats in fixed point: largest |v| (as the bit pattern of a double) into
// slot's vmax; q = RNE(v 2^f) as int64 or int32 (q null: not written) with
// q's range in slot (flag:
// NaN or infinity; vmax INT64_MAX: some |v 2^f| >= 2^62 or q outside the
// output type); out = q 2^-f (slots initialised by launch_range_init)
hipError_t launch_float_absmax(const void *v, int dtype, uint64_t n, RangeSlot *slot,
                               hipStream_t s);
hipError_t launch_quantize(const void *v, int dtype, uint64_t n, int frac_bits, void *q,
                           int qdtype, RangeSlot *slot, hipStream_t s);
hipError_t launch_dequantize(const int64_t *q, uint64_t n, int frac_bits, int dtype, void *out,
                             hipStream_t s);
// packs RNE(v 2^f) at `bits` straight from n floats (values checked before)
hipError_t launch_compress_fx(const void *v, int dtype, uint64_t n, int frac_bits, int bits,
                              uint32_t *out, uint64_t cap32, hipStream_t s);

// ---------------------------------------------------------------------------
// Results whose width stays on the device.  A reduced range (the spread
// slots) is folded on the device into a ccm_result (exact extremes, width,
// word count, status); the packing launchers below read the width from it.
// ---------------------------------------------------------------------------

// res <- the folded range of slot as a rows x cols result; with check_flag a
// set overflow flag gives status CCM_E_OVERFLOW (and bits 0).
hipError_t launch_result_finalize(const RangeSlot *slot, int64_t rows, int64_t cols,
                                  int check_flag, ccm_result *res, hipStream_t s);
// Packs dense at res->bits (skipped when res->status != CCM_OK); the grid is
// sized for any width up to max_bits.
hipError_t launch_compress_dev(const void *dense, int dtype, uint64_t n, int max_bits,
                               uint32_t *out, const ccm_result *res, hipStream_t s);
// Elementwise packing at res->bits, skipped when res->status != CCM_OK or
// res->bits == skip_bits (the payload already holds that width); max_bits
// bounds res->bits.
hipError_t launch_ewise_pack_dev(int op, PackedOperand a, PackedOperand b, int64_t scalar,
                                 uint64_t n, int vclass, int max_bits, int skip_bits,
                                 uint32_t *out, const ccm_result *res, hipStream_t s);

// matvec: y = A x.  x dtype CCM_I32 / CCM_I64.
hipError_t launch_matvec(const uint32_t *w, int64_t rows, int64_t cols, int bits, int sgn,
                         const void *x, int xdtype, int64_t *y, hipStream_t s);

// y = A^T x over a row-major stream (x: rows values, y: cols).  Rows are
// split over at most kMaxSplitsT blocks per column panel; with part (device,
// part_words >= kMaxSplitsT * cols int64) the splits store partial column
// sums there and a second kernel adds them into y, otherwise they add into a
// zeroed y with atomics.
constexpr int kMaxSplitsT = 32;
hipError_t launch_matvec_t(const uint32_t *w, int64_t rows, int64_t cols, int bits, int sgn,
                           const void *x, int xdtype, int64_t *y, int64_t *part,
                           uint64_t part_words, hipStream_t s);
// The library's own partial-sum buffer for y = A^T x (columns up to
// kNoAllocColsT): its device address on the current device and its size in
// int64 words.
constexpr int64_t kNoAllocColsT = 65536;
hipError_t static_matvec_t_scratch(int64_t **ptr, uint64_t *words);
// y[c] = sum over s < splits of part[s * cols + c] (mod 2^64).
hipError_t launch_sum_splits(const int64_t *part, int64_t splits, int64_t cols, int64_t *y,
                             hipStream_t s);

// Packs a dense row-major rows x cols matrix unravelled by column (the
// row-major stream of its transpose) into out[0, cap32).
hipError_t launch_compress_cm(const void *dense, int dtype, int64_t rows, int64_t cols,
                              int bits, uint32_t *out, uint64_t cap32, hipStream_t s);

// matmul into dense scratch (int32 if out32 else int64) with its range.
hipError_t launch_matmul(const uint32_t *aw, int abits, int asgn, const uint32_t *bw,
                         int bbits, int bsgn, int64_t M, int64_t K, int64_t N, int use_i8,
                         int out32, void *scratch, RangeSlot *slot, hipStream_t s);

// int8 MFMA matmul (operands whose values fit int8, K*max|A|*max|B| < 2^31):
// The int8 MFMA path decodes A (M x K) and B^T (N x K) into int8 scratch,
// K padded to a multiple of 128: matmul_i8_bytes bytes.
uint64_t matmul_i8_bytes(int64_t M, int64_t K, int64_t N);
hipError_t launch_matmul_i8(const uint32_t *aw, int abits, int asgn, const uint32_t *bw,
                            int bbits, int bsgn, int64_t M, int64_t K, int64_t N, int out32,
                            void *scratch_c, int8_t *scratch_i8, RangeSlot *slot, hipStream_t s);

// Method 2 (variable length blocks): stream, index and shape of one matrix.
struct VlbView {
  const uint32_t *w;        // the stream as 32-bit words
  const uint64_t *row_bit;  // rows + 1 row start bits
  const uint32_t *grp;      // rows x ngr group offsets within the row
  int64_t rows, cols, ngr;  // ngr = ceil(cols / 32)
  int k;                    // length-field width
  int bmax;                 // largest element width
  int sgn;
  uint64_t gmax;            // bits of the longest group
  uint64_t nbits;           // stream bits
};
uint64_t vlb_ngr(int64_t cols);
// pass 1: grp[i][g] = bits of group g of row i (sum of k + b_e); the largest
// folds into slot's vmax (slot initialised by launch_range_init)
hipError_t launch_vlb_sizes(const void *dense, int dtype, int64_t rows, int64_t cols, int k,
                            int sgn, uint32_t *grp, RangeSlot *slot, hipStream_t s);
// pass 2: counts -> offsets within rows, row starts and the total in row_bit
hipError_t launch_vlb_scan(int64_t rows, int64_t cols, uint32_t *grp, uint64_t *row_bit,
                           hipStream_t s);
// pass 3: the stream (zeroes cap32 words first)
hipError_t launch_vlb_pack(const void *dense, int dtype, const VlbView &a, uint32_t *out,
                           uint64_t cap32, uint64_t nbits, hipStream_t s);
hipError_t launch_vlb_decode(const VlbView &a, int64_t *out, hipStream_t s);
hipError_t launch_vlb_get(const VlbView &a, int64_t i, int64_t j, int64_t *out, hipStream_t s);
hipError_t launch_vlb_matvec(const VlbView &a, const void *x, int xdtype, int64_t *y,
                             hipStream_t s);

// One pass for the method choice: (min, max) into slot (initialised by
// launch_range_init) and, into the spread pairs `sums`, the sums of the
// unsigned and of the two's complement element widths (zeroed here).
hipError_t launch_method_stats(const void *dense, int dtype, uint64_t n, RangeSlot *slot,
                               uint64_t *sums, hipStream_t s);

// synthetic data
hipError_t launch_fill_uniform(void *dense, int dtype, uint64_t n, int64_t lo, uint64_t span,
                               uint64_t seed, uint64_t stream_id, uint64_t start,
                               hipStream_t s);
hipError_t launch_gen_range(uint64_t n, int64_t lo, uint64_t span, uint64_t seed,
                            uint64_t stream_id, RangeSlot *slot, hipStream_t s);
hipError_t launch_gen_pack(uint64_t n, int64_t lo, uint64_t span, uint64_t seed,
                           uint64_t stream_id, int bits, uint32_t *out, uint64_t cap32,
                           hipStream_t s);

// SplitMix64 draw `ctr` of the sequence starting at `seed`, mapped to
// [lo, lo + span) with span <= 2^32.
__host__ __device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t ctr) {
  uint64_t z = seed + (ctr + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline int64_t uniform_at(uint64_t seed, uint64_t stream_id, uint64_t idx,
                                              int64_t lo, uint64_t span) {
  const uint64_t h = splitmix64_at(seed, (stream_id << 40) + idx);
  return lo + (int64_t)(((h >> 32) * span) >> 32);
}

}  // namespace ccm
