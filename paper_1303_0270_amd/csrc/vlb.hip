// Method 2 of the paper (Variable Length Blocks): every element is stored in
// its own minimal width b_e, preceded by a fixed k-bit length field holding
// b_e, with k the bit-length of the largest b_e (Methods, "Method 2"; Eq. 16
// counts the bits).  Elements follow each other in row-major order, least
// significant bit first, straddling 64-bit bitstrings as in Method 1.
//
// The stream alone can only be read from its start.  For random access and
// data-parallel decoding the library keeps an index beside it:
//   row_bit[i]   (uint64, rows + 1 entries): stream bit where row i starts;
//                row_bit[rows] is the total bit count;
//   grp_off[i][g] (uint32, rows x ceil(cols/32)): bit offset of element
//                (i, 32g) from the start of row i.
// A "group" is 32 consecutive elements of one row (the last group of a row
// may be shorter).  A lane that owns a group knows where it starts and walks
// its 32 (length, value) pairs; where the next one starts depends on the
// length just read, so the walk is serial within a group and parallel across
// groups.
//
// Encoding runs in three passes: group bit counts (sum of k + b_e), scans
// (within rows, then over rows) that turn the counts into the index, and the
// packing pass, where a block assembles the bits of 64 consecutive groups in
// LDS (a half-wave per group places its pairs with a prefix sum of their
// lengths) and writes them out: the words its stretch covers entirely with
// plain stores, the two it shares with its neighbours with atomic ORs into
// the zeroed payload.
#include <hip/hip_runtime.h>

#include "ccm_internal.hpp"

namespace ccm {
namespace {

constexpr int kVG = 32;          // elements per index group
constexpr int kVThreads = 256;   // threads per block of every VLB kernel

__device__ __forceinline__ int bitlen64(uint64_t u) { return u ? 64 - __clzll((long long)u) : 0; }

// b_e of one value: Eq. 1 on the element when the matrix has no negative
// value; otherwise the smallest two's complement width holding it.
__device__ __forceinline__ int elem_width(int64_t v, int sgn) {
  if (!sgn) {
    const int L = bitlen64((uint64_t)v);
    return L > 1 ? L : 1;
  }
  const uint64_t m = v < 0 ? ~(uint64_t)v : (uint64_t)v;
  return 1 + bitlen64(m);
}

template <typename T>
__device__ __forceinline__ int64_t load_dense(const T *d, uint64_t e) {
  return (int64_t)d[e];
}

// nb (1..64) stream bits starting at bit p, zero-extended.  Reads words
// p/32 .. p/32 + 2, which stay inside the payload capacity for any field
// that starts inside the stream.
__device__ __forceinline__ uint64_t bits_at(const uint32_t *w, uint64_t p, int nb) {
  const uint64_t q = p >> 5;
  const int off = (int)(p & 31u);
  uint64_t v = ((uint64_t)w[q] | ((uint64_t)w[q + 1] << 32)) >> off;
  if (off + nb > 64) v |= (uint64_t)w[q + 2] << (64 - off);
  return v & mask64(nb);
}

// ---- pass 1: bits per group --------------------------------------------

// Half-wave h of a wave owns one group: lane l reads element 32g + l, and the
// 32 lanes sum k + b_e.  The grid-stride step is a multiple of 32 and the
// total a multiple of 32, so a group's lanes are always active together.
template <typename T>
__global__ __launch_bounds__(kVThreads) void k_vlb_sizes(const T *__restrict__ dense, int64_t rows,
                                                         int64_t cols, int64_t ngr, int k, int sgn,
                                                         uint32_t *__restrict__ grp,
                                                         RangeSlot *slot) {
  const uint64_t total = (uint64_t)rows * (uint64_t)ngr * kVG;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  // group gi = (row i, group g of the row), advanced by the grid step with
  // one division up front (a 64-bit division per element would cost more
  // than the element's own work)
  const uint64_t gstep = stride >> 5;
  const uint64_t di = gstep / (uint64_t)ngr, dg = gstep - di * (uint64_t)ngr;
  uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t i = (t >> 5) / (uint64_t)ngr, g = (t >> 5) - i * (uint64_t)ngr;
  const int l = (int)(t & 31u);
  uint32_t gmax = 0;
  // kSizeSteps grid steps per iteration: their loads (unconditional, with
  // clamped row and column) are all issued before any is used.  A step's
  // validity is the same for the 32 lanes of a group (total and the step are
  // multiples of 32), so the group's shuffles always run together.
  constexpr int kSizeSteps = 4;
  for (; t < total; t += kSizeSteps * stride) {
    int64_t v[kSizeSteps];
    bool live[kSizeSteps], valid[kSizeSteps];
#pragma unroll
    for (int u = 0; u < kSizeSteps; ++u) {
      valid[u] = t + u * stride < total;
      const uint64_t j = g * kVG + (uint64_t)l;
      live[u] = valid[u] && j < (uint64_t)cols;
      const uint64_t ic = valid[u] ? i : (uint64_t)rows - 1;
      v[u] = load_dense(dense, ic * (uint64_t)cols + (live[u] ? j : (uint64_t)cols - 1));
      g += dg;
      i += di;
      if (g >= (uint64_t)ngr) {
        g -= (uint64_t)ngr;
        ++i;
      }
    }
#pragma unroll
    for (int u = 0; u < kSizeSteps; ++u) {
      uint32_t nb = live[u] ? (uint32_t)(k + elem_width(v[u], sgn)) : 0u;
#pragma unroll
      for (int m = 16; m >= 1; m >>= 1) nb += (uint32_t)__shfl_xor((int)nb, m, 32);
      if (l == 0 && valid[u]) grp[(t + u * stride) >> 5] = nb;
      gmax = nb > gmax ? nb : gmax;
    }
  }
  // the longest group (sizes the staging buffers of the matvec kernel)
  block_range_commit(0, (int64_t)gmax, 0, slot);
}

// ---- pass 2: scans ----------------------------------------------------------

// Inclusive block-wide scan of one value per thread (uint64), with the block
// total.  Every thread must call it.
__device__ __forceinline__ uint64_t block_scan_incl(uint64_t v, uint64_t *total) {
  __shared__ uint64_t s_wave[kVThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  if (lane == 63) s_wave[wave] = v;
  __syncthreads();
  uint64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kVThreads / 64; ++w) {
    const uint64_t s = s_wave[w];
    before += w < wave ? s : 0;
    all += s;
  }
  __syncthreads();  // s_wave is reused by the next call
  *total = all;
  return v + before;
}

// Row i's group counts become exclusive offsets from the row start; the row's
// total goes to row_bit[i + 1] (pass 3 turns those into starts).
__global__ __launch_bounds__(kVThreads) void k_vlb_row_scan(int64_t rows, int64_t ngr,
                                                            uint32_t *__restrict__ grp,
                                                            uint64_t *__restrict__ row_bit) {
  for (int64_t i = blockIdx.x; i < rows; i += gridDim.x) {
    uint32_t *gp = grp + (uint64_t)i * (uint64_t)ngr;
    uint64_t carry = 0;
    for (int64_t c0 = 0; c0 < ngr; c0 += kVThreads) {
      const int64_t g = c0 + threadIdx.x;
      const uint64_t v = g < ngr ? gp[g] : 0;
      uint64_t tot = 0;
      const uint64_t inc = block_scan_incl(v, &tot);
      if (g < ngr) gp[g] = (uint32_t)(carry + inc - v);
      carry += tot;
    }
    if (threadIdx.x == 0) row_bit[i + 1] = carry;
  }
}

// row_bit[0] = 0 and row_bit[i + 1] = sum of the first i + 1 row totals.  One
// block.
__global__ __launch_bounds__(kVThreads) void k_vlb_rows_scan(int64_t rows,
                                                             uint64_t *__restrict__ row_bit) {
  uint64_t carry = 0;
  for (int64_t c0 = 0; c0 < rows; c0 += kVThreads) {
    const int64_t i = c0 + threadIdx.x;
    const uint64_t v = i < rows ? row_bit[i + 1] : 0;
    uint64_t tot = 0;
    const uint64_t inc = block_scan_incl(v, &tot);
    if (i < rows) row_bit[i + 1] = carry + inc;
    carry += tot;
  }
  if (threadIdx.x == 0) row_bit[0] = 0;
}

// ---- pass 3: packing -----------------------------------------------------------

__global__ void k_zero_u32(uint32_t *p, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) p[e] = 0;
}

// ORs the low nb (1..64) bits of val into an LDS bit span at bit pos (at
// most three words; LDS atomics, since neighbouring lanes share words).
__device__ __forceinline__ void lds_or_bits(uint32_t *span, uint32_t pos, uint64_t val, int nb) {
  val &= mask64(nb);
  const uint32_t q = pos >> 5, sh = pos & 31u;
  const uint64_t lo = val << sh;
  const uint32_t hi = sh ? (uint32_t)(val >> (64u - sh)) : 0u;
  const int nw = (int)((sh + (uint32_t)nb + 31u) >> 5);
  if ((uint32_t)lo) atomicOr(&span[q], (uint32_t)lo);
  if (nw > 1 && (uint32_t)(lo >> 32)) atomicOr(&span[q + 1], (uint32_t)(lo >> 32));
  if (nw > 2 && hi) atomicOr(&span[q + 2], hi);
}

// A block assembles the stream of kPackGroups consecutive groups (a
// contiguous stretch of bits [S, E)) in LDS, then writes it out.
//   * A half-wave per group: lane l reads element 32g + l (coalesced), takes
//     its width b_e, and a 32-lane prefix sum of k + b_e places its pair
//     (length field, then value) inside the group, which starts at the bit
//     the index gives.  The pair is ORed into the LDS stretch.
//   * Write-out: the words the stretch covers entirely are plain coalesced
//     stores; its first and last words, shared with the neighbouring blocks,
//     are atomic ORs into the zeroed payload.
constexpr int kPackGroups = 64;

template <typename T>
__global__ __launch_bounds__(kVThreads) void k_vlb_pack(const T *__restrict__ dense, int64_t rows,
                                                        int64_t cols, int64_t ngr, int k, int sgn,
                                                        const uint64_t *__restrict__ row_bit,
                                                        const uint32_t *__restrict__ grp,
                                                        uint64_t nbits, int span_words,
                                                        uint32_t *__restrict__ out) {
  extern __shared__ uint32_t span[];
  const uint64_t total = (uint64_t)rows * (uint64_t)ngr;
  const int half = threadIdx.x >> 5, l = threadIdx.x & 31;
  for (uint64_t gb = (uint64_t)blockIdx.x * kPackGroups; gb < total;
       gb += (uint64_t)gridDim.x * kPackGroups) {
    const uint64_t ge = gb + kPackGroups < total ? gb + kPackGroups : total;
    // stretch [S, E) of groups gb .. ge - 1
    const uint64_t ib = gb / (uint64_t)ngr;
    const uint64_t S = row_bit[ib] + grp[gb];
    uint64_t E;
    if (ge < total) {
      const uint64_t ie = ge / (uint64_t)ngr;
      E = row_bit[ie] + grp[ge];
    } else {
      E = nbits;
    }
    const uint64_t q0 = S >> 5;
    const int nwords = (int)(((E + 31u) >> 5) - q0);
    for (int w = threadIdx.x; w < span_words; w += blockDim.x) span[w] = 0;
    __syncthreads();
    // This half-wave's groups of the stretch (at most kPackPer): their
    // elements and start bits are requested first, with clamped addresses,
    // then placed one group at a time.  (row, group) advance from one
    // division per stretch.
    constexpr int kPackPer = kPackGroups / (kVThreads / 32);
    const uint64_t gi0 = gb + (uint64_t)half;
    uint64_t i = gi0 / (uint64_t)ngr, g = gi0 - i * (uint64_t)ngr;
    int64_t v[kPackPer];
    uint64_t gstart[kPackPer];
    bool live[kPackPer];
#pragma unroll
    for (int u = 0; u < kPackPer; ++u) {
      const uint64_t gi = gi0 + (uint64_t)u * (kVThreads / 32);
      const bool valid = gi < ge;
      const uint64_t j = g * kVG + (uint64_t)l;
      live[u] = valid && j < (uint64_t)cols;
      const uint64_t ic = valid ? i : (uint64_t)rows - 1;
      v[u] = load_dense(dense, ic * (uint64_t)cols + (live[u] ? j : (uint64_t)cols - 1));
      gstart[u] = row_bit[ic] + grp[valid ? gi : total - 1];
      g += kVThreads / 32;
      while (g >= (uint64_t)ngr) {
        g -= (uint64_t)ngr;
        ++i;
      }
    }
#pragma unroll
    for (int u = 0; u < kPackPer; ++u) {
      // the same for the 32 lanes of a group, so its shuffles run together
      if (gi0 + (uint64_t)u * (kVThreads / 32) >= ge) break;
      const int b = live[u] ? elem_width(v[u], sgn) : 0;
      const uint32_t len = live[u] ? (uint32_t)(k + b) : 0u;
      // exclusive prefix sum over the 32 lanes of the group
      uint32_t inc = len;
#pragma unroll
      for (int d = 1; d < 32; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)inc, d, 32);
        if (l >= d) inc += o;
      }
      const uint32_t pos = (uint32_t)(gstart[u] - q0 * 32u) + (inc - len);
      if (live[u]) {
        lds_or_bits(span, pos, (uint64_t)b, k);                   // the length field
        lds_or_bits(span, pos + (uint32_t)k, (uint64_t)v[u], b);  // then the value
      }
    }
    __syncthreads();
    for (int w = threadIdx.x; w < nwords; w += blockDim.x) {
      const uint64_t q = q0 + (uint64_t)w;
      const uint32_t val = span[w];
      if (q * 32u >= S && q * 32u + 32u <= E)
        out[q] = val;
      else if (val)
        atomicOr(&out[q], val);
    }
    __syncthreads();  // the span is cleared for the next stretch
  }
}

// ---- decode, get ------------------------------------------------------------

// One (length, value) pair at stream bit *p; advances *p.
__device__ __forceinline__ int64_t vlb_read(const uint32_t *w, uint64_t *p, int k, int sgn) {
  const int b = (int)bits_at(w, *p, k);
  const uint64_t u = bits_at(w, *p + (uint64_t)k, b);
  *p += (uint64_t)(k + b);
  return sgn ? sext64(u, b) : (int64_t)u;
}

__global__ __launch_bounds__(kVThreads) void k_vlb_decode(const uint32_t *__restrict__ w,
                                                          const uint64_t *__restrict__ row_bit,
                                                          const uint32_t *__restrict__ grp,
                                                          int64_t rows, int64_t cols, int64_t ngr,
                                                          int k, int sgn, int64_t *__restrict__ out) {
  const uint64_t total = (uint64_t)rows * (uint64_t)ngr;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t gi = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < total; gi += stride) {
    const int64_t i = (int64_t)(gi / (uint64_t)ngr);
    const int64_t g = (int64_t)(gi - (uint64_t)i * (uint64_t)ngr);
    uint64_t p = row_bit[i] + grp[gi];
    const int64_t j0 = g * kVG;
    const int n = cols - j0 < kVG ? (int)(cols - j0) : kVG;
    int64_t *dst = out + (uint64_t)i * (uint64_t)cols + (uint64_t)j0;
    for (int l = 0; l < n; ++l) dst[l] = vlb_read(w, &p, k, sgn);
  }
}

__global__ void k_vlb_get(const uint32_t *__restrict__ w, const uint64_t *__restrict__ row_bit,
                          const uint32_t *__restrict__ grp, int64_t ngr, int64_t i, int64_t j,
                          int k, int sgn, int64_t *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t g = j / kVG;
  uint64_t p = row_bit[i] + grp[(uint64_t)i * (uint64_t)ngr + (uint64_t)g];
  int64_t v = 0;
  for (int64_t l = g * kVG; l <= j; ++l) v = vlb_read(w, &p, k, sgn);
  *out = v;
}

// ---- matvec ------------------------------------------------------------------

// General form: any k + b_e, int32 or int64 x.  Block (chunk c, row i) walks
// groups 256c .. 256c + 255 of row i, one per lane, reading the stream
// straight from memory; the block's sum goes to y[i] (atomically when a row
// has more than one chunk; y was zeroed).
template <typename XT>
__global__ __launch_bounds__(kVThreads) void k_vlb_mv_gen(
    const uint32_t *__restrict__ w, const uint64_t *__restrict__ row_bit,
    const uint32_t *__restrict__ grp, int64_t rows, int64_t cols, int64_t ngr, int k, int sgn,
    const XT *__restrict__ x, int64_t *__restrict__ y) {
  __shared__ uint64_t s_part[kVThreads / 64];
  const int64_t nchunk = (ngr + kVThreads - 1) / kVThreads;
  const uint64_t nblk = (uint64_t)rows * (uint64_t)nchunk;
  for (uint64_t bi = blockIdx.x; bi < nblk; bi += gridDim.x) {
    const int64_t i = (int64_t)(bi / (uint64_t)nchunk);
    const int64_t c = (int64_t)(bi - (uint64_t)i * (uint64_t)nchunk);
    const int64_t g = c * kVThreads + threadIdx.x;
    uint64_t acc = 0;
    if (g < ngr) {
      uint64_t p = row_bit[i] + grp[(uint64_t)i * (uint64_t)ngr + (uint64_t)g];
      const int64_t j0 = g * kVG;
      const int n = cols - j0 < kVG ? (int)(cols - j0) : kVG;
      for (int l = 0; l < n; ++l) {
        const int64_t a = vlb_read(w, &p, k, sgn);
        acc += (uint64_t)a * (uint64_t)(int64_t)x[j0 + l];
      }
    }
    const int64_t ws = wave_sum((int64_t)acc);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = (uint64_t)ws;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t t = 0;
#pragma unroll
      for (int v = 0; v < kVThreads / 64; ++v) t += s_part[v];
      if (nchunk > 1)
        atomicAdd((unsigned long long *)&y[i], (unsigned long long)t);
      else
        y[i] = (int64_t)t;
    }
    __syncthreads();
  }
}

// Both of (a == b ? x0 : y0) and (a == b ? x1 : y1) from one compare and
// two v_cndmask.  As plain C the compiler turns the select of two values just
// read from LDS into a select of their addresses and demotes the chain state
// to scratch.
__device__ __forceinline__ void select_eq2(uint32_t a, uint32_t b, uint32_t x0, uint32_t y0,
                                           uint32_t x1, uint32_t y1, uint32_t &r0,
                                           uint32_t &r1) {
  asm("v_cmp_eq_u32 vcc, %2, %3\n\t"
      "v_cndmask_b32 %0, %5, %4, vcc\n\t"
      "v_cndmask_b32 %1, %7, %6, vcc"
      : "=&v"(r0), "=v"(r1)
      : "v"(a), "v"(b), "v"(x0), "v"(y0), "v"(x1), "v"(y1)
      : "vcc");
}

// 64 stream bits from bit pv of a staged stretch (reads three words).
__device__ __forceinline__ uint64_t lds_bits64(const uint32_t *seg, uint32_t pv) {
  const uint32_t q = pv >> 5;
  const uint32_t w0 = seg[q], w1 = seg[q + 1], w2 = seg[q + 2];
  const uint32_t lo = __builtin_amdgcn_alignbit(w1, w0, pv & 31u);
  const uint32_t hi = __builtin_amdgcn_alignbit(w2, w1, pv & 31u);
  return ((uint64_t)hi << 32) | lo;
}

// Staged form for int32 x on a 16-byte boundary, any widths.
//   * Block (panel p, row slice) owns groups [256 GPT p, 256 GPT (p + 1)) of
//     the rows it visits; lane t owns groups 256 GPT p + GPT t + u (u < GPT),
//     GPT independent chains (instruction-level parallelism in the serial
//     walks), and keeps their 32 GPT x values in registers for all rows.
//   * Per row the block copies the panel's stretch of the stream (contiguous:
//     the panel's groups follow each other) into LDS with 16-byte
//     memory-to-LDS loads (global_load_lds_dwordx4, no registers), issued
//     right after the walks of the previous row.  One buffer: a second one,
//     filled a row ahead, measured slower, since it halves the blocks per CU
//     and the other resident blocks already cover a block's copy.
//   * A chain keeps the two stream words around its position in registers
//     (w0 = word q, w1 = word q + 1).  Per element: a funnel shift
//     (v_alignbit) gives the 32 bits at the pair's start; the length is their
//     low k bits; the value is one bit-field extract of the same word
//     (sign-extending when signed) and the product one 32x32->64
//     multiply-add.  A pair of at most 32 bits moves the position by at most
//     one word, so the window advances with a select and ONE new LDS word per
//     element.  A longer pair (rare in the paper's bit-length distributions)
//     takes a branch that reads the 64 bits at the value's start, corrects
//     the product and reloads the window.
//   * Rows visited: blockIdx.y, blockIdx.y + gridDim.y, ... (resident
//     blocks only, so x is loaded once per block).  Wave partial sums of row
//     r are folded and stored after the barrier that opens row r + 1.
//   * CLAMP: some chain of the panel is shorter than 32 elements or absent
//     (ragged row end, partial panel); its walk then continues through bits
//     of the next group or past the stretch, with x = 0 for those elements,
//     and its reads are clamped inside the staged buffer.
template <bool SGN, int GPT, bool CLAMP, bool WIDE>
__global__ __launch_bounds__(kVThreads) void k_vlb_mv_lds(
    const uint32_t *__restrict__ w, const uint64_t *__restrict__ row_bit,
    const uint32_t *__restrict__ grp, int64_t rows, int64_t cols, int64_t ngr, int k,
    int seg_words, const int32_t *__restrict__ x, int64_t *__restrict__ y, int atomic_out) {
  extern __shared__ uint4 seg4[];
  // the stretch buffer (seg_words words), then the wave partial sums of two
  // rows
  uint64_t *s_part = (uint64_t *)((uint32_t *)seg4 + seg_words);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t g0 = (int64_t)blockIdx.x * kVThreads * GPT;
  const int64_t ge = g0 + kVThreads * GPT < ngr ? g0 + kVThreads * GPT : ngr;
  const uint32_t kmask = (1u << k) - 1u;
  const uint32_t narrow = 32u - (uint32_t)k;  // largest b read from one 32-bit window
  const uint32_t qmax = (uint32_t)seg_words - 4u;
  const uint32_t pmax = qmax * 32u;
  const uint32_t pmaxw = ((uint32_t)seg_words - 5u) * 32u;  // four-word reads

  int32_t xr[GPT][kVG];
#pragma unroll
  for (int u = 0; u < GPT; ++u) {
    const int64_t c0 = (g0 + (int64_t)GPT * t + u) * kVG;
    if (c0 + kVG <= cols) {
      const int4 *xv = (const int4 *)(x + c0);
#pragma unroll
      for (int q = 0; q < kVG / 4; ++q) {
        const int4 v = xv[q];
        xr[u][4 * q] = v.x;
        xr[u][4 * q + 1] = v.y;
        xr[u][4 * q + 2] = v.z;
        xr[u][4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < kVG; ++j) xr[u][j] = c0 + j < cols ? x[c0 + j] : 0;
    }
  }

  // Row r's stage: its start bit, first staged word (16-byte aligned) and
  // 16-byte vector count; the lanes' raw group offsets (clamped loads,
  // branch-free) and the copy of the stretch into the buffer.
  uint64_t nb_base = 0, nb_ws = 0;
  uint32_t graw[GPT];
  auto stage = [&](int64_t r) {
    const uint64_t base = row_bit[r];
    const uint32_t *gr = grp + (uint64_t)r * (uint64_t)ngr;
    const uint64_t s = base + gr[g0];
    const uint64_t e = ge < ngr ? base + gr[ge] : row_bit[r + 1];
    const uint64_t ws = (s >> 5) & ~3ull;
    const uint64_t we = ((e + 31u) >> 5) + 2u;  // two guard words for the 64-bit reads
    const int nvec = (int)((we - ws + 3u) >> 2);
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      int64_t g = g0 + (int64_t)GPT * t + u;
      g = g < ngr ? g : ngr - 1;
      graw[u] = gr[g];
    }
    const uint4 *src = (const uint4 *)(w + ws);
    uint4 *dst = seg4;
    for (int v0 = 0; v0 < nvec; v0 += kVThreads) {
      const int v = v0 + t;
      if (v < nvec)
        __builtin_amdgcn_global_load_lds(
            (const void *)(src + v),
            (__attribute__((address_space(3))) void *)(dst + v0 + 64 * wave), 16, 0, 0);
    }
    nb_base = base;
    nb_ws = ws;
  };

  int64_t r = blockIdx.y;
  if (r < rows) stage(r);
  int cur = 0;
  int64_t prev = -1;  // row whose wave sums wait in s_part[cur ^ 1]
  while (r < rows) {
    __builtin_amdgcn_s_waitcnt(0);  // all counters to zero: this lane's copies have landed
    __syncthreads();                // everyone's copies have landed
    if (prev >= 0 && t == 0) {
      uint64_t sum = 0;
#pragma unroll
      for (int v = 0; v < kVThreads / 64; ++v) sum += s_part[4 * (cur ^ 1) + v];
      if (atomic_out)
        atomicAdd((unsigned long long *)&y[prev], (unsigned long long)sum);
      else
        y[prev] = (int64_t)sum;
    }
    uint32_t p[GPT];
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int64_t g = g0 + (int64_t)GPT * t + u;
      p[u] = g < ngr ? (uint32_t)(nb_base + graw[u] - nb_ws * 32u) : 0u;
    }
    const int64_t rn = r + gridDim.y;

    // x stays in 32-bit registers: without this the compiler hoists the
    // sign extensions out of the row loop and doubles the register count
#pragma unroll
    for (int u = 0; u < GPT; ++u)
#pragma unroll
      for (int j = 0; j < kVG; ++j) asm volatile("" : "+v"(xr[u][j]));

    const uint32_t *seg = (const uint32_t *)seg4;
    int64_t acc[GPT];
    // the window: words q, q + 1 around the position and q + 2 requested
    // ahead (a pair of at most 32 bits moves the position by at most a
    // word, so the next window is (w0, w1) or (w1, w2), never a word still
    // in flight)
    // The four-word walk keeps the four words at its (clamped) read
    // position q in w0..w3, and requests the next element's as soon as the
    // length is known, before the value and the product.
    uint32_t q[GPT], w0[GPT], w1[GPT], w2[GPT], w3[GPT];
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      acc[u] = 0;
      if constexpr (WIDE) {
        q[u] = CLAMP && p[u] > pmaxw ? pmaxw : p[u];
        const uint32_t qc = q[u] >> 5;
        w0[u] = seg[qc];
        w1[u] = seg[qc + 1];
        w2[u] = seg[qc + 2];
        w3[u] = seg[qc + 3];
      } else {
        q[u] = p[u] >> 5;
        w0[u] = seg[q[u]];
        w1[u] = seg[q[u] + 1];
        w2[u] = seg[q[u] + 2];
        w3[u] = 0u;
      }
    }
#pragma unroll
    for (int j = 0; j < kVG; ++j) {
#pragma unroll
      for (int u = 0; u < GPT; ++u) {
        if constexpr (WIDE) {
          // four words at the pair's start give 96 bits: the length and a
          // value of up to 64 bits, with no branch
          const uint32_t sh = q[u] & 31u;
          const uint32_t a0 = __builtin_amdgcn_alignbit(w1[u], w0[u], sh);
          const uint32_t a1 = __builtin_amdgcn_alignbit(w2[u], w1[u], sh);
          const uint32_t a2 = __builtin_amdgcn_alignbit(w3[u], w2[u], sh);
          const uint32_t b = a0 & kmask;
          p[u] += (uint32_t)k + b;
          // the next pair's words, requested before this one's value and
          // product (kept here: the scheduler would sink them to their use)
          q[u] = CLAMP && p[u] > pmaxw ? pmaxw : p[u];
          const uint32_t qc = q[u] >> 5;
          w0[u] = seg[qc];
          w1[u] = seg[qc + 1];
          w2[u] = seg[qc + 2];
          w3[u] = seg[qc + 3];
          __builtin_amdgcn_sched_barrier(0);
          const int nb = b < 64u ? (int)b : 64;
          const uint64_t lo = ((uint64_t)a1 << 32) | a0;
          uint64_t v = ((lo >> k) | ((uint64_t)a2 << (64 - k))) & mask64(nb);
          if (SGN) v = (uint64_t)sext64(v, nb > 0 ? nb : 1);
          acc[u] += (int64_t)(v * (uint64_t)(int64_t)xr[u][j]);
          asm volatile("" : "+v"(acc[u]));
          continue;
        }
        const uint32_t wv = __builtin_amdgcn_alignbit(w1[u], w0[u], p[u] & 31u);
        const uint32_t b = wv & kmask;
        int32_t a;
        if (SGN)
          a = opaque_i32(__builtin_amdgcn_sbfe((int32_t)wv, k, b));
        else
          a = (int32_t)__builtin_amdgcn_ubfe(wv, k, b);
        acc[u] += (int64_t)a * (int64_t)xr[u][j];
        // one v_add3 (the compiler otherwise keeps p + k apart for the rare
        // branch and spends two adds on every element)
        uint32_t pn;
        asm("v_add3_u32 %0, %1, %2, %3" : "=v"(pn) : "v"(p[u]), "s"((uint32_t)k), "v"(b));
        uint32_t qn = pn >> 5;
        if (CLAMP) qn = qn < qmax ? qn : qmax;
        // the word after the next window, requested as early as its address
        // is known (kept here: left to itself the scheduler sinks the
        // request to its use in the next element, which then waits for it)
        const uint32_t w2n = seg[qn + 2];
        __builtin_amdgcn_sched_barrier(0);
        uint32_t w0n, w1n;
        select_eq2(qn, q[u], w0[u], w1[u], w1[u], w2[u], w0n, w1n);
        if (__builtin_expect(b > narrow, 0)) {
          // the value runs past the 32 bits read: replace a by the full
          // value, and reload the window where the next pair starts
          uint32_t pv = p[u] + (uint32_t)k;
          if (CLAMP) pv = pv < pmax ? pv : pmax;
          const int nb = b < 64u ? (int)b : 64;
          uint64_t v = lds_bits64(seg, pv) & mask64(nb);
          if (SGN) v = (uint64_t)sext64(v, nb);
          int32_t xw = xr[u][j];
          asm volatile("" : "+v"(xw));  // sign-extend here, not hoisted
          acc[u] += (int64_t)((v - (uint64_t)(int64_t)a) * (uint64_t)(int64_t)xw);
          w0n = seg[qn];
          w1n = seg[qn + 1];
          // wait for these two here, on the rare path: a wait at the merge
          // would also wait for the prefetch on the common one
          __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
        }
        asm volatile("" : "+v"(acc[u]));  // accumulate in place, element by element
        w2[u] = w2n;
        w1[u] = w1n;
        w0[u] = w0n;
        q[u] = qn;
        p[u] = pn;
      }
    }
    int64_t tot = 0;
#pragma unroll
    for (int u = 0; u < GPT; ++u) tot += acc[u];
    tot = wave_sum(tot);
    if (lane == 0) s_part[4 * cur + wave] = (uint64_t)tot;
    __syncthreads();  // every walk is done before the copy overwrites the buffer
    if (rn < rows) stage(rn);
    prev = r;
    r = rn;
    cur ^= 1;
  }
  __syncthreads();
  if (prev >= 0 && t == 0) {
    uint64_t sum = 0;
#pragma unroll
    for (int v = 0; v < kVThreads / 64; ++v) sum += s_part[4 * (cur ^ 1) + v];
    if (atomic_out)
      atomicAdd((unsigned long long *)&y[prev], (unsigned long long)sum);
    else
      y[prev] = (int64_t)sum;
  }
}

int compute_units() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n < 1)
      n = 256;
    cus = n;
  }
  return cus;
}

constexpr size_t kMaxLds = 160 * 1024 - 64;

// A panel's stretch: at most 256 GPT gmax bits, plus the alignment of its
// first word down to 16 bytes, the two guard words after its last, the
// rounding to whole 16-byte vectors and the clamp margin.
int stage_words(uint64_t gmax, int gpt) {
  return (int)(((uint64_t)kVThreads * gpt * gmax + 31u) / 32u + 16u) & ~3;
}

// The stretch buffer and the wave partial sums of two rows.
size_t stage_lds(uint64_t gmax, int gpt) {
  return (size_t)stage_words(gmax, gpt) * 4u + 2u * (kVThreads / 64) * 8u;
}

template <bool SGN, int GPT, bool CLAMP, bool WIDE>
int resident_lds(size_t lds) {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_vlb_mv_lds<SGN, GPT, CLAMP, WIDE>,
                                                   kVThreads, lds) != hipSuccess ||
      occ < 1)
    occ = 1;
  return occ * compute_units();
}

template <bool SGN, int GPT, bool CLAMP, bool WIDE>
hipError_t launch_mv_lds(const VlbView &a, const int32_t *x, int64_t *y, hipStream_t s) {
  const int64_t per_panel = (int64_t)kVThreads * GPT;
  const int64_t npanels = (a.ngr + per_panel - 1) / per_panel;
  if (npanels > 65535) return hipErrorInvalidValue;
  const int seg_words = stage_words(a.gmax, GPT);
  const size_t lds = stage_lds(a.gmax, GPT);
  if (lds > kMaxLds) return hipErrorInvalidValue;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void *)k_vlb_mv_lds<SGN, GPT, CLAMP, WIDE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (npanels > 1) {
    hipError_t e = launch_fill_i64(y, (uint64_t)a.rows, 0, s);
    if (e != hipSuccess) return e;
  }
  int64_t gy = resident_lds<SGN, GPT, CLAMP, WIDE>(lds) / npanels;
  gy = gy < 1 ? 1 : (gy > a.rows ? a.rows : gy);
  if (gy > 65535) gy = 65535;
  dim3 grid((unsigned)npanels, (unsigned)gy);
  k_vlb_mv_lds<SGN, GPT, CLAMP, WIDE><<<grid, kVThreads, lds, s>>>(
      a.w, a.row_bit, a.grp, a.rows, a.cols, a.ngr, a.k, seg_words, x, y, npanels > 1 ? 1 : 0);
  return hipGetLastError();
}

template <bool SGN, int GPT, bool WIDE>
hipError_t launch_mv_lds_c(const VlbView &a, const int32_t *x, int64_t *y, hipStream_t s) {
  const bool clamp = (a.cols % ((int64_t)kVThreads * GPT * kVG)) != 0;
  return clamp ? launch_mv_lds<SGN, GPT, true, WIDE>(a, x, y, s)
               : launch_mv_lds<SGN, GPT, false, WIDE>(a, x, y, s);
}

// Staged matvec: one group per lane (256 groups of at most 32 * 71 bits
// always fit in LDS), or two when that keeps strictly more chains resident
// per CU (blocks per CU from registers and LDS, times 256 GPT).  At equal
// chain counts one group per lane measured faster: twice the waves to hide
// the LDS latency of the walks.  Matrices whose pairs average more than 24
// bits (so that most pairs pass 32 bits, as with uniform bit-lengths) take
// the branch-free four-word walk.
template <bool SGN, bool WIDE>
hipError_t launch_mv_staged_w(const VlbView &a, const int32_t *x, int64_t *y, hipStream_t s) {
  const int64_t chains1 = (int64_t)resident_lds<SGN, 1, true, WIDE>(stage_lds(a.gmax, 1));
  int64_t chains2 = 0;
  if (stage_lds(a.gmax, 2) <= kMaxLds)
    chains2 = 2 * (int64_t)resident_lds<SGN, 2, true, WIDE>(stage_lds(a.gmax, 2));
  return chains2 > chains1 ? launch_mv_lds_c<SGN, 2, WIDE>(a, x, y, s)
                           : launch_mv_lds_c<SGN, 1, WIDE>(a, x, y, s);
}

template <bool SGN>
hipError_t launch_mv_staged(const VlbView &a, const int32_t *x, int64_t *y, hipStream_t s) {
  const uint64_t n = (uint64_t)a.rows * (uint64_t)a.cols;
  return a.nbits > 24u * n ? launch_mv_staged_w<SGN, true>(a, x, y, s)
                           : launch_mv_staged_w<SGN, false>(a, x, y, s);
}

unsigned vgrid(uint64_t work, uint64_t per_block, unsigned cap) {
  uint64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

uint64_t vlb_ngr(int64_t cols) { return ((uint64_t)cols + kVG - 1) / kVG; }

hipError_t launch_vlb_sizes(const void *dense, int dtype, int64_t rows, int64_t cols, int k,
                            int sgn, uint32_t *grp, RangeSlot *slot, hipStream_t s) {
  const int64_t ngr = (int64_t)vlb_ngr(cols);
  const unsigned grid = vgrid((uint64_t)rows * (uint64_t)ngr * kVG, kVThreads * 4, 4096);
  if (dtype == CCM_I64)
    k_vlb_sizes<int64_t><<<grid, kVThreads, 0, s>>>((const int64_t *)dense, rows, cols, ngr, k,
                                                    sgn, grp, slot);
  else
    k_vlb_sizes<int32_t><<<grid, kVThreads, 0, s>>>((const int32_t *)dense, rows, cols, ngr, k,
                                                    sgn, grp, slot);
  return hipGetLastError();
}

hipError_t launch_vlb_scan(int64_t rows, int64_t cols, uint32_t *grp, uint64_t *row_bit,
                           hipStream_t s) {
  const int64_t ngr = (int64_t)vlb_ngr(cols);
  const unsigned grid = vgrid((uint64_t)rows, 1, 16384);
  k_vlb_row_scan<<<grid, kVThreads, 0, s>>>(rows, ngr, grp, row_bit);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_vlb_rows_scan<<<1, kVThreads, 0, s>>>(rows, row_bit);
  return hipGetLastError();
}

hipError_t launch_vlb_pack(const void *dense, int dtype, const VlbView &a, uint32_t *out,
                           uint64_t cap32, uint64_t nbits, hipStream_t s) {
  k_zero_u32<<<vgrid(cap32, kVThreads * 8, 8192), kVThreads, 0, s>>>(out, cap32);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // a stretch of kPackGroups groups spans at most kPackGroups * gmax bits
  // and one word more
  const int span_words = (int)(((uint64_t)kPackGroups * a.gmax + 31u) / 32u + 2u);
  const size_t lds = (size_t)span_words * 4u;
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  const uint64_t total = (uint64_t)a.rows * (uint64_t)a.ngr;
  const unsigned grid = vgrid(total, kPackGroups, 65536);
  if (dtype == CCM_I64)
    k_vlb_pack<int64_t><<<grid, kVThreads, lds, s>>>((const int64_t *)dense, a.rows, a.cols,
                                                     a.ngr, a.k, a.sgn, a.row_bit, a.grp, nbits,
                                                     span_words, out);
  else
    k_vlb_pack<int32_t><<<grid, kVThreads, lds, s>>>((const int32_t *)dense, a.rows, a.cols,
                                                     a.ngr, a.k, a.sgn, a.row_bit, a.grp, nbits,
                                                     span_words, out);
  return hipGetLastError();
}

hipError_t launch_vlb_decode(const VlbView &a, int64_t *out, hipStream_t s) {
  const unsigned grid = vgrid((uint64_t)a.rows * (uint64_t)a.ngr, kVThreads, 65536);
  k_vlb_decode<<<grid, kVThreads, 0, s>>>(a.w, a.row_bit, a.grp, a.rows, a.cols, a.ngr, a.k,
                                          a.sgn, out);
  return hipGetLastError();
}

hipError_t launch_vlb_get(const VlbView &a, int64_t i, int64_t j, int64_t *out, hipStream_t s) {
  k_vlb_get<<<1, 64, 0, s>>>(a.w, a.row_bit, a.grp, a.ngr, i, j, a.k, a.sgn, out);
  return hipGetLastError();
}

hipError_t launch_vlb_matvec(const VlbView &a, const void *x, int xdtype, int64_t *y,
                             hipStream_t s) {
  const bool staged = xdtype == CCM_I32 && ((uintptr_t)x % 16) == 0;
  if (staged) {
    const int32_t *xi = (const int32_t *)x;
    return a.sgn ? launch_mv_staged<true>(a, xi, y, s) : launch_mv_staged<false>(a, xi, y, s);
  }
  const int64_t nchunk = (a.ngr + kVThreads - 1) / kVThreads;
  if (nchunk > 1) {
    hipError_t e = launch_fill_i64(y, (uint64_t)a.rows, 0, s);
    if (e != hipSuccess) return e;
  }
  const unsigned grid = vgrid((uint64_t)a.rows * (uint64_t)nchunk, 1, 65536);
  if (xdtype == CCM_I64)
    k_vlb_mv_gen<int64_t><<<grid, kVThreads, 0, s>>>(a.w, a.row_bit, a.grp, a.rows, a.cols, a.ngr,
                                                     a.k, a.sgn, (const int64_t *)x, y);
  else
    k_vlb_mv_gen<int32_t><<<grid, kVThreads, 0, s>>>(a.w, a.row_bit, a.grp, a.rows, a.cols, a.ngr,
                                                     a.k, a.sgn, (const int32_t *)x, y);
  return hipGetLastError();
}

}  // namespace ccm
