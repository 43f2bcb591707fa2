// Column-major unravel (Methods, "Matrix compression": a matrix may be
// unravelled by column as well as by row).  A matrix A (R x C) unravelled by
// column has exactly the stream of A^T (C x R) unravelled by row, so the
// library describes it by A^T's row-major descriptor and needs two kernels
// beyond the row-major ones:
//   * packing a dense row-major A column by column, and
//   * y = A^T x over a row-major stream (matvec_t_impl.hpp), which is y = A x
//     for the column-major matrix.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "ccm_internal.hpp"
#include "group_codec.hpp"

namespace ccm {
namespace mvt {

int compute_units_t() {
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

hipError_t launch_t_widths_1(const uint32_t *, int64_t, int64_t, int, int, const void *, int,
                             int64_t *, int64_t *, uint64_t, hipStream_t);
hipError_t launch_t_widths_2(const uint32_t *, int64_t, int64_t, int, int, const void *, int,
                             int64_t *, int64_t *, uint64_t, hipStream_t);
hipError_t launch_t_widths_3(const uint32_t *, int64_t, int64_t, int, int, const void *, int,
                             int64_t *, int64_t *, uint64_t, hipStream_t);
hipError_t launch_t_widths_4(const uint32_t *, int64_t, int64_t, int, int, const void *, int,
                             int64_t *, int64_t *, uint64_t, hipStream_t);

}  // namespace mvt

namespace {

constexpr int kCmThreads = 128;

__global__ void k_zero_tail(uint32_t *p, uint64_t from, uint64_t to) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = from + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < to; e += stride)
    p[e] = 0;
}

// rows % 32 == 0: group g = j * (rows / 32) + q holds rows 32q .. 32q + 31 of
// column j.  Block (column block, q): lane t owns column j = 128 * bx + t and
// reads its 32 values row by row, so each load instruction of a wave reads 64
// consecutive columns of one row.
template <typename T>
__global__ __launch_bounds__(kCmThreads) void k_compress_cm_tile(const T *__restrict__ d,
                                                                 int64_t rows, int64_t cols,
                                                                 int bits,
                                                                 uint32_t *__restrict__ out,
                                                                 uint64_t cap32) {
  const int64_t j = (int64_t)blockIdx.x * kCmThreads + threadIdx.x;
  const int64_t q = blockIdx.y;
  if (j >= cols) return;
  int64_t v[kGroup];
  const T *src = d + (uint64_t)(32 * q) * (uint64_t)cols + (uint64_t)j;
#pragma unroll
  for (int i = 0; i < kGroup; ++i) v[i] = (int64_t)src[(uint64_t)i * (uint64_t)cols];
  const uint64_t g = (uint64_t)j * (uint64_t)(rows / kGroup) + (uint64_t)q;
  const uint64_t w0 = g * (uint64_t)bits;
  codec::encode_rt(v, bits, out + w0, cap32 - w0);
}

// Any shape: lane g packs stream elements 32g .. 32g + 31, element e being
// (e % rows, e / rows); groups past the last element write zeros, so every
// word of the capacity is written.
template <typename T>
__global__ __launch_bounds__(kCmThreads) void k_compress_cm_gen(const T *__restrict__ d,
                                                                int64_t rows, int64_t cols,
                                                                int bits,
                                                                uint32_t *__restrict__ out,
                                                                uint64_t cap32,
                                                                uint64_t ngroups) {
  const uint64_t n = (uint64_t)rows * (uint64_t)cols;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups; g += stride) {
    const uint64_t e0 = g * kGroup;
    uint64_t j = e0 / (uint64_t)rows;
    uint64_t i = e0 - j * (uint64_t)rows;
    int64_t v[kGroup];
#pragma unroll
    for (int t = 0; t < kGroup; ++t) {
      v[t] = e0 + t < n ? (int64_t)d[i * (uint64_t)cols + j] : 0;
      if (++i == (uint64_t)rows) {
        i = 0;
        ++j;
      }
    }
    const uint64_t w0 = g * (uint64_t)bits;
    codec::encode_rt(v, bits, out + w0, cap32 - w0);
  }
}

// Column totals of the row splits' partial sums.  Block = 64 columns x 4
// waves: wave q adds splits q, q + 4, ... of its lane's column (loads
// coalesced across the columns, all of a lane's in flight together), and the
// four partials meet in LDS.
__global__ __launch_bounds__(256) void k_sum_splits(const int64_t *__restrict__ part,
                                                    int64_t splits, int64_t cols,
                                                    int64_t *__restrict__ y) {
  __shared__ uint64_t red[4][64];
  const int q = threadIdx.x >> 6, cl = threadIdx.x & 63;
  for (uint64_t c0 = (uint64_t)blockIdx.x * 64; c0 < (uint64_t)cols;
       c0 += (uint64_t)gridDim.x * 64) {
    const uint64_t c = c0 + cl;
    uint64_t t = 0;
    if (c < (uint64_t)cols) {
#pragma unroll 8
      for (int64_t k = q; k < splits; k += 4)
        t += (uint64_t)part[(uint64_t)k * (uint64_t)cols + c];
    }
    red[q][cl] = t;
    __syncthreads();
    if (q == 0 && c < (uint64_t)cols)
      y[c] = (int64_t)(red[0][cl] + red[1][cl] + red[2][cl] + red[3][cl]);
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_compress_cm(const void *dense, int dtype, int64_t rows, int64_t cols,
                              int bits, uint32_t *out, uint64_t cap32, hipStream_t s) {
  const uint64_t n = (uint64_t)rows * (uint64_t)cols;
  if (rows % kGroup == 0 && rows / kGroup <= 65535) {
    dim3 grid((unsigned)((cols + kCmThreads - 1) / kCmThreads), (unsigned)(rows / kGroup));
    if (dtype == CCM_I64)
      k_compress_cm_tile<int64_t><<<grid, kCmThreads, 0, s>>>((const int64_t *)dense, rows, cols,
                                                              bits, out, cap32);
    else
      k_compress_cm_tile<int32_t><<<grid, kCmThreads, 0, s>>>((const int32_t *)dense, rows, cols,
                                                              bits, out, cap32);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint64_t used = n / kGroup * (uint64_t)bits;  // whole groups: n % 32 == 0
    if (used < cap32) {
      uint64_t g = (cap32 - used + 255) / 256;
      k_zero_tail<<<(unsigned)(g < 4096 ? g : 4096), 256, 0, s>>>(out, used, cap32);
      e = hipGetLastError();
    }
    return e;
  }
  const uint64_t ngroups = (cap32 + bits - 1) / bits;
  uint64_t grid = (ngroups + kCmThreads - 1) / kCmThreads;
  grid = grid < 1 ? 1 : (grid > 65536 ? 65536 : grid);
  if (dtype == CCM_I64)
    k_compress_cm_gen<int64_t><<<(unsigned)grid, kCmThreads, 0, s>>>(
        (const int64_t *)dense, rows, cols, bits, out, cap32, ngroups);
  else
    k_compress_cm_gen<int32_t><<<(unsigned)grid, kCmThreads, 0, s>>>(
        (const int32_t *)dense, rows, cols, bits, out, cap32, ngroups);
  return hipGetLastError();
}

hipError_t launch_matvec_t(const uint32_t *w, int64_t rows, int64_t cols, int bits, int sgn,
                           const void *x, int xdtype, int64_t *y, int64_t *part,
                           uint64_t part_words, hipStream_t s) {
  if (bits <= 16)
    return mvt::launch_t_widths_1(w, rows, cols, bits, sgn, x, xdtype, y, part, part_words, s);
  if (bits <= 32)
    return mvt::launch_t_widths_2(w, rows, cols, bits, sgn, x, xdtype, y, part, part_words, s);
  if (bits <= 48)
    return mvt::launch_t_widths_3(w, rows, cols, bits, sgn, x, xdtype, y, part, part_words, s);
  return mvt::launch_t_widths_4(w, rows, cols, bits, sgn, x, xdtype, y, part, part_words, s);
}

// Library-owned partial sums of y = A^T x for callers that cannot allocate:
// kMaxSplitsT rows of kNoAllocColsT int64 (16 MB per device, held until the
// process ends).  In host code `scratch` names a host-side stand-in, never
// the device array: its device address is looked up once per device below
// and only that address reaches kernels.  Calls that overlap on one device
// share (and race on) it.
static __device__ __align__(256) int64_t scratch[kMaxSplitsT * kNoAllocColsT];

hipError_t static_matvec_t_scratch(int64_t **ptr, uint64_t *words) {
  static std::mutex mu;
  static std::vector<int64_t *> per_dev;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  if ((size_t)dev >= per_dev.size()) per_dev.resize((size_t)dev + 1, nullptr);
  if (!per_dev[(size_t)dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    per_dev[(size_t)dev] = (int64_t *)p;
  }
  *ptr = per_dev[(size_t)dev];
  *words = (uint64_t)kMaxSplitsT * (uint64_t)kNoAllocColsT;
  return hipSuccess;
}

hipError_t launch_sum_splits(const int64_t *part, int64_t splits, int64_t cols, int64_t *y,
                             hipStream_t s) {
  uint64_t g = ((uint64_t)cols + 63) / 64;
  g = g < 1 ? 1 : (g > 65536 ? 65536 : g);
  k_sum_splits<<<(unsigned)g, 256, 0, s>>>(part, splits, cols, y);
  return hipGetLastError();
}

}  // namespace ccm
