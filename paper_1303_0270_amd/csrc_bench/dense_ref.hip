// Comparison kernels for the benchmark, outside the compressed-matrix
// library: a dense int32 matvec (the "Gelem/s vs dense int32" reference, laid
// out like the packed kernel: x panel in LDS, 4 rows per wave, 16-byte loads)
// and an HBM read-bandwidth probe.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 256, kRows = 4, kPanel = 8192;

__global__ __launch_bounds__(kThreads) void k_dense_mv(const int32_t *__restrict__ A, int64_t rows,
                                                       int64_t cols, const int32_t *__restrict__ x,
                                                       int64_t *__restrict__ y, int atomic_out) {
  __shared__ int4 xs[kPanel / 4];
  const int64_t c0 = (int64_t)blockIdx.y * kPanel;
  const int64_t pc = cols - c0 < kPanel ? cols - c0 : kPanel;
  int32_t *xs32 = reinterpret_cast<int32_t *>(xs);
  for (int q = threadIdx.x; q < (int)((pc + 3) / 4 * 4); q += kThreads)
    xs32[q] = q < pc ? x[c0 + q] : 0;
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nrb = (rows + 4 * kRows - 1) / (4 * kRows);
  const bool vec = (cols % 4) == 0;
  for (int64_t rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
    const int64_t r0 = rb * 4 * kRows + wave * kRows;
    int64_t acc[kRows] = {0, 0, 0, 0};
    if (vec) {
      for (int q = lane; q < (int)(pc / 4); q += 64) {
        const int4 xv = xs[q];
#pragma unroll
        for (int rr = 0; rr < kRows; ++rr) {
          if (r0 + rr < rows) {
            const int4 a = *reinterpret_cast<const int4 *>(A + (r0 + rr) * cols + c0 + 4 * q);
            acc[rr] += (int64_t)a.x * xv.x + (int64_t)a.y * xv.y + (int64_t)a.z * xv.z +
                       (int64_t)a.w * xv.w;
          }
        }
      }
    } else {
      for (int q = lane; q < (int)pc; q += 64) {
        const int32_t xv = xs32[q];
#pragma unroll
        for (int rr = 0; rr < kRows; ++rr)
          if (r0 + rr < rows) acc[rr] += (int64_t)A[(r0 + rr) * cols + c0 + q] * xv;
      }
    }
#pragma unroll
    for (int rr = 0; rr < kRows; ++rr) {
      int64_t v = acc[rr];
      for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
      if (lane == 0 && r0 + rr < rows) {
        if (atomic_out)
          atomicAdd((unsigned long long *)&y[r0 + rr], (unsigned long long)v);
        else
          y[r0 + rr] = v;
      }
    }
  }
}

__global__ void k_zero(int64_t *y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 0;
}

__global__ __launch_bounds__(256) void k_read(const uint4 *__restrict__ p, uint64_t n16,
                                              uint32_t *sink) {
  uint32_t acc = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
    const uint4 v = p[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x9e3779b9u) sink[0] = acc;  // keeps the loads; practically never stores
}

}  // namespace

extern "C" int ccmb_dense_matvec_i32(const int32_t *A, int64_t rows, int64_t cols,
                                     const int32_t *x, int64_t *y, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const int64_t npanels = (cols + kPanel - 1) / kPanel;
  const int64_t nrb = (rows + 4 * kRows - 1) / (4 * kRows);
  int64_t gx = nrb < 1024 ? nrb : 1024;
  if (npanels > 1) {
    k_zero<<<(unsigned)((rows + 255) / 256), 256, 0, s>>>(y, rows);
    gx = gx < 2048 / npanels ? gx : (2048 / npanels > 0 ? 2048 / npanels : 1);
  }
  k_dense_mv<<<dim3((unsigned)gx, (unsigned)npanels), kThreads, 0, s>>>(A, rows, cols, x, y,
                                                                       npanels > 1);
  return hipGetLastError() == hipSuccess ? 0 : -6;
}

extern "C" int ccmb_read_bytes(const void *buf, uint64_t nbytes, uint32_t *sink, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  k_read<<<4096, 256, 0, s>>>((const uint4 *)buf, nbytes / 16, sink);
  return hipGetLastError() == hipSuccess ? 0 : -6;
}
