// Floats in fixed point (the Conclusion allows floats if some precision is
// given up): the quantization that turns a float matrix into the integer
// matrix Method 1 packs, the exact largest magnitude that picks its scale,
// and the conversion of integer results back to floats (gfx950).
//
//   q = round-half-to-even(v * 2^f): v_ldexp_f64 scales exactly (or leaves
//   the double range: then |v 2^f| is far beyond 2^62, or below 2^-1022,
//   where the rounding gives 0 either way), v_rndne_f64 rounds half to even.
//   Back: int64 -> double rounds half to even (one rounding: the high half
//   scaled by 2^32 plus the exact low half), ldexp by -f, and for float32 one
//   more rounding (v_cvt_f32_f64, round to nearest even).
#include "ccm_internal.hpp"
#include "group_codec.hpp"

#include <cmath>

namespace ccm {
namespace {

constexpr int kFxThreads = 256;

// |v| as the bit pattern of a non-negative double: these order like the
// values, and NaN and the infinities have the largest ones (>= 0x7FF0...).
__device__ __forceinline__ int64_t abs_bits(double v) {
  return __double_as_longlong(fabs(v));
}

template <typename F>
__global__ __launch_bounds__(kFxThreads) void k_float_absmax(const F *__restrict__ v, uint64_t n,
                                                             RangeSlot *slot) {
  int64_t hi = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // four loads in flight per lane, then the tail
  for (; i + 3 * stride < n; i += 4 * stride) {
    F t[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) t[u] = v[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t b = abs_bits((double)t[u]);
      hi = b > hi ? b : hi;
    }
  }
  for (; i < n; i += stride) {
    const int64_t b = abs_bits((double)v[i]);
    hi = b > hi ? b : hi;
  }
  block_range_commit(INT64_MAX, hi, 0, slot);
}

// q = RNE(v 2^f) with the range of q folded into slot.  A NaN or infinity
// sets the slot's flag; a |v 2^f| >= 2^62, or for int32 output a q outside
// int32, folds INT64_MAX into the maximum (every valid q is below 2^62 in
// magnitude).
// q may be null: the range and the checks only (the pass before packing
// straight from the floats)
template <typename F, typename Q>
__global__ __launch_bounds__(kFxThreads) void k_quantize(const F *__restrict__ v, uint64_t n,
                                                         int f, Q *__restrict__ q,
                                                         RangeSlot *slot) {
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  int bad = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  auto one = [&](F x, uint64_t e) {
    const double d = (double)x;
    const double t = ldexp(d, f);
    int64_t r = 0;
    if (!isfinite(d)) {
      bad = 1;
    } else if (!(fabs(t) < 0x1p62)) {
      hi = INT64_MAX;
    } else {
      r = (int64_t)rint(t);
      if (sizeof(Q) == 4 && (r < INT32_MIN || r > INT32_MAX)) {
        hi = INT64_MAX;
        r = 0;
      } else {
        lo = r < lo ? r : lo;
        hi = r > hi ? r : hi;
      }
    }
    if (q) q[e] = (Q)r;
  };
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    F t[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) t[u] = v[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) one(t[u], i + u * stride);
  }
  for (; i < n; i += stride) one(v[i], i);
  block_range_commit(lo, hi, bad, slot);
}

template <typename F>
__global__ __launch_bounds__(kFxThreads) void k_dequantize(const int64_t *__restrict__ q,
                                                           uint64_t n, int f,
                                                           F *__restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    int64_t t[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) t[u] = q[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) out[i + u * stride] = (F)ldexp((double)t[u], -f);
  }
  for (; i < n; i += stride) out[i] = (F)ldexp((double)q[i], -f);
}

// Packs RNE(v 2^f) at `bits` straight from the floats: a block stages its
// 32 x 128 floats through LDS with 16-byte loads, then lane g quantizes group
// g's 32 values and encodes its b words (as the integer packing kernel does).
// The values were checked by the range pass before (finite, inside the
// width), so no test is repeated here.
constexpr int kFxTile = 128;
constexpr int kFxPad = kGroup + 1;

template <typename F>
__global__ __launch_bounds__(kFxTile) void k_compress_fx(const F *__restrict__ d, uint64_t n,
                                                         int f, int bits,
                                                         uint32_t *__restrict__ out,
                                                         uint64_t cap32, uint64_t ngroups,
                                                         int aligned16) {
  constexpr int PER = 16 / sizeof(F);
  constexpr int NLOAD = kFxTile * kGroup / (kFxTile * PER);
  // the input tile, reused for the block's packed words (up to 64 a group)
  constexpr size_t kBytes = sizeof(F) * kFxTile * kFxPad > 4 * (size_t)kFxTile * 64
                                ? sizeof(F) * kFxTile * kFxPad
                                : 4 * (size_t)kFxTile * 64;
  __shared__ __align__(16) unsigned char lds[kBytes];
  F *tile = reinterpret_cast<F *>(lds);
  const uint64_t g0 = (uint64_t)blockIdx.x * kFxTile;
  const uint64_t e0 = g0 * kGroup;
  if (aligned16 && e0 + (uint64_t)kFxTile * kGroup <= n) {
    const uint4 *src = reinterpret_cast<const uint4 *>(d + e0);
    uint4 r[NLOAD];
#pragma unroll
    for (int j = 0; j < NLOAD; ++j) r[j] = src[threadIdx.x + j * kFxTile];
#pragma unroll
    for (int j = 0; j < NLOAD; ++j) {
      const int q = (threadIdx.x + j * kFxTile) * PER;
      const F *t = reinterpret_cast<const F *>(&r[j]);
#pragma unroll
      for (int u = 0; u < PER; ++u) tile[q + u + (q >> 5)] = t[u];
    }
  } else {
    for (int q = threadIdx.x; q < kFxTile * kGroup; q += kFxTile) {
      const uint64_t e = e0 + q;
      tile[q + (q >> 5)] = e < n ? d[e] : F(0);
    }
  }
  __syncthreads();
  int64_t v[kGroup];
  const F *row = tile + threadIdx.x * kFxPad;
#pragma unroll
  for (int i = 0; i < kGroup; ++i) v[i] = (int64_t)rint(ldexp((double)row[i], f));
  // group g into LDS, then the block's contiguous run of words (as the
  // integer packing kernel)
  __syncthreads();
  uint32_t *s_out = reinterpret_cast<uint32_t *>(lds);
  codec::encode_rt(v, bits, s_out + threadIdx.x * bits, (uint64_t)bits);
  __syncthreads();
  store_block_run(s_out, bits, out, cap32);
  (void)ngroups;
}

unsigned fx_grid(uint64_t n) {
  const uint64_t g = (n + 4ull * kFxThreads - 1) / (4ull * kFxThreads);
  return (unsigned)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

}  // namespace

hipError_t launch_float_absmax(const void *v, int dtype, uint64_t n, RangeSlot *slot,
                               hipStream_t s) {
  if (dtype == CCM_F64)
    k_float_absmax<double><<<fx_grid(n), kFxThreads, 0, s>>>((const double *)v, n, slot);
  else
    k_float_absmax<float><<<fx_grid(n), kFxThreads, 0, s>>>((const float *)v, n, slot);
  return hipGetLastError();
}

hipError_t launch_quantize(const void *v, int dtype, uint64_t n, int frac_bits, void *q,
                           int qdtype, RangeSlot *slot, hipStream_t s) {
  const unsigned g = fx_grid(n);
  if (dtype == CCM_F64 && qdtype == CCM_I64)
    k_quantize<double, int64_t><<<g, kFxThreads, 0, s>>>((const double *)v, n, frac_bits,
                                                         (int64_t *)q, slot);
  else if (dtype == CCM_F64)
    k_quantize<double, int32_t><<<g, kFxThreads, 0, s>>>((const double *)v, n, frac_bits,
                                                         (int32_t *)q, slot);
  else if (qdtype == CCM_I64)
    k_quantize<float, int64_t><<<g, kFxThreads, 0, s>>>((const float *)v, n, frac_bits,
                                                        (int64_t *)q, slot);
  else
    k_quantize<float, int32_t><<<g, kFxThreads, 0, s>>>((const float *)v, n, frac_bits,
                                                        (int32_t *)q, slot);
  return hipGetLastError();
}

hipError_t launch_compress_fx(const void *v, int dtype, uint64_t n, int frac_bits, int bits,
                              uint32_t *out, uint64_t cap32, hipStream_t s) {
  const uint64_t ngroups = (cap32 + bits - 1) / bits;
  const uint64_t grid = (ngroups + kFxTile - 1) / kFxTile;
  if (grid > 0x7fffffffull) return hipErrorInvalidValue;
  const int al = ((uintptr_t)v % 16) == 0;
  if (dtype == CCM_F64)
    k_compress_fx<double><<<(unsigned)grid, kFxTile, 0, s>>>((const double *)v, n, frac_bits,
                                                             bits, out, cap32, ngroups, al);
  else
    k_compress_fx<float><<<(unsigned)grid, kFxTile, 0, s>>>((const float *)v, n, frac_bits,
                                                            bits, out, cap32, ngroups, al);
  return hipGetLastError();
}

hipError_t launch_dequantize(const int64_t *q, uint64_t n, int frac_bits, int dtype, void *out,
                             hipStream_t s) {
  if (dtype == CCM_F64)
    k_dequantize<double><<<fx_grid(n), kFxThreads, 0, s>>>(q, n, frac_bits, (double *)out);
  else
    k_dequantize<float><<<fx_grid(n), kFxThreads, 0, s>>>(q, n, frac_bits, (float *)out);
  return hipGetLastError();
}

}  // namespace ccm
