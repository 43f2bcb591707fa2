// Group codec: a group of 32 consecutive elements at field width b is exactly
// b 32-bit words (see ccm_internal.hpp).  With b a compile-time constant the
// lane loads all b words at once and every field sits at a fixed offset:
// one v_bfe (plus a v_alignbit when it straddles a word) per field for
// b <= 32, a two-word funnel for b > 32.  The runtime-width entry points
// dispatch over b with a switch, so each wave runs straight-line code for
// its width.
#pragma once

#include "ccm_internal.hpp"

namespace ccm {
namespace codec {

// Unsigned field i of a group held in w[0..B-1].
template <int B>
__device__ __forceinline__ uint64_t field(const uint32_t *w, int i) {
  const int p = i * B;
  const int k = p >> 5;
  const int off = p & 31;
  if constexpr (B <= 32) {
    uint32_t src;
    if (off + B <= 32)
      src = w[k] >> off;
    else
      src = __builtin_amdgcn_alignbit(w[k + 1], w[k], off);
    return (uint64_t)(B == 32 ? src : (src & ((1u << (B & 31)) - 1u)));
  } else {
    const uint32_t lo = off ? __builtin_amdgcn_alignbit(w[k + 1], w[k], off) : w[k];
    uint32_t hi;
    if (off + B > 64)
      hi = __builtin_amdgcn_alignbit(w[k + 2], w[k + 1], off);
    else
      hi = w[k + 1] >> off;
    if constexpr (B < 64) hi &= (1u << (B - 32)) - 1u;
    return ((uint64_t)hi << 32) | lo;
  }
}

template <int B>
__device__ __forceinline__ void decode(const uint32_t *__restrict__ p, int sgn, int64_t *v) {
  uint32_t w[B];
#pragma unroll
  for (int k = 0; k < B; ++k) w[k] = p[k];
#pragma unroll
  for (int i = 0; i < kGroup; ++i) {
    const uint64_t u = field<B>(w, i);
    v[i] = sgn ? sext64(u, B) : (int64_t)u;
  }
}

// Packs v[0..31] at width B (low B bits of each two's complement) into
// out[0..B-1]; stores past `limit` words (counted from out) are dropped.
template <int B>
__device__ __forceinline__ void encode(const int64_t *v, uint32_t *__restrict__ out,
                                       uint64_t limit) {
  uint32_t w[B];
#pragma unroll
  for (int k = 0; k < B; ++k) w[k] = 0;
#pragma unroll
  for (int i = 0; i < kGroup; ++i) {
    const uint64_t u = (uint64_t)v[i] & mask64(B);
    const int p = i * B;
    const int k = p >> 5;
    const int off = p & 31;
    w[k] |= (uint32_t)(u << off);
    if (off + B > 32) w[k + 1] |= (uint32_t)(u >> (32 - off));
    if (off + B > 64) w[k + 2] |= (uint32_t)(u >> (64 - off));
  }
  if (limit >= (uint64_t)B) {
    if constexpr (B % 4 == 0) {
#pragma unroll
      for (int k = 0; k < B; k += 4)
        *reinterpret_cast<uint4 *>(out + k) = make_uint4(w[k], w[k + 1], w[k + 2], w[k + 3]);
    } else if constexpr (B % 2 == 0) {
#pragma unroll
      for (int k = 0; k < B; k += 2)
        *reinterpret_cast<uint2 *>(out + k) = make_uint2(w[k], w[k + 1]);
    } else {
#pragma unroll
      for (int k = 0; k < B; ++k) out[k] = w[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < B; ++k)
      if ((uint64_t)k < limit) out[k] = w[k];
  }
}

// Field i of a group as a 32-bit value: one bit-field extract (v_bfe_i32
// sign-extending when S, v_bfe_u32 otherwise), after a funnel shift when the
// field straddles two words.
template <int B, bool S>
__device__ __forceinline__ uint32_t field32(const uint32_t *w, int i) {
  const int p = i * B;
  const int k = p >> 5;
  const int off = p & 31;
  if constexpr (B == 32) {
    return w[k];
  } else {
    uint32_t src;
    int o;
    if (off + B <= 32) {
      src = w[k];
      o = off;
    } else {
      src = __builtin_amdgcn_alignbit(w[k + 1], w[k], off);
      o = 0;
    }
    if constexpr (S)
      return (uint32_t)__builtin_amdgcn_sbfe((int32_t)src, o, B);
    else
      return __builtin_amdgcn_ubfe(src, o, B);
  }
}

// 32-bit values (b <= 32): fields zero-extended, or sign-extended when sgn
// (tested once per group, not per field).
template <int B>
__device__ __forceinline__ void decode32(const uint32_t *__restrict__ p, int sgn, uint32_t *v) {
  static_assert(B <= 32, "32-bit decode");
  uint32_t w[B];
#pragma unroll
  for (int k = 0; k < B; ++k) w[k] = p[k];
  if (sgn) {
#pragma unroll
    for (int i = 0; i < kGroup; ++i) v[i] = field32<B, true>(w, i);
  } else {
#pragma unroll
    for (int i = 0; i < kGroup; ++i) v[i] = field32<B, false>(w, i);
  }
}

template <int B>
__device__ __forceinline__ void encode32(const uint32_t *v, uint32_t *__restrict__ out,
                                         uint64_t limit) {
  static_assert(B <= 32, "32-bit encode");
  uint32_t w[B];
#pragma unroll
  for (int k = 0; k < B; ++k) w[k] = 0;
#pragma unroll
  for (int i = 0; i < kGroup; ++i) {
    const uint32_t u = B == 32 ? v[i] : (v[i] & ((1u << (B & 31)) - 1u));
    const int p = i * B;
    const int k = p >> 5;
    const int off = p & 31;
    w[k] |= u << off;
    if (off + B > 32) w[k + 1] |= u >> (32 - off);
  }
  if (limit >= (uint64_t)B) {
    if constexpr (B % 4 == 0) {
#pragma unroll
      for (int k = 0; k < B; k += 4)
        *reinterpret_cast<uint4 *>(out + k) = make_uint4(w[k], w[k + 1], w[k + 2], w[k + 3]);
    } else if constexpr (B % 2 == 0) {
#pragma unroll
      for (int k = 0; k < B; k += 2)
        *reinterpret_cast<uint2 *>(out + k) = make_uint2(w[k], w[k + 1]);
    } else {
#pragma unroll
      for (int k = 0; k < B; ++k) out[k] = w[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < B; ++k)
      if ((uint64_t)k < limit) out[k] = w[k];
  }
}

#define CCM_WIDTH_CASES_32(X)                                                                \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)   \
  X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30)      \
  X(31) X(32)

#define CCM_WIDTH_CASES(X)                                                                   \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)   \
  X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30)      \
  X(31) X(32) X(33) X(34) X(35) X(36) X(37) X(38) X(39) X(40) X(41) X(42) X(43) X(44)      \
  X(45) X(46) X(47) X(48) X(49) X(50) X(51) X(52) X(53) X(54) X(55) X(56) X(57) X(58)      \
  X(59) X(60) X(61) X(62) X(63) X(64)

// Runtime-width entry points (b is wave-uniform).
__device__ __forceinline__ void decode_rt(const uint32_t *__restrict__ p, int bits, int sgn,
                                          int64_t *v) {
  switch (bits) {
#define CCM_DEC_CASE(b) \
  case b:               \
    decode<b>(p, sgn, v); \
    break;
    CCM_WIDTH_CASES(CCM_DEC_CASE)
#undef CCM_DEC_CASE
    default:
      break;
  }
}

__device__ __forceinline__ void encode_rt(const int64_t *v, int bits, uint32_t *__restrict__ out,
                                          uint64_t limit) {
  switch (bits) {
#define CCM_ENC_CASE(b)        \
  case b:                      \
    encode<b>(v, out, limit);  \
    break;
    CCM_WIDTH_CASES(CCM_ENC_CASE)
#undef CCM_ENC_CASE
    default:
      break;
  }
}

__device__ __forceinline__ void decode32_rt(const uint32_t *__restrict__ p, int bits, int sgn,
                                            uint32_t *v) {
  switch (bits) {
#define CCM_DEC32_CASE(b)    \
  case b:                    \
    decode32<b>(p, sgn, v);  \
    break;
    CCM_WIDTH_CASES_32(CCM_DEC32_CASE)
#undef CCM_DEC32_CASE
    default:
      break;
  }
}

__device__ __forceinline__ void encode32_rt(const uint32_t *v, int bits, uint32_t *__restrict__ out,
                                            uint64_t limit) {
  switch (bits) {
#define CCM_ENC32_CASE(b)         \
  case b:                         \
    encode32<b>(v, out, limit);   \
    break;
    CCM_WIDTH_CASES_32(CCM_ENC32_CASE)
#undef CCM_ENC32_CASE
    default:
      break;
  }
}

}  // namespace codec
}  // namespace ccm
