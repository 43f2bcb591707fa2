// C ABI of libccm: argument and descriptor validation, width arithmetic, the
// blocking range ("plan") passes and kernel dispatch.  See include/ccm.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "ccm.h"
#include "ccm_internal.hpp"

namespace {

bool log_enabled() {
  static const bool on = std::getenv("CCM_LOG") != nullptr;
  return on;
}

int dev_err(hipError_t e, const char *where) {
  if (e == hipSuccess) return CCM_OK;
  if (log_enabled()) std::fprintf(stderr, "ccm: %s: %s\n", where, hipGetErrorString(e));
  if (e == hipErrorOutOfMemory) return CCM_E_NOMEM;
  return CCM_E_DEVICE;
}

#define CCM_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return dev_err(e_, #call);    \
  } while (0)

// Blocking reductions share one device slot and one pinned host mirror per
// device, used under a lock (each use ends with a stream synchronize).
struct DeviceCtx {
  ccm::RangeSlot *slot = nullptr;
  ccm::RangeSlot *host = nullptr;
  int64_t *one = nullptr;    // single-element get
  uint64_t *sums = nullptr;  // spread sum pairs (method choice)
};
std::mutex g_mu;
std::vector<DeviceCtx> g_ctx;

int device_ctx(DeviceCtx **out) {
  int dev = 0;
  CCM_HIP(hipGetDevice(&dev));
  if ((size_t)dev >= g_ctx.size()) g_ctx.resize((size_t)dev + 1);
  DeviceCtx &c = g_ctx[(size_t)dev];
  if (!c.slot) {
    void *p = nullptr;
    CCM_HIP(hipMalloc(&p, ccm::kRangeBytes + 256 + ccm::kSumBytes));
    c.slot = (ccm::RangeSlot *)p;
    c.one = (int64_t *)((char *)p + ccm::kRangeBytes);
    c.sums = (uint64_t *)((char *)p + ccm::kRangeBytes + 256);
    void *h = nullptr;
    CCM_HIP(hipHostMalloc(&h, ccm::kRangeBytes + 64 + ccm::kSumBytes, hipHostMallocDefault));
    c.host = (ccm::RangeSlot *)h;
  }
  *out = &c;
  return CCM_OK;
}

// Copies the spread range slots back and folds them into one result.
int read_slot(DeviceCtx *c, hipStream_t s, ccm::RangeSlot *res) {
  CCM_HIP(hipMemcpyAsync(c->host, c->slot, ccm::kRangeBytes, hipMemcpyDeviceToHost, s));
  CCM_HIP(hipStreamSynchronize(s));
  ccm::RangeSlot r = c->host[0];
  for (int i = 1; i < ccm::kRangeSpread; ++i) {
    const ccm::RangeSlot &t = c->host[ccm::kRangeStride * i];
    r.vmin = t.vmin < r.vmin ? t.vmin : r.vmin;
    r.vmax = t.vmax > r.vmax ? t.vmax : r.vmax;
    r.flag |= t.flag;
  }
  *res = r;
  return CCM_OK;
}

int width_rule(int64_t vmin, int64_t vmax, int32_t *bits, int32_t *sgn) {
  if (vmin > vmax) return CCM_E_INVAL;
  auto bitlen = [](uint64_t u) {
    int L = 0;
    while (L < 64 && (u >> L) != 0) ++L;
    return L;
  };
  if (vmin >= 0) {
    *sgn = 0;
    *bits = vmax <= 1 ? 1 : bitlen((uint64_t)vmax);
  } else {
    const int lo = bitlen(~(uint64_t)vmin);  // -(vmin+1)
    const int hi = vmax > 0 ? bitlen((uint64_t)vmax) : 0;
    *sgn = 1;
    *bits = 1 + (lo > hi ? lo : hi);
  }
  return CCM_OK;
}

bool shape_ok(int64_t rows, int64_t cols) {
  if (rows < 1 || cols < 1) return false;
  // keep rows*cols*64 inside uint64
  const unsigned __int128 n = (unsigned __int128)rows * (unsigned __int128)cols;
  return n <= ((unsigned __int128)1 << 57);
}

uint64_t nelem(const ccm_desc *d) { return (uint64_t)d->rows * (uint64_t)d->cols; }

// A descriptor is valid when its width is the width rule of its range and the
// word count matches; with need_payload, payload must be set.
int check_desc(const ccm_desc *d, bool need_payload) {
  if (!d) return CCM_E_INVAL;
  if (!shape_ok(d->rows, d->cols)) return CCM_E_INVAL;
  int32_t b = 0, s = 0;
  if (width_rule(d->vmin, d->vmax, &b, &s) != CCM_OK) return CCM_E_INVAL;
  if (b != d->bits || s != d->is_signed) return CCM_E_INVAL;
  if (d->words != ccm_words(d->rows, d->cols, d->bits)) return CCM_E_INVAL;
  if (need_payload && !d->payload) return CCM_E_INVAL;
  return CCM_OK;
}

int fill_desc(int64_t rows, int64_t cols, int64_t vmin, int64_t vmax, ccm_desc *out) {
  int32_t b = 0, s = 0;
  int rc = width_rule(vmin, vmax, &b, &s);
  if (rc != CCM_OK) return rc;
  out->rows = rows;
  out->cols = cols;
  out->vmin = vmin;
  out->vmax = vmax;
  out->bits = b;
  out->is_signed = s;
  out->words = ccm_words(rows, cols, b);
  out->payload = nullptr;
  return CCM_OK;
}

ccm::PackedOperand operand(const ccm_desc *d) {
  return ccm::PackedOperand{(const uint32_t *)d->payload, d->bits, d->is_signed};
}

uint64_t max_abs(int64_t lo, int64_t hi) {
  const uint64_t a = lo < 0 ? 0 - (uint64_t)lo : (uint64_t)lo;
  const uint64_t b = hi < 0 ? 0 - (uint64_t)hi : (uint64_t)hi;
  return a > b ? a : b;
}

// The matmul overflow rule: K * max|A| * max|B| >= 2^63 is rejected.
bool matmul_bound(const ccm_desc *a, const ccm_desc *b, unsigned __int128 *bound) {
  const unsigned __int128 lim = (unsigned __int128)1 << 63;
  const unsigned __int128 p =
      (unsigned __int128)max_abs(a->vmin, a->vmax) * (unsigned __int128)max_abs(b->vmin, b->vmax);
  if (p >= lim) return false;
  *bound = p * (unsigned __int128)(uint64_t)a->cols;
  return *bound < lim;
}

bool fits_i8(const ccm_desc *d) { return d->vmin >= -128 && d->vmax <= 127; }

}  // namespace

extern "C" {

int ccm_version(void) { return 10000; }

const char *ccm_status_str(int status) {
  switch (status) {
    case CCM_OK: return "ok";
    case CCM_E_INVAL: return "invalid argument";
    case CCM_E_SHAPE: return "shape mismatch";
    case CCM_E_RANGE: return "index out of range";
    case CCM_E_OVERFLOW: return "result overflows int64";
    case CCM_E_NOMEM: return "out of memory or buffer too small";
    case CCM_E_DEVICE: return "HIP runtime error";
    case CCM_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

uint64_t ccm_words(int64_t rows, int64_t cols, int32_t bits) {
  if (!shape_ok(rows, cols) || bits < 1 || bits > 64) return 0;
  return ((uint64_t)rows * (uint64_t)cols * (uint64_t)bits) / 64u + 1u;
}

uint64_t ccm_packed_bytes(int64_t rows, int64_t cols, int32_t bits) {
  const uint64_t w = ccm_words(rows, cols, bits);
  return w ? 64u + 8u * w : 0u;
}

uint64_t ccm_payload_capacity(int64_t rows, int64_t cols, int32_t bits) {
  if (!ccm_words(rows, cols, bits)) return 0;
  return 4u * ccm::cap_words32((uint64_t)rows * (uint64_t)cols, bits);
}

int ccm_width(int64_t vmin, int64_t vmax, int32_t *bits, int32_t *is_signed) {
  if (!bits || !is_signed) return CCM_E_INVAL;
  return width_rule(vmin, vmax, bits, is_signed);
}

int ccm_header_encode(const ccm_desc *d, uint8_t out[64]) {
  if (!out) return CCM_E_INVAL;
  int rc = check_desc(d, false);
  if (rc != CCM_OK) return rc;
  std::memset(out, 0, 64);
  std::memcpy(out, "CCM1", 4);
  out[4] = 1;
  out[5] = 0;
  out[6] = (uint8_t)d->bits;
  out[7] = (uint8_t)(d->is_signed ? 1 : 0);
  auto put = [&](int at, uint64_t v) {
    for (int k = 0; k < 8; ++k) out[at + k] = (uint8_t)(v >> (8 * k));
  };
  put(8, (uint64_t)d->rows);
  put(16, (uint64_t)d->cols);
  put(24, (uint64_t)d->vmin);
  put(32, (uint64_t)d->vmax);
  put(40, d->words);
  return CCM_OK;
}

int ccm_header_decode(const uint8_t in[64], ccm_desc *d) {
  if (!in || !d) return CCM_E_INVAL;
  if (std::memcmp(in, "CCM1", 4) != 0 || in[4] != 1 || in[5] != 0) return CCM_E_INVAL;
  if (in[7] & ~1u) return CCM_E_INVAL;
  for (int k = 48; k < 64; ++k)
    if (in[k]) return CCM_E_INVAL;
  auto get = [&](int at) {
    uint64_t v = 0;
    for (int k = 0; k < 8; ++k) v |= (uint64_t)in[at + k] << (8 * k);
    return v;
  };
  ccm_desc t;
  t.rows = (int64_t)get(8);
  t.cols = (int64_t)get(16);
  t.vmin = (int64_t)get(24);
  t.vmax = (int64_t)get(32);
  t.bits = in[6];
  t.is_signed = in[7] & 1;
  t.words = get(40);
  t.payload = nullptr;
  int rc = check_desc(&t, false);
  if (rc != CCM_OK) return rc;
  *d = t;
  return CCM_OK;
}

int ccm_range(const void *dense, int32_t dtype, int64_t n, int64_t *vmin, int64_t *vmax,
              void *stream) {
  if (!dense || !vmin || !vmax || n < 1 || (dtype != CCM_I32 && dtype != CCM_I64))
    return CCM_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx *c = nullptr;
  int rc = device_ctx(&c);
  if (rc != CCM_OK) return rc;
  CCM_HIP(ccm::launch_range_init(c->slot, s));
  CCM_HIP(ccm::launch_range_dense(dense, dtype, (uint64_t)n, c->slot, s));
  ccm::RangeSlot r;
  rc = read_slot(c, s, &r);
  if (rc != CCM_OK) return rc;
  *vmin = r.vmin;
  *vmax = r.vmax;
  return CCM_OK;
}

int ccm_compress_plan(const void *dense, int32_t dtype, int64_t rows, int64_t cols,
                      ccm_desc *out, void *stream) {
  if (!out || !shape_ok(rows, cols)) return CCM_E_INVAL;
  int64_t lo = 0, hi = 0;
  int rc = ccm_range(dense, dtype, rows * cols, &lo, &hi, stream);
  if (rc != CCM_OK) return rc;
  return fill_desc(rows, cols, lo, hi, out);
}

int ccm_compress(const void *dense, int32_t dtype, const ccm_desc *out, void *stream) {
  if (!dense || (dtype != CCM_I32 && dtype != CCM_I64)) return CCM_E_INVAL;
  int rc = check_desc(out, true);
  if (rc != CCM_OK) return rc;
  const uint64_t n = nelem(out);
  CCM_HIP(ccm::launch_compress(dense, dtype, n, out->bits, (uint32_t *)out->payload,
                               ccm::cap_words32(n, out->bits), (hipStream_t)stream));
  return CCM_OK;
}

int ccm_decompress(const ccm_desc *a, int64_t *dense_out, void *stream) {
  int rc = check_desc(a, true);
  if (rc != CCM_OK) return rc;
  if (!dense_out) return CCM_E_INVAL;
  CCM_HIP(ccm::launch_decompress((const uint32_t *)a->payload, nelem(a), a->bits, a->is_signed,
                                 dense_out, (hipStream_t)stream));
  return CCM_OK;
}

int ccm_get(const ccm_desc *a, int64_t i, int64_t j, int64_t *value, void *stream) {
  int rc = check_desc(a, true);
  if (rc != CCM_OK) return rc;
  if (!value) return CCM_E_INVAL;
  if (i < 0 || i >= a->rows || j < 0 || j >= a->cols) return CCM_E_RANGE;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx *c = nullptr;
  rc = device_ctx(&c);
  if (rc != CCM_OK) return rc;
  CCM_HIP(ccm::launch_get_one((const uint32_t *)a->payload, (uint64_t)(i * a->cols + j), a->bits,
                              a->is_signed, c->one, s));
  int64_t *h = (int64_t *)((char *)c->host + ccm::kRangeBytes);
  CCM_HIP(hipMemcpyAsync(h, c->one, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  CCM_HIP(hipStreamSynchronize(s));
  *value = *h;
  return CCM_OK;
}

int ccm_gather(const ccm_desc *a, const int64_t *ii, const int64_t *jj, int64_t n,
               int64_t *out, int32_t *bad, void *stream) {
  int rc = check_desc(a, true);
  if (rc != CCM_OK) return rc;
  if (n < 0 || (n > 0 && (!ii || !jj || !out))) return CCM_E_INVAL;
  CCM_HIP(ccm::launch_gather((const uint32_t *)a->payload, a->rows, a->cols, a->bits,
                             a->is_signed, ii, jj, n, out, bad, (hipStream_t)stream));
  return CCM_OK;
}

// Value class of an elementwise pass from the operands' exact ranges: 32-bit
// arithmetic when every operand value and every possible result fits.
static bool in_i32(__int128 v) { return v >= (__int128)INT32_MIN && v <= (__int128)INT32_MAX; }

static int add_class(const ccm_desc *a, const ccm_desc *b) {
  const __int128 lo = (__int128)a->vmin + b->vmin, hi = (__int128)a->vmax + b->vmax;
  if (in_i32(a->vmin) && in_i32(a->vmax) && in_i32(b->vmin) && in_i32(b->vmax) && in_i32(lo) &&
      in_i32(hi))
    return ccm::EW_I32;
  if (a->vmin >= 0 && b->vmin >= 0 && hi <= (__int128)UINT32_MAX) return ccm::EW_U32;
  return ccm::EW_I64;
}

static int scale_class(const ccm_desc *a, int64_t s) {
  const __int128 p = (__int128)a->vmin * s, q = (__int128)a->vmax * s;
  const __int128 lo = p < q ? p : q, hi = p < q ? q : p;
  if (in_i32(a->vmin) && in_i32(a->vmax) && in_i32(s) && in_i32(lo) && in_i32(hi))
    return ccm::EW_I32;
  if (a->vmin >= 0 && s >= 0 && s <= (int64_t)UINT32_MAX && hi <= (__int128)UINT32_MAX)
    return ccm::EW_U32;
  return ccm::EW_I64;
}

int ccm_add_plan(const ccm_desc *a, const ccm_desc *b, ccm_desc *out, void *stream) {
  int rc = check_desc(a, true);
  if (rc == CCM_OK) rc = check_desc(b, true);
  if (rc != CCM_OK) return rc;
  if (!out) return CCM_E_INVAL;
  if (a->rows != b->rows || a->cols != b->cols) return CCM_E_SHAPE;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx *c = nullptr;
  rc = device_ctx(&c);
  if (rc != CCM_OK) return rc;
  CCM_HIP(ccm::launch_range_init(c->slot, s));
  CCM_HIP(ccm::launch_ewise_range(ccm::EW_ADD, operand(a), operand(b), 0, nelem(a),
                                  add_class(a, b), c->slot, s));
  ccm::RangeSlot r;
  rc = read_slot(c, s, &r);
  if (rc != CCM_OK) return rc;
  if (r.flag) return CCM_E_OVERFLOW;
  return fill_desc(a->rows, a->cols, r.vmin, r.vmax, out);
}

static int check_result(const ccm_desc *out, int64_t rows, int64_t cols) {
  int rc = check_desc(out, true);
  if (rc != CCM_OK) return rc;
  if (out->rows != rows || out->cols != cols) return CCM_E_SHAPE;
  return CCM_OK;
}

int ccm_add(const ccm_desc *a, const ccm_desc *b, const ccm_desc *out, void *stream) {
  int rc = check_desc(a, true);
  if (rc == CCM_OK) rc = check_desc(b, true);
  if (rc != CCM_OK) return rc;
  if (a->rows != b->rows || a->cols != b->cols) return CCM_E_SHAPE;
  rc = check_result(out, a->rows, a->cols);
  if (rc != CCM_OK) return rc;
  const uint64_t n = nelem(a);
  CCM_HIP(ccm::launch_ewise_pack(ccm::EW_ADD, operand(a), operand(b), 0, n, add_class(a, b),
                                 out->bits,
                                 (uint32_t *)out->payload, ccm::cap_words32(n, out->bits),
                                 (hipStream_t)stream));
  return CCM_OK;
}

// The result range the headers bound: [a.min + b.min, a.max + b.max], or
// false when it leaves int64 (some sum may overflow).
static bool add_bound(const ccm_desc *a, const ccm_desc *b, int64_t *lo, int64_t *hi) {
  const __int128 l = (__int128)a->vmin + b->vmin, h = (__int128)a->vmax + b->vmax;
  if (l < (__int128)INT64_MIN || h > (__int128)INT64_MAX) return false;
  *lo = (int64_t)l;
  *hi = (int64_t)h;
  return true;
}

uint64_t ccm_add_capacity(const ccm_desc *a, const ccm_desc *b) {
  if (check_desc(a, false) != CCM_OK || check_desc(b, false) != CCM_OK) return 0;
  if (a->rows != b->rows || a->cols != b->cols) return 0;
  int64_t lo, hi;
  int32_t bits = 64, sgn = 0;
  if (add_bound(a, b, &lo, &hi) && width_rule(lo, hi, &bits, &sgn) != CCM_OK) return 0;
  return ccm_payload_capacity(a->rows, a->cols, bits);
}

int ccm_add_onepass(const ccm_desc *a, const ccm_desc *b, ccm_desc *out, void *stream) {
  int rc = check_desc(a, true);
  if (rc == CCM_OK) rc = check_desc(b, true);
  if (rc != CCM_OK) return rc;
  if (!out || !out->payload) return CCM_E_INVAL;
  if (a->rows != b->rows || a->cols != b->cols) return CCM_E_SHAPE;
  void *payload = out->payload;
  const uint64_t n = nelem(a);
  const int vclass = add_class(a, b);
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx *c = nullptr;
  rc = device_ctx(&c);
  if (rc != CCM_OK) return rc;
  ccm_desc bound, exact;
  int64_t lo, hi;
  ccm::RangeSlot r;
  if (n > 0 && add_bound(a, b, &lo, &hi) &&
      fill_desc(a->rows, a->cols, lo, hi, &bound) == CCM_OK) {
    // one pass: pack at the bounded width, learn the exact range meanwhile
    CCM_HIP(ccm::launch_range_init(c->slot, s));
    CCM_HIP(ccm::launch_add_pack_range(operand(a), operand(b), n, vclass, bound.bits,
                                       (uint32_t *)payload, ccm::cap_words32(n, bound.bits),
                                       c->slot, s));
    rc = read_slot(c, s, &r);
    if (rc != CCM_OK) return rc;
    rc = fill_desc(a->rows, a->cols, r.vmin, r.vmax, &exact);
    if (rc != CCM_OK) return rc;
    exact.payload = payload;
    if (exact.bits > bound.bits) return CCM_E_DEVICE;  // sums outside the bound: a failed pass
    if (exact.bits != bound.bits || exact.is_signed != bound.is_signed) {
      // the bound was loose: pack again at the exact width (it is narrower,
      // so the payload holds it)
      CCM_HIP(ccm::launch_ewise_pack(ccm::EW_ADD, operand(a), operand(b), 0, n, vclass,
                                     exact.bits, (uint32_t *)payload,
                                     ccm::cap_words32(n, exact.bits), s));
    }
    *out = exact;
    return CCM_OK;
  }
  // a bound past int64: the range pass first (it detects overflow), then the pack
  CCM_HIP(ccm::launch_range_init(c->slot, s));
  CCM_HIP(ccm::launch_ewise_range(ccm::EW_ADD, operand(a), operand(b), 0, n, vclass, c->slot, s));
  rc = read_slot(c, s, &r);
  if (rc != CCM_OK) return rc;
  if (r.flag) return CCM_E_OVERFLOW;
  rc = fill_desc(a->rows, a->cols, r.vmin, r.vmax, &exact);
  if (rc != CCM_OK) return rc;
  exact.payload = payload;
  CCM_HIP(ccm::launch_ewise_pack(ccm::EW_ADD, operand(a), operand(b), 0, n, vclass, exact.bits,
                                 (uint32_t *)payload, ccm::cap_words32(n, exact.bits), s));
  *out = exact;
  return CCM_OK;
}

int ccm_scale_plan(const ccm_desc *a, int64_t s, ccm_desc *out) {
  int rc = check_desc(a, false);
  if (rc != CCM_OK) return rc;
  if (!out) return CCM_E_INVAL;
  const __int128 p = (__int128)a->vmin * s, q = (__int128)a->vmax * s;
  const __int128 lo = p < q ? p : q, hi = p < q ? q : p;
  if (lo < (__int128)INT64_MIN || hi > (__int128)INT64_MAX) return CCM_E_OVERFLOW;
  return fill_desc(a->rows, a->cols, (int64_t)lo, (int64_t)hi, out);
}

int ccm_scale(const ccm_desc *a, int64_t s, const ccm_desc *out, void *stream) {
  int rc = check_desc(a, true);
  if (rc != CCM_OK) return rc;
  ccm_desc expect;
  rc = ccm_scale_plan(a, s, &expect);
  if (rc != CCM_OK) return rc;
  rc = check_result(out, a->rows, a->cols);
  if (rc != CCM_OK) return rc;
  if (out->bits != expect.bits || out->vmin != expect.vmin || out->vmax != expect.vmax)
    return CCM_E_INVAL;
  const uint64_t n = nelem(a);
  ccm::PackedOperand none{nullptr, 0, 0};
  CCM_HIP(ccm::launch_ewise_pack(ccm::EW_SCALE, operand(a), none, s, n, scale_class(a, s),
                                 out->bits,
                                 (uint32_t *)out->payload, ccm::cap_words32(n, out->bits),
                                 (hipStream_t)stream));
  return CCM_OK;
}

int ccm_matvec(const ccm_desc *a, const void *x, int32_t xdtype, int64_t *y, void *stream) {
  int rc = check_desc(a, true);
  if (rc != CCM_OK) return rc;
  if (!x || !y || (xdtype != CCM_I32 && xdtype != CCM_I64)) return CCM_E_INVAL;
  CCM_HIP(ccm::launch_matvec((const uint32_t *)a->payload, a->rows, a->cols, a->bits,
                             a->is_signed, x, xdtype, y, (hipStream_t)stream));
  return CCM_OK;
}

// Scratch layout of a matmul: dense C (int32 when the bound allows, else
// int64), rounded up to 256 bytes, then -- on the int8 MFMA path -- A and
// B^T decoded to int8.  The MFMA path is taken when both operands' values
// fit int8 and the bound K*max|A|*max|B| < 2^31 keeps int32 sums exact.
struct MatmulPlan {
  int out32, use_i8;
  uint64_t c_bytes, total;
};

static bool matmul_layout(const ccm_desc *a, const ccm_desc *b, MatmulPlan *p) {
  unsigned __int128 bound = 0;
  if (!matmul_bound(a, b, &bound)) return false;
  p->out32 = bound < ((unsigned __int128)1 << 31) ? 1 : 0;
  p->use_i8 = (p->out32 && fits_i8(a) && fits_i8(b)) ? 1 : 0;
  const uint64_t c = (p->out32 ? 4u : 8u) * (uint64_t)a->rows * (uint64_t)b->cols;
  p->c_bytes = (c + 255u) / 256u * 256u;
  p->total = p->c_bytes + (p->use_i8 ? ccm::matmul_i8_bytes(a->rows, a->cols, b->cols) : 0u);
  return true;
}

uint64_t ccm_matmul_scratch_bytes(const ccm_desc *a, const ccm_desc *b) {
  if (check_desc(a, false) != CCM_OK || check_desc(b, false) != CCM_OK) return 0;
  if (a->cols != b->rows) return 0;
  MatmulPlan p;
  if (!matmul_layout(a, b, &p)) return 0;
  return p.total;
}

static int matmul_common(const ccm_desc *a, const ccm_desc *b, uint64_t scratch_bytes,
                         const void *scratch, MatmulPlan *p) {
  int rc = check_desc(a, true);
  if (rc == CCM_OK) rc = check_desc(b, true);
  if (rc != CCM_OK) return rc;
  if (a->cols != b->rows) return CCM_E_SHAPE;
  if (!shape_ok(a->rows, b->cols)) return CCM_E_INVAL;
  if (!matmul_layout(a, b, p)) return CCM_E_OVERFLOW;
  if (!scratch) return CCM_E_INVAL;
  if (scratch_bytes < p->total) return CCM_E_NOMEM;
  return CCM_OK;
}

int ccm_matmul_plan(const ccm_desc *a, const ccm_desc *b, ccm_desc *out, void *scratch,
                    uint64_t scratch_bytes, void *stream) {
  MatmulPlan mp;
  int rc = matmul_common(a, b, scratch_bytes, scratch, &mp);
  if (rc != CCM_OK) return rc;
  if (!out) return CCM_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx *c = nullptr;
  rc = device_ctx(&c);
  if (rc != CCM_OK) return rc;
  CCM_HIP(ccm::launch_range_init(c->slot, s));
  CCM_HIP(ccm::launch_matmul((const uint32_t *)a->payload, a->bits, a->is_signed,
                             (const uint32_t *)b->payload, b->bits, b->is_signed, a->rows,
                             a->cols, b->cols, mp.use_i8, mp.out32, scratch, c->slot, s));
  ccm::RangeSlot r;
  rc = read_slot(c, s, &r);
  if (rc != CCM_OK) return rc;
  return fill_desc(a->rows, b->cols, r.vmin, r.vmax, out);
}

int ccm_matmul(const ccm_desc *a, const ccm_desc *b, const ccm_desc *out, const void *scratch,
               uint64_t scratch_bytes, void *stream) {
  MatmulPlan mp;
  int rc = matmul_common(a, b, scratch_bytes, scratch, &mp);
  if (rc != CCM_OK) return rc;
  rc = check_result(out, a->rows, b->cols);
  if (rc != CCM_OK) return rc;
  const uint64_t n = nelem(out);
  CCM_HIP(ccm::launch_compress(scratch, mp.out32 ? CCM_I32 : CCM_I64, n, out->bits,
                               (uint32_t *)out->payload, ccm::cap_words32(n, out->bits),
                               (hipStream_t)stream));
  return CCM_OK;
}

// ---- results whose width stays on the device ----------------------------
// ws layout: the ccm_result at byte 0, the spread range slots from byte 256.
constexpr uint64_t kWsSlots = 256;

uint64_t ccm_async_ws_bytes(void) { return kWsSlots + ccm::kRangeBytes; }

static int async_ws(void *ws, ccm::RangeSlot **slots, ccm_result **res) {
  if (!ws || ((uintptr_t)ws % 256) != 0) return CCM_E_INVAL;
  *res = (ccm_result *)ws;
  *slots = (ccm::RangeSlot *)((char *)ws + kWsSlots);
  return CCM_OK;
}

int ccm_add_async(const ccm_desc *a, const ccm_desc *b, void *payload, uint64_t payload_bytes,
                  void *ws, void *stream) {
  int rc = check_desc(a, true);
  if (rc == CCM_OK) rc = check_desc(b, true);
  if (rc != CCM_OK) return rc;
  if (a->rows != b->rows || a->cols != b->cols) return CCM_E_SHAPE;
  if (!payload) return CCM_E_INVAL;
  ccm::RangeSlot *slots = nullptr;
  ccm_result *res = nullptr;
  rc = async_ws(ws, &slots, &res);
  if (rc != CCM_OK) return rc;
  if (payload_bytes < ccm_add_capacity(a, b)) return CCM_E_NOMEM;
  const uint64_t n = nelem(a);
  const int vclass = add_class(a, b);
  hipStream_t s = (hipStream_t)stream;
  uint32_t *out = (uint32_t *)payload;
  ccm_desc bound;
  int64_t lo, hi;
  CCM_HIP(ccm::launch_range_init(slots, s));
  if (add_bound(a, b, &lo, &hi) && fill_desc(a->rows, a->cols, lo, hi, &bound) == CCM_OK) {
    // pack at the bounded width while the exact range folds into the slots;
    // the device then repacks only if the exact width is narrower
    CCM_HIP(ccm::launch_add_pack_range(operand(a), operand(b), n, vclass, bound.bits, out,
                                       ccm::cap_words32(n, bound.bits), slots, s));
    CCM_HIP(ccm::launch_result_finalize(slots, a->rows, a->cols, 0, res, s));
    CCM_HIP(ccm::launch_ewise_pack_dev(ccm::EW_ADD, operand(a), operand(b), 0, n, vclass,
                                       bound.bits, bound.bits, out, res, s));
    return CCM_OK;
  }
  // a bound past int64: the range pass (which flags overflow), then the pack
  CCM_HIP(ccm::launch_ewise_range(ccm::EW_ADD, operand(a), operand(b), 0, n, vclass, slots, s));
  CCM_HIP(ccm::launch_result_finalize(slots, a->rows, a->cols, 1, res, s));
  CCM_HIP(ccm::launch_ewise_pack_dev(ccm::EW_ADD, operand(a), operand(b), 0, n, vclass, 64, 0,
                                     out, res, s));
  return CCM_OK;
}

// Widest width a product can take under the overflow rule's bound.
static bool matmul_max_bits(const ccm_desc *a, const ccm_desc *b, int32_t *bits) {
  unsigned __int128 bound = 0;
  if (!matmul_bound(a, b, &bound)) return false;
  int32_t sg = 0;
  return width_rule(-(int64_t)bound, (int64_t)bound, bits, &sg) == CCM_OK;
}

uint64_t ccm_matmul_capacity(const ccm_desc *a, const ccm_desc *b) {
  if (check_desc(a, false) != CCM_OK || check_desc(b, false) != CCM_OK) return 0;
  if (a->cols != b->rows || !shape_ok(a->rows, b->cols)) return 0;
  int32_t bits = 0;
  if (!matmul_max_bits(a, b, &bits)) return 0;
  return ccm_payload_capacity(a->rows, b->cols, bits);
}

int ccm_matmul_async(const ccm_desc *a, const ccm_desc *b, void *payload,
                     uint64_t payload_bytes, void *scratch, uint64_t scratch_bytes, void *ws,
                     void *stream) {
  MatmulPlan mp;
  int rc = matmul_common(a, b, scratch_bytes, scratch, &mp);
  if (rc != CCM_OK) return rc;
  if (!payload) return CCM_E_INVAL;
  ccm::RangeSlot *slots = nullptr;
  ccm_result *res = nullptr;
  rc = async_ws(ws, &slots, &res);
  if (rc != CCM_OK) return rc;
  int32_t max_bits = 0;
  if (!matmul_max_bits(a, b, &max_bits)) return CCM_E_OVERFLOW;
  if (payload_bytes < ccm_payload_capacity(a->rows, b->cols, max_bits)) return CCM_E_NOMEM;
  hipStream_t s = (hipStream_t)stream;
  CCM_HIP(ccm::launch_range_init(slots, s));
  CCM_HIP(ccm::launch_matmul((const uint32_t *)a->payload, a->bits, a->is_signed,
                             (const uint32_t *)b->payload, b->bits, b->is_signed, a->rows,
                             a->cols, b->cols, mp.use_i8, mp.out32, scratch, slots, s));
  CCM_HIP(ccm::launch_result_finalize(slots, a->rows, b->cols, 0, res, s));
  CCM_HIP(ccm::launch_compress_dev(scratch, mp.out32 ? CCM_I32 : CCM_I64,
                                   (uint64_t)a->rows * (uint64_t)b->cols, max_bits,
                                   (uint32_t *)payload, res, s));
  return CCM_OK;
}

int ccm_result_desc(const ccm_result *r, void *payload, ccm_desc *out) {
  if (!r || !out) return CCM_E_INVAL;
  if (r->status != CCM_OK) return r->status;
  ccm_desc d;
  int rc = fill_desc(r->rows, r->cols, r->vmin, r->vmax, &d);
  if (rc != CCM_OK) return CCM_E_INVAL;
  if (!shape_ok(r->rows, r->cols) || d.bits != r->bits || d.is_signed != r->is_signed ||
      d.words != r->words)
    return CCM_E_INVAL;
  d.payload = payload;
  *out = d;
  return CCM_OK;
}

int ccm_fill_uniform(void *dense, int32_t dtype, int64_t n, int64_t lo, int64_t hi,
                     uint64_t seed, uint64_t stream_id, uint64_t start, void *stream) {
  if (!dense || n < 0 || (dtype != CCM_I32 && dtype != CCM_I64)) return CCM_E_INVAL;
  if (hi <= lo) return CCM_E_INVAL;
  const uint64_t span = (uint64_t)hi - (uint64_t)lo;
  if (span > (1ull << 32)) return CCM_E_INVAL;
  if (dtype == CCM_I32 && (lo < INT32_MIN || hi - 1 > INT32_MAX)) return CCM_E_INVAL;
  CCM_HIP(ccm::launch_fill_uniform(dense, dtype, (uint64_t)n, lo, span, seed, stream_id, start,
                                   (hipStream_t)stream));
  return CCM_OK;
}

int ccm_generate_plan(int64_t rows, int64_t cols, int64_t lo, int64_t hi, uint64_t seed,
                      uint64_t stream_id, ccm_desc *out, void *stream) {
  if (!out || !shape_ok(rows, cols) || hi <= lo) return CCM_E_INVAL;
  const uint64_t span = (uint64_t)hi - (uint64_t)lo;
  if (span > (1ull << 32)) return CCM_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx *c = nullptr;
  int rc = device_ctx(&c);
  if (rc != CCM_OK) return rc;
  CCM_HIP(ccm::launch_range_init(c->slot, s));
  CCM_HIP(ccm::launch_gen_range((uint64_t)rows * (uint64_t)cols, lo, span, seed, stream_id,
                                c->slot, s));
  ccm::RangeSlot r;
  rc = read_slot(c, s, &r);
  if (rc != CCM_OK) return rc;
  return fill_desc(rows, cols, r.vmin, r.vmax, out);
}

int ccm_generate(const ccm_desc *out, int64_t lo, int64_t hi, uint64_t seed,
                 uint64_t stream_id, void *stream) {
  int rc = check_desc(out, true);
  if (rc != CCM_OK) return rc;
  if (hi <= lo) return CCM_E_INVAL;
  const uint64_t span = (uint64_t)hi - (uint64_t)lo;
  if (span > (1ull << 32)) return CCM_E_INVAL;
  const uint64_t n = nelem(out);
  CCM_HIP(ccm::launch_gen_pack(n, lo, span, seed, stream_id, out->bits,
                               (uint32_t *)out->payload, ccm::cap_words32(n, out->bits),
                               (hipStream_t)stream));
  return CCM_OK;
}

// ---- choosing the method -------------------------------------------------

}  // extern "C"

namespace {
void vlb_widths(int64_t vmin, int64_t vmax, int32_t *bmax, int32_t *k);
}  // namespace

extern "C" {

int ccm_method_plan(const void *dense, int32_t dtype, int64_t rows, int64_t cols,
                    ccm_method_info *out, void *stream) {
  if (!dense || !out || !shape_ok(rows, cols) || (dtype != CCM_I32 && dtype != CCM_I64))
    return CCM_E_INVAL;
  const uint64_t n = (uint64_t)rows * (uint64_t)cols;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx *c = nullptr;
  int rc = device_ctx(&c);
  if (rc != CCM_OK) return rc;
  CCM_HIP(ccm::launch_range_init(c->slot, s));
  CCM_HIP(ccm::launch_method_stats(dense, dtype, n, c->slot, c->sums, s));
  uint64_t *hs = (uint64_t *)((char *)c->host + ccm::kRangeBytes + 64);
  CCM_HIP(hipMemcpyAsync(hs, c->sums, ccm::kSumBytes, hipMemcpyDeviceToHost, s));
  ccm::RangeSlot r;
  rc = read_slot(c, s, &r);  // synchronizes the stream
  if (rc != CCM_OK) return rc;
  uint64_t su = 0, ss = 0;
  for (int i = 0; i < ccm::kRangeSpread; ++i) {
    su += hs[2 * ccm::kSumStride * i];
    ss += hs[2 * ccm::kSumStride * i + 1];
  }
  int32_t b = 0, sgn = 0, bmax = 0, k = 0;
  rc = width_rule(r.vmin, r.vmax, &b, &sgn);
  if (rc != CCM_OK) return rc;
  vlb_widths(r.vmin, r.vmax, &bmax, &k);
  out->vmin = r.vmin;
  out->vmax = r.vmax;
  out->sm_bits = b;
  out->vlb_k = k;
  out->sm_nbits = n * (uint64_t)b;
  out->vlb_nbits = n * (uint64_t)k + (sgn ? ss : su);
  out->eta1 = 1.0 - (double)out->sm_nbits / (64.0 * (double)n);
  out->eta2 = 1.0 - (double)out->vlb_nbits / (64.0 * (double)n);
  out->method = out->vlb_nbits < out->sm_nbits ? 2 : 1;
  out->reserved = 0;
  return CCM_OK;
}

// ---- column-major unravel and y = A^T x ----------------------------------

uint64_t ccm_matvec_t_scratch_bytes(const ccm_desc *a) {
  if (check_desc(a, false) != CCM_OK) return 0;
  return 8ull * (uint64_t)ccm::kMaxSplitsT * (uint64_t)a->cols;
}

int ccm_matvec_t(const ccm_desc *a, const void *x, int32_t xdtype, int64_t *y, void *scratch,
                 uint64_t scratch_bytes, void *stream) {
  int rc = check_desc(a, true);
  if (rc != CCM_OK) return rc;
  if (!x || !y || (xdtype != CCM_I32 && xdtype != CCM_I64)) return CCM_E_INVAL;
  if (scratch && (uintptr_t)scratch % 8 != 0) return CCM_E_INVAL;
  if (scratch && scratch_bytes < ccm_matvec_t_scratch_bytes(a)) return CCM_E_NOMEM;
  CCM_HIP(ccm::launch_matvec_t((const uint32_t *)a->payload, a->rows, a->cols, a->bits,
                               a->is_signed, x, xdtype, y, (int64_t *)scratch,
                               scratch ? scratch_bytes / 8 : 0, (hipStream_t)stream));
  return CCM_OK;
}

int ccm_matvec_t_noalloc(const ccm_desc *a, const void *x, int32_t xdtype, int64_t *y,
                         void *stream) {
  int rc = check_desc(a, true);
  if (rc != CCM_OK) return rc;
  if (!x || !y || (xdtype != CCM_I32 && xdtype != CCM_I64)) return CCM_E_INVAL;
  if (a->cols > ccm::kNoAllocColsT) return CCM_E_NOMEM;
  int64_t *part = nullptr;
  uint64_t words = 0;
  CCM_HIP(ccm::static_matvec_t_scratch(&part, &words));
  CCM_HIP(ccm::launch_matvec_t((const uint32_t *)a->payload, a->rows, a->cols, a->bits,
                               a->is_signed, x, xdtype, y, part, words, (hipStream_t)stream));
  return CCM_OK;
}

int ccm_compress_cm(const void *dense, int32_t dtype, const ccm_desc *out, void *stream) {
  if (!dense || (dtype != CCM_I32 && dtype != CCM_I64)) return CCM_E_INVAL;
  int rc = check_desc(out, true);
  if (rc != CCM_OK) return rc;
  // dense is A (out->cols x out->rows, row-major); out describes A^T
  CCM_HIP(ccm::launch_compress_cm(dense, dtype, out->cols, out->rows, out->bits,
                                  (uint32_t *)out->payload,
                                  ccm::cap_words32(nelem(out), out->bits), (hipStream_t)stream));
  return CCM_OK;
}

int ccm_header_encode_cm(const ccm_desc *at, uint8_t out[64]) {
  if (!at) return CCM_E_INVAL;
  ccm_desc a = *at;
  a.rows = at->cols;
  a.cols = at->rows;
  int rc = ccm_header_encode(&a, out);
  if (rc != CCM_OK) return rc;
  out[7] = (uint8_t)(out[7] | 2u);
  return CCM_OK;
}

int ccm_header_decode_cm(const uint8_t in[64], ccm_desc *at) {
  if (!in || !at) return CCM_E_INVAL;
  if (!(in[7] & 2u)) return CCM_E_INVAL;
  uint8_t h[64];
  std::memcpy(h, in, 64);
  h[7] = (uint8_t)(h[7] & ~2u);
  ccm_desc a;
  int rc = ccm_header_decode(h, &a);
  if (rc != CCM_OK) return rc;
  ccm_desc t = a;
  t.rows = a.cols;
  t.cols = a.rows;
  *at = t;
  return CCM_OK;
}

// ---- floats in fixed point (Conclusion) ----------------------------------

int ccm_float_absmax(const void *v, int32_t dtype, int64_t n, double *absmax, void *stream) {
  if (!v || !absmax || n < 1 || (dtype != CCM_F32 && dtype != CCM_F64)) return CCM_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx *c = nullptr;
  int rc = device_ctx(&c);
  if (rc != CCM_OK) return rc;
  CCM_HIP(ccm::launch_range_init(c->slot, s));
  CCM_HIP(ccm::launch_float_absmax(v, dtype, (uint64_t)n, c->slot, s));
  ccm::RangeSlot r;
  rc = read_slot(c, s, &r);
  if (rc != CCM_OK) return rc;
  if (r.vmax >= 0x7FF0000000000000ll) return CCM_E_RANGE;  // NaN or infinity
  double a;
  std::memcpy(&a, &r.vmax, sizeof a);
  *absmax = a;
  return CCM_OK;
}

int ccm_float_frac_bits(double absmax, int32_t sig_bits, int32_t *frac_bits) {
  if (!frac_bits || sig_bits < 1 || sig_bits > 62 || !(absmax >= 0.0) || std::isinf(absmax))
    return CCM_E_INVAL;
  if (absmax == 0.0) {
    *frac_bits = 0;
    return CCM_OK;
  }
  int ex = 0;
  (void)std::frexp(absmax, &ex);  // absmax = m 2^ex, 1/2 <= m < 1
  *frac_bits = sig_bits - ex;     // sig_bits - 1 - floor(log2 absmax)
  return CCM_OK;
}

int ccm_quantize(const void *v, int32_t dtype, int64_t n, int32_t frac_bits, void *q,
                 int32_t qdtype, int64_t *qmin, int64_t *qmax, void *stream) {
  if (!v || !qmin || !qmax || n < 1 || (dtype != CCM_F32 && dtype != CCM_F64) ||
      (q && qdtype != CCM_I32 && qdtype != CCM_I64) || frac_bits < -1200 || frac_bits > 1200)
    return CCM_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx *c = nullptr;
  int rc = device_ctx(&c);
  if (rc != CCM_OK) return rc;
  CCM_HIP(ccm::launch_range_init(c->slot, s));
  CCM_HIP(ccm::launch_quantize(v, dtype, (uint64_t)n, frac_bits, q, qdtype, c->slot, s));
  ccm::RangeSlot r;
  rc = read_slot(c, s, &r);
  if (rc != CCM_OK) return rc;
  if (r.flag) return CCM_E_RANGE;
  if (r.vmax == INT64_MAX) return CCM_E_OVERFLOW;
  *qmin = r.vmin;
  *qmax = r.vmax;
  return CCM_OK;
}

int ccm_compress_fx(const void *v, int32_t dtype, int32_t frac_bits, const ccm_desc *out,
                    void *stream) {
  if (!v || (dtype != CCM_F32 && dtype != CCM_F64) || frac_bits < -1200 || frac_bits > 1200)
    return CCM_E_INVAL;
  int rc = check_desc(out, true);
  if (rc != CCM_OK) return rc;
  const uint64_t n = nelem(out);
  CCM_HIP(ccm::launch_compress_fx(v, dtype, n, frac_bits, out->bits, (uint32_t *)out->payload,
                                  ccm::cap_words32(n, out->bits), (hipStream_t)stream));
  return CCM_OK;
}

int ccm_dequantize(const int64_t *q, int64_t n, int32_t frac_bits, int32_t dtype, void *out,
                   void *stream) {
  if (!q || !out || n < 1 || (dtype != CCM_F32 && dtype != CCM_F64) || frac_bits < -2400 ||
      frac_bits > 2400)
    return CCM_E_INVAL;
  CCM_HIP(ccm::launch_dequantize(q, (uint64_t)n, frac_bits, dtype, out, (hipStream_t)stream));
  return CCM_OK;
}

int ccm_header_encode_fx(const ccm_desc *d, int32_t frac_bits, uint8_t out[64]) {
  if (frac_bits < -1200 || frac_bits > 1200) return CCM_E_INVAL;
  int rc = ccm_header_encode(d, out);
  if (rc != CCM_OK) return rc;
  out[7] = (uint8_t)(out[7] | 4u);
  const uint16_t f = (uint16_t)(int16_t)frac_bits;
  out[48] = (uint8_t)(f & 0xFFu);
  out[49] = (uint8_t)(f >> 8);
  return CCM_OK;
}

int ccm_header_decode_fx(const uint8_t in[64], ccm_desc *d, int32_t *frac_bits) {
  if (!in || !d || !frac_bits) return CCM_E_INVAL;
  if (!(in[7] & 4u)) return CCM_E_INVAL;
  uint8_t h[64];
  std::memcpy(h, in, 64);
  h[7] = (uint8_t)(h[7] & ~4u);
  const int32_t f = (int16_t)(uint16_t)(in[48] | ((uint16_t)in[49] << 8));
  h[48] = h[49] = 0;
  if (f < -1200 || f > 1200) return CCM_E_INVAL;
  ccm_desc t;
  int rc = ccm_header_decode(h, &t);  // also rejects any other reserved byte or flag
  if (rc != CCM_OK) return rc;
  *d = t;
  *frac_bits = f;
  return CCM_OK;
}

// ---- Method 2: variable length blocks -----------------------------------

}  // extern "C"

namespace {

int bitlen_u(uint64_t u) {
  int L = 0;
  while (L < 64 && (u >> L) != 0) ++L;
  return L;
}

// Largest element width of a matrix with range [vmin, vmax] (widths grow with
// |v| on each side of zero, so an extreme has it) and the length-field width
// k = its bit-length.
void vlb_widths(int64_t vmin, int64_t vmax, int32_t *bmax, int32_t *k) {
  int b;
  if (vmin >= 0) {
    b = vmax <= 1 ? 1 : bitlen_u((uint64_t)vmax);
  } else {
    const int lo = 1 + bitlen_u(~(uint64_t)vmin);
    const int hi = 1 + bitlen_u(vmax < 0 ? ~(uint64_t)vmax : (uint64_t)vmax);
    b = lo > hi ? lo : hi;
  }
  *bmax = b;
  *k = bitlen_u((uint64_t)b);
}

constexpr int kVlbGroup = 32;

uint64_t vlb_grp_offset(int64_t rows) { return ((uint64_t)(rows + 1) * 8u + 255u) / 256u * 256u; }

uint64_t vlb_cap32(uint64_t nbits) { return ((nbits + 31u) / 32u + 16u + 63u) / 64u * 64u; }

int check_vlb(const ccm_vlb_desc *d) {
  if (!d || !d->payload || !d->index) return CCM_E_INVAL;
  if (!shape_ok(d->rows, d->cols) || d->vmin > d->vmax) return CCM_E_INVAL;
  if (d->is_signed != (d->vmin < 0 ? 1 : 0)) return CCM_E_INVAL;
  int32_t bmax = 0, k = 0;
  vlb_widths(d->vmin, d->vmax, &bmax, &k);
  if (k != d->k) return CCM_E_INVAL;
  const unsigned __int128 n = (unsigned __int128)d->rows * (unsigned __int128)d->cols;
  if ((unsigned __int128)d->nbits < n * (unsigned __int128)(k + 1) ||
      (unsigned __int128)d->nbits > n * (unsigned __int128)(k + bmax))
    return CCM_E_INVAL;
  if (d->words != d->nbits / 64u + 1u) return CCM_E_INVAL;
  if (d->gmax < (uint64_t)(k + 1) || d->gmax > (uint64_t)kVlbGroup * (uint64_t)(k + bmax) ||
      d->gmax > d->nbits)
    return CCM_E_INVAL;
  return CCM_OK;
}

ccm::VlbView vlb_view(const ccm_vlb_desc *d) {
  ccm::VlbView v;
  v.w = (const uint32_t *)d->payload;
  v.row_bit = (const uint64_t *)d->index;
  v.grp = (const uint32_t *)((const char *)d->index + vlb_grp_offset(d->rows));
  v.rows = d->rows;
  v.cols = d->cols;
  v.ngr = (int64_t)ccm::vlb_ngr(d->cols);
  int32_t bmax = 0, k = 0;
  vlb_widths(d->vmin, d->vmax, &bmax, &k);
  v.k = k;
  v.bmax = bmax;
  v.sgn = d->is_signed;
  v.gmax = d->gmax;
  v.nbits = d->nbits;
  return v;
}

}  // namespace

extern "C" {

uint64_t ccm_vlb_index_bytes(int64_t rows, int64_t cols) {
  if (!shape_ok(rows, cols)) return 0;
  const uint64_t g = (uint64_t)rows * ccm::vlb_ngr(cols) * 4u;
  return vlb_grp_offset(rows) + (g + 255u) / 256u * 256u;
}

uint64_t ccm_vlb_payload_capacity(uint64_t nbits) { return vlb_cap32(nbits) * 4u; }

int ccm_vlb_compress_plan(const void *dense, int32_t dtype, int64_t rows, int64_t cols,
                          void *index, ccm_vlb_desc *out, void *stream) {
  if (!out || !index || !shape_ok(rows, cols)) return CCM_E_INVAL;
  int64_t lo = 0, hi = 0;
  int rc = ccm_range(dense, dtype, rows * cols, &lo, &hi, stream);
  if (rc != CCM_OK) return rc;
  int32_t bmax = 0, k = 0;
  vlb_widths(lo, hi, &bmax, &k);
  // group offsets within a row are 32-bit
  if ((unsigned __int128)cols * (unsigned __int128)(k + bmax) >= ((unsigned __int128)1 << 32))
    return CCM_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  uint64_t *row_bit = (uint64_t *)index;
  uint32_t *grp = (uint32_t *)((char *)index + vlb_grp_offset(rows));
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx *c = nullptr;
  rc = device_ctx(&c);
  if (rc != CCM_OK) return rc;
  CCM_HIP(ccm::launch_range_init(c->slot, s));
  CCM_HIP(ccm::launch_vlb_sizes(dense, dtype, rows, cols, k, lo < 0 ? 1 : 0, grp, c->slot, s));
  CCM_HIP(ccm::launch_vlb_scan(rows, cols, grp, row_bit, s));
  uint64_t *h = (uint64_t *)((char *)c->host + ccm::kRangeBytes);
  CCM_HIP(hipMemcpyAsync(h, row_bit + rows, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  ccm::RangeSlot gr;
  rc = read_slot(c, s, &gr);  // synchronizes the stream
  if (rc != CCM_OK) return rc;
  out->rows = rows;
  out->cols = cols;
  out->vmin = lo;
  out->vmax = hi;
  out->k = k;
  out->is_signed = lo < 0 ? 1 : 0;
  out->nbits = *h;
  out->words = out->nbits / 64u + 1u;
  out->gmax = (uint64_t)gr.vmax;
  out->payload = nullptr;
  out->index = index;
  return CCM_OK;
}

int ccm_vlb_compress(const void *dense, int32_t dtype, const ccm_vlb_desc *out, void *stream) {
  if (!dense || (dtype != CCM_I32 && dtype != CCM_I64)) return CCM_E_INVAL;
  int rc = check_vlb(out);
  if (rc != CCM_OK) return rc;
  CCM_HIP(ccm::launch_vlb_pack(dense, dtype, vlb_view(out), (uint32_t *)out->payload,
                               vlb_cap32(out->nbits), out->nbits, (hipStream_t)stream));
  return CCM_OK;
}

int ccm_vlb_decompress(const ccm_vlb_desc *a, int64_t *dense_out, void *stream) {
  int rc = check_vlb(a);
  if (rc != CCM_OK) return rc;
  if (!dense_out) return CCM_E_INVAL;
  CCM_HIP(ccm::launch_vlb_decode(vlb_view(a), dense_out, (hipStream_t)stream));
  return CCM_OK;
}

int ccm_vlb_get(const ccm_vlb_desc *a, int64_t i, int64_t j, int64_t *value, void *stream) {
  int rc = check_vlb(a);
  if (rc != CCM_OK) return rc;
  if (!value) return CCM_E_INVAL;
  if (i < 0 || i >= a->rows || j < 0 || j >= a->cols) return CCM_E_RANGE;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx *c = nullptr;
  rc = device_ctx(&c);
  if (rc != CCM_OK) return rc;
  CCM_HIP(ccm::launch_vlb_get(vlb_view(a), i, j, c->one, s));
  int64_t *h = (int64_t *)((char *)c->host + ccm::kRangeBytes);
  CCM_HIP(hipMemcpyAsync(h, c->one, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  CCM_HIP(hipStreamSynchronize(s));
  *value = *h;
  return CCM_OK;
}

int ccm_vlb_matvec(const ccm_vlb_desc *a, const void *x, int32_t xdtype, int64_t *y,
                   void *stream) {
  int rc = check_vlb(a);
  if (rc != CCM_OK) return rc;
  if (!x || !y || (xdtype != CCM_I32 && xdtype != CCM_I64)) return CCM_E_INVAL;
  CCM_HIP(ccm::launch_vlb_matvec(vlb_view(a), x, xdtype, y, (hipStream_t)stream));
  return CCM_OK;
}

}  // extern "C"
