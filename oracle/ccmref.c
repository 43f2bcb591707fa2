/*
 * ccmref.c -- CPU oracle for SM-compressed integer matrices.
 *
 * TEST INFRASTRUCTURE ONLY (see ccmref.h).  Every routine here is the plain
 * definition, one bit or one element at a time, with no blocking or fusion.
 * The two OpenMP pragmas only split independent output rows / entries over
 * threads; the per-row code is the same with or without them.
 */
#include "ccmref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- bit-length and width (Eq. 1, Table 1) ------------------------------ */

int ccmref_bitlen(uint64_t u) {
  int L = 0;
  while (L < 64 && (u >> L) != 0) L++;
  return L;
}

int ccmref_sm_width(uint64_t sup) {
  if (sup == 0 || sup == 1) return 1;     /* Eq. 1, first case */
  return ccmref_bitlen(sup);              /* floor(log2(sup)) + 1 */
}

int ccmref_width(int64_t vmin, int64_t vmax, int32_t *bits, int32_t *is_signed) {
  if (vmin > vmax) return CCMREF_E_INVAL;
  if (vmin >= 0) {
    /* The paper's case: every element is non-negative, b = b(sup M). */
    *is_signed = 0;
    *bits = ccmref_sm_width((uint64_t)vmax);
  } else {
    /* Two's complement: smallest b with -2^(b-1) <= vmin and vmax < 2^(b-1).
     * -(vmin+1) < 2^(b-1)  <=>  bitlen(-(vmin+1)) <= b-1. */
    int lo = ccmref_bitlen((uint64_t)(-(vmin + 1)));
    int hi = vmax > 0 ? ccmref_bitlen((uint64_t)vmax) : 0;
    *is_signed = 1;
    *bits = 1 + (lo > hi ? lo : hi);
  }
  return CCMREF_OK;
}

uint64_t ccmref_words(int64_t rows, int64_t cols, int32_t bits) {
  uint64_t n = (uint64_t)rows * (uint64_t)cols;
  return (n * (uint64_t)bits) / 64u + 1u;
}

/* ---- the bitstream (Eq. 3 and the straddle step) ------------------------ */

/* Stream bit p is bit (p mod 64) of bitstring floor(p/64); bit 0 is the
 * rightmost (least significant) bit. */
static void put_bit(uint64_t *words, uint64_t p, int bit) {
  if (bit) words[p / 64u] |= (uint64_t)1 << (p % 64u);
}

static int get_bit(const uint64_t *words, uint64_t p) {
  return (int)((words[p / 64u] >> (p % 64u)) & 1u);
}

/* Field e occupies stream bits [e*b, e*b + b); field bit t is stream bit e*b+t.
 * The field holds the low b bits of the value's two's complement. */
static void put_field(uint64_t *words, uint64_t e, int32_t bits, int64_t v) {
  uint64_t u = (uint64_t)v;
  uint64_t p0 = e * (uint64_t)bits;
  for (int t = 0; t < bits; t++) put_bit(words, p0 + (uint64_t)t, (int)((u >> t) & 1u));
}

static int64_t get_field(const uint64_t *words, uint64_t e, int32_t bits, int32_t is_signed) {
  uint64_t p0 = e * (uint64_t)bits;
  uint64_t u = 0;
  for (int t = 0; t < bits; t++) u |= (uint64_t)get_bit(words, p0 + (uint64_t)t) << t;
  if (is_signed && ((u >> (bits - 1)) & 1u)) {
    /* v = u - 2^b, evaluated modulo 2^64 */
    if (bits < 64) u = u - ((uint64_t)1 << bits);
  }
  return (int64_t)u;
}

void ccmref_encode_run(const int64_t *vals, int64_t n, int32_t bits, uint64_t *words) {
  for (int64_t e = 0; e < n; e++) put_field(words, (uint64_t)e, bits, vals[e]);
}

void ccmref_decode_run(const uint64_t *words, int64_t n, int32_t bits, int32_t is_signed,
                       int64_t *vals) {
  for (int64_t e = 0; e < n; e++) vals[e] = get_field(words, (uint64_t)e, bits, is_signed);
}

/* ---- compress / decompress / get --------------------------------------- */

int ccmref_plan(const int64_t *dense, int64_t rows, int64_t cols, ccmref_matrix *m) {
  if (rows < 1 || cols < 1 || !dense || !m) return CCMREF_E_INVAL;
  int64_t n = rows * cols;
  int64_t lo = dense[0], hi = dense[0];
  for (int64_t e = 1; e < n; e++) {
    if (dense[e] < lo) lo = dense[e];
    if (dense[e] > hi) hi = dense[e];
  }
  m->rows = rows;
  m->cols = cols;
  m->vmin = lo;
  m->vmax = hi;
  ccmref_width(lo, hi, &m->bits, &m->is_signed);
  m->words = ccmref_words(rows, cols, m->bits);
  return CCMREF_OK;
}

int ccmref_compress(const int64_t *dense, ccmref_matrix *m) {
  if (!dense || !m || !m->payload) return CCMREF_E_INVAL;
  memset(m->payload, 0, m->words * sizeof(uint64_t));
  ccmref_encode_run(dense, m->rows * m->cols, m->bits, m->payload);
  return CCMREF_OK;
}

int ccmref_decompress(const ccmref_matrix *m, int64_t *dense) {
  if (!dense || !m || !m->payload) return CCMREF_E_INVAL;
  ccmref_decode_run(m->payload, m->rows * m->cols, m->bits, m->is_signed, dense);
  return CCMREF_OK;
}

int ccmref_get(const ccmref_matrix *m, int64_t i, int64_t j, int64_t *out) {
  if (!m || !out) return CCMREF_E_INVAL;
  if (i < 0 || i >= m->rows || j < 0 || j >= m->cols) return CCMREF_E_RANGE;
  *out = get_field(m->payload, (uint64_t)(i * m->cols + j), m->bits, m->is_signed);
  return CCMREF_OK;
}

static void put_le(uint8_t *dst, uint64_t v, int nbytes) {
  for (int k = 0; k < nbytes; k++) dst[k] = (uint8_t)(v >> (8 * k));
}

void ccmref_header(const ccmref_matrix *m, uint8_t out[64]) {
  memset(out, 0, 64);
  out[0] = 'C';
  out[1] = 'C';
  out[2] = 'M';
  out[3] = '1';
  put_le(out + 4, 1u, 2);
  out[6] = (uint8_t)m->bits;
  out[7] = (uint8_t)(m->is_signed ? 1u : 0u);
  put_le(out + 8, (uint64_t)m->rows, 8);
  put_le(out + 16, (uint64_t)m->cols, 8);
  put_le(out + 24, (uint64_t)m->vmin, 8);
  put_le(out + 32, (uint64_t)m->vmax, 8);
  put_le(out + 40, m->words, 8);
}

/* ---- arithmetic on the decoded values ---------------------------------- */

static int fits_i64(__int128 v) {
  return v >= (__int128)INT64_MIN && v <= (__int128)INT64_MAX;
}

int ccmref_add_dense(const ccmref_matrix *a, const ccmref_matrix *b, int64_t *out) {
  if (!a || !b || !out) return CCMREF_E_INVAL;
  if (a->rows != b->rows || a->cols != b->cols) return CCMREF_E_SHAPE;
  int64_t n = a->rows * a->cols;
  for (int64_t e = 0; e < n; e++) {
    __int128 s = (__int128)get_field(a->payload, (uint64_t)e, a->bits, a->is_signed) +
                 (__int128)get_field(b->payload, (uint64_t)e, b->bits, b->is_signed);
    if (!fits_i64(s)) return CCMREF_E_OVERFLOW;
    out[e] = (int64_t)s;
  }
  return CCMREF_OK;
}

int ccmref_scale_dense(const ccmref_matrix *a, int64_t s, int64_t *out) {
  if (!a || !out) return CCMREF_E_INVAL;
  int64_t n = a->rows * a->cols;
  for (int64_t e = 0; e < n; e++) {
    __int128 p = (__int128)get_field(a->payload, (uint64_t)e, a->bits, a->is_signed) * (__int128)s;
    if (!fits_i64(p)) return CCMREF_E_OVERFLOW;
    out[e] = (int64_t)p;
  }
  return CCMREF_OK;
}

int ccmref_matvec_rows(const ccmref_matrix *a, const int64_t *x, int64_t row_begin,
                       int64_t row_end, int64_t *y) {
  if (!a || !x || !y) return CCMREF_E_INVAL;
  if (row_begin < 0 || row_end > a->rows || row_begin > row_end) return CCMREF_E_RANGE;
  int64_t r;
#pragma omp parallel for schedule(dynamic, 1)
  for (r = row_begin; r < row_end; r++) {
    /* Accumulate modulo 2^128 (unsigned, no undefined overflow); the low 64
     * bits are the sum modulo 2^64. */
    unsigned __int128 acc = 0;
    for (int64_t j = 0; j < a->cols; j++) {
      int64_t v = get_field(a->payload, (uint64_t)(r * a->cols + j), a->bits, a->is_signed);
      acc += (unsigned __int128)((__int128)v * (__int128)x[j]);
    }
    y[r - row_begin] = (int64_t)(uint64_t)acc;
  }
  return CCMREF_OK;
}

static uint64_t max_abs(int64_t lo, int64_t hi) {
  uint64_t a = lo < 0 ? (uint64_t)0 - (uint64_t)lo : (uint64_t)lo;
  uint64_t b = hi < 0 ? (uint64_t)0 - (uint64_t)hi : (uint64_t)hi;
  return a > b ? a : b;
}

int ccmref_matmul_check(const ccmref_matrix *a, const ccmref_matrix *b) {
  if (!a || !b) return CCMREF_E_INVAL;
  if (a->cols != b->rows) return CCMREF_E_SHAPE;
  unsigned __int128 p = (unsigned __int128)max_abs(a->vmin, a->vmax) *
                        (unsigned __int128)max_abs(b->vmin, b->vmax);
  const unsigned __int128 lim = (unsigned __int128)1 << 63;
  if (p >= lim) return CCMREF_E_OVERFLOW;
  if (p * (unsigned __int128)(uint64_t)a->cols >= lim) return CCMREF_E_OVERFLOW;
  return CCMREF_OK;
}

static int64_t matmul_entry(const ccmref_matrix *a, const ccmref_matrix *b, int64_t i,
                            int64_t j) {
  __int128 acc = 0;
  for (int64_t k = 0; k < a->cols; k++) {
    int64_t av = get_field(a->payload, (uint64_t)(i * a->cols + k), a->bits, a->is_signed);
    int64_t bv = get_field(b->payload, (uint64_t)(k * b->cols + j), b->bits, b->is_signed);
    acc += (__int128)av * (__int128)bv;
  }
  return (int64_t)acc; /* fits: guaranteed by ccmref_matmul_check */
}

int ccmref_matmul_dense(const ccmref_matrix *a, const ccmref_matrix *b, int64_t *out) {
  int rc = ccmref_matmul_check(a, b);
  if (rc != CCMREF_OK) return rc;
  if (!out) return CCMREF_E_INVAL;
  int64_t i;
#pragma omp parallel for schedule(dynamic, 1)
  for (i = 0; i < a->rows; i++)
    for (int64_t j = 0; j < b->cols; j++) out[i * b->cols + j] = matmul_entry(a, b, i, j);
  return CCMREF_OK;
}

int ccmref_matmul_entries(const ccmref_matrix *a, const ccmref_matrix *b, const int64_t *ii,
                          const int64_t *jj, int64_t n, int64_t *out) {
  int rc = ccmref_matmul_check(a, b);
  if (rc != CCMREF_OK) return rc;
  if (!ii || !jj || !out) return CCMREF_E_INVAL;
  for (int64_t t = 0; t < n; t++)
    if (ii[t] < 0 || ii[t] >= a->rows || jj[t] < 0 || jj[t] >= b->cols) return CCMREF_E_RANGE;
  int64_t t;
#pragma omp parallel for schedule(dynamic, 16)
  for (t = 0; t < n; t++) out[t] = matmul_entry(a, b, ii[t], jj[t]);
  return CCMREF_OK;
}

/* ---- column-major unravel ------------------------------------------------ */

/* Stream index of element (i, j) when the matrix is unravelled by column. */
static uint64_t cm_index(const ccmref_matrix *m, int64_t i, int64_t j) {
  return (uint64_t)(j * m->rows + i);
}

int ccmref_compress_cm(const int64_t *dense, ccmref_matrix *m) {
  if (!dense || !m || !m->payload) return CCMREF_E_INVAL;
  memset(m->payload, 0, m->words * sizeof(uint64_t));
  for (int64_t i = 0; i < m->rows; i++)
    for (int64_t j = 0; j < m->cols; j++)
      put_field(m->payload, cm_index(m, i, j), m->bits, dense[i * m->cols + j]);
  return CCMREF_OK;
}

int ccmref_decompress_cm(const ccmref_matrix *m, int64_t *dense) {
  if (!dense || !m || !m->payload) return CCMREF_E_INVAL;
  for (int64_t i = 0; i < m->rows; i++)
    for (int64_t j = 0; j < m->cols; j++)
      dense[i * m->cols + j] = get_field(m->payload, cm_index(m, i, j), m->bits, m->is_signed);
  return CCMREF_OK;
}

int ccmref_get_cm(const ccmref_matrix *m, int64_t i, int64_t j, int64_t *out) {
  if (!m || !out || !m->payload) return CCMREF_E_INVAL;
  if (i < 0 || i >= m->rows || j < 0 || j >= m->cols) return CCMREF_E_RANGE;
  *out = get_field(m->payload, cm_index(m, i, j), m->bits, m->is_signed);
  return CCMREF_OK;
}

int ccmref_matvec_cm(const ccmref_matrix *a, const int64_t *x, int64_t *y) {
  if (!a || !x || !y || !a->payload) return CCMREF_E_INVAL;
  int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
  for (i = 0; i < a->rows; i++) {
    unsigned __int128 acc = 0;
    for (int64_t j = 0; j < a->cols; j++) {
      int64_t v = get_field(a->payload, cm_index(a, i, j), a->bits, a->is_signed);
      acc += (unsigned __int128)((__int128)v * (__int128)x[j]);
    }
    y[i] = (int64_t)(uint64_t)acc;
  }
  return CCMREF_OK;
}

int ccmref_matvec_t(const ccmref_matrix *a, const int64_t *x, int64_t *y) {
  if (!a || !x || !y || !a->payload) return CCMREF_E_INVAL;
  int64_t j;
#pragma omp parallel for schedule(dynamic, 16)
  for (j = 0; j < a->cols; j++) {
    unsigned __int128 acc = 0;
    for (int64_t i = 0; i < a->rows; i++) {
      int64_t v = get_field(a->payload, (uint64_t)(i * a->cols + j), a->bits, a->is_signed);
      acc += (unsigned __int128)((__int128)v * (__int128)x[i]);
    }
    y[j] = (int64_t)(uint64_t)acc;
  }
  return CCMREF_OK;
}

int ccmref_matvec_t_cm(const ccmref_matrix *a, const int64_t *x, int64_t *y) {
  if (!a || !x || !y || !a->payload) return CCMREF_E_INVAL;
  int64_t j;
#pragma omp parallel for schedule(dynamic, 16)
  for (j = 0; j < a->cols; j++) {
    unsigned __int128 acc = 0;
    for (int64_t i = 0; i < a->rows; i++) {
      int64_t v = get_field(a->payload, cm_index(a, i, j), a->bits, a->is_signed);
      acc += (unsigned __int128)((__int128)v * (__int128)x[i]);
    }
    y[j] = (int64_t)(uint64_t)acc;
  }
  return CCMREF_OK;
}

void ccmref_header_cm(const ccmref_matrix *m, uint8_t out[64]) {
  ccmref_header(m, out);
  out[7] = (uint8_t)(out[7] | 2u);
}

/* ---- Method 2: Variable Length Blocks ----------------------------------- */

int ccmref_vlb_width(int64_t v, int32_t is_signed) {
  if (!is_signed) return ccmref_sm_width((uint64_t)v); /* Eq. 1 on the element */
  int32_t b = 0, s = 0;
  /* the width of the one-value range [v, v] in two's complement, with the
   * sign bit even for v >= 0 */
  if (v < 0) {
    ccmref_width(v, v, &b, &s);
  } else {
    b = 1 + ccmref_bitlen((uint64_t)v);
  }
  return b;
}

/* Bits [p, p+bits) of the stream get the low bits of u. */
static void put_bits(uint64_t *words, uint64_t p, int32_t bits, uint64_t u) {
  for (int t = 0; t < bits; t++) put_bit(words, p + (uint64_t)t, (int)((u >> t) & 1u));
}

static uint64_t get_bits(const uint64_t *words, uint64_t p, int32_t bits) {
  uint64_t u = 0;
  for (int t = 0; t < bits; t++) u |= (uint64_t)get_bit(words, p + (uint64_t)t) << t;
  return u;
}

int ccmref_vlb_plan(const int64_t *dense, int64_t rows, int64_t cols, ccmref_vlb *m) {
  if (!dense || !m || rows < 1 || cols < 1) return CCMREF_E_INVAL;
  int64_t n = rows * cols;
  int64_t lo = dense[0], hi = dense[0];
  for (int64_t e = 1; e < n; e++) {
    if (dense[e] < lo) lo = dense[e];
    if (dense[e] > hi) hi = dense[e];
  }
  m->rows = rows;
  m->cols = cols;
  m->vmin = lo;
  m->vmax = hi;
  m->is_signed = lo < 0;
  int32_t bmax = 1;
  uint64_t sum_b = 0;
  for (int64_t e = 0; e < n; e++) {
    int32_t b = ccmref_vlb_width(dense[e], m->is_signed);
    if (b > bmax) bmax = b;
    sum_b += (uint64_t)b;
  }
  m->k = ccmref_bitlen((uint64_t)bmax);
  m->nbits = (uint64_t)n * (uint64_t)m->k + sum_b;
  m->words = m->nbits / 64u + 1u;
  return CCMREF_OK;
}

int ccmref_vlb_compress(const int64_t *dense, ccmref_vlb *m) {
  if (!dense || !m || !m->payload) return CCMREF_E_INVAL;
  memset(m->payload, 0, m->words * sizeof(uint64_t));
  uint64_t p = 0;
  for (int64_t e = 0; e < m->rows * m->cols; e++) {
    int32_t b = ccmref_vlb_width(dense[e], m->is_signed);
    put_bits(m->payload, p, m->k, (uint64_t)b); /* the fixed-size length chunk */
    p += (uint64_t)m->k;
    put_bits(m->payload, p, b, (uint64_t)dense[e]); /* then the element itself */
    p += (uint64_t)b;
  }
  return CCMREF_OK;
}

/* Decodes the element starting at stream bit *p and advances *p. */
static int64_t vlb_next(const ccmref_vlb *m, uint64_t *p) {
  int32_t b = (int32_t)get_bits(m->payload, *p, m->k);
  *p += (uint64_t)m->k;
  uint64_t u = get_bits(m->payload, *p, b);
  *p += (uint64_t)b;
  if (m->is_signed && ((u >> (b - 1)) & 1u) && b < 64) u -= (uint64_t)1 << b;
  return (int64_t)u;
}

int ccmref_vlb_decompress(const ccmref_vlb *m, int64_t *dense) {
  if (!m || !dense || !m->payload) return CCMREF_E_INVAL;
  uint64_t p = 0;
  for (int64_t e = 0; e < m->rows * m->cols; e++) dense[e] = vlb_next(m, &p);
  return CCMREF_OK;
}

int ccmref_vlb_get(const ccmref_vlb *m, int64_t i, int64_t j, int64_t *out) {
  if (!m || !out || !m->payload) return CCMREF_E_INVAL;
  if (i < 0 || i >= m->rows || j < 0 || j >= m->cols) return CCMREF_E_RANGE;
  uint64_t p = 0;
  int64_t v = 0;
  for (int64_t e = 0; e <= i * m->cols + j; e++) v = vlb_next(m, &p);
  *out = v;
  return CCMREF_OK;
}

int ccmref_vlb_offsets(const ccmref_vlb *m, int64_t group, uint64_t *out) {
  if (!m || !out || !m->payload || group < 1) return CCMREF_E_INVAL;
  uint64_t p = 0;
  int64_t t = 0;
  for (int64_t i = 0; i < m->rows; i++)
    for (int64_t j = 0; j < m->cols; j++) {
      if (j % group == 0) out[t++] = p;
      (void)vlb_next(m, &p);
    }
  return CCMREF_OK;
}

int ccmref_vlb_matvec(const ccmref_vlb *m, const int64_t *x, int64_t *y) {
  if (!m || !x || !y || !m->payload) return CCMREF_E_INVAL;
  uint64_t p = 0;
  for (int64_t i = 0; i < m->rows; i++) {
    unsigned __int128 acc = 0;
    for (int64_t j = 0; j < m->cols; j++) {
      int64_t a = vlb_next(m, &p);
      acc += (unsigned __int128)((__int128)a * (__int128)x[j]);
    }
    y[i] = (int64_t)(uint64_t)acc;
  }
  return CCMREF_OK;
}

/* ---- choosing the method ---------------------------------------------------- */

int ccmref_method_info_of(const int64_t *dense, int64_t rows, int64_t cols,
                          ccmref_method_info *out) {
  if (!dense || !out || rows < 1 || cols < 1) return CCMREF_E_INVAL;
  ccmref_matrix m1;
  int rc = ccmref_plan(dense, rows, cols, &m1);
  if (rc != CCMREF_OK) return rc;
  ccmref_vlb m2;
  rc = ccmref_vlb_plan(dense, rows, cols, &m2);
  if (rc != CCMREF_OK) return rc;
  const uint64_t n = (uint64_t)rows * (uint64_t)cols;
  out->vmin = m1.vmin;
  out->vmax = m1.vmax;
  out->sm_bits = m1.bits;
  out->vlb_k = m2.k;
  out->sm_nbits = n * (uint64_t)m1.bits;
  out->vlb_nbits = m2.nbits;
  out->eta1 = 1.0 - (double)out->sm_nbits / (64.0 * (double)n);
  out->eta2 = 1.0 - (double)out->vlb_nbits / (64.0 * (double)n);
  out->method = out->vlb_nbits < out->sm_nbits ? 2 : 1;
  out->pad = 0;
  return CCMREF_OK;
}

double ccmref_eta2_model(const double *p, int32_t k) {
  double mean = 0.0;
  for (int b = 1; b <= 64; b++) mean += (double)b * p[b - 1];
  return 1.0 - mean / 64.0 - (double)k / 64.0;
}

/* ---- floats in fixed point ------------------------------------------------ */

int ccmref_frac_bits(double absmax, int32_t sig_bits, int32_t *frac_bits) {
  if (!frac_bits || sig_bits < 1 || sig_bits > 62 || !(absmax >= 0.0) || isinf(absmax))
    return CCMREF_E_INVAL;
  if (absmax == 0.0) {
    *frac_bits = 0;
    return CCMREF_OK;
  }
  int ex = 0;
  (void)frexp(absmax, &ex); /* absmax = m 2^ex, 1/2 <= m < 1: e = ex - 1 */
  *frac_bits = sig_bits - 1 - (ex - 1);
  return CCMREF_OK;
}

/* round half to even of a finite double, written out: the floor, the
 * fraction above it (exact), then the nearer neighbour or the even one */
static double round_half_even(double t) {
  const double fl = floor(t);
  const double d = t - fl;
  if (d > 0.5) return fl + 1.0;
  if (d < 0.5) return fl;
  return fmod(fl, 2.0) == 0.0 ? fl : fl + 1.0;
}

static int quantize_one(double v, int32_t f, int64_t *q) {
  const double t = ldexp(v, f); /* exact unless it leaves the double range */
  if (!(fabs(t) < 0x1p62)) return CCMREF_E_OVERFLOW;
  *q = (int64_t)round_half_even(t);
  return CCMREF_OK;
}

int ccmref_quantize_f64(const double *v, int64_t n, int32_t frac_bits, int64_t *q) {
  if (!v || !q || n < 0) return CCMREF_E_INVAL;
  for (int64_t i = 0; i < n; i++)
    if (isnan(v[i]) || isinf(v[i])) return CCMREF_E_RANGE;
  for (int64_t i = 0; i < n; i++) {
    const int rc = quantize_one(v[i], frac_bits, &q[i]);
    if (rc != CCMREF_OK) return rc;
  }
  return CCMREF_OK;
}

int ccmref_quantize_f32(const float *v, int64_t n, int32_t frac_bits, int64_t *q) {
  if (!v || !q || n < 0) return CCMREF_E_INVAL;
  for (int64_t i = 0; i < n; i++)
    if (isnan(v[i]) || isinf(v[i])) return CCMREF_E_RANGE;
  for (int64_t i = 0; i < n; i++) {
    const int rc = quantize_one((double)v[i], frac_bits, &q[i]);
    if (rc != CCMREF_OK) return rc;
  }
  return CCMREF_OK;
}

void ccmref_dequantize_f64(const int64_t *q, int64_t n, int32_t frac_bits, double *v) {
  for (int64_t i = 0; i < n; i++) v[i] = ldexp((double)q[i], -frac_bits);
}

void ccmref_dequantize_f32(const int64_t *q, int64_t n, int32_t frac_bits, float *v) {
  for (int64_t i = 0; i < n; i++) v[i] = (float)ldexp((double)q[i], -frac_bits);
}

void ccmref_header_fx(const ccmref_matrix *m, int32_t frac_bits, uint8_t out[64]) {
  ccmref_header(m, out);
  out[7] = (uint8_t)(out[7] | 4u);
  put_le(out + 48, (uint64_t)(uint16_t)(int16_t)frac_bits, 2);
}
