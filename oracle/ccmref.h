/*
 * ccmref.h -- CPU oracle for Supreme-Minimum (SM) compressed integer matrices.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Paper: Paixao & Codeco Coelho, "Computable Compressed Matrices"
 * (arXiv 1303.0270).  Section references below are to that paper.
 *
 * Encoding (Methods, "Matrix compression" and "Method 1: The Supreme Minimum"):
 *   - one fixed field width b per matrix, b = b(sup M) from Eq. 1;
 *   - elements unravelled row-major and written as adjacent b-bit chunks,
 *     least significant bit first ("read from right to left"), with a chunk
 *     that does not fit in the current 64-bit bitstring straddling into the
 *     next one (Eq. 3 and the step-by-step example that follows it);
 *   - floor(dim(M) * b / 64) + 1 bitstrings (text after Table 1).
 *
 * Readings where the paper is silent (each is also listed in the design notes):
 *   - negative values: two's complement in b bits with a per-matrix signed flag,
 *     set iff min < 0; non-negative matrices encode exactly as in the paper;
 *   - all bits of the payload past rows*cols*b are zero;
 *   - operations (add, scale, matvec, matmul) are exact integer arithmetic on
 *     the decoded values, and every matrix result is re-encoded at the minimal
 *     width of its own values (signedness also from the result values);
 *   - overflow: add/scale fail iff an exact result leaves int64; matmul fails
 *     iff K*max|A|*max|B| >= 2^63 (an O(1) bound from the headers); matvec
 *     wraps modulo 2^64.
 *
 * Parity pins (all in tests/, run without a GPU):
 *   bitlen / width: Table 1's eight bit-lengths, Eq. 1's {0,1} case, brute force
 *     against Python's int.bit_length;
 *   encode / decode / size: the worked example's two bitstrings (Eq. 3 and the
 *     straddle step), round trips, closed-form size, zero padding, width
 *     minimality;
 *   signed encoding: the paper treats positive integers only, so no printed
 *     value covers it; pinned by round trips, minimality and brute force;
 *   add / scale / matvec / matmul: the paper prints no arithmetic example;
 *     pinned by brute force against uncompressed Python integer arithmetic
 *     and by algebraic identities.
 */
#ifndef CCMREF_H
#define CCMREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CCMREF_OK = 0,
  CCMREF_E_INVAL = -1,
  CCMREF_E_SHAPE = -2,
  CCMREF_E_RANGE = -3,
  CCMREF_E_OVERFLOW = -4
};

/* A compressed matrix "m" (lower-case name for the compressed form of M,
 * Method 1).  The payload is host memory owned by the caller, `words`
 * 64-bit bitstrings long. */
typedef struct {
  int64_t rows, cols;
  int64_t vmin, vmax;   /* exact extremes of the values */
  int32_t bits;         /* field width b */
  int32_t is_signed;    /* 1 iff vmin < 0 */
  uint64_t words;       /* floor(rows*cols*bits/64) + 1 */
  uint64_t *payload;
} ccmref_matrix;

/* Smallest L with u < 2^L (so bitlen(0) == 0). */
int ccmref_bitlen(uint64_t u);

/* Eq. 1: b(sup M) = 1 if sup M is 0 or 1, else floor(log2(sup M)) + 1. */
int ccmref_sm_width(uint64_t sup);

/* Width rule for a value range: Eq. 1 applied to sup M when min >= 0,
 * otherwise the smallest two's-complement width that holds [min, max]. */
int ccmref_width(int64_t vmin, int64_t vmax, int32_t *bits, int32_t *is_signed);

/* Number of 64-bit bitstrings, floor(n*b/64) + 1 (text after Table 1). */
uint64_t ccmref_words(int64_t rows, int64_t cols, int32_t bits);

/* Fill rows, cols, vmin, vmax, bits, is_signed and words from dense values
 * (row-major, rows*cols int64).  Does not touch payload. */
int ccmref_plan(const int64_t *dense, int64_t rows, int64_t cols, ccmref_matrix *m);

/* Write the SM bitstrings of dense into m->payload (m from ccmref_plan). */
int ccmref_compress(const int64_t *dense, ccmref_matrix *m);

/* Decode every element of m into dense (row-major). */
int ccmref_decompress(const ccmref_matrix *m, int64_t *dense);

/* Element access by row i and column j (both 0-based). */
int ccmref_get(const ccmref_matrix *m, int64_t i, int64_t j, int64_t *out);

/* Write / read n fields of width b starting at stream bit 0 of words
 * (a run of adjacent chunks; the building block of compress/decompress). */
void ccmref_encode_run(const int64_t *vals, int64_t n, int32_t bits, uint64_t *words);
void ccmref_decode_run(const uint64_t *words, int64_t n, int32_t bits, int32_t is_signed,
                       int64_t *vals);

/* The 64-byte little-endian header: "CCM1", u16 version 1, u8 bits,
 * u8 flags (bit 0 signed), i64 rows, cols, min, max, u64 words, 16 zero bytes. */
void ccmref_header(const ccmref_matrix *m, uint8_t out[64]);

/* Exact elementwise results as dense int64 (to be re-encoded with
 * ccmref_plan + ccmref_compress). */
int ccmref_add_dense(const ccmref_matrix *a, const ccmref_matrix *b, int64_t *out);
int ccmref_scale_dense(const ccmref_matrix *a, int64_t s, int64_t *out);

/* y[i] = sum_j a[i][j] * x[j] modulo 2^64, for rows [row_begin, row_end). */
int ccmref_matvec_rows(const ccmref_matrix *a, const int64_t *x, int64_t row_begin,
                       int64_t row_end, int64_t *y);

/* Overflow rule for C = A*B (see the header comment). */
int ccmref_matmul_check(const ccmref_matrix *a, const ccmref_matrix *b);

/* Dense C = A*B, exact (after ccmref_matmul_check). */
int ccmref_matmul_dense(const ccmref_matrix *a, const ccmref_matrix *b, int64_t *out);

/* Selected entries C[ii[t]][jj[t]] of A*B, exact. */
int ccmref_matmul_entries(const ccmref_matrix *a, const ccmref_matrix *b, const int64_t *ii,
                          const int64_t *jj, int64_t n, int64_t *out);

/* ---- Column-major unravel ------------------------------------------------
 *
 * The matrix may be unravelled by column (Fortran order) instead of by row
 * (Methods, "Matrix compression").  Same widths, fields, bit order and word
 * count; element (i, j) is stream element j*rows + i.  rows and cols stay
 * those of A; the header sets flags bit 1.  The y = A^T x products are the
 * plain definition y[j] = sum_i a[i][j] * x[i] modulo 2^64.
 */

/* dense is row-major rows*cols (m from ccmref_plan over the same values). */
int ccmref_compress_cm(const int64_t *dense, ccmref_matrix *m);
/* Decode to row-major dense. */
int ccmref_decompress_cm(const ccmref_matrix *m, int64_t *dense);
int ccmref_get_cm(const ccmref_matrix *m, int64_t i, int64_t j, int64_t *out);
/* y = A x (x: cols, y: rows) for a column-major matrix. */
int ccmref_matvec_cm(const ccmref_matrix *a, const int64_t *x, int64_t *y);
/* y = A^T x (x: rows, y: cols) for a row-major / column-major matrix. */
int ccmref_matvec_t(const ccmref_matrix *a, const int64_t *x, int64_t *y);
int ccmref_matvec_t_cm(const ccmref_matrix *a, const int64_t *x, int64_t *y);
/* The header of a column-major matrix (flags bit 1 set). */
void ccmref_header_cm(const ccmref_matrix *m, uint8_t out[64]);

/* ---- Method 2: Variable Length Blocks (VLB) ----------------------------
 *
 * Each element gets its own minimal width b_e, stored in a length field of a
 * fixed k bits that precedes the element's b_e value bits; k is the
 * bit-length of the largest b_e (Methods, "Method 2": the fixed chunk holds
 * the bit-length of sup M, 10 -> 4 bits in the worked example).  Elements are
 * adjacent in row-major order, least significant bit first, fields
 * straddling bitstrings exactly as in Method 1.
 *
 * Readings where the paper is silent:
 *   - b_e is Eq. 1 applied to the single element (0 and 1 take one bit); for
 *     a matrix with a negative element every b_e is a two's complement width
 *     (one bit more than the magnitude's bit-length), decoded by sign
 *     extension from b_e bits;
 *   - the length field holds b_e itself (1..64), so k = bitlen(max b_e) <= 7;
 *   - floor(total_bits / 64) + 1 bitstrings, as for Method 1; bits past the
 *     last field are zero;
 *   - random access (get) is a scan from the first element: the paper gives
 *     no index.
 * Pins: the worked example's two bitstrings (the layout gives 91 bits; the
 * paper's text says 87), round trips, the closed-form bit count, brute force.
 */
typedef struct {
  int64_t rows, cols;
  int64_t vmin, vmax;
  int32_t k;          /* length-field width */
  int32_t is_signed;  /* 1 iff vmin < 0 */
  uint64_t nbits;     /* sum over elements of k + b_e */
  uint64_t words;     /* floor(nbits / 64) + 1 */
  uint64_t *payload;
} ccmref_vlb;

/* b_e of one value under the matrix's signedness. */
int ccmref_vlb_width(int64_t v, int32_t is_signed);

/* Fills everything but payload. */
int ccmref_vlb_plan(const int64_t *dense, int64_t rows, int64_t cols, ccmref_vlb *m);

/* Writes m->payload (m->words bitstrings, caller-allocated) after ccmref_vlb_plan. */
int ccmref_vlb_compress(const int64_t *dense, ccmref_vlb *m);

int ccmref_vlb_decompress(const ccmref_vlb *m, int64_t *dense);

int ccmref_vlb_get(const ccmref_vlb *m, int64_t i, int64_t j, int64_t *out);

/* Stream bit where element (i, j) starts, for every i and every j that is a
 * multiple of `group` (row-major over (i, j / group)); out holds
 * rows * ceil(cols / group) entries.  Used to check the GPU's index. */
int ccmref_vlb_offsets(const ccmref_vlb *m, int64_t group, uint64_t *out);

/* y[i] = sum_j a[i][j] * x[j] modulo 2^64 for every row. */
int ccmref_vlb_matvec(const ccmref_vlb *m, const int64_t *x, int64_t *y);

/* ---- Choosing the method (Eq. 14-17; Discussion, "Calculating
 * Efficiencies") ----------------------------------------------------------
 *
 * Efficiency is eta = (bits allocated - bits used) / bits allocated against
 * 64-bit storage (Eq. 14).  Method 1 uses n*b bits (eta_1 = (64 - b)/64,
 * Eq. 15); Method 2 uses sum over elements of (k + b_e) (Eq. 16, 17).  The
 * method chosen is the one using fewer bits; on a tie Method 1 (its fields
 * need no index to reach).  The bit counts are exact integers; the eta values
 * are doubles computed from them as 1 - used / (64 n).
 */
typedef struct {
  int64_t vmin, vmax;
  int32_t sm_bits;      /* Method 1 width b */
  int32_t vlb_k;        /* Method 2 length-field width */
  uint64_t sm_nbits;    /* n * b */
  uint64_t vlb_nbits;   /* sum of k + b_e */
  double eta1, eta2;
  int32_t method;       /* 1 or 2 */
  int32_t pad;
} ccmref_method_info;

int ccmref_method_info_of(const int64_t *dense, int64_t rows, int64_t cols,
                          ccmref_method_info *out);

/* ---- Floats in fixed point (Conclusion) --------------------------------
 *
 * The Conclusion says floats fit the framework if some precision is given
 * up, and gives no encoding.  Reading: a float matrix is stored as the integer
 * matrix q = round-half-to-even(v * 2^f) (f "fraction bits", one per
 * matrix), which Method 1 then packs like any integer matrix; the only
 * loss is that rounding, |v - q 2^-f| <= 2^-(f+1).  Everything after it is
 * exact integer arithmetic on q, and a float result is the exact integer
 * result converted back: to double with round-half-to-even, scaled by 2^-f
 * (exact unless the result is subnormal, then rounded once), and for float32
 * rounded once more to float.  The user picks f directly or as the number of
 * significant bits p the largest magnitude keeps: with 2^e <= max|v| <
 * 2^(e+1), f = p - 1 - e.
 * Pins: exact rational arithmetic (Python Fractions) on every rounding and
 * conversion, ties, subnormals, the error bound, a hand-computed header.
 */

/* f = sig_bits - 1 - e, 2^e <= absmax < 2^(e+1); f = 0 for absmax 0.
 * CCMREF_E_INVAL unless 1 <= sig_bits <= 62 and absmax is finite, >= 0. */
int ccmref_frac_bits(double absmax, int32_t sig_bits, int32_t *frac_bits);

/* q[i] = round-half-to-even(v[i] * 2^frac_bits).  CCMREF_E_RANGE when any
 * value is NaN or infinite, else CCMREF_E_OVERFLOW when some
 * |v * 2^f| >= 2^62. */
int ccmref_quantize_f64(const double *v, int64_t n, int32_t frac_bits, int64_t *q);
int ccmref_quantize_f32(const float *v, int64_t n, int32_t frac_bits, int64_t *q);

/* v[i] = q[i] * 2^-frac_bits as above (double, or rounded on to float). */
void ccmref_dequantize_f64(const int64_t *q, int64_t n, int32_t frac_bits, double *v);
void ccmref_dequantize_f32(const int64_t *q, int64_t n, int32_t frac_bits, float *v);

/* Header of a fixed-point matrix (this library's format): the integer
 * matrix's header with flags bit 2 set and f as a little-endian int16 at
 * bytes 48..49. */
void ccmref_header_fx(const ccmref_matrix *m, int32_t frac_bits, uint8_t out[64]);

/* Eq. 29: expected eta_2 for a bit-length distribution, p[b-1] = P(bit-length
 * = b) for b = 1..64, with a fixed k: 1 - sum_b b p_b / 64 - k / 64.  The
 * paper's analytic tables fix k = 7. */
double ccmref_eta2_model(const double *p, int32_t k);

#ifdef __cplusplus
}
#endif

#endif
