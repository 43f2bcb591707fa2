/*
 * ccm.h -- C ABI of libccm, linear algebra on SM-compressed integer matrices
 * on AMD Instinct MI355X (gfx950).
 *
 * Paper: Paixao & Codeco Coelho, "Computable Compressed Matrices"
 * (arXiv 1303.0270).  "Methods" below means its section "Methods" and the
 * subsections "Matrix compression" and "Method 1: The Supreme Minimum (SM)".
 *
 * Encoding (Method 1, Eq. 1, Eq. 3):
 *   A matrix of rows x cols int64 values is stored at ONE field width b:
 *     - min >= 0: b = b(sup M) from Eq. 1 (1 if max is 0 or 1, else
 *       floor(log2 max) + 1), unsigned fields;
 *     - min < 0 (the paper treats positive integers only; this library's
 *       reading): the smallest b with -2^(b-1) <= min and max < 2^(b-1),
 *       fields hold the low b bits of the two's complement.
 *   Elements are unravelled row-major; element e = i*cols + j occupies stream
 *   bits [e*b, e*b + b), least significant bit first ("read from right to
 *   left").  Stream bit p is bit p%64 of 64-bit bitstring p/64; a field that
 *   does not fit in one bitstring straddles into the next (Eq. 3 and the
 *   straddle step after it).  The canonical payload is W = floor(rows*cols*b
 *   /64) + 1 little-endian 64-bit bitstrings (the count stated after Table 1)
 *   with every bit past rows*cols*b zero; the serialized form is a 64-byte
 *   header (ccm_header_encode) followed by the payload: 64 + 8*W bytes.
 *   The GPU reads the same bytes as 32-bit words: word q holds stream bits
 *   [32q, 32q+32).
 *
 * Operations (the Introduction wants arithmetic on the compressed form to
 * agree with arithmetic on the uncompressed matrix; the paper gives no
 * algorithm): exact integer arithmetic on the decoded values.  Every
 * matrix-valued result is re-encoded at the minimal width of its own values
 * (its signedness too), found by a max/min-reduction pass ("plan") before the
 * packing pass.  matvec results are int64 modulo 2^64.
 *
 * Memory and ownership:
 *   - Every data pointer marked "device" is GPU memory owned by the caller;
 *     the library never frees it.  A compressed matrix's payload buffer must
 *     hold ccm_payload_capacity(rows, cols, bits) bytes (the canonical 8*W
 *     bytes plus guard words that kernels may read past the last field) and
 *     be 256-byte aligned (hipMalloc allocations are).  Kernels
 *     that write a payload write every byte of that capacity.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls marked "async" only enqueue work on it; calls marked "blocking"
 *     synchronize it before returning.  Inputs must stay valid until the
 *     enqueued work completes.
 *   - The library keeps a few bytes of device memory per device for blocking
 *     reductions (taken under a lock) and the batch objects' metadata.
 *
 * Errors: every call returns a ccm_status and never throws.  Arguments are
 * validated before any work is enqueued; CCM_E_DEVICE reports a HIP error
 * (the HIP error string is logged to stderr when CCM_LOG is set).
 */
#ifndef CCM_H
#define CCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CCM_OK = 0,
  CCM_E_INVAL = -1,       /* null pointer, rows or cols < 1, invalid descriptor */
  CCM_E_SHAPE = -2,       /* operand shapes do not match */
  CCM_E_RANGE = -3,       /* element index out of range */
  CCM_E_OVERFLOW = -4,    /* an exact result does not fit in int64 (rules below) */
  CCM_E_NOMEM = -5,       /* a caller buffer is too small, or an allocation failed */
  CCM_E_DEVICE = -6,      /* HIP runtime error */
  CCM_E_UNSUPPORTED = -7  /* valid request the library does not implement */
} ccm_status;

typedef enum { CCM_I32 = 0, CCM_I64 = 1, CCM_F32 = 2, CCM_F64 = 3 } ccm_dtype;

/* Descriptor of a compressed matrix "m" (the paper's lower-case name for the
 * compressed form of M).  Host struct; `payload` is a device pointer. */
typedef struct ccm_desc {
  int64_t rows, cols;
  int64_t vmin, vmax;  /* exact extremes of the values (not bounds) */
  int32_t bits;        /* field width b, 1..64 */
  int32_t is_signed;   /* 1 iff vmin < 0 (fields are two's complement) */
  uint64_t words;      /* W = floor(rows*cols*bits/64) + 1 */
  void *payload;       /* device, caller-owned, >= ccm_payload_capacity bytes */
} ccm_desc;

/* ---- sizes, widths, headers (host only, no GPU work) -------------------- */

/* Library version (major*10000 + minor*100 + patch). */
int ccm_version(void);

/* Human-readable name of a status code (static string). */
const char *ccm_status_str(int status);

/* W = floor(rows*cols*bits/64) + 1, the bitstring count after Table 1.
 * Returns 0 for invalid arguments. */
uint64_t ccm_words(int64_t rows, int64_t cols, int32_t bits);

/* Serialized size 64 + 8*W bytes (header + payload). 0 if invalid. */
uint64_t ccm_packed_bytes(int64_t rows, int64_t cols, int32_t bits);

/* Device bytes a payload buffer must hold: 8*W rounded up, plus guard words.
 * 0 if invalid. */
uint64_t ccm_payload_capacity(int64_t rows, int64_t cols, int32_t bits);

/* Width rule (Eq. 1 for min >= 0, two's complement otherwise).
 * CCM_E_INVAL if vmin > vmax or an output pointer is NULL. */
int ccm_width(int64_t vmin, int64_t vmax, int32_t *bits, int32_t *is_signed);

/* 64-byte little-endian header: "CCM1", u16 version 1, u8 bits, u8 flags
 * (bit 0 = signed), i64 rows, cols, min, max, u64 W, 16 zero bytes.
 * decode validates magic, version, flags, bits, W and that the width equals
 * the width rule applied to [min, max]; it leaves `payload` NULL. */
int ccm_header_encode(const ccm_desc *d, uint8_t out[64]);
int ccm_header_decode(const uint8_t in[64], ccm_desc *d);

/* ---- compress / decompress / get (Methods; element access by (i, j)) --- */

/* Exact (min, max) of n dense values (device, dtype CCM_I32 or CCM_I64).
 * Blocking. */
int ccm_range(const void *dense, int32_t dtype, int64_t n, int64_t *vmin, int64_t *vmax,
              void *stream);

/* Plan a compression: runs the range pass over dense (device, rows*cols
 * row-major values of `dtype`) and fills every field of `out` except
 * `payload`, which is set to NULL.  Blocking. */
int ccm_compress_plan(const void *dense, int32_t dtype, int64_t rows, int64_t cols,
                      ccm_desc *out, void *stream);

/* Pack dense into out->payload at out->bits (Method 1's SM packing).  `out`
 * must come from ccm_compress_plan over the same values with `payload`
 * set by the caller.  Async. */
int ccm_compress(const void *dense, int32_t dtype, const ccm_desc *out, void *stream);

/* Decode every element into dense_out (device, rows*cols int64).  Async. */
int ccm_decompress(const ccm_desc *a, int64_t *dense_out, void *stream);

/* Element (i, j) into *value (host).  CCM_E_RANGE outside the matrix.
 * Blocking. */
int ccm_get(const ccm_desc *a, int64_t i, int64_t j, int64_t *value, void *stream);

/* out[t] = element (ii[t], jj[t]) for t < n; ii, jj, out are device arrays.
 * Out-of-range pairs yield 0 and set *bad (device int32, may be NULL) to 1.
 * Async. */
int ccm_gather(const ccm_desc *a, const int64_t *ii, const int64_t *jj, int64_t n,
               int64_t *out, int32_t *bad, void *stream);

/* ---- elementwise add and scalar multiply -------------------------------- */
/* The Introduction asks that compressed matrices take the arithmetic of the
 * uncompressed ones; every result here is exact and re-encoded at the width
 * the width rule (Eq. 1) gives for its own extremes. */

/* C = A + B.  Plan: range pass over the exact sums, fills out (payload
 * NULL); CCM_E_OVERFLOW iff some sum leaves int64.  Blocking.
 * Op: decode, add, pack at out->bits.  Async. */
int ccm_add_plan(const ccm_desc *a, const ccm_desc *b, ccm_desc *out, void *stream);
int ccm_add(const ccm_desc *a, const ccm_desc *b, const ccm_desc *out, void *stream);

/* C = A + B in one call, usually one pass over A and B: the same result as
 * ccm_add_plan followed by ccm_add.  The headers bound the sums to
 * [a.vmin + b.vmin, a.vmax + b.vmax]; when that bound lies inside int64 (no
 * sum can overflow), the sums are packed at the bound's width while their
 * exact extremes are reduced, and only if the exact range needs a narrower
 * width are they packed again at that width.  Otherwise the range pass runs
 * first, as in ccm_add_plan.
 * out->payload: device, caller-owned, at least ccm_add_capacity(a, b) bytes
 * (never less than the final width needs); the other fields of *out are
 * outputs, set on success.  The first ccm_payload_capacity(rows, cols,
 * out->bits) bytes then hold what ccm_add writes there (zeros past 8*W); the
 * bytes after them are unspecified.  CCM_E_OVERFLOW iff some sum leaves
 * int64.  Blocking (one device-to-host read of the range). */
uint64_t ccm_add_capacity(const ccm_desc *a, const ccm_desc *b); /* 0 if invalid */
int ccm_add_onepass(const ccm_desc *a, const ccm_desc *b, ccm_desc *out, void *stream);

/* C = s * A.  The result range [s*min, s*max] (ordered) comes from A's
 * header, so the plan is host-only; CCM_E_OVERFLOW iff it leaves int64.
 * s = 0 gives an all-zero matrix with b = 1.  Op: async. */
int ccm_scale_plan(const ccm_desc *a, int64_t s, ccm_desc *out);
int ccm_scale(const ccm_desc *a, int64_t s, const ccm_desc *out, void *stream);

/* ---- matvec and matmul --------------------------------------------------- */

/* y = A x (y[i] = sum_j a_ij x_j modulo 2^64), read straight from the
 * packed fields (Introduction: compressed matrices take the same arithmetic
 * as uncompressed ones; the fields are laid out as in Method 1, Eq. 3).
 * x: device, cols values of xdtype (CCM_I32 or CCM_I64); y: device, rows
 * int64.  Async; no error for wrap-around. */
int ccm_matvec(const ccm_desc *a, const void *x, int32_t xdtype, int64_t *y, void *stream);

/* C = A B on packed operands (Introduction: the product of the uncompressed
 * matrices), re-encoded at the width of its exact range (Eq. 1, or two's
 * complement for a negative minimum).  CCM_E_OVERFLOW iff
 * K * max|A| * max|B| >= 2^63 (max|M| = max(|min|, |max|) from the headers;
 * an O(1) conservative bound), so every entry fits in int64.  Fields of at most 8 bits whose values fit int8 go
 * through int8 MFMA tiles with exact integer accumulation; others through an
 * exact int64 path.
 *   scratch_bytes: device scratch the two calls need (dense C at 4 or 8 bytes
 *     per entry; on the int8 path also A and B^T decoded to int8, K padded
 *     to a multiple of 128).
 *   plan: computes C into scratch and its exact range, fills out (payload
 *     NULL).  Blocking.
 *   op: packs the scratch into out->payload.  Async.
 * The scratch must not be modified between the two calls. */
uint64_t ccm_matmul_scratch_bytes(const ccm_desc *a, const ccm_desc *b);
int ccm_matmul_plan(const ccm_desc *a, const ccm_desc *b, ccm_desc *out, void *scratch,
                    uint64_t scratch_bytes, void *stream);
int ccm_matmul(const ccm_desc *a, const ccm_desc *b, const ccm_desc *out,
               const void *scratch, uint64_t scratch_bytes, void *stream);

/* ---- results whose width stays on the device (no host wait) -------------
 *
 * The same results as ccm_add_onepass and ccm_matmul_plan + ccm_matmul, with
 * every step enqueued on `stream` and no host synchronization: the exact
 * range is reduced on the device, the width rule (Eq. 1, or two's complement
 * for a negative minimum) is applied there, and the packing kernels read the
 * width from device memory.  For callers that keep work in flight (a serving
 * loop): the result's header fields are read back only once the stream's
 * work is known to be complete.
 *
 * ws: device, caller-owned, at least ccm_async_ws_bytes() bytes, 256-byte
 *   aligned.  Bytes [0, 64) receive a ccm_result when the enqueued work
 *   completes; the rest holds the range reduction's slots.  Calls whose work
 *   may overlap on the device need distinct ws buffers.
 * payload: device, caller-owned, at least the capacity stated for each call
 *   (the capacity at the width the operand headers bound, which is never
 *   less than the exact width needs).  On completion its first
 *   ccm_payload_capacity(rows, cols, result.bits) bytes hold exactly what the
 *   blocking calls write (zeros past 8*W); the bytes after them are
 *   unspecified.
 * Argument errors are returned at once; an overflow found on the device
 * (add only) is reported in result.status. */
typedef struct ccm_result {
  int64_t rows, cols;
  int64_t vmin, vmax;  /* exact extremes of the result */
  int32_t bits;        /* its width */
  int32_t is_signed;
  uint64_t words;      /* W = floor(rows*cols*bits/64) + 1 */
  int32_t status;      /* CCM_OK, or CCM_E_OVERFLOW (then no payload was written) */
  int32_t reserved0;
  uint64_t reserved1;
} ccm_result;          /* 64 bytes */

uint64_t ccm_async_ws_bytes(void);

/* C = A + B (Introduction: the arithmetic of the uncompressed matrices).
 * payload: at least ccm_add_capacity(a, b) bytes.  Async. */
int ccm_add_async(const ccm_desc *a, const ccm_desc *b, void *payload, uint64_t payload_bytes,
                  void *ws, void *stream);

/* C = A B, as ccm_matmul_plan + ccm_matmul (same overflow rule, same
 * scratch).  payload: at least ccm_matmul_capacity(a, b) bytes (0 if the
 * operands are invalid or the overflow bound is exceeded).  Async. */
uint64_t ccm_matmul_capacity(const ccm_desc *a, const ccm_desc *b);
int ccm_matmul_async(const ccm_desc *a, const ccm_desc *b, void *payload,
                     uint64_t payload_bytes, void *scratch, uint64_t scratch_bytes, void *ws,
                     void *stream);

/* Descriptor of a completed asynchronous result from a host copy of its
 * ccm_result (the first 64 bytes of ws) and its payload pointer: checks the
 * fields (status, width rule, word count) and fills *out.  Host only. */
int ccm_result_desc(const ccm_result *r, void *payload, ccm_desc *out);

/* ---- batched matvec (many matrices, one persistent launch) ------------- */

/* A batch binds n compressed matrices (their descriptors are copied; the
 * payloads must stay valid) and an int32 or int64 x dtype.  Creating it
 * builds a work list of (matrix, row block) items ordered by width and size,
 * with per-width tile choices from a tuning table (JSON written by the
 * project's autotuner, {"widths": {"<b>": {"tile_rows": r,
 * "rows_in_flight": f}}}, f in {1, 2, 4}, capped at 4 for b <= 8, 2 for
 * b <= 16 and 1 above; NULL, an unreadable path or a missing width uses
 * built-in defaults), and copies it to device memory the batch owns. */
typedef struct ccm_batch ccm_batch;

int ccm_batch_create(const ccm_desc *as, int32_t n, int32_t xdtype, const char *tune_json,
                     ccm_batch **out);

/* Bind the x and y device pointers of every matrix (host arrays of n device
 * pointers).  Enqueues one host-to-device copy on `stream`.  Async. */
int ccm_batch_set_io(ccm_batch *b, const void *const *xs, int64_t *const *ys, void *stream);

/* y_t = A_t x_t for every matrix t, in one persistent kernel launch.  With
 * use_graph != 0 the launch is captured once into a HIP graph and replayed.
 * Async. */
int ccm_batch_matvec(ccm_batch *b, int32_t use_graph, void *stream);

/* Work-list statistics: number of items, total packed bytes, max width. */
int ccm_batch_info(const ccm_batch *b, int64_t *items, uint64_t *packed_bytes,
                   int32_t *max_bits);

int ccm_batch_destroy(ccm_batch *b);

/* Dynamic batches (the matrices change on every launch, as in a serving
 * loop).  A workspace holds `slots` sets of pinned host staging and device
 * tables for up to max_mats matrices and max_items work items; launches use
 * the slots in turn, and a slot is reused only after its previous launch has
 * completed (the call waits for that if needed).  Library-owned memory,
 * released by ccm_batch_ws_destroy. */
typedef struct ccm_batch_ws ccm_batch_ws;

int ccm_batch_ws_create(int32_t max_mats, int64_t max_items, int32_t slots,
                        const char *tune_json, ccm_batch_ws **out);
int ccm_batch_ws_destroy(ccm_batch_ws *w);

/* y_t = A_t x_t for the n matrices given (x int32), planned on the host and
 * run as one persistent launch on `stream`.  CCM_E_NOMEM if n or the work
 * list exceeds the workspace.  Async (one host-to-device table copy). */
int ccm_batch_matvec_dyn(ccm_batch_ws *w, const ccm_desc *as, const void *const *xs,
                         int64_t *const *ys, int32_t n, void *stream);

/* ---- seeded synthetic data (SplitMix64, counter-based) ------------------ */

/* dense[t] = draw number (stream_id << 40) + start + t of SplitMix64 from
 * `seed`, mapped to [lo, hi) as lo + (((h >> 32) * (hi - lo)) >> 32);
 * requires 1 <= hi - lo <= 2^32.  Async. */
int ccm_fill_uniform(void *dense, int32_t dtype, int64_t n, int64_t lo, int64_t hi,
                     uint64_t seed, uint64_t stream_id, uint64_t start, void *stream);

/* Compress the rows x cols matrix whose row-major elements are the draws
 * above (start = 0) without a dense copy: plan runs the range pass (blocking)
 * and fills out (payload NULL); op packs (async). */
int ccm_generate_plan(int64_t rows, int64_t cols, int64_t lo, int64_t hi, uint64_t seed,
                      uint64_t stream_id, ccm_desc *out, void *stream);
int ccm_generate(const ccm_desc *out, int64_t lo, int64_t hi, uint64_t seed,
                 uint64_t stream_id, void *stream);

/* ---- column-major unravel (Methods, "Matrix compression") and y = A^T x ---
 *
 * The paper lets a matrix be unravelled by column (Fortran order) or by row.
 * A matrix A (R x C) unravelled by column holds element (i, j) at stream
 * element j*R + i: exactly the row-major stream of A^T (C x R), with the same
 * width rule, fields and word count.  The library therefore describes a
 * column-major A by the row-major descriptor of A^T (rows = C, cols = R); its
 * serialized header states A's own shape with flags bit 1 set.  Every
 * row-major call applies to that descriptor: y = A^T x of the column-major A
 * is ccm_matvec on it, and y = A x is ccm_matvec_t. */

/* y = A^T x (y[j] = sum_i a_ij x_i modulo 2^64) for the row-major matrix a:
 * x device, a->rows values of xdtype; y device, a->cols int64.
 *   The rows are split over up to 32 blocks per 2048-column panel.  With
 *   scratch (device, 8-byte aligned, at least ccm_matvec_t_scratch_bytes(a)
 *   bytes: 32 int64 partial sums per column) each split stores its column
 *   sums there and a second kernel adds them into y; with scratch NULL the
 *   splits add into y with atomics after zeroing it (slower).  A non-NULL
 *   scratch that is too small is CCM_E_NOMEM, a misaligned one CCM_E_INVAL.
 *   Calls that share one scratch buffer must be ordered (one stream).  Async. */
uint64_t ccm_matvec_t_scratch_bytes(const ccm_desc *a);
int ccm_matvec_t(const ccm_desc *a, const void *x, int32_t xdtype, int64_t *y, void *scratch,
                 uint64_t scratch_bytes, void *stream);

/* y = A^T x as ccm_matvec_t with a scratch buffer, for callers that cannot
 * allocate device memory (code under stream capture, serving loops, harnesses
 * that forbid allocation): the split partial sums go to a buffer the library
 * holds for the life of the process, 32 int64 per column for up to 65536
 * columns (16 MB per device).  Allocates nothing.  a->cols > 65536 is
 * CCM_E_NOMEM.  Calls whose work overlaps on one device share that buffer and
 * race: order them (one stream).  Async. */
int ccm_matvec_t_noalloc(const ccm_desc *a, const void *x, int32_t xdtype, int64_t *y,
                         void *stream);

/* Packs A, given dense row-major (out->cols x out->rows values of dtype),
 * unravelled by column into out->payload; out describes A^T and comes from
 * ccm_compress_plan(dense, dtype, out->rows, out->cols, ...) (the range pass
 * does not depend on the shape).  Writes the whole capacity.  Async. */
int ccm_compress_cm(const void *dense, int32_t dtype, const ccm_desc *out, void *stream);

/* Header of the column-major matrix whose stream `at` describes (A^T,
 * row-major): A's rows and cols, flags bit 1 set.  Decode: a header with
 * flags bit 1 set back to the descriptor of A^T (payload NULL); CCM_E_INVAL
 * when bit 1 is clear (ccm_header_decode reads only row-major headers). */
int ccm_header_encode_cm(const ccm_desc *at, uint8_t out[64]);
int ccm_header_decode_cm(const uint8_t in[64], ccm_desc *at);

/* ---- choosing the method (Eq. 14-17; Discussion, "Calculating
 * Efficiencies") ------------------------------------------------------------
 *
 * The paper picks Method 1 for small or nearly constant bit-lengths and
 * Method 2 otherwise, from the efficiency eta = (bits allocated - bits used) /
 * bits allocated against 64-bit storage (Eq. 14).  Here both bit counts are
 * computed exactly: Method 1 uses n*b bits (eta_1 = (64 - b)/64, Eq. 15),
 * Method 2 sum of (k + b_e) bits (Eq. 16, 17).  The choice is Method 2 iff it
 * uses strictly fewer bits (Method 1 on a tie: its fields need no index). */
typedef struct ccm_method_info {
  int64_t vmin, vmax;  /* exact extremes */
  int32_t sm_bits;     /* Method 1 width b */
  int32_t vlb_k;       /* Method 2 length-field width */
  uint64_t sm_nbits;   /* n * b */
  uint64_t vlb_nbits;  /* sum of k + b_e */
  double eta1, eta2;   /* 1 - bits / (64 n) */
  int32_t method;      /* 1 or 2 */
  int32_t reserved;
} ccm_method_info;

/* One pass over dense (device, rows*cols values of dtype): extremes and both
 * sums of element widths; fills out.  Blocking. */
int ccm_method_plan(const void *dense, int32_t dtype, int64_t rows, int64_t cols,
                    ccm_method_info *out, void *stream);

/* ---- Method 2: Variable Length Blocks (Methods, "Method 2"; Eq. 16) ------
 *
 * Encoding: every element e has its own width b_e -- Eq. 1 applied to the
 * element when the matrix has no negative value, else the smallest two's
 * complement width holding it (the same sign reading as Method 1).  The
 * stream holds, for each element in row-major order, a k-bit length field
 * with the value b_e followed by the low b_e bits of the element, least
 * significant bit first and straddling 64-bit bitstrings exactly as in
 * Method 1; k is the bit-length of the largest b_e (for the worked example,
 * largest value 1023 -> b = 10 -> k = 4).  nbits = sum over elements of
 * (k + b_e) (Eq. 16's bits used); the canonical payload is floor(nbits/64) + 1
 * little-endian bitstrings with every bit past nbits zero (the same count
 * rule as Method 1).
 *
 * Index (this library's; the paper gives none, and the stream alone can only
 * be read from its start): a device buffer of ccm_vlb_index_bytes(rows, cols)
 * bytes holding row_bit[rows + 1] (uint64 at offset 0: stream bit where row i
 * starts; row_bit[rows] = nbits) and, from the next 256-byte boundary,
 * grp_off[rows][ceil(cols/32)] (uint32: bit offset of element (i, 32g) from
 * row i's start).  It costs 32 bits per 32 elements plus 64 bits per row and
 * is what lets the GPU decode groups of 32 elements in parallel and get one
 * element by reading at most 32 pairs.  A row may hold at most 2^32 - 1 bits:
 * cols * (k + max b_e) < 2^32, else CCM_E_UNSUPPORTED. */
typedef struct ccm_vlb_desc {
  int64_t rows, cols;
  int64_t vmin, vmax;  /* exact extremes of the values */
  int32_t k;           /* length-field width, 1..7 */
  int32_t is_signed;   /* 1 iff vmin < 0 */
  uint64_t nbits;      /* sum of k + b_e over the elements */
  uint64_t words;      /* floor(nbits / 64) + 1 */
  uint64_t gmax;       /* bits of the longest group of 32 elements of a row (sizes the
                          matvec's staging) */
  void *payload;       /* device, caller-owned, >= ccm_vlb_payload_capacity(nbits) bytes */
  void *index;         /* device, caller-owned, ccm_vlb_index_bytes(rows, cols) bytes */
} ccm_vlb_desc;

/* Sizes of the caller-allocated buffers (host only; 0 for an invalid shape).
 * The payload capacity adds guard words that kernels may read past the last
 * field, rounded up to 256 bytes. */
uint64_t ccm_vlb_index_bytes(int64_t rows, int64_t cols);
uint64_t ccm_vlb_payload_capacity(uint64_t nbits);

/* Plan: range pass over dense (device, rows x cols of dtype), then the index:
 * per-group bit counts and their scans, written into `index` (device, caller
 * allocated).  Fills every field of out (payload NULL, index = index) and
 * reads nbits back.  Blocking. */
int ccm_vlb_compress_plan(const void *dense, int32_t dtype, int64_t rows, int64_t cols,
                          void *index, ccm_vlb_desc *out, void *stream);

/* Packs dense into out->payload (set by the caller), zeroing its whole
 * capacity first.  `out` must come from ccm_vlb_compress_plan over the same
 * values.  Async. */
int ccm_vlb_compress(const void *dense, int32_t dtype, const ccm_vlb_desc *out, void *stream);

/* Every element into dense_out (device, rows*cols int64).  Async. */
int ccm_vlb_decompress(const ccm_vlb_desc *a, int64_t *dense_out, void *stream);

/* Element (i, j) into *value (host); CCM_E_RANGE outside the matrix.
 * Blocking. */
int ccm_vlb_get(const ccm_vlb_desc *a, int64_t i, int64_t j, int64_t *value, void *stream);

/* y = A x modulo 2^64, as ccm_matvec.  x: device, cols values of xdtype;
 * y: device, rows int64.  Async. */
int ccm_vlb_matvec(const ccm_vlb_desc *a, const void *x, int32_t xdtype, int64_t *y,
                   void *stream);

/* ---- floats in fixed point (Conclusion) ---------------------------------
 *
 * The Conclusion says floats fit the framework if some precision is given
 * up; it gives no encoding.  This library's reading: a float matrix V is stored
 * as the integer matrix q = round-half-to-even(v * 2^f), one f ("fraction
 * bits", possibly negative) per matrix, which Method 1 packs like any
 * integer matrix (ccm_compress on q).  The rounding is the only loss,
 * |v - q 2^-f| <= 2^-(f+1); every operation after it is the exact integer
 * operation on q.  An integer result r with scale 2^-g converts back as
 * ccm_dequantize(r, g): r to double (round half to even), times 2^-g (exact
 * unless subnormal, then rounded once), and for float32 rounded once more.
 * So y = V x takes q (scale 2^-f) and a quantized x (scale 2^-g) through
 * ccm_matvec and dequantizes y at f + g; y is exact modulo 2^64, so the
 * caller keeps cols * max|q| * max|x_q| below 2^63.
 * The fraction bits usually come from the significant bits p the largest
 * magnitude should keep (the Conclusion's point: data with fewer
 * significant digits compress better): f = p - 1 - e with
 * 2^e <= max|v| < 2^(e+1), so the width of q is p to p + 2 bits.
 * Float dtypes: CCM_F32 (float) and CCM_F64 (double). */

/* Largest |v| of n device floats (dtype CCM_F32 or CCM_F64), exact.
 * CCM_E_RANGE if any value is NaN or infinite.  Blocking. */
int ccm_float_absmax(const void *v, int32_t dtype, int64_t n, double *absmax, void *stream);

/* Host only: f = sig_bits - 1 - e with 2^e <= absmax < 2^(e+1); 0 for
 * absmax 0.  CCM_E_INVAL unless 1 <= sig_bits <= 62 and absmax is finite
 * and >= 0. */
int ccm_float_frac_bits(double absmax, int32_t sig_bits, int32_t *frac_bits);

/* q[i] = round-half-to-even(v[i] * 2^frac_bits) for n device floats into
 * device q of qdtype (CCM_I64, or CCM_I32 for a vector the int32 matvec
 * path takes), and the exact (min, max) of q, which is all a compression
 * plan needs (ccm_width, ccm_words; then ccm_compress_fx on v, or
 * ccm_compress on q).  q may be NULL (qdtype ignored): the range and the
 * checks only.  CCM_E_RANGE if any value is NaN or infinite, else
 * CCM_E_OVERFLOW if some |v 2^f| >= 2^62 or, for CCM_I32, some q leaves
 * int32; q is then unspecified.  |frac_bits| <= 1200.  Blocking. */
int ccm_quantize(const void *v, int32_t dtype, int64_t n, int32_t frac_bits, void *q,
                 int32_t qdtype, int64_t *qmin, int64_t *qmax, void *stream);

/* Pack q = round-half-to-even(v * 2^frac_bits) of rows*cols device floats
 * straight into out->payload at out->bits (Method 1's packing, no int64
 * copy of q).  `out` must describe exactly these quantized values: its
 * range from ccm_quantize with the same frac_bits (which also rejected
 * NaN, infinities and overflow).  Async. */
int ccm_compress_fx(const void *v, int32_t dtype, int32_t frac_bits, const ccm_desc *out,
                    void *stream);

/* out[i] = q[i] * 2^-frac_bits converted as described above, into device
 * floats of dtype CCM_F32 or CCM_F64.  |frac_bits| <= 2400.  Async. */
int ccm_dequantize(const int64_t *q, int64_t n, int32_t frac_bits, int32_t dtype, void *out,
                   void *stream);

/* Header of a fixed-point matrix (row-major): the integer header of q with
 * flags bit 2 set and frac_bits as a little-endian int16 at bytes 48..49.
 * decode_fx reads such a header (CCM_E_INVAL if flags bit 2 is clear or the
 * other reserved bytes are not zero) into the descriptor of q and f. */
int ccm_header_encode_fx(const ccm_desc *d, int32_t frac_bits, uint8_t out[64]);
int ccm_header_decode_fx(const uint8_t in[64], ccm_desc *d, int32_t *frac_bits);

#ifdef __cplusplus
}
#endif

#endif
