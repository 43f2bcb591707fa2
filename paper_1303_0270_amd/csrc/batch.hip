// Batched matvec: y_t = A_t x_t for many SM-packed matrices of uneven shapes
// and widths in one persistent kernel launch (optionally a captured HIP graph).
//
// Host planner (ccm_batch_create): every matrix is cut into items of at most
// `tile_rows` rows; items are sorted by width, then by size (largest first),
// so that a block keeps running one width's code and the big items start
// early.  Per-width tile_rows and rows-in-flight come from a tuning table
// (JSON written by the autotuner, or built-in defaults).
//
// Kernel: persistent blocks pull items from an atomic counter.  For an item,
// the block stages the matrix's x into LDS (zero-padded to whole groups,
// int16-range check as in the single-matrix kernel), then each wave works on
// rows.  A row of g groups is handled by L = next_pow2(g) lanes (at most 64),
// so narrow matrices put several rows on one wave; each lane decodes one
// group per row with the width's compile-time decoder (funnel-shifted by the
// row's own bit offset) and the row sum is a segmented shuffle reduction over
// its L lanes.  Widths above 32 use a runtime-width decoder.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "ccm.h"
#include "ccm_internal.hpp"
#include "matvec_impl.hpp"

namespace ccm {
namespace bt {

constexpr int kThreads = 256;
constexpr int kMaxCols = 8192;  // widest matrix a batch accepts (x is staged whole in LDS)
constexpr int kPitch = kGroup + 4;

struct Mat {
  const uint32_t *w;
  const void *x;
  int64_t *y;
  int64_t rows, cols;
  int32_t bits, sgn;
};

struct Item {
  int32_t mat;
  int32_t row0;
  int32_t nrows;
  int32_t rif;  // rows in flight per lane (1 or 2)
};

// Sum over aligned segments of L lanes (L a power of two); lane j%L == 0
// holds the segment's total.
__device__ __forceinline__ int64_t seg_sum(int64_t v, int L) {
  uint64_t u = (uint64_t)v;
  for (int m = 1; m < L; m <<= 1) u += (uint64_t)__shfl_xor((int64_t)u, m, 64);
  return (int64_t)u;
}

// Dot product of one group held in w[0..B] (B + 1 words from the group's
// first word), funnel-shifted by the row's bit offset s (0 leaves the words).
template <int B, bool SGN, bool FAST>
__device__ __forceinline__ uint64_t group_words_dot(uint32_t *w, int s, const int32_t *xg) {
#pragma unroll
  for (int k = 0; k < B; ++k) w[k] = __builtin_amdgcn_alignbit(w[k + 1], w[k], s);
  if constexpr (FAST && B <= 16)
    return mv::group_dot_small<B, SGN>(w, xg);
  else
    return mv::group_dot_wide<B, SGN, int32_t>(w, xg);
}

// Rows [row0, row0+nrows) of matrix m; x staged in xs.  FAST: every x of the
// matrix is in int16 range (exact int32 runs, see the single-matrix kernel).
// Each lane has RIF rows in flight: the words of all of them are requested
// before any is decoded, with rows past the item clamped to its last row
// (decoded and dropped), so the loads are unconditional and the compiler
// waits for them together instead of one row at a time.
template <int B, bool SGN, int RIF, bool FAST>
__device__ __forceinline__ void item_rows(const Mat &m, int row0, int nrows, const int32_t *xs) {
  const int ng = (int)((m.cols + kGroup - 1) / kGroup);
  int L = 1;
  while (L < ng && L < 64) L <<= 1;
  const int sub_per_wave = 64 / L;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sub = lane / L, j0 = lane % L;
  const int rows_per_pass = (kThreads / 64) * sub_per_wave * RIF;
  for (int base = 0; base < nrows; base += rows_per_pass) {
    uint64_t acc[RIF];
    int rr[RIF];
#pragma unroll
    for (int q = 0; q < RIF; ++q) {
      acc[q] = 0;
      rr[q] = base + ((wave * RIF + q) * sub_per_wave + sub);
    }
    for (int j = j0; j < ng; j += L) {
      uint32_t w[RIF][B + 1];
      int sh[RIF];
#pragma unroll
      for (int q = 0; q < RIF; ++q) {
        const int64_t r = row0 + (rr[q] < nrows ? rr[q] : nrows - 1);
        const uint64_t bit = ((uint64_t)r * (uint64_t)m.cols + (uint64_t)j * kGroup) * B;
        const uint32_t *gp = m.w + (bit >> 5);
        sh[q] = (int)(bit & 31u);
#pragma unroll
        for (int k = 0; k <= B; ++k) w[q][k] = gp[k];
      }
#pragma unroll
      for (int q = 0; q < RIF; ++q) {
        const uint64_t d = group_words_dot<B, SGN, FAST>(w[q], sh[q], xs + j * kPitch);
        acc[q] += rr[q] < nrows ? d : 0u;
      }
    }
#pragma unroll
    for (int q = 0; q < RIF; ++q) {
      const int64_t tot = seg_sum((int64_t)acc[q], L);
      if (j0 == 0 && rr[q] < nrows) m.y[row0 + rr[q]] = tot;
    }
  }
}

// Runtime-width rows (fields wider than 32 bits): one element per lane step.
__device__ void item_rows_rt(const Mat &m, int row0, int nrows, const int32_t *xs) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int rr = wave; rr < nrows; rr += kThreads / 64) {
    const int64_t r = row0 + rr;
    uint64_t acc = 0;
    for (int64_t c = lane; c < m.cols; c += 64) {
      const int64_t a = value_at(m.w, (uint64_t)(r * m.cols + c), m.bits, m.sgn);
      acc += (uint64_t)a * (uint64_t)(int64_t)xs[(c >> 5) * kPitch + (c & 31)];
    }
    const int64_t tot = wave_sum((int64_t)acc);
    if (lane == 0) m.y[r] = tot;
  }
}

// Rows in flight per lane: up to 4 for widths to 8, 2 to 16, 1 above (the
// words of every row in flight are held in registers, and one kernel holds
// every width's code, so the widest case sets the register count).
template <int B>
constexpr int max_rif() {
  return B <= 8 ? 4 : B <= 16 ? 2 : 1;
}

template <int B, bool SGN, bool FAST>
__device__ __forceinline__ void item_width(const Mat &m, const Item &it, const int32_t *xs) {
  if constexpr (max_rif<B>() >= 4) {
    if (it.rif >= 4) {
      item_rows<B, SGN, 4, FAST>(m, it.row0, it.nrows, xs);
      return;
    }
  }
  if constexpr (max_rif<B>() >= 2) {
    if (it.rif >= 2) {
      item_rows<B, SGN, 2, FAST>(m, it.row0, it.nrows, xs);
      return;
    }
  }
  item_rows<B, SGN, 1, FAST>(m, it.row0, it.nrows, xs);
}

template <bool SGN, bool FAST>
__device__ __forceinline__ void dispatch(const Mat &m, const Item &it, const int32_t *xs) {
  switch (m.bits) {
#define CCM_B(b) \
  case b:        \
    item_width<b, SGN, FAST>(m, it, xs); \
    return;
    CCM_B(1) CCM_B(2) CCM_B(3) CCM_B(4) CCM_B(5) CCM_B(6) CCM_B(7) CCM_B(8) CCM_B(9)
    CCM_B(10) CCM_B(11) CCM_B(12) CCM_B(13) CCM_B(14) CCM_B(15) CCM_B(16) CCM_B(17)
    CCM_B(18) CCM_B(19) CCM_B(20) CCM_B(21) CCM_B(22) CCM_B(23) CCM_B(24) CCM_B(25)
    CCM_B(26) CCM_B(27) CCM_B(28) CCM_B(29) CCM_B(30) CCM_B(31) CCM_B(32)
#undef CCM_B
    default:
      item_rows_rt(m, it.row0, it.nrows, xs);
      return;
  }
}

__global__ void k_counter_reset(int *counter) { *counter = 0; }

// Every block loops until the shared counter passes the item count; the exit
// test is block-uniform (item index broadcast through LDS).  A block stops
// at its first index past the end, so every block exits.
__global__ __launch_bounds__(kThreads) void k_batch(const Mat *__restrict__ mats,
                                                    const Item *__restrict__ items, int nitems,
                                                    int *counter) {
  __shared__ __align__(16) int32_t xs[(kMaxCols / kGroup) * kPitch];
  __shared__ int s_item;
  // The next item's index is requested when an item starts and read when it
  // ends, so the atomic's round trip overlaps the item's work.
  int next = 0;
  if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
  for (;;) {
    __syncthreads();
    const int it = s_item;
    if (it >= nitems) break;
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    const Item item = items[it];
    const Mat m = mats[item.mat];
    const int ng = (int)((m.cols + kGroup - 1) / kGroup);
    const int32_t *x = (const int32_t *)m.x;
    int small = 1;
    // stage x with eight independent loads in flight per lane
    for (int q0 = threadIdx.x; q0 < ng * kGroup; q0 += kThreads * 8) {
      int32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * kThreads;
        v[u] = q < m.cols ? x[q] : 0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * kThreads;
        if (q < ng * kGroup) {
          xs[(q >> 5) * kPitch + (q & 31)] = v[u];
          small &= (v[u] >= -32768 && v[u] <= 32767);
        }
      }
    }
    const bool fast = __syncthreads_and(small);
    if (fast) {
      if (m.sgn)
        dispatch<true, true>(m, item, xs);
      else
        dispatch<false, true>(m, item, xs);
    } else {
      if (m.sgn)
        dispatch<true, false>(m, item, xs);
      else
        dispatch<false, false>(m, item, xs);
    }
    __syncthreads();  // xs and s_item are rewritten by the next item
    if (threadIdx.x == 0) s_item = next;
  }
}

}  // namespace bt
}  // namespace ccm

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

using ccm::bt::Item;
using ccm::bt::Mat;

struct ccm_batch {
  int n = 0;
  int32_t xdtype = CCM_I32;
  std::vector<Mat> mats;  // host copy (x, y filled by set_io)
  std::vector<Item> items;
  uint64_t packed_bytes = 0;
  int32_t max_bits = 0;
  Mat *d_mats = nullptr;
  Item *d_items = nullptr;
  int *d_counter = nullptr;
  int grid = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool io_set = false;
};

namespace {

struct TuneEntry {
  int tile_rows = 256;
  int rif = 1;
};

// Defaults: small widths need more rows per item to amortize staging x.
TuneEntry default_tune(int bits) {
  TuneEntry t;
  t.tile_rows = bits <= 4 ? 512 : bits <= 12 ? 256 : 128;
  t.rif = bits <= 8 ? 4 : bits <= 16 ? 2 : 1;
  return t;
}

// Reads {"widths": {"<b>": {"tile_rows": r, "rows_in_flight": f}, ...}}; any
// parse problem leaves the defaults in place.
void load_tune(const char *path, TuneEntry table[65]) {
  for (int b = 1; b <= 64; ++b) table[b] = default_tune(b);
  if (!path) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  for (int b = 1; b <= 64; ++b) {
    const std::string key = "\"" + std::to_string(b) + "\"";
    size_t p = s.find(key);
    if (p == std::string::npos) continue;
    const size_t end = s.find('}', p);
    auto field = [&](const char *name, int *out) {
      const size_t q = s.find(name, p);
      if (q == std::string::npos || q > end) return;
      const size_t c = s.find(':', q);
      if (c == std::string::npos || c > end) return;
      const int v = std::atoi(s.c_str() + c + 1);
      if (v > 0) *out = v;
    };
    field("\"tile_rows\"", &table[b].tile_rows);
    field("\"rows_in_flight\"", &table[b].rif);
    if (table[b].rif != 2 && table[b].rif != 4) table[b].rif = 1;
    if (table[b].tile_rows < 1) table[b].tile_rows = 1;
  }
}

int hip_status(hipError_t e) {
  if (e == hipSuccess) return CCM_OK;
  if (std::getenv("CCM_LOG")) std::fprintf(stderr, "ccm batch: %s\n", hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? CCM_E_NOMEM : CCM_E_DEVICE;
}

int check_batch_descs(const ccm_desc *as, int32_t n) {
  for (int t = 0; t < n; ++t) {
    const ccm_desc &d = as[t];
    int32_t b = 0, s = 0;
    if (!d.payload || d.rows < 1 || d.cols < 1 || ccm_width(d.vmin, d.vmax, &b, &s) != CCM_OK ||
        b != d.bits || s != d.is_signed || d.words != ccm_words(d.rows, d.cols, d.bits))
      return CCM_E_INVAL;
    if (d.cols > ccm::bt::kMaxCols || d.rows > 0x7fffffff) return CCM_E_UNSUPPORTED;
  }
  return CCM_OK;
}

// Work list: items of at most tile_rows rows, ordered by width then size.
void plan_items(const std::vector<Mat> &mats, const TuneEntry *table, std::vector<Item> *items) {
  items->clear();
  for (size_t t = 0; t < mats.size(); ++t) {
    const Mat &d = mats[t];
    const TuneEntry te = table[d.bits];
    for (int64_t r = 0; r < d.rows; r += te.tile_rows) {
      const int nr = (int)std::min<int64_t>(te.tile_rows, d.rows - r);
      items->push_back(Item{(int32_t)t, (int32_t)r, nr, te.rif});
    }
  }
  std::stable_sort(items->begin(), items->end(), [&](const Item &x, const Item &y) {
    const Mat &a = mats[x.mat], &c = mats[y.mat];
    if (a.bits != c.bits) return a.bits < c.bits;
    const uint64_t sa = (uint64_t)x.nrows * a.cols, sc = (uint64_t)y.nrows * c.cols;
    return sa > sc;
  });
}

int resident_grid() {
  int occ = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, ccm::bt::k_batch, ccm::bt::kThreads, 0) !=
          hipSuccess ||
      occ < 1)
    occ = 1;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  return occ * cus;
}

}  // namespace

// Reusable device workspace for batches whose matrices change on every launch
// (the serving loop): a ring of slots, each with pinned host staging, device
// tables and a completion event that guards its reuse.
struct ccm_batch_ws {
  struct Slot {
    Mat *h_mats = nullptr, *d_mats = nullptr;
    Item *h_items = nullptr, *d_items = nullptr;
    int *d_counter = nullptr;
    hipEvent_t done = nullptr;
    bool used = false;
  };
  int max_mats = 0;
  int64_t max_items = 0;
  int grid = 0;
  int next = 0;
  TuneEntry table[65];
  std::vector<Slot> slots;
  std::vector<Mat> mats;
  std::vector<Item> items;
};

namespace {
void free_ws(ccm_batch_ws *w) {
  for (auto &s : w->slots) {
    if (s.h_mats) (void)hipHostFree(s.h_mats);
    if (s.h_items) (void)hipHostFree(s.h_items);
    if (s.d_mats) (void)hipFree(s.d_mats);
    if (s.d_items) (void)hipFree(s.d_items);
    if (s.d_counter) (void)hipFree(s.d_counter);
    if (s.done) (void)hipEventDestroy(s.done);
  }
  delete w;
}
}  // namespace

extern "C" {

int ccm_batch_create(const ccm_desc *as, int32_t n, int32_t xdtype, const char *tune_json,
                     ccm_batch **out) {
  if (!as || n < 1 || !out) return CCM_E_INVAL;
  if (xdtype != CCM_I32) return CCM_E_UNSUPPORTED;
  int rc = check_batch_descs(as, n);
  if (rc != CCM_OK) return rc;
  TuneEntry table[65];
  load_tune(tune_json, table);
  ccm_batch *b = new ccm_batch();
  b->n = n;
  b->xdtype = xdtype;
  b->mats.resize(n);
  for (int t = 0; t < n; ++t) {
    const ccm_desc &d = as[t];
    b->mats[t] = Mat{(const uint32_t *)d.payload, nullptr, nullptr, d.rows, d.cols, d.bits,
                     d.is_signed};
    b->packed_bytes += 8u * d.words;
    b->max_bits = std::max(b->max_bits, d.bits);
  }
  plan_items(b->mats, table, &b->items);
  rc = hip_status(hipMalloc(&b->d_mats, sizeof(Mat) * n));
  if (rc == CCM_OK) rc = hip_status(hipMalloc(&b->d_items, sizeof(Item) * b->items.size()));
  if (rc == CCM_OK) rc = hip_status(hipMalloc(&b->d_counter, 256));
  if (rc == CCM_OK)
    rc = hip_status(hipMemcpy(b->d_items, b->items.data(), sizeof(Item) * b->items.size(),
                              hipMemcpyHostToDevice));
  if (rc == CCM_OK) rc = hip_status(hipMemcpy(b->d_mats, b->mats.data(), sizeof(Mat) * n,
                                              hipMemcpyHostToDevice));
  if (rc == CCM_OK) b->grid = resident_grid();
  if (rc == CCM_OK) rc = hip_status(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  if (rc != CCM_OK) {
    ccm_batch_destroy(b);
    return rc;
  }
  *out = b;
  return CCM_OK;
}

int ccm_batch_set_io(ccm_batch *b, const void *const *xs, int64_t *const *ys, void *stream) {
  if (!b || !xs || !ys) return CCM_E_INVAL;
  for (int t = 0; t < b->n; ++t) {
    if (!xs[t] || !ys[t]) return CCM_E_INVAL;
    b->mats[t].x = xs[t];
    b->mats[t].y = ys[t];
  }
  // from pageable memory: the runtime stages the bytes before returning, and
  // the copy is ordered before later work on `stream`
  int rc = hip_status(hipMemcpyAsync(b->d_mats, b->mats.data(), sizeof(Mat) * b->n,
                                     hipMemcpyHostToDevice, (hipStream_t)stream));
  if (rc == CCM_OK) b->io_set = true;
  return rc;
}

static int batch_enqueue(ccm_batch *b, hipStream_t s) {
  ccm::bt::k_counter_reset<<<1, 1, 0, s>>>(b->d_counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e);
  ccm::bt::k_batch<<<b->grid, ccm::bt::kThreads, 0, s>>>(b->d_mats, b->d_items,
                                                        (int)b->items.size(), b->d_counter);
  return hip_status(hipGetLastError());
}

int ccm_batch_matvec(ccm_batch *b, int32_t use_graph, void *stream) {
  if (!b) return CCM_E_INVAL;
  if (!b->io_set) return CCM_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  if (!use_graph) return batch_enqueue(b, s);
  if (!b->exec) {
    int rc = hip_status(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    if (rc != CCM_OK) return rc;
    rc = batch_enqueue(b, b->cap_stream);
    hipGraph_t g = nullptr;
    const int rc2 = hip_status(hipStreamEndCapture(b->cap_stream, &g));
    if (rc != CCM_OK || rc2 != CCM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc != CCM_OK ? rc : rc2;
    }
    b->graph = g;
    rc = hip_status(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    if (rc != CCM_OK) return rc;
  }
  return hip_status(hipGraphLaunch(b->exec, s));
}

int ccm_batch_info(const ccm_batch *b, int64_t *items, uint64_t *packed_bytes,
                   int32_t *max_bits) {
  if (!b) return CCM_E_INVAL;
  if (items) *items = (int64_t)b->items.size();
  if (packed_bytes) *packed_bytes = b->packed_bytes;
  if (max_bits) *max_bits = b->max_bits;
  return CCM_OK;
}

int ccm_batch_ws_create(int32_t max_mats, int64_t max_items, int32_t slots, const char *tune_json,
                        ccm_batch_ws **out) {
  if (max_mats < 1 || max_items < 1 || slots < 1 || slots > 64 || !out) return CCM_E_INVAL;
  ccm_batch_ws *w = new ccm_batch_ws();
  w->max_mats = max_mats;
  w->max_items = max_items;
  load_tune(tune_json, w->table);
  w->slots.resize(slots);
  int rc = CCM_OK;
  for (auto &sl : w->slots) {
    if (rc == CCM_OK) rc = hip_status(hipHostMalloc((void **)&sl.h_mats, sizeof(Mat) * max_mats,
                                                    hipHostMallocDefault));
    if (rc == CCM_OK) rc = hip_status(hipHostMalloc((void **)&sl.h_items,
                                                    sizeof(Item) * max_items,
                                                    hipHostMallocDefault));
    if (rc == CCM_OK) rc = hip_status(hipMalloc((void **)&sl.d_mats, sizeof(Mat) * max_mats));
    if (rc == CCM_OK) rc = hip_status(hipMalloc((void **)&sl.d_items, sizeof(Item) * max_items));
    if (rc == CCM_OK) rc = hip_status(hipMalloc((void **)&sl.d_counter, 256));
    if (rc == CCM_OK) rc = hip_status(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
  }
  if (rc == CCM_OK) w->grid = resident_grid();
  if (rc != CCM_OK) {
    free_ws(w);
    return rc;
  }
  *out = w;
  return CCM_OK;
}

int ccm_batch_ws_destroy(ccm_batch_ws *w) {
  if (!w) return CCM_E_INVAL;
  for (auto &sl : w->slots)
    if (sl.used) (void)hipEventSynchronize(sl.done);
  free_ws(w);
  return CCM_OK;
}

int ccm_batch_matvec_dyn(ccm_batch_ws *w, const ccm_desc *as, const void *const *xs,
                         int64_t *const *ys, int32_t n, void *stream) {
  if (!w || !as || !xs || !ys || n < 1) return CCM_E_INVAL;
  if (n > w->max_mats) return CCM_E_NOMEM;
  int rc = check_batch_descs(as, n);
  if (rc != CCM_OK) return rc;
  w->mats.resize(n);
  for (int t = 0; t < n; ++t) {
    if (!xs[t] || !ys[t]) return CCM_E_INVAL;
    const ccm_desc &d = as[t];
    w->mats[t] = Mat{(const uint32_t *)d.payload, xs[t], ys[t], d.rows, d.cols, d.bits,
                     d.is_signed};
  }
  plan_items(w->mats, w->table, &w->items);
  if ((int64_t)w->items.size() > w->max_items) return CCM_E_NOMEM;
  ccm_batch_ws::Slot &sl = w->slots[w->next];
  w->next = (w->next + 1) % (int)w->slots.size();
  if (sl.used) {
    rc = hip_status(hipEventSynchronize(sl.done));  // its previous upload has been consumed
    if (rc != CCM_OK) return rc;
  }
  std::memcpy(sl.h_mats, w->mats.data(), sizeof(Mat) * n);
  std::memcpy(sl.h_items, w->items.data(), sizeof(Item) * w->items.size());
  hipStream_t s = (hipStream_t)stream;
  rc = hip_status(hipMemcpyAsync(sl.d_mats, sl.h_mats, sizeof(Mat) * n, hipMemcpyHostToDevice, s));
  if (rc == CCM_OK)
    rc = hip_status(hipMemcpyAsync(sl.d_items, sl.h_items, sizeof(Item) * w->items.size(),
                                   hipMemcpyHostToDevice, s));
  if (rc != CCM_OK) return rc;
  ccm::bt::k_counter_reset<<<1, 1, 0, s>>>(sl.d_counter);
  rc = hip_status(hipGetLastError());
  if (rc != CCM_OK) return rc;
  ccm::bt::k_batch<<<w->grid, ccm::bt::kThreads, 0, s>>>(sl.d_mats, sl.d_items,
                                                        (int)w->items.size(), sl.d_counter);
  rc = hip_status(hipGetLastError());
  if (rc != CCM_OK) return rc;
  rc = hip_status(hipEventRecord(sl.done, s));
  sl.used = (rc == CCM_OK);
  return rc;
}

int ccm_batch_destroy(ccm_batch *b) {
  if (!b) return CCM_E_INVAL;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->d_mats) (void)hipFree(b->d_mats);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_counter) (void)hipFree(b->d_counter);
  delete b;
  return CCM_OK;
}

}  // extern "C"
