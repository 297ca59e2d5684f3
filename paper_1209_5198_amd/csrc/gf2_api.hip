// gf2_api.hip -- C ABI of libgf2 (include/gf2.h): validation, workspace and the
// host-side sequence of kernels for each call.
//
// Decomposition driver (Section 4, non-recursive block loop): the columns are
// processed in trailing-update panels of s sub-panels of 64 columns.  For each
// sub-panel the panel kernel selects the pivots (buildZ, Sections 4.2-4.4) and
// the rows kernel stores the multipliers and updates the rest of the panel;
// then the panel's row exchanges are applied to every other column (P^(j)),
// the pivot rows are brought to echelon form right of the panel (k_trsm), and
// the Schur complement A^(j+1) = E xor Y*C (eq. (Aj)) is formed by the
// Four-Russians product (Section 6).  Every size that depends on the data (the
// rank so far, the number of pivots of a sub-panel) stays on the device: the
// host enqueues a fixed sequence of launches and only the caller reads results.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <limits.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "gf2_internal.h"

namespace gf2 {
namespace {

thread_local std::string g_err;
// set for the duration of an allocation-free call: no profiling events
thread_local bool g_noalloc = false;
int g_panel_words = 0;  // 0: automatic (the tuned width of the size class, else 8)
// Strassen-Winograd recursion while every dimension of the current product is
// at least this many bits (0: never).  Measured on MI355X: one level pays at
// 65536^3 (56 ms against 62 ms), none at 32768^3 (10.3 ms against 8 ms).
int64_t g_strassen_cutoff = 65536;
int g_gemm_variant = -1;        // product-kernel variant for gf2_matmul (-1: automatic)
int g_panel_gemm_variant = -1;  // product-kernel variant for the trailing update (-1: automatic)
// Panels per super-panel (0: the one-level schedule): the words outside a
// super-panel and the next one are updated once per super-panel, by products
// of inner dimension up to 64 * panel_words * sp_panels bits (at most
// kSpSubMax sub-panels).  Measured on MI355X at 65536^2: 56.7 ms one-level
// against 65.3 (2), 66.4 (1) and 69.1 ms (4) with super-panels.
int g_sp_panels = 0;
// one-level schedule: product tiles by the wall-time rule instead of the
// largest tile that still gives every CU a workgroup
// Trailing-update tiles by the wall-time rule (rounds x fitted step time)
// instead of the largest tile that fills the CUs: 0 never, 1 always (the
// default), 2 for launches of at most 16384 active rows whose wall-rule tile
// fits the CUs in one round.  Since a trailing update's workgroups without rows
// come last in its grid, "always" is the fastest: 65536^2 43.7-43.9 against
// 44.3-44.4 ms for 2, 32768^2 11.54-11.57 against 11.87-12.16 ms, the planted
// rank-20000 32768 x 65536 matrix 18.00-18.06 against 18.08-18.13 ms, 16384^2
// and 2048^2 unchanged.  (With those workgroups first, 2 was the best: always
// cost 32768^2 12.6 against 12.4 ms.)
int g_wall_tiles = 1;
// near-update size (table lookups) from which a panel's update of the near
// words beyond the next panel starts right after the row exchanges, beside
// the next panel's columns and its pivot chain, instead of after them
double g_overlap_lookups = 3e8;
// (one-level schedule) bulk-update size (table lookups) from which the next
// panel's k_post runs on the bulk stream right after that update (then waiting
// for the next chain), instead of on the main stream after a hop from the bulk
// stream: where the bulk update is the longer path this takes two stream hops
// per panel off it (-1 = never; measured on MI355X at 65536^2: 57.1-57.4 ms at
// 1.5e9 against 58.2 ms never, 59.5 ms always, 58.2 ms at 5e9)
double g_post_follow_lookups = 1.5e9;
// Product-kernel tile per size class, written by gf2_autotune: rows class r
// (active rows in [256 << r, 512 << r), clamped to 0..8) x column-block class c
// (1, 2-3, 4-15, 16+ blocks of 16 words); -1 = the built-in rule.
constexpr int kTuneRows = 9, kTuneBlocks = 4;
int g_tuned[kTuneRows][kTuneBlocks];
// Panel width (sub-panels of 64 columns) per decomposition size class
// (max(n, m) <= 4096, <= 16384, larger), written by gf2_autotune.
constexpr int kWClasses = 3;
constexpr int64_t kWClassMax[kWClasses] = {4096, 16384, INT64_MAX};
constexpr int64_t kWClassProbe[kWClasses] = {2048, 16384, 32768};  // the size each class is timed at
int g_tuned_W[kWClasses] = {0, 0, 0};
int w_class(int64_t n, int64_t m) {
  const int64_t s = n > m ? n : m;
  int c = 0;
  while (c + 1 < kWClasses && s > kWClassMax[c]) ++c;
  return c;
}
bool g_tuned_valid = false;  // a table was measured
bool g_tuned_on = false;     // ... and is used

// Panel width of an n x m decomposition: the knob when set, else the tuned
// width of its size class while the tuned table is in use, else 8.
int panel_words_for(int64_t n, int64_t m) {
  if (g_panel_words > 0) return g_panel_words;
  const int t = g_tuned_W[w_class(n, m)];
  return (g_tuned_on && t > 0) ? t : kMaxPanelWords;
}
int tune_row_class(int64_t rows) {
  int r = 0;
  while (r + 1 < kTuneRows && rows >= ((int64_t)512 << r)) ++r;
  return r;
}
int tune_block_class(int blocks) { return blocks <= 1 ? 0 : (blocks <= 3 ? 1 : (blocks <= 15 ? 2 : 3)); }

// Per (device, caller stream): the two internal streams of the look-ahead
// pipeline of a decomposition (main: row exchanges, next panel's columns and
// pivot chains; bulk: each panel's update of the other near words and the
// super-panels' far work); events order them.  Calls made on
// different caller streams get different sets, so their factorizations can
// run concurrently.  All streams have the default priority and no CU mask.
// gf2_release() destroys them.
struct Pipe {
  hipStream_t gemm = nullptr, chain = nullptr;
  std::vector<hipEvent_t> ring;      // links that involve the caller's stream
  std::vector<hipEvent_t> ring_dev;  // links between the pipe's own two streams
  size_t next = 0, next_dev = 0;
};
std::map<std::pair<int, hipStream_t>, Pipe> g_pipes;

struct Workspace {
  void *ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

struct ProfState {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  std::vector<hipEvent_t> pool;  // events created once and reused by later profiling sessions
  size_t used = 0;               // events of the pool taken in this session
  unsigned long long *work_dev = nullptr;
  int64_t launches = 0;
} g_prof;


// Descriptors of a batch travel through one pinned host buffer; a copy is
// complete (event) before the buffer is refilled by the next batched call.
struct Staging {
  void *host = nullptr;
  size_t bytes = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};
Staging g_stage;
std::mutex g_stage_mu;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return GF2_EHIP;
}

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #x);  \
  } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int check_mat(const gf2_mat *M, const char *name) {
  if (!M) return fail(GF2_EINVAL, std::string(name) + ": null descriptor");
  if (M->rows < 0 || M->cols < 0) return fail(GF2_EINVAL, std::string(name) + ": negative shape");
  if (M->w < 1) return fail(GF2_EINVAL, std::string(name) + ": w must be >= 1");
  if (M->ld < M->rows) return fail(GF2_EINVAL, std::string(name) + ": ld < rows");
  if (M->rows > 0 && M->cols > 0 && !M->data) return fail(GF2_EINVAL, std::string(name) + ": null data");
  if (M->rows >= (1ll << 31)) return fail(GF2_EINVAL, std::string(name) + ": rows must be < 2^31");
  return GF2_OK;
}

// Workspace of (device, stream), grown on demand.  Growing synchronises the
// device before the old buffer is released.
int get_workspace(hipStream_t s, size_t bytes, void **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace &w = g_ws[std::make_pair(dev, s)];
  if (w.bytes < bytes) {
    if (w.ptr) {
      HIPCHK(hipDeviceSynchronize());
      HIPCHK(hipFree(w.ptr));
      w.ptr = nullptr;
      w.bytes = 0;
    }
    size_t want = align256(bytes + bytes / 8);
    if (hipMalloc(&w.ptr, want) != hipSuccess) {
      (void)hipGetLastError();
      w.ptr = nullptr;
      if (hipMalloc(&w.ptr, align256(bytes)) != hipSuccess) {
        (void)hipGetLastError();
        w.ptr = nullptr;
        return fail(GF2_ENOMEM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
      }
      want = align256(bytes);
    }
    w.bytes = want;
  }
  *out = w.ptr;
  return GF2_OK;
}

struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base((char *)b) {}
  template <typename T>
  T *take(size_t count) {
    T *p = (T *)(base + off);
    off += align256(count * sizeof(T));
    return p;
  }
};

size_t decomp_bytes(int64_t n, int64_t m, int64_t ldw, int64_t Mw, int64_t NB) {
  size_t b = 0;
  b += align256((size_t)NB * ldw * TW * 8);
  b += align256(sizeof(DecState));
  b += align256((size_t)Mw * sizeof(SubInfo));
  b += 2 * align256((size_t)Mw * 64 * 8);
  b += align256((size_t)n * 8);
  b += align256((size_t)Mw * 64 * 8);
  b += 2 * align256((size_t)n * 4);
  b += align256((size_t)kMaxPanelWords * 64 * 2 * 4);
  b += align256((size_t)(Mw + 1) * 4);
  b += align256((size_t)n * 4);
  b += align256((size_t)kPanelTabWords * 8);
  b += 2 * align256((size_t)2 * n * 4);
  b += align256((size_t)2 * kSpListMax * 4);
  b += align256((size_t)2 * 4);
  (void)m;
  return b;
}

void carve_decomp(Carver &c, DecWork &w) {
  w.W = c.take<uint64_t>((size_t)w.NB * w.ldw * TW);
  w.st = c.take<DecState>(1);
  w.sub = c.take<SubInfo>(w.Mw);
  w.Zc = c.take<uint64_t>((size_t)w.Mw * 64);
  w.Linv = c.take<uint64_t>((size_t)w.Mw * 64);
  w.perm = c.take<int64_t>(w.n);
  w.pivcols = c.take<int64_t>((size_t)w.Mw * 64);
  w.bp_src = c.take<int32_t>(w.n);
  w.bp_mark = c.take<int32_t>(w.n);
  w.bp_list = c.take<int32_t>((size_t)kMaxPanelWords * 64 * 2);
  w.nzflag = c.take<uint32_t>((size_t)w.Mw + 1);
  w.lvl = c.take<int32_t>(w.n);
  w.ptab = c.take<uint64_t>(kPanelTabWords);
  w.sp_src = c.take<int32_t>((size_t)2 * w.n);
  w.sp_mark = c.take<int32_t>((size_t)2 * w.n);
  w.sp_list = c.take<int32_t>((size_t)2 * kSpListMax);
  w.sp_count = c.take<int32_t>(2);
}

// the next event of the profiling pool (created the first time it is needed)
int prof_event(hipEvent_t *e) {
  if (g_prof.used == g_prof.pool.size()) {
    hipEvent_t n = nullptr;
    HIPCHK(hipEventCreate(&n));
    g_prof.pool.push_back(n);
  }
  *e = g_prof.pool[g_prof.used++];
  return GF2_OK;
}

bool prof_on() { return g_prof.on && !g_noalloc; }

int profile_begin(hipStream_t s, hipEvent_t *a) {
  if (!prof_on()) return GF2_OK;
  int rc = prof_event(a);
  if (rc) return rc;
  HIPCHK(hipEventRecord(*a, s));
  return GF2_OK;
}

int profile_end(hipStream_t s, hipEvent_t a) {
  if (!prof_on()) return GF2_OK;
  hipEvent_t b;
  int rc = prof_event(&b);
  if (rc) return rc;
  HIPCHK(hipEventRecord(b, s));
  g_prof.ev.emplace_back(a, b);
  g_prof.launches += 1;
  return GF2_OK;
}

int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
    cached[dev] = prop.multiProcessorCount;
  }
  return cached[dev];
}

// active_rows: rows expected to do work (used only to pick a tile size)
int run_gemm(GemmArgs &a, int64_t nrows_max, int variant, int64_t active_rows, hipStream_t s) {
  if (variant < 0 && g_tuned_on && !(a.qc0 % 8 == 0 && a.qc1 - a.qc0 <= 8)) {
    const int blocks = ((a.qc1 - 1) >> 4) - (a.qc0 >> 4) + 1;
    variant = g_tuned[tune_row_class(active_rows)][tune_block_class(blocks)];
  }
  if (variant < 0 || variant >= kGemmVariants) variant = gemm_auto_variant(active_rows, a.qc0, a.qc1, gf2::device_cus());
  // A narrow accumulating product that runs alone (kparts = -1 on entry) and
  // whose workgroups leave CUs idle is split over its inner words (up to 8
  // parts, the launch still one round): each workgroup's chain of dependent
  // table steps is what it waits for.
  const bool may_split = a.kparts < 0;
  a.kparts = 1;
  if (may_split && (variant == 4 || variant == 5) && a.accumulate) {
    const int tm = gemm_tile_rows(variant);
    const int64_t wgs = ((active_rows + tm - 1) / tm) * (((a.qc1 - 1) >> 3) - (a.qc0 >> 3) + 1);
    while (a.kparts < 8 && 2 * a.kparts <= a.kwords && wgs * 2 * a.kparts <= gf2::device_cus()) a.kparts *= 2;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool prof = prof_on();
  if (prof) {  // the launch records the kernel's own start and end
    int rc = prof_event(&e0);
    if (!rc) rc = prof_event(&e1);
    if (rc) return rc;
  }
  a.work = prof ? g_prof.work_dev : nullptr;
  HIPCHK(launch_gemm(a, nrows_max, variant, s, e0, e1));
  if (prof) {
    g_prof.ev.emplace_back(e0, e1);
    g_prof.launches += 1;
  }
  return GF2_OK;
}

// The fp4 matrix-core product for a plain B of bwords words per row; ws is
// mfma_ws_bytes(a.kwords, bwords, rows) bytes of workspace.
int run_gemm_mfma(GemmArgs &a, int64_t bwords, uint64_t *ws, hipStream_t s) {
  hipEvent_t e0 = nullptr;
  int rc = profile_begin(s, &e0);
  if (rc) return rc;
  a.work = prof_on() ? g_prof.work_dev : nullptr;
  HIPCHK(launch_gemm_mfma(a, bwords, ws, gf2::device_cus(), s));
  return profile_end(s, e0);
}

int get_pipe(hipStream_t user, Pipe **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  Pipe &p = g_pipes[std::make_pair(dev, user)];
  if (!p.gemm) {
    HIPCHK(hipStreamCreateWithFlags(&p.gemm, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&p.chain, hipStreamNonBlocking));
    p.ring.assign(64, nullptr);
    for (auto &e : p.ring) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // Both ends of these links are kernels of this device, so the events skip
    // the system-scope fence (the caller's stream, which may hand results to
    // the host or another device, is linked through the ring above).
    p.ring_dev.assign(64, nullptr);
    for (auto &e : p.ring_dev)
      HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventDisableSystemFence));
  }
  *out = &p;
  return GF2_OK;
}

// Where a call's launches go: the caller's stream and the two look-ahead
// streams of its pipe, or (P == nullptr) everything in order on the caller's
// stream, which needs no stream or event of the library's own.
struct Exec {
  hipStream_t user = nullptr, G = nullptr, Cs = nullptr;
  Pipe *P = nullptr;
};

int make_exec(hipStream_t user, bool single, Exec &x) {
  x.user = user;
  if (single) {
    x.G = x.Cs = user;
    x.P = nullptr;
    return GF2_OK;
  }
  int rc = get_pipe(user, &x.P);
  if (rc) return rc;
  x.G = x.P->gemm;
  x.Cs = x.P->chain;
  return GF2_OK;
}

// At most two panels: the event links of the look-ahead streams cost more than
// the overlap they buy (one stream: 0.283 against 0.336 ms at 1024^2, equal at
// 2048^2, slower from 4096^2 on), so such factorizations run on the caller's
// stream alone.  S as in the panel loop.
bool few_panels(const DecWork &w, const gf2_mat *A) {
  const int S = panel_words_for(w.n, A->cols);
  return (w.Mw + S - 1) / S <= 2;
}

// an event marking everything enqueued so far on s (null on a single stream);
// device_only: its waiter is the pipe's other stream
int mark(const Exec &x, hipStream_t s, hipEvent_t *e, bool device_only = false) {
  *e = nullptr;
  if (!x.P) return GF2_OK;
  *e = device_only ? x.P->ring_dev[x.P->next_dev++ % x.P->ring_dev.size()]
                   : x.P->ring[x.P->next++ % x.P->ring.size()];
  HIPCHK(hipEventRecord(*e, s));
  return GF2_OK;
}

int wait_mark(hipStream_t waiter, hipEvent_t e) {
  if (e) HIPCHK(hipStreamWaitEvent(waiter, e, 0));
  return GF2_OK;
}

// make `waiter` wait for everything enqueued so far on `signaller` (nothing to
// do when both are the same stream)
int link(const Exec &x, hipStream_t signaller, hipStream_t waiter) {
  if (signaller == waiter) return GF2_OK;
  hipEvent_t e = nullptr;
  const bool device_only = signaller != x.user && waiter != x.user;
  int rc = mark(x, signaller, &e, device_only);
  return rc ? rc : wait_mark(waiter, e);
}

// C words [qc0, qc1) of every row below the pivots of sub-panels [q0, q0 + nsub)
// ^= (their multipliers in words [q0, q0 + nsub)) * (the pivot rows' words):
// eq. (Aj) for those sub-panels.  nz: flag slot ORed with "a written word is
// nonzero"; skip: flag slot whose zero means the Schur complement is zero
// (-1: none).
// split_ok: nothing runs beside this launch (the inner dimension of a narrow
// product may then be split over idle CUs)
int trailing_gemm(DecWork &w, int q0, int nsub, int nz, int skip, int qc0, int qc1, hipStream_t s,
                  bool split_ok = false) {
  if (qc1 <= qc0) return GF2_OK;
  GemmArgs a;
  memset(&a, 0, sizeof(a));
  a.A = w.W; a.ldA = w.ldw; a.a_word0 = q0;
  a.B = w.W; a.ldB = w.ldw; a.b_rows = 0; a.bsub = w.sub + q0;
  a.C = w.W; a.ldC = w.ldw;
  a.row_tile0 = 0; a.row_end = w.n;
  a.kwords = nsub;
  a.qc0 = qc0; a.qc1 = qc1;
  a.accumulate = 1;
  a.nzflag = w.nzflag + nz;
  a.skip_flag = skip >= 0 ? w.nzflag + skip : nullptr;
  a.kparts = split_ok ? -1 : 1;
  // at most 64 pivots per sub-panel so far: a lower bound on the rows left
  int64_t active = w.n - 64ll * (q0 + nsub);
  if (active < 1) active = 1;
  int v = g_panel_gemm_variant;
  if (v < 0 && !g_tuned_on) {
    const int ncu = gf2::device_cus();
    if (g_sp_panels > 0 || g_wall_tiles == 1) {
      v = gemm_wall_variant(active, qc0, qc1, ncu);
    } else if (g_wall_tiles == 2 && active <= 16384 && !gemm_narrow_ok(qc0, qc1)) {
      const int vw = gemm_wall_variant(active, qc0, qc1, ncu), tm = gemm_tile_rows(vw);
      const int64_t wgs = ((active + tm - 1) / tm) * (int64_t)(((qc1 - 1) >> 4) - (qc0 >> 4) + 1);
      if (wgs <= ncu) v = vw;
    }
  }
  return run_gemm(a, w.n, v, active, s);
}

int chain(DecWork &w, int q0, int s_eff, int flag, int spb, hipStream_t s) {
  HIPCHK(launch_panel(w, q0, s_eff, flag, spb, s));
  return GF2_OK;
}

// Factor A into the working state w (which the caller sized with decomp_bytes).
//
// Columns go in super-panels of sp_panels panels (SPW words); the near words
// of super-panel k are its own and those of super-panel k+1.  Per panel J:
//   G:  post(J)     row exchanges and pivot rows in echelon form on the near
//                   words, the rows' multipliers in the panel words
//       narrow      the next panel's columns get panel J's update
//       chain(J+1)  pivots of the next panel (look-ahead)
//   Cs: near bulk   the other near words right of the next panel get panel
//                   J's update, then a slice of the previous super-panel's
//                   far work; post(J+1) waits for Cs
// so the bulk work overlaps only the pivot chain (one workgroup), never the
// row exchanges or the next panel's columns.  Closing super-panel k (Cs, after
// its last near bulk): its net permutation on all other words (they kept the
// super-panel's starting row order), its pivot rows in echelon form on the
// far words and the update of super-panel k+2's words, which become near for
// super-panel k+1, with inner dimension 64 * SPW; the update of the remaining
// far words follows in slices during super-panel k+1's panels.
// Zero test: flag slot k is ORed by the products that write the final state
// of super-panel k's Schur complement (its last panel's near products and
// its far products), so slot k == 0 means that everything after is zero; a
// launch only reads a slot whose writers are certainly finished.  Returns
// with `user` ordered after all the work.
// What the working matrix holds: A; [A | I] (w sized for A->cols + A->rows
// columns, A square: the augmented form the inverse is read from); or A^T (w
// sized for A->cols x A->rows: the rank of a wide matrix, equal to that of its
// transpose, with fewer panels).
enum class Pack { kPlain, kIdentityRight, kTransposed };

// far words [q0, q1) of super-panel k (sub-panels [s0, s0 + nsub)) still to
// be brought up to date, in `left` slices
struct FarWork {
  int k = -1, s0 = 0, nsub = 0, q0 = 0, q1 = 0, left = 0;
};

int far_slice(DecWork &w, FarWork &f, hipStream_t s) {
  if (f.left <= 0 || f.q1 <= f.q0) {
    f.left = 0;
    return GF2_OK;
  }
  // whole 16-word blocks where possible
  int take = (f.q1 - f.q0 + f.left - 1) / f.left;
  take = (take + TW - 1) / TW * TW;
  const int qe = f.q0 + take < f.q1 ? f.q0 + take : f.q1;
  int rc = trailing_gemm(w, f.s0, f.nsub, f.k, f.k >= 1 ? f.k - 1 : -1, f.q0, qe, s);
  f.q0 = qe;
  --f.left;
  return rc;
}

// One-level schedule (sp_panels = 0): every panel's update of all words right
// of the next panel is one product of inner dimension 64 * panel_words.
// Main stream G: post(J), next panel's columns, chain(J+1), in order (no
// stream hop before the chain).  Bulk stream Cs: the rest of panel J's
// update, started after post(J) when it clearly outlasts the chain (it then
// runs beside the next panel's columns and the chain), else after the next
// panel's columns.  post(J+1) waits for it: on G, or, after a bulk update of
// at least g_post_follow_lookups, on Cs right behind it (then waiting for
// chain(J+1) instead), with G continuing after post(J+1).  On a single
// stream the same launches run in this order, one after the other.  The
// zero-tail test of a panel's chain reads the flag of the panel two steps
// back, the last one whose trailing update is certainly complete.
int factor_panels(const gf2_mat *A, DecWork &w, const Exec &x, Pack pack) {
  int rc;
  const hipStream_t G = x.G, Cs = x.Cs;
  if ((rc = link(x, x.user, G))) return rc;
  HIPCHK(launch_init_state(w, G));
  if (pack == Pack::kTransposed) {
    HIPCHK(launch_pack_transposed(*A, w.W, w.ldw, w.NB, G));
  } else {
    HIPCHK(launch_pack(*A, w.W, w.ldw, w.n, A->cols, w.NB, G));
    if (pack == Pack::kIdentityRight) HIPCHK(launch_set_identity(w.W, w.ldw, w.n, A->cols, G));
  }
  const int S = panel_words_for(w.n, A->cols);
  int prev = -1;
  // Main stream G: post(J), next panel's columns, chain(J+1), in order (no
  // stream hop before the chain).  Bulk stream Cs: the rest of panel J's
  // update, started after post(J) when it clearly outlasts the chain (it then
  // runs beside the next panel's columns and the chain), else after the next
  // panel's columns.  post(J+1) waits for it: on G, or, after a bulk update of
  // at least g_post_follow_lookups, on Cs right behind it (then waiting for
  // chain(J+1) instead), with G continuing after post(J+1).  On a single
  // stream the same launches run in this order, one after the other.
  if ((rc = chain(w, 0, w.Mw < S ? w.Mw : S, -1, -1, G))) return rc;
  bool post_on_cs = false;  // k_post of this panel follows the previous bulk update on Cs
  for (int q0 = 0; q0 < w.Mw; q0 += S) {
    const int s_eff = (w.Mw - q0) < S ? (w.Mw - q0) : S;
    if (post_on_cs) {
      // Cs already follows the previous bulk update; wait for this chain
      if ((rc = link(x, G, Cs))) return rc;
      HIPCHK(launch_post(w, q0, s_eff, 0, w.Mw, gf2::device_cus(), Cs));
      if ((rc = link(x, Cs, G))) return rc;
    } else {
      HIPCHK(launch_post(w, q0, s_eff, 0, w.Mw, gf2::device_cus(), G));  // row exchanges, multipliers, pivot rows in echelon form
    }
    const int nq0 = q0 + s_eff;
    bool next_on_cs = false;
    if (nq0 < w.Mw) {
      const int ns = (w.Mw - nq0) < S ? (w.Mw - nq0) : S;
      // lookups of the bulk update (rows left >= n - 64 * sub-panels done)
      const int64_t rows_left = w.n - 64ll * nq0;
      const double bulk = (double)(rows_left > 0 ? rows_left : 0) * (double)(w.Mw - nq0 - ns) * 8.0 * s_eff;
      const bool early = bulk >= g_overlap_lookups;
      if (early && !post_on_cs && (rc = link(x, G, Cs))) return rc;
      // next panel's columns (alone on the chip unless the bulk update started early)
      if ((rc = trailing_gemm(w, q0, s_eff, q0, prev, nq0, nq0 + ns, G, !early))) return rc;
      if (!early && (rc = link(x, G, Cs))) return rc;
      if ((rc = chain(w, nq0, ns, prev, -1, G))) return rc;                           // look-ahead
      if ((rc = trailing_gemm(w, q0, s_eff, q0, prev, nq0 + ns, w.Mw, Cs))) return rc; // the rest
      next_on_cs = g_post_follow_lookups >= 0.0 && bulk >= g_post_follow_lookups;
      if (!next_on_cs && (rc = link(x, Cs, G))) return rc;
    }
    post_on_cs = next_on_cs;
    prev = q0;
  }
  return link(x, G, x.user);
}

int factor(const gf2_mat *A, DecWork &w, const Exec &x, Pack pack = Pack::kPlain) {
  if (g_sp_panels <= 0) return factor_panels(A, w, x, pack);
  int rc;
  const hipStream_t G = x.G, Cs = x.Cs;
  if ((rc = link(x, x.user, G))) return rc;
  HIPCHK(launch_init_state(w, G));
  if (pack == Pack::kTransposed) {
    HIPCHK(launch_pack_transposed(*A, w.W, w.ldw, w.NB, G));
  } else {
    HIPCHK(launch_pack(*A, w.W, w.ldw, w.n, A->cols, w.NB, G));
    if (pack == Pack::kIdentityRight) HIPCHK(launch_set_identity(w.W, w.ldw, w.n, A->cols, G));
  }
  const int S = panel_words_for(w.n, A->cols);
  int P = g_sp_panels;
  if (P * S > kSpSubMax) P = kSpSubMax / S;
  const int SPW = P * S;
  const int Mw = w.Mw, dummy = Mw;  // flag slot that nothing reads
  // flag slot a launch of super-panel k may read: the products of k-2 (k-3
  // for the first chain of k, which is launched before k's first post)
  auto zslot = [](int k, int back) { return k - back >= 0 ? k - back : -1; };
  FarWork far;
  if ((rc = chain(w, 0, Mw < S ? Mw : S, -1, 0, G))) return rc;
  int k = 0;
  for (int sp0 = 0; sp0 < Mw; sp0 += SPW, ++k) {
    const int sp1 = sp0 + SPW < Mw ? sp0 + SPW : Mw;
    const int n1 = sp1 + SPW < Mw ? sp1 + SPW : Mw;
    for (int q0 = sp0; q0 < sp1; q0 += S) {
      const int s_eff = sp1 - q0 < S ? sp1 - q0 : S;
      const bool last = q0 + s_eff == sp1;
      if ((rc = link(x, Cs, G))) return rc;  // the previous bulk work
      HIPCHK(launch_post(w, q0, s_eff, sp0, n1, gf2::device_cus(), G));
      const int nq0 = q0 + s_eff;
      if (nq0 < Mw) {
        const int ns = Mw - nq0 < S ? Mw - nq0 : S;
        const int nz = last ? k : dummy, skip = zslot(k, 2);
        const int nk = last ? k + 1 : k;  // super-panel of the next panel
        const double near =
            (double)(w.n - 64ll * nq0 > 0 ? w.n - 64ll * nq0 : 0) * (double)(n1 - nq0 - ns) * 8.0 * s_eff;
        const bool early = near >= g_overlap_lookups;
        if (early && (rc = link(x, G, Cs))) return rc;
        if ((rc = trailing_gemm(w, q0, s_eff, nz, skip, nq0, nq0 + ns, G))) return rc;  // next panel's columns
        if (!early && (rc = link(x, G, Cs))) return rc;
        if ((rc = chain(w, nq0, ns, zslot(nk, last ? 3 : 2), nk & 1, G))) return rc;
        if ((rc = trailing_gemm(w, q0, s_eff, nz, skip, nq0 + ns, n1, Cs))) return rc;  // the other near words
      } else if ((rc = link(x, G, Cs))) {
        return rc;
      }
      // a slice of the previous super-panel's far words (the last panel takes what is left)
      if (last)
        while (far.left > 0)
          if ((rc = far_slice(w, far, Cs))) return rc;
      if ((rc = far_slice(w, far, Cs))) return rc;
    }
    // ---- close super-panel k (Cs, after its last near bulk and the previous
    // super-panel's far work)
    HIPCHK(launch_sp_swap(w, k & 1, sp0, n1, Cs));
    HIPCHK(launch_sp_reset(w, k & 1, Cs));
    if (n1 < Mw) {
      const int nsub = sp1 - sp0, n2 = n1 + SPW < Mw ? n1 + SPW : Mw;
      HIPCHK(launch_trsm_far(w, sp0, nsub, n1, Mw, Cs));  // all far words: one word per workgroup
      if ((rc = trailing_gemm(w, sp0, nsub, k, zslot(k, 1), n1, n2, Cs))) return rc;
      far.k = k;
      far.s0 = sp0;
      far.nsub = nsub;
      far.q0 = n2;
      far.q1 = Mw;
      far.left = n2 < Mw ? P : 0;
    }
  }
  while (far.left > 0)
    if ((rc = far_slice(w, far, Cs))) return rc;
  if ((rc = link(x, Cs, G))) return rc;
  return link(x, G, x.user);
}

// Working state of an n x m factorization carved from `ws` (at least
// decomp_bytes(n, m) + extra bytes); *extra_ptr receives the extra bytes.
void layout_decomp(int64_t n, int64_t m, DecWork &w) {
  memset(&w, 0, sizeof(w));
  w.n = n;
  w.m = m;
  w.Mw = (int32_t)ceil_div(m, 64);
  w.NB = (int32_t)ceil_div(w.Mw, TW);
  w.ldw = ceil_div(n > 0 ? n : 1, 256) * 256;
}

size_t decomp_bytes(int64_t n, int64_t m) {
  DecWork w;
  layout_decomp(n, m, w);
  return decomp_bytes(n, m, w.ldw, w.Mw, w.NB);
}

void prepare_decomp(int64_t n, int64_t m, void *ws, DecWork &w, size_t extra, void **extra_ptr) {
  layout_decomp(n, m, w);
  Carver c(ws);
  carve_decomp(c, w);
  if (extra_ptr) *extra_ptr = c.take<char>(extra);
}

// A caller workspace must be 256-byte aligned and at least `need` bytes.
int check_ws(const void *ws, size_t ws_bytes, size_t need, const char *who) {
  if (need == 0) return GF2_OK;
  if (!ws) return fail(GF2_EINVAL, std::string(who) + ": null workspace");
  if (((uintptr_t)ws & 255u) != 0) return fail(GF2_EINVAL, std::string(who) + ": workspace must be 256-byte aligned");
  if (ws_bytes < need)
    return fail(GF2_EINVAL, std::string(who) + ": workspace of " + std::to_string(ws_bytes) + " bytes, " +
                                std::to_string(need) + " needed");
  return GF2_OK;
}

// Reduced row echelon form of A in the working layout: the decomposition's E
// (extracted into ldE-row blocks), then R = U^-1 E bottom-up in blocks of 512
// pivot rows (diagonal-block back-substitution, then one 512-bit-inner product
// per block for every row above it).
struct RrefWork {
  uint64_t *E = nullptr;   // kmin x m, working layout, ldE rows per block: E, then R
  int64_t ldE = 0;
  uint64_t *G = nullptr;   // kmin x kmin: E restricted to the pivot columns
  uint64_t *Bb = nullptr;  // 512 x m: one block of R as a product operand
  int64_t *piv = nullptr, *rank = nullptr, *tw0 = nullptr, *freecols = nullptr;
  uint64_t *bitmap = nullptr;
  int64_t Mw = 0, NBE = 0, Gw = 0;
};

// augment: reduce [A | I] instead of A (A square), for the inverse
int rref_run(const gf2_mat *A, hipStream_t s, RrefWork &rw, bool augment = false) {
  gf2_mat shape = *A;
  if (augment) shape.cols = A->cols + A->rows;
  const int64_t n = shape.rows, m = shape.cols, kmin = n < m ? n : m;
  rw.Mw = ceil_div(m, 64);
  rw.ldE = ceil_div(kmin, 256) * 256;
  rw.NBE = ceil_div(rw.Mw, TW);
  rw.Gw = ceil_div(kmin, 64);
  const int64_t NBG = ceil_div(rw.Gw, TW);
  const size_t bE = align256((size_t)rw.NBE * rw.ldE * TW * 8), bG = align256((size_t)NBG * rw.ldE * TW * 8),
               bB = align256((size_t)rw.NBE * 512 * TW * 8), bI = align256((size_t)(kmin + 2) * 8),
               bM = align256((size_t)(rw.Mw + 1) * 8), bF = align256((size_t)(m + 1) * 8);
  const size_t extra_bytes = bE + bG + bB + bI + 2 * bM + bF + 256;
  void *ws = nullptr;
  int rc = get_workspace(s, decomp_bytes(n, m) + align256(extra_bytes), &ws);
  if (rc) return rc;
  DecWork w;
  void *extra = nullptr;
  prepare_decomp(n, m, ws, w, extra_bytes, &extra);
  Exec x;
  if ((rc = make_exec(s, few_panels(w, A), x))) return rc;
  char *p = (char *)extra;
  rw.E = (uint64_t *)p; p += bE;
  rw.G = (uint64_t *)p; p += bG;
  rw.Bb = (uint64_t *)p; p += bB;
  rw.piv = (int64_t *)p; p += bI;
  rw.bitmap = (uint64_t *)p; p += bM;
  rw.tw0 = (int64_t *)p; p += bM;
  rw.freecols = (int64_t *)p; p += bF;
  rw.rank = (int64_t *)p;
  if ((rc = factor(A, w, x, augment ? Pack::kIdentityRight : Pack::kPlain))) return rc;
  HIPCHK(launch_finish(w, nullptr, rw.piv, rw.rank, s));
  const gf2_mat Em{rw.E, kmin, m, TW, rw.ldE};
  HIPCHK(launch_extract_E(w, Em, s));
  HIPCHK(launch_gather_pivcols(rw.E, rw.ldE, rw.piv, rw.rank, rw.G, kmin, rw.Gw, s));
  const int nJ = (int)ceil_div(kmin, 512);
  for (int J = nJ - 1; J >= 0; --J) {
    HIPCHK(launch_rref_diag(rw.E, rw.ldE, rw.G, rw.rank, J, rw.Mw, s));
    if (J == 0) break;
    HIPCHK(launch_copy_block_rows(rw.E, rw.ldE, rw.rank, 512ll * J, rw.Bb, rw.NBE, s));
    GemmArgs a;
    memset(&a, 0, sizeof(a));
    a.A = rw.G; a.ldA = rw.ldE; a.a_word0 = 8 * J;
    a.B = rw.Bb; a.ldB = 512; a.b_rows = 512; a.bsub = nullptr;
    a.C = rw.E; a.ldC = rw.ldE;
    a.row_tile0 = 0; a.row_end = 512ll * J;
    a.kwords = (int32_t)std::min<int64_t>(8, rw.Gw - 8ll * J);
    // rows of block J are zero left of their pivots, which lie at or beyond
    // column 512 J: only words from 8 J change
    a.qc0 = 8 * J; a.qc1 = (int32_t)rw.Mw;
    a.accumulate = 1;
    if ((rc = run_gemm(a, 512ll * J, -1, 512ll * J, s))) return rc;
  }
  return GF2_OK;
}

}  // namespace
}  // namespace gf2

using namespace gf2;

extern "C" {

const char *gf2_version(void) { return "libgf2 0.1 (gfx950)"; }

const char *gf2_last_error(void) { return g_err.c_str(); }

int gf2_set_param(const char *name, int64_t value) {
  if (!name) return fail(GF2_EINVAL, "null parameter name");
  if (!strcmp(name, "panel_words")) {
    if (value < 0 || value > kMaxPanelWords) return fail(GF2_EINVAL, "panel_words must be in 0..8");
    g_panel_words = (int)value;
    return GF2_OK;
  }
  if (!strcmp(name, "gemm_variant")) {
    if (value < -1 || value > kGemmMfma) return fail(GF2_EINVAL, "gemm_variant out of range");
    g_gemm_variant = (int)value;
    return GF2_OK;
  }
  if (!strcmp(name, "panel_gemm_variant")) {
    if (value < -1 || value >= kGemmVariants) return fail(GF2_EINVAL, "panel_gemm_variant out of range");
    g_panel_gemm_variant = (int)value;
    return GF2_OK;
  }
  if (!strcmp(name, "autotuned")) {
    if (value < 0 || value > 1) return fail(GF2_EINVAL, "autotuned must be 0 or 1");
    g_tuned_on = value == 1 && g_tuned_valid;
    return GF2_OK;
  }
  if (!strcmp(name, "sp_panels")) {
    if (value < 0 || value > kSpSubMax) return fail(GF2_EINVAL, "sp_panels must be in 0..32");
    g_sp_panels = (int)value;
    return GF2_OK;
  }
  if (!strcmp(name, "wall_tiles")) {
    if (value < 0 || value > 2) return fail(GF2_EINVAL, "wall_tiles must be 0, 1 or 2");
    g_wall_tiles = (int)value;
    return GF2_OK;
  }
  if (!strcmp(name, "wide_threads")) {
    if (value != 512 && value != 1024) return fail(GF2_EINVAL, "wide_threads must be 512 or 1024");
    g_wide_threads = (int)value;
    return GF2_OK;
  }
  if (!strcmp(name, "post_follow_lookups")) {
    if (value < -1) return fail(GF2_EINVAL, "post_follow_lookups must be >= -1");
    g_post_follow_lookups = (double)value;
    return GF2_OK;
  }
  if (!strcmp(name, "overlap_lookups")) {
    if (value < 0) return fail(GF2_EINVAL, "overlap_lookups must be >= 0");
    g_overlap_lookups = (double)value;
    return GF2_OK;
  }
  if (!strcmp(name, "chain_cus")) {
    // CU-masked chain streams were removed: a masked product launch left the
    // reserved CUs idle and unbalanced their XCD (measured slower)
    if (value != 0) return fail(GF2_EINVAL, "chain_cus: CU-masked streams are not supported (only 0)");
    return GF2_OK;
  }
  if (!strcmp(name, "strassen_cutoff")) {
    if (value < 0) return fail(GF2_EINVAL, "strassen_cutoff must be >= 0");
    g_strassen_cutoff = value;
    return GF2_OK;
  }
  return fail(GF2_EINVAL, std::string("unknown parameter ") + name);
}

int gf2_profile(int enable) {
  // a new session reuses the pool's events once the previous session's are done
  for (auto &p : g_prof.ev) HIPCHK(hipEventSynchronize(p.second));
  g_prof.ev.clear();
  g_prof.used = 0;
  g_prof.launches = 0;
  if (enable && !g_prof.work_dev) {
    HIPCHK(hipMalloc((void **)&g_prof.work_dev, sizeof(unsigned long long)));
  }
  if (g_prof.work_dev) HIPCHK(hipMemset(g_prof.work_dev, 0, sizeof(unsigned long long)));
  g_prof.on = enable != 0;
  return GF2_OK;
}

int gf2_profile_read(double *ms, int64_t *launches, double *lookups) {
  double total = 0.0;
  for (auto &p : g_prof.ev) {
    HIPCHK(hipEventSynchronize(p.second));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, p.first, p.second));
    total += t;
  }
  unsigned long long work = 0;
  if (g_prof.work_dev) HIPCHK(hipMemcpy(&work, g_prof.work_dev, sizeof(work), hipMemcpyDeviceToHost));
  if (ms) *ms = total;
  if (launches) *launches = g_prof.launches;
  if (lookups) *lookups = (double)work;
  return GF2_OK;
}

int gf2_microbench(int kind, int64_t bytes, int iters, double *rate, double *ms, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  if (kind < 0 || kind >= kProbeKinds || !rate || !ms) return fail(GF2_EINVAL, "gf2_microbench: bad kind or null output");
  if (kind <= 1 && (bytes < 65536 || bytes % 65536 != 0))
    return fail(GF2_EINVAL, "gf2_microbench: bytes must be a positive multiple of 65536");
  if (kind >= 2 && (iters < 1 || iters > (1 << 24))) return fail(GF2_EINVAL, "gf2_microbench: iters out of range");
  const int ncu = gf2::device_cus();
  void *buf = nullptr;
  uint32_t *sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = GF2_OK;
  do {
    hipError_t e;
    if ((e = hipMalloc(&sink, 256)) != hipSuccess) { rc = hip_fail(e, "hipMalloc"); break; }
    if (kind <= 1 && (e = hipMalloc(&buf, (size_t)bytes)) != hipSuccess) { rc = hip_fail(e, "hipMalloc"); break; }
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
      rc = hip_fail(e, "hipEventCreate");
      break;
    }
    double work = 0.0;
    constexpr int kReps = 3;
    if ((e = launch_probe(kind, buf, (size_t)bytes, iters, ncu, sink, s, &work)) != hipSuccess) {  // warm-up
      rc = hip_fail(e, "launch_probe");
      break;
    }
    if ((e = hipEventRecord(e0, s)) != hipSuccess) { rc = hip_fail(e, "hipEventRecord"); break; }
    for (int r = 0; r < kReps && e == hipSuccess; ++r) e = launch_probe(kind, buf, (size_t)bytes, iters, ncu, sink, s, &work);
    if (e != hipSuccess) { rc = hip_fail(e, "launch_probe"); break; }
    if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) {
      rc = hip_fail(e, "hipEventSynchronize");
      break;
    }
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) { rc = hip_fail(e, "hipEventElapsedTime"); break; }
    *ms = (double)t / kReps;
    *rate = *ms > 0.0 ? work / (*ms * 1e-3) : 0.0;
  } while (false);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (buf || sink) (void)hipStreamSynchronize(s);
  if (buf) (void)hipFree(buf);
  if (sink) (void)hipFree(sink);
  return rc;
}

int gf2_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  // every device that holds a workspace or a pipe finishes its work first
  std::vector<int> devs;
  for (auto &kv : g_ws) devs.push_back(kv.first.first);
  for (auto &kv : g_pipes) devs.push_back(kv.first.first);
  std::sort(devs.begin(), devs.end());
  devs.erase(std::unique(devs.begin(), devs.end()), devs.end());
  for (int d : devs) {
    HIPCHK(hipSetDevice(d));
    HIPCHK(hipDeviceSynchronize());
  }
  for (auto &kv : g_ws) {
    if (kv.second.ptr) {
      HIPCHK(hipSetDevice(kv.first.first));
      HIPCHK(hipFree(kv.second.ptr));
    }
  }
  g_ws.clear();
  for (auto &kv : g_pipes) {
    HIPCHK(hipSetDevice(kv.first.first));
    for (hipEvent_t e : kv.second.ring)
      if (e) HIPCHK(hipEventDestroy(e));
    for (hipEvent_t e : kv.second.ring_dev)
      if (e) HIPCHK(hipEventDestroy(e));
    if (kv.second.gemm) HIPCHK(hipStreamDestroy(kv.second.gemm));
    if (kv.second.chain) HIPCHK(hipStreamDestroy(kv.second.chain));
  }
  g_pipes.clear();
  HIPCHK(hipSetDevice(cur));
  if (!g_prof.on) {
    for (hipEvent_t e : g_prof.pool) HIPCHK(hipEventDestroy(e));
    g_prof.pool.clear();
    g_prof.ev.clear();
    g_prof.used = 0;
  }
  {
    std::lock_guard<std::mutex> ls(g_stage_mu);
    if (g_stage.ev) {
      HIPCHK(hipEventSynchronize(g_stage.ev));
      HIPCHK(hipEventDestroy(g_stage.ev));
    }
    if (g_stage.host) HIPCHK(hipHostFree(g_stage.host));
    g_stage = Staging();
  }
  return GF2_OK;
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------- batches
int stage_descs(const std::vector<BatchDesc> &v, BatchDesc *dev, hipStream_t s) {
  const size_t bytes = v.size() * sizeof(BatchDesc);
  std::lock_guard<std::mutex> lk(g_stage_mu);
  if (g_stage.pending) {
    HIPCHK(hipEventSynchronize(g_stage.ev));
    g_stage.pending = false;
  }
  if (g_stage.bytes < bytes) {
    if (g_stage.host) HIPCHK(hipHostFree(g_stage.host));
    g_stage.host = nullptr;
    g_stage.bytes = 0;
    HIPCHK(hipHostMalloc(&g_stage.host, bytes));
    g_stage.bytes = bytes;
  }
  if (!g_stage.ev) HIPCHK(hipEventCreateWithFlags(&g_stage.ev, hipEventDisableTiming));
  memcpy(g_stage.host, v.data(), bytes);
  HIPCHK(hipMemcpyAsync(dev, g_stage.host, bytes, hipMemcpyHostToDevice, s));
  HIPCHK(hipEventRecord(g_stage.ev, s));
  g_stage.pending = true;
  return GF2_OK;
}

// Words of one batched worker slot for an n x m item: the working copy with
// rows padded to 64-byte segments.
int64_t batch_slot_words(int64_t n, int64_t m) { return n * ((ceil_div(m, 64) + 7) / 8 * 8); }

// Validate the items and order them by decreasing work (n * m * min(n, m)),
// so that a persistent launch starts the largest matrices first.
int batch_descs(const gf2_batch_item *items, int64_t count, bool solve, std::vector<BatchDesc> &out,
                int64_t *max_words) {
  if (count < 0 || count > (int64_t)INT32_MAX) return fail(GF2_EINVAL, "batch: count out of range");
  if (count > 0 && !items) return fail(GF2_EINVAL, "batch: null items");
  std::vector<std::pair<double, int32_t>> key((size_t)count);
  int64_t mw = 0;
  for (int64_t i = 0; i < count; ++i) {
    const gf2_batch_item &it = items[i];
    if (it.rows < 0 || it.rows > GF2_BATCH_MAX_DIM || it.cols < 0 || it.cols > GF2_BATCH_MAX_DIM)
      return fail(GF2_EINVAL, "batch item " + std::to_string(i) + ": rows and cols must be in [0, " +
                                  std::to_string(GF2_BATCH_MAX_DIM) + "]");
    if (it.a < 0 || it.l < 0 || it.e < 0 || it.p < 0 || it.c < 0 || (solve && (it.b < 0 || it.x < 0)))
      return fail(GF2_EINVAL, "batch item " + std::to_string(i) + ": negative offset");
    const double n = (double)it.rows, m = (double)it.cols;
    key[(size_t)i] = std::make_pair(n * m * (n < m ? n : m) + n + m, (int32_t)i);
    mw = std::max(mw, batch_slot_words(it.rows, it.cols));
  }
  std::stable_sort(key.begin(), key.end(),
                   [](const std::pair<double, int32_t> &x, const std::pair<double, int32_t> &y) {
                     return x.first > y.first;
                   });
  out.resize((size_t)count);
  for (int64_t j = 0; j < count; ++j) {
    const gf2_batch_item &it = items[key[(size_t)j].second];
    BatchDesc &d = out[(size_t)j];
    d.n = (int32_t)it.rows;
    d.m = (int32_t)it.cols;
    d.idx = key[(size_t)j].second;
    d.pad = 0;
    d.a = it.a;
    d.l = it.l;
    d.e = it.e;
    d.p = it.p;
    d.c = it.c;
    d.b = solve ? it.b : 0;
    d.x = solve ? it.x : 0;
  }
  *max_words = mw;
  return GF2_OK;
}

int device_cus(int *ncu) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(ncu, hipDeviceAttributeMultiprocessorCount, dev));
  if (*ncu < 1) *ncu = 1;
  return GF2_OK;
}

// ---------------------------------------------------------------- Strassen-Winograd
// One level on quadrant views (Winograd's form: 7 products, 15 additions;
// over GF(2) every addition and subtraction is an exclusive or):
//   S1 = A21+A22, S2 = S1+A11, S3 = A11+A21, S4 = A12+S2
//   T1 = B12+B11, T2 = B22+T1, T3 = B22+B12, T4 = T2+B21
//   P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4, P5 = S1 T1, P6 = S2 T2, P7 = S3 T3
//   C11 = P1+P2, U2 = P1+P6, U3 = U2+P7, C12 = U2+P5+P3, C21 = U3+P4, C22 = U3+P5
// Products recurse while levels remain; leaves are single Four-Russians launches.
// Temporaries come from a stack (`top`) that a level releases when it returns:
// all launches go to one stream, so later work reuses the memory only after the
// earlier kernels that read it.
struct Stack {
  char *base;
  size_t top, cap;
};

BView quad(const BView &v, int i, int j) {
  BView q;
  q.ld = v.ld;
  q.rows = v.rows / 2;
  q.words = v.words / 2;
  q.p = v.p + ((int64_t)j * (q.words / TW) * v.ld + (int64_t)i * q.rows) * TW;
  return q;
}

BView temp(Stack &st, int64_t rows, int64_t words) {
  BView t;
  t.ld = rows;
  t.rows = rows;
  t.words = words;
  t.p = (uint64_t *)(st.base + st.top);
  st.top += align256((size_t)(words / TW) * rows * TW * 8);
  return t;
}

size_t strassen_bytes(int64_t n, int64_t kw, int64_t mw, int depth) {
  size_t b = 0;
  for (int d = 0; d < depth; ++d) {
    n /= 2;
    kw /= 2;
    mw /= 2;
    const int64_t kr = kw * 64;
    b += 4 * align256((size_t)(kw / TW) * n * TW * 8) + 4 * align256((size_t)(mw / TW) * kr * TW * 8) +
         7 * align256((size_t)(mw / TW) * n * TW * 8);
  }
  return b;
}

int gemm_view(const BView &C, const BView &A, const BView &B, int acc, hipStream_t s) {
  GemmArgs a;
  memset(&a, 0, sizeof(a));
  a.A = A.p; a.ldA = A.ld; a.a_word0 = 0;
  a.B = B.p; a.ldB = B.ld; a.b_rows = B.rows; a.bsub = nullptr;
  a.C = C.p; a.ldC = C.ld;
  a.row_tile0 = 0; a.row_end = C.rows;
  a.kwords = (int32_t)A.words;
  a.qc0 = 0; a.qc1 = (int32_t)C.words;
  a.accumulate = acc;
  return run_gemm(a, C.rows, g_gemm_variant, C.rows, s);
}

int strassen(const BView &C, const BView &A, const BView &B, int depth, int acc, Stack &st, hipStream_t s) {
  if (depth == 0) return gemm_view(C, A, B, acc, s);
  const size_t mark = st.top;
  const BView A11 = quad(A, 0, 0), A12 = quad(A, 0, 1), A21 = quad(A, 1, 0), A22 = quad(A, 1, 1);
  const BView B11 = quad(B, 0, 0), B12 = quad(B, 0, 1), B21 = quad(B, 1, 0), B22 = quad(B, 1, 1);
  const BView C11 = quad(C, 0, 0), C12 = quad(C, 0, 1), C21 = quad(C, 1, 0), C22 = quad(C, 1, 1);
  BView S[4], T[4], P[7];
  for (auto &x : S) x = temp(st, A11.rows, A11.words);
  for (auto &x : T) x = temp(st, B11.rows, B11.words);
  for (auto &x : P) x = temp(st, C11.rows, C11.words);
  HIPCHK(launch_xor_view(S[0], A21, A22, nullptr, 0, s));
  HIPCHK(launch_xor_view(S[1], S[0], A11, nullptr, 0, s));
  HIPCHK(launch_xor_view(S[2], A11, A21, nullptr, 0, s));
  HIPCHK(launch_xor_view(S[3], A12, S[1], nullptr, 0, s));
  HIPCHK(launch_xor_view(T[0], B12, B11, nullptr, 0, s));
  HIPCHK(launch_xor_view(T[1], B22, T[0], nullptr, 0, s));
  HIPCHK(launch_xor_view(T[2], B22, B12, nullptr, 0, s));
  HIPCHK(launch_xor_view(T[3], T[1], B21, nullptr, 0, s));
  int rc;
  if ((rc = strassen(P[0], A11, B11, depth - 1, 0, st, s)) || (rc = strassen(P[1], A12, B21, depth - 1, 0, st, s)) ||
      (rc = strassen(P[2], S[3], B22, depth - 1, 0, st, s)) || (rc = strassen(P[3], A22, T[3], depth - 1, 0, st, s)) ||
      (rc = strassen(P[4], S[0], T[0], depth - 1, 0, st, s)) || (rc = strassen(P[5], S[1], T[1], depth - 1, 0, st, s)) ||
      (rc = strassen(P[6], S[2], T[2], depth - 1, 0, st, s)))
    return rc;
  HIPCHK(launch_xor_view(C11, P[0], P[1], nullptr, acc, s));
  HIPCHK(launch_xor_view(P[5], P[0], P[5], nullptr, 0, s));  // U2
  HIPCHK(launch_xor_view(P[6], P[5], P[6], nullptr, 0, s));  // U3
  HIPCHK(launch_xor_view(C12, P[5], P[4], &P[2], acc, s));
  HIPCHK(launch_xor_view(C21, P[6], P[3], nullptr, acc, s));
  HIPCHK(launch_xor_view(C22, P[6], P[4], nullptr, acc, s));
  st.top = mark;
  return GF2_OK;
}

// ---------------------------------------------------------------- plans and bodies of the calls
// Everything a gf2_matmul call lays out in its workspace.
struct MatmulPlan {
  int depth = 0;
  bool mfma = false;
  int64_t np = 0, kp = 0, mp = 0, Kw = 0, Mw = 0, NBa = 0, NBb = 0, lda = 0, ldb = 0;
  size_t ba = 0, bb = 0, bc = 0, bs = 0, bt = 0;
  size_t total() const { return ba + bb + bc + bs + bt; }
};

MatmulPlan matmul_plan(int64_t n, int64_t k, int64_t m) {
  MatmulPlan p;
  if (n == 0 || m == 0) return p;
  // Strassen-Winograd levels: while every dimension of the (halved) problem is
  // at least the cutoff (Section 6: the recursion pays only for large products)
  if (g_strassen_cutoff > 0)
    while (p.depth < 4 && std::min(n, std::min(k, m)) >> p.depth >= g_strassen_cutoff) ++p.depth;
  // padded shape: rows a multiple of 256 * 2^depth, inner and output columns of
  // 1024 * 2^depth bits (so every quadrant is a whole number of 16-word blocks)
  const int64_t rq = (int64_t)256 << p.depth, cq = (int64_t)1024 << p.depth;
  p.np = ceil_div(n, rq) * rq;
  p.kp = p.depth ? ceil_div(k, cq) * cq : k;
  p.mp = p.depth ? ceil_div(m, cq) * cq : m;
  p.Kw = ceil_div(p.kp, 64);
  p.Mw = ceil_div(p.mp, 64);
  p.NBa = ceil_div(p.Kw > 0 ? p.Kw : 1, TW);
  p.NBb = ceil_div(p.Mw, TW);
  p.lda = p.np;
  p.ldb = ceil_div(p.kp > 0 ? p.kp : 1, 256) * 256;
  p.ba = align256((size_t)p.NBa * p.lda * TW * 8);
  p.bb = align256((size_t)p.NBb * p.ldb * TW * 8);
  p.bc = align256((size_t)p.NBb * p.lda * TW * 8);
  p.bs = p.depth ? strassen_bytes(p.np, p.NBa * TW, p.NBb * TW, p.depth) : 0;
  // the fp4 matrix-core product when forced, or automatically where the table
  // kernels cannot fill the chip with 1024-row tiles and the inner dimension is
  // long enough to amortise its transpose and epilogue (measured crossover)
  p.mfma = p.depth == 0 && k > 0 &&
           (g_gemm_variant == kGemmMfma ||
            (g_gemm_variant < 0 && k >= 1024 && ceil_div(n, 1024) * ceil_div(m, 1024) < gf2::device_cus()));
  p.bt = p.mfma ? align256(mfma_ws_bytes(p.Kw, p.Mw, n)) : 0;
  return p;
}

int matmul_check(const gf2_mat *C, const gf2_mat *A, const gf2_mat *B) {
  int rc;
  if ((rc = check_mat(C, "C")) || (rc = check_mat(A, "A")) || (rc = check_mat(B, "B"))) return rc;
  if (A->cols != B->rows || C->rows != A->rows || C->cols != B->cols)
    return fail(GF2_EINVAL, "gf2_matmul: shapes do not match (C n x m, A n x k, B k x m)");
  return GF2_OK;
}

int matmul_body(const gf2_mat *C, const gf2_mat *A, const gf2_mat *B, int accumulate, const MatmulPlan &p, void *ws,
                hipStream_t s) {
  int rc;
  const int64_t n = A->rows, k = A->cols, m = B->cols;
  if (n == 0 || m == 0) return GF2_OK;
  uint64_t *Aw = (uint64_t *)ws, *Bw = (uint64_t *)((char *)ws + p.ba), *Cw = (uint64_t *)((char *)ws + p.ba + p.bb);
  HIPCHK(launch_pack(*A, Aw, p.lda, n, k, (int32_t)p.NBa, s));
  HIPCHK(launch_pack(*B, Bw, p.ldb, k, m, (int32_t)p.NBb, s));
  if (accumulate) HIPCHK(launch_pack(*C, Cw, p.lda, n, m, (int32_t)p.NBb, s));
  if (p.depth > 0) {
    Stack st{(char *)ws + p.ba + p.bb + p.bc, 0, p.bs};
    const BView Cv{Cw, p.lda, p.np, p.NBb * TW}, Av{Aw, p.lda, p.np, p.NBa * TW}, Bv{Bw, p.ldb, p.NBa * TW * 64, p.NBb * TW};
    if ((rc = strassen(Cv, Av, Bv, p.depth, accumulate ? 1 : 0, st, s))) return rc;
  } else if (k > 0 || accumulate) {
    GemmArgs a;
    memset(&a, 0, sizeof(a));
    a.A = Aw; a.ldA = p.lda; a.a_word0 = 0;
    a.B = Bw; a.ldB = p.ldb; a.b_rows = k; a.bsub = nullptr;
    a.C = Cw; a.ldC = p.lda;
    a.row_tile0 = 0; a.row_end = n;
    a.kwords = (int32_t)p.Kw;
    a.qc0 = 0; a.qc1 = (int32_t)p.Mw;
    a.accumulate = accumulate ? 1 : 0;
    if (p.mfma) {
      if (!accumulate && mfma_splits_inner(a, gf2::device_cus())) {  // split inner dimension: XORs into a zeroed C
        HIPCHK(launch_zero(Cw, p.bc / 8, s));
        a.accumulate = 1;
      }
      if ((rc = run_gemm_mfma(a, p.Mw, (uint64_t *)((char *)ws + p.ba + p.bb + p.bc), s))) return rc;
    } else if ((rc = run_gemm(a, n, g_gemm_variant, n, s))) {
      return rc;
    }
  } else {
    HIPCHK(launch_zero(Cw, p.bc / 8, s));
  }
  HIPCHK(launch_unpack(Cw, p.lda, *C, s));
  return GF2_OK;
}

int decompose_check(const gf2_mat *A, const gf2_mat *L, const gf2_mat *E) {
  int rc;
  if ((rc = check_mat(A, "A"))) return rc;
  const int64_t n = A->rows, m = A->cols, kmin = n < m ? n : m;
  if (L) {
    if ((rc = check_mat(L, "L"))) return rc;
    if (L->rows != n || L->cols != kmin) return fail(GF2_EINVAL, "gf2_decompose: L must be n x min(n,m)");
  }
  if (E) {
    if ((rc = check_mat(E, "E"))) return rc;
    if (E->rows != kmin || E->cols != m) return fail(GF2_EINVAL, "gf2_decompose: E must be min(n,m) x m");
  }
  return GF2_OK;
}

size_t decompose_need(const gf2_mat *A) {
  return (A->rows == 0 || A->cols == 0) ? 0 : decomp_bytes(A->rows, A->cols);
}

// single: every launch in order on the caller's stream (no look-ahead streams)
int decompose_body(const gf2_mat *A, const gf2_mat *L, const gf2_mat *E, int64_t *perm, int64_t *pivcols,
                   int64_t *rank, void *ws, hipStream_t s, bool single) {
  int rc;
  const int64_t n = A->rows, m = A->cols;
  if (n == 0 || m == 0) {  // rank 0, P = I; L and E have no entries (min(n, m) = 0)
    HIPCHK(launch_empty_outputs(perm, n, rank, s));
    return GF2_OK;
  }
  DecWork w;
  prepare_decomp(n, m, ws, w, 0, nullptr);
  Exec x;
  if ((rc = make_exec(s, single || few_panels(w, A), x))) return rc;
  if ((rc = factor(A, w, x))) return rc;
  if (E && L && x.P) {
    // both outputs are HBM-bound copies of disjoint parts of the working
    // matrix: E on the pipe's main stream beside L on the caller's stream
    // (the main stream already follows every launch of the factorization,
    // and the caller's stream holds nothing newer)
    HIPCHK(launch_extract_E(w, *E, x.G));
    HIPCHK(launch_extract_L(w, *L, s));
    if ((rc = link(x, x.G, s))) return rc;
  } else {
    if (E) HIPCHK(launch_extract_E(w, *E, s));
    if (L) HIPCHK(launch_extract_L(w, *L, s));
  }
  HIPCHK(launch_finish(w, perm, pivcols, rank, s));
  return GF2_OK;
}

// ---------------------------------------------------------------- allocation-free decomposition
// The working state of gf2_decompose_noalloc lives in this file-scope device
// array: every GPU the library runs on holds its own copy from the time the
// code object is loaded there until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol): the device address comes from hipGetSymbolAddress, once per device,
// with that device current.
constexpr size_t kScratchBytes = GF2_NOALLOC_MAX_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");
static __device__ __align__(256) uint64_t scratch[kScratchBytes / 8];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

// the current device's copy of `scratch`
int scratch_ptr(void **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GF2_EINVAL, "gf2_decompose_noalloc: device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "gf2_decompose_noalloc: hipGetSymbolAddress(scratch)");
    if (!p || ((uintptr_t)p & 255u) != 0)
      return fail(GF2_EHIP, "gf2_decompose_noalloc: scratch address is null or not 256-byte aligned");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GF2_OK;
}

int rank_check(const gf2_mat *A, const int64_t *rank) {
  int rc;
  if ((rc = check_mat(A, "A"))) return rc;
  if (!rank) return fail(GF2_EINVAL, "gf2_rank: null rank pointer");
  if (A->cols > A->rows && A->cols >= (1ll << 31)) return fail(GF2_EINVAL, "gf2_rank: cols must be < 2^31 when cols > rows");
  return GF2_OK;
}

// rank A = rank A^T: a wide matrix is factored transposed, which needs
// ceil(rows / 512) panels instead of ceil(cols / 512) (the panels past the
// rank still cost their launches)
size_t rank_need(const gf2_mat *A) {
  if (A->rows == 0 || A->cols == 0) return 0;
  const bool wide = A->cols > A->rows;
  return wide ? decomp_bytes(A->cols, A->rows) : decomp_bytes(A->rows, A->cols);
}

int rank_body(const gf2_mat *A, int64_t *rank, void *ws, hipStream_t s) {
  int rc;
  if (A->rows == 0 || A->cols == 0) {
    HIPCHK(launch_empty_outputs(nullptr, 0, rank, s));
    return GF2_OK;
  }
  const bool wide = A->cols > A->rows;
  DecWork w;
  if (wide) prepare_decomp(A->cols, A->rows, ws, w, 0, nullptr);
  else prepare_decomp(A->rows, A->cols, ws, w, 0, nullptr);
  Exec x;
  if ((rc = make_exec(s, few_panels(w, A), x))) return rc;
  if ((rc = factor(A, w, x, wide ? Pack::kTransposed : Pack::kPlain))) return rc;
  HIPCHK(launch_finish(w, nullptr, nullptr, rank, s));
  return GF2_OK;
}

int solve_check(const gf2_mat *A, const gf2_mat *B, const gf2_mat *X, const uint64_t *consistent) {
  int rc;
  if ((rc = check_mat(A, "A")) || (rc = check_mat(B, "B")) || (rc = check_mat(X, "X"))) return rc;
  if (!consistent) return fail(GF2_EINVAL, "gf2_solve: null consistent pointer");
  const int64_t n = A->rows, m = A->cols, k = B->cols;
  if (B->rows != n || X->rows != m || X->cols != k)
    return fail(GF2_EINVAL, "gf2_solve: shapes do not match (A n x m, B n x k, X m x k)");
  if (n == 0 || m == 0 || k == 0) return fail(GF2_EINVAL, "gf2_solve: empty systems are not supported");
  return GF2_OK;
}

// right-hand sides after P, then Y (n x ceil(k/64) words), and the residual flags
size_t solve_extra(int64_t n, int64_t k) {
  const int64_t kw = ceil_div(k, 64);
  return align256((size_t)n * kw * 8) + align256((size_t)kw * 8);
}

size_t solve_need(int64_t n, int64_t m, int64_t k) { return decomp_bytes(n, m) + align256(solve_extra(n, k)); }

int solve_body(const gf2_mat *A, const gf2_mat *B, const gf2_mat *X, uint64_t *consistent, int64_t *rank, void *ws,
               hipStream_t s) {
  int rc;
  const int64_t n = A->rows, m = A->cols, k = B->cols;
  const int64_t kw = ceil_div(k, 64);
  DecWork w;
  void *extra = nullptr;
  prepare_decomp(n, m, ws, w, solve_extra(n, k), &extra);
  Exec x;
  if ((rc = make_exec(s, few_panels(w, A), x))) return rc;
  if ((rc = factor(A, w, x))) return rc;
  SolveWork sw;
  sw.Y = (uint64_t *)extra;
  sw.kw = kw;
  sw.k = k;
  sw.bad = (uint64_t *)((char *)extra + align256((size_t)n * kw * 8));
  HIPCHK(launch_solve(w, *B, *X, sw, consistent, s));
  HIPCHK(launch_finish(w, nullptr, nullptr, rank, s));
  return GF2_OK;
}

// A batched decomposition's workspace: the sorted descriptors, the queue head
// and one working-copy slot per persistent workgroup (slot sized for the
// largest item, rounded to 32 words).
size_t batch_dec_need(int64_t count, int64_t max_words, int workers) {
  if (count <= 0) return 0;
  const int64_t wslot = (std::max<int64_t>(max_words, 1) + 31) / 32 * 32;
  return align256((size_t)count * sizeof(BatchDesc)) + 256 + align256((size_t)workers * (size_t)wslot * 8);
}

int batch_dec_body(const std::vector<BatchDesc> &descs, int64_t max_words, int workers, const uint64_t *A, uint64_t *L,
                   uint64_t *E, int64_t *perm, int64_t *pivcols, int64_t *rank, void *ws, hipStream_t s) {
  int rc;
  const int64_t count = (int64_t)descs.size();
  const int64_t wslot = (std::max<int64_t>(max_words, 1) + 31) / 32 * 32;
  Carver c(ws);
  BatchDesc *dd = c.take<BatchDesc>((size_t)count);
  uint32_t *ctr = c.take<uint32_t>(64);
  uint64_t *W = c.take<uint64_t>((size_t)workers * (size_t)wslot);
  if ((rc = stage_descs(descs, dd, s))) return rc;
  BatchArgs a;
  a.d = dd;
  a.count = (int32_t)count;
  a.counter = ctr;
  a.A = A;
  a.L = L;
  a.E = E;
  a.perm = perm;
  a.pivcols = pivcols;
  a.rank = rank;
  a.W = W;
  a.wslot = wslot;
  HIPCHK(launch_batch_dec(a, workers, s));
  return GF2_OK;
}

int batch_workers_for(int64_t count, int *workers) {
  int ncu = 1;
  int rc = device_cus(&ncu);
  if (rc) return rc;
  *workers = (int)std::min<int64_t>(std::max<int64_t>(count, 1), batch_workers(ncu));
  return GF2_OK;
}

int batch_solve_body(const std::vector<BatchDesc> &descs, const uint64_t *L, const uint64_t *E, const int64_t *perm,
                     const int64_t *pivcols, const int64_t *rank, const uint64_t *B, uint64_t *X, int32_t *consistent,
                     void *ws, hipStream_t s) {
  int rc;
  BatchDesc *dd = (BatchDesc *)ws;
  if ((rc = stage_descs(descs, dd, s))) return rc;
  BatchSolveArgs a;
  a.d = dd;
  a.count = (int32_t)descs.size();
  a.L = L;
  a.E = E;
  a.perm = perm;
  a.pivcols = pivcols;
  a.rank = rank;
  a.B = B;
  a.X = X;
  a.consistent = consistent;
  HIPCHK(launch_batch_solve(a, s));
  return GF2_OK;
}

}  // namespace

namespace {
int batch_dec_check(const gf2_batch_item *items, int64_t count, const uint64_t *A, const int64_t *rank,
                    std::vector<BatchDesc> &descs, int64_t *maxw) {
  int rc = batch_descs(items, count, false, descs, maxw);
  if (rc) return rc;
  if (count == 0) return GF2_OK;
  if (!rank) return fail(GF2_EINVAL, "gf2_decompose_batched: null rank");
  if (*maxw > 0 && !A) return fail(GF2_EINVAL, "gf2_decompose_batched: null A");
  return GF2_OK;
}

int batch_solve_check(const gf2_batch_item *items, int64_t count, const uint64_t *L, const uint64_t *E,
                      const int64_t *perm, const int64_t *pivcols, const int64_t *rank, const uint64_t *B,
                      const uint64_t *X, const int32_t *consistent, std::vector<BatchDesc> &descs) {
  int64_t maxw = 0;
  int rc = batch_descs(items, count, true, descs, &maxw);
  if (rc) return rc;
  if (count == 0) return GF2_OK;
  if (!L || !E || !perm || !pivcols || !rank || !B || !X || !consistent)
    return fail(GF2_EINVAL, "gf2_solve_batched: null pointer argument");
  return GF2_OK;
}
}  // namespace

extern "C" {

size_t gf2_workspace_bytes(int op, int64_t rows, int64_t cols, int64_t k) {
  if (rows < 0 || cols < 0 || k < 0) {
    fail(GF2_EINVAL, "gf2_workspace_bytes: negative size");
    return SIZE_MAX;
  }
  switch (op) {
    case GF2_OP_MATMUL:
      return matmul_plan(rows, k, cols).total();
    case GF2_OP_DECOMPOSE:
      return (rows == 0 || cols == 0) ? 0 : decomp_bytes(rows, cols);
    case GF2_OP_RANK: {
      gf2_mat a{nullptr, rows, cols, 1, rows};
      return rank_need(&a);
    }
    case GF2_OP_SOLVE:
      return (rows == 0 || cols == 0 || k == 0) ? 0 : solve_need(rows, cols, k);
    case GF2_OP_DECOMPOSE_BATCHED: {
      if (cols > GF2_BATCH_MAX_DIM || k > GF2_BATCH_MAX_DIM) break;
      int workers = 1;
      if (batch_workers_for(rows, &workers)) return SIZE_MAX;
      return batch_dec_need(rows, batch_slot_words(k, cols), workers);
    }
    case GF2_OP_SOLVE_BATCHED:
      return rows > 0 ? align256((size_t)rows * sizeof(BatchDesc)) : 0;
    default:
      break;
  }
  fail(GF2_EINVAL, "gf2_workspace_bytes: unknown operation or size out of range");
  return SIZE_MAX;
}

int gf2_matmul(const gf2_mat *C, const gf2_mat *A, const gf2_mat *B, int accumulate, void *stream) {
  int rc;
  if ((rc = matmul_check(C, A, B))) return rc;
  const MatmulPlan p = matmul_plan(A->rows, A->cols, B->cols);
  void *ws = nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (p.total() && (rc = get_workspace(s, p.total(), &ws))) return rc;
  return matmul_body(C, A, B, accumulate, p, ws, s);
}

int gf2_matmul_ws(const gf2_mat *C, const gf2_mat *A, const gf2_mat *B, int accumulate, void *workspace,
                  size_t workspace_bytes, void *stream) {
  int rc;
  if ((rc = matmul_check(C, A, B))) return rc;
  const MatmulPlan p = matmul_plan(A->rows, A->cols, B->cols);
  if ((rc = check_ws(workspace, workspace_bytes, p.total(), "gf2_matmul_ws"))) return rc;
  return matmul_body(C, A, B, accumulate, p, workspace, (hipStream_t)stream);
}

int gf2_decompose(const gf2_mat *A, const gf2_mat *L, const gf2_mat *E, int64_t *perm,
                  int64_t *pivcols, int64_t *rank, void *stream) {
  int rc;
  if ((rc = decompose_check(A, L, E))) return rc;
  hipStream_t s = (hipStream_t)stream;
  void *ws = nullptr;
  const size_t need = decompose_need(A);
  if (need && (rc = get_workspace(s, need, &ws))) return rc;
  return decompose_body(A, L, E, perm, pivcols, rank, ws, s, false);
}

int gf2_decompose_ws(const gf2_mat *A, const gf2_mat *L, const gf2_mat *E, int64_t *perm, int64_t *pivcols,
                     int64_t *rank, void *workspace, size_t workspace_bytes, void *stream) {
  int rc;
  if ((rc = decompose_check(A, L, E))) return rc;
  if ((rc = check_ws(workspace, workspace_bytes, decompose_need(A), "gf2_decompose_ws"))) return rc;
  return decompose_body(A, L, E, perm, pivcols, rank, workspace, (hipStream_t)stream, false);
}

int gf2_decompose_noalloc(const gf2_mat *A, const gf2_mat *L, const gf2_mat *E, int64_t *perm, int64_t *pivcols,
                          int64_t *rank, void *stream) {
  int rc;
  if ((rc = decompose_check(A, L, E))) return rc;
  const size_t need = decompose_need(A);
  if (need > kScratchBytes)
    return fail(GF2_EINVAL, "gf2_decompose_noalloc: a " + std::to_string(A->rows) + " x " +
                                std::to_string(A->cols) + " decomposition needs " + std::to_string(need) +
                                " bytes of working state; the static scratch holds " +
                                std::to_string(kScratchBytes) + " (GF2_NOALLOC_MAX_BYTES)");
  void *ws = nullptr;
  if (need && (rc = scratch_ptr(&ws))) return rc;
  // every launch in order on the caller's stream, no profiling events
  g_noalloc = true;
  rc = decompose_body(A, L, E, perm, pivcols, rank, ws, (hipStream_t)stream, true);
  g_noalloc = false;
  return rc;
}

// A captured decomposition: the instantiated graph of one gf2_decompose_ws
// call with every launch in order on the capturing stream.  (Capturing the
// look-ahead streams through their events ended in a host-side crash inside
// the runtime during capture on MI355X; that form is not used.)
struct gf2_graph_s {
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

int gf2_decompose_graph(const gf2_mat *A, const gf2_mat *L, const gf2_mat *E, int64_t *perm, int64_t *pivcols,
                        int64_t *rank, void *workspace, size_t workspace_bytes, void *stream, gf2_graph *graph) {
  int rc;
  if (!graph) return fail(GF2_EINVAL, "gf2_decompose_graph: null graph pointer");
  *graph = nullptr;
  if (!stream) return fail(GF2_EINVAL, "gf2_decompose_graph: capture needs a stream other than the null stream");
  if ((rc = decompose_check(A, L, E))) return rc;
  if ((rc = check_ws(workspace, workspace_bytes, decompose_need(A), "gf2_decompose_graph"))) return rc;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  const bool prof = g_noalloc;
  g_noalloc = true;  // no profiling events inside a capture
  rc = decompose_body(A, L, E, perm, pivcols, rank, workspace, s, true);
  g_noalloc = prof;
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(s, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (ec != hipSuccess) return hip_fail(ec, "gf2_decompose_graph: hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return hip_fail(ei, "gf2_decompose_graph: hipGraphInstantiate");
  gf2_graph h = new gf2_graph_s;
  h->exec = exec;
  h->device = dev;
  *graph = h;
  return GF2_OK;
}

int gf2_graph_launch(gf2_graph graph, void *stream) {
  if (!graph || !graph->exec) return fail(GF2_EINVAL, "gf2_graph_launch: null graph");
  HIPCHK(hipGraphLaunch(graph->exec, (hipStream_t)stream));
  return GF2_OK;
}

int gf2_graph_destroy(gf2_graph graph) {
  if (!graph) return GF2_OK;
  int rc = GF2_OK;
  if (graph->exec) {
    const hipError_t e = hipGraphExecDestroy(graph->exec);
    if (e != hipSuccess) rc = hip_fail(e, "gf2_graph_destroy");
  }
  delete graph;
  return rc;
}

int gf2_rank(const gf2_mat *A, int64_t *rank, void *stream) {
  int rc;
  if ((rc = rank_check(A, rank))) return rc;
  hipStream_t s = (hipStream_t)stream;
  void *ws = nullptr;
  const size_t need = rank_need(A);
  if (need && (rc = get_workspace(s, need, &ws))) return rc;
  return rank_body(A, rank, ws, s);
}

int gf2_rank_ws(const gf2_mat *A, int64_t *rank, void *workspace, size_t workspace_bytes, void *stream) {
  int rc;
  if ((rc = rank_check(A, rank))) return rc;
  if ((rc = check_ws(workspace, workspace_bytes, rank_need(A), "gf2_rank_ws"))) return rc;
  return rank_body(A, rank, workspace, (hipStream_t)stream);
}

int gf2_solve(const gf2_mat *A, const gf2_mat *B, const gf2_mat *X, uint64_t *consistent,
              int64_t *rank, void *stream) {
  int rc;
  if ((rc = solve_check(A, B, X, consistent))) return rc;
  hipStream_t s = (hipStream_t)stream;
  void *ws = nullptr;
  if ((rc = get_workspace(s, solve_need(A->rows, A->cols, B->cols), &ws))) return rc;
  return solve_body(A, B, X, consistent, rank, ws, s);
}

int gf2_solve_ws(const gf2_mat *A, const gf2_mat *B, const gf2_mat *X, uint64_t *consistent, int64_t *rank,
                 void *workspace, size_t workspace_bytes, void *stream) {
  int rc;
  if ((rc = solve_check(A, B, X, consistent))) return rc;
  if ((rc = check_ws(workspace, workspace_bytes, solve_need(A->rows, A->cols, B->cols), "gf2_solve_ws"))) return rc;
  return solve_body(A, B, X, consistent, rank, workspace, (hipStream_t)stream);
}


int gf2_decompose_batched(const gf2_batch_item *items, int64_t count, const uint64_t *A,
                          uint64_t *L, uint64_t *E, int64_t *perm, int64_t *pivcols,
                          int64_t *rank, void *stream) {
  std::vector<BatchDesc> descs;
  int64_t maxw = 0;
  int rc = batch_dec_check(items, count, A, rank, descs, &maxw);
  if (rc || count == 0) return rc;
  int workers = 1;
  if ((rc = batch_workers_for(count, &workers))) return rc;
  hipStream_t s = (hipStream_t)stream;
  void *ws = nullptr;
  if ((rc = get_workspace(s, batch_dec_need(count, maxw, workers), &ws))) return rc;
  return batch_dec_body(descs, maxw, workers, A, L, E, perm, pivcols, rank, ws, s);
}

int gf2_decompose_batched_ws(const gf2_batch_item *items, int64_t count, const uint64_t *A, uint64_t *L, uint64_t *E,
                             int64_t *perm, int64_t *pivcols, int64_t *rank, void *workspace,
                             size_t workspace_bytes, void *stream) {
  std::vector<BatchDesc> descs;
  int64_t maxw = 0;
  int rc = batch_dec_check(items, count, A, rank, descs, &maxw);
  if (rc || count == 0) return rc;
  int workers = 1;
  if ((rc = batch_workers_for(count, &workers))) return rc;
  if ((rc = check_ws(workspace, workspace_bytes, batch_dec_need(count, maxw, workers), "gf2_decompose_batched_ws")))
    return rc;
  return batch_dec_body(descs, maxw, workers, A, L, E, perm, pivcols, rank, workspace, (hipStream_t)stream);
}

int gf2_solve_batched(const gf2_batch_item *items, int64_t count, const uint64_t *L,
                      const uint64_t *E, const int64_t *perm, const int64_t *pivcols,
                      const int64_t *rank, const uint64_t *B, uint64_t *X, int32_t *consistent,
                      void *stream) {
  std::vector<BatchDesc> descs;
  int rc = batch_solve_check(items, count, L, E, perm, pivcols, rank, B, X, consistent, descs);
  if (rc || count == 0) return rc;
  hipStream_t s = (hipStream_t)stream;
  void *ws = nullptr;
  if ((rc = get_workspace(s, align256((size_t)count * sizeof(BatchDesc)), &ws))) return rc;
  return batch_solve_body(descs, L, E, perm, pivcols, rank, B, X, consistent, ws, s);
}

int gf2_solve_batched_ws(const gf2_batch_item *items, int64_t count, const uint64_t *L, const uint64_t *E,
                         const int64_t *perm, const int64_t *pivcols, const int64_t *rank, const uint64_t *B,
                         uint64_t *X, int32_t *consistent, void *workspace, size_t workspace_bytes, void *stream) {
  std::vector<BatchDesc> descs;
  int rc = batch_solve_check(items, count, L, E, perm, pivcols, rank, B, X, consistent, descs);
  if (rc || count == 0) return rc;
  if ((rc = check_ws(workspace, workspace_bytes, align256((size_t)count * sizeof(BatchDesc)),
                     "gf2_solve_batched_ws")))
    return rc;
  return batch_solve_body(descs, L, E, perm, pivcols, rank, B, X, consistent, workspace, (hipStream_t)stream);
}

int gf2_autotune(int64_t max_size, void *stream) {
  if (max_size < 256) return fail(GF2_EINVAL, "gf2_autotune: max_size must be >= 256");
  hipStream_t s = (hipStream_t)stream;
  int rc = GF2_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto timed = [&](auto &&launch, float *ms) -> int {
    int r = launch();  // warm-up
    if (r) return r;
    HIPCHK(hipEventRecord(e0, s));
    for (int i = 0; i < 3; ++i)
      if ((r = launch())) return r;
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(ms, e0, e1));
    return GF2_OK;
  };

  // ---- product-kernel tile per size class, at the decomposition's inner
  // dimension (one 512-column panel) on synthetic operands
  const int cand[4] = {0, 1, 2, 3};
  const int bsel[kTuneBlocks] = {1, 3, 8, 32};
  int nr = 0;
  while (nr < kTuneRows && ((int64_t)256 << nr) <= max_size) ++nr;
  const int64_t rows_max = ((int64_t)256 << (nr - 1)) * 3 / 2;
  const int64_t ldA = ceil_div(rows_max, 256) * 256, ldB = 512;
  const size_t wA = (size_t)ldA * TW, wB = (size_t)32 * ldB * TW, wC = (size_t)32 * ldA * TW;
  uint64_t *buf = nullptr;
  HIPCHK(hipMalloc(&buf, (wA + wB + wC) * 8));
  uint64_t *bA = buf, *bB = buf + wA, *bC = buf + wA + wB;
  int table[kTuneRows][kTuneBlocks];
  do {
    if (launch_fill_bits(buf, wA + wB + wC, 0x5eed, s) != hipSuccess) { rc = fail(GF2_EHIP, "fill"); break; }
    for (int r = 0; r < nr && !rc; ++r) {
      const int64_t rows = ((int64_t)256 << r) * 3 / 2;
      for (int c = 0; c < kTuneBlocks && !rc; ++c) {
        float best_ms = 1e30f;
        int best = -1;
        for (int v : cand) {
          GemmArgs a;
          memset(&a, 0, sizeof(a));
          a.A = bA; a.ldA = ldA; a.a_word0 = 0;
          a.B = bB; a.ldB = ldB; a.b_rows = 512;
          a.C = bC; a.ldC = ldA;
          a.row_tile0 = 0; a.row_end = rows;
          a.kwords = 8;
          a.qc0 = 0; a.qc1 = bsel[c] * TW;
          a.accumulate = 1;
          float ms = 0.f;
          rc = timed([&]() -> int { HIPCHK(launch_gemm(a, rows, v, s)); return GF2_OK; }, &ms);
          if (rc) break;
          if (ms < best_ms) { best_ms = ms; best = v; }
        }
        table[r][c] = best;
      }
    }
  } while (0);
  (void)hipFree(buf);
  if (rc) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return rc; }
  for (int r = 0; r < kTuneRows; ++r)
    for (int c = 0; c < kTuneBlocks; ++c) g_tuned[r][c] = table[r < nr ? r : nr - 1][c];
  g_tuned_valid = g_tuned_on = true;

  // ---- Strassen-Winograd cutoff: one level against the plain product on
  // square operands; the smallest size where the level pays becomes the cutoff
  int64_t cutoff = 0, largest = 0;
  for (int64_t n = 32768; n <= 65536 && n <= max_size && !rc; n *= 2) {
    largest = n;
    const int64_t nw = n / 64;
    const size_t wm = (size_t)n * nw, st_bytes = strassen_bytes(n, nw, nw, 1);
    char *sb = nullptr;
    if (hipMalloc(&sb, 3 * wm * 8 + st_bytes) != hipSuccess) {
      (void)hipGetLastError();
      break;  // not enough memory to compare at this size: keep the previous answer
    }
    uint64_t *mA = (uint64_t *)sb, *mB = mA + wm, *mC = mB + wm;
    if (launch_fill_bits(mA, 2 * wm, 0x5eed + n, s) != hipSuccess) rc = fail(GF2_EHIP, "fill");
    const BView Av{mA, n, n, nw}, Bv{mB, n, n, nw}, Cv{mC, n, n, nw};
    float plain = 0.f, one = 0.f;
    if (!rc) rc = timed([&]() -> int { return gemm_view(Cv, Av, Bv, 0, s); }, &plain);
    if (!rc) {
      rc = timed([&]() -> int {
        Stack st{sb + 3 * wm * 8, 0, st_bytes};
        return strassen(Cv, Av, Bv, 1, 0, st, s);
      }, &one);
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(sb);
    if (!rc && one < plain) {
      cutoff = n;
      break;
    }
  }
  if (rc) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return rc; }
  if (largest > 0) g_strassen_cutoff = cutoff > 0 ? cutoff : 2 * largest;

  // ---- panel width (sub-panels of 64 columns, W) per decomposition size
  // class: one decomposition of a random square matrix at the class's probe
  // size (up to max_size) for W = 2, 4, 8; the fastest becomes the class's
  // width.  Classes above max_size keep the default (8).
  const int saved_w = g_panel_words;
  const bool saved_on = g_tuned_on;
  g_tuned_on = false;
  for (int c = 0; c < kWClasses && !rc; ++c) {
    const int64_t n = kWClassProbe[c];
    if (n > max_size) {
      g_tuned_W[c] = 0;
      continue;
    }
    const int64_t nw = n / 64;
    const size_t words = (size_t)n * (size_t)nw;
    char *mem = nullptr;
    if (hipMalloc(&mem, 3 * words * 8 + (size_t)(2 * n + 1) * 8) != hipSuccess) {
      (void)hipGetLastError();
      g_tuned_W[c] = 0;
      break;  // not enough memory at this size: the larger classes keep the default
    }
    uint64_t *dA = (uint64_t *)mem, *dL = dA + words, *dE = dL + words;
    int64_t *perm = (int64_t *)(dE + words), *piv = perm + n, *rk = piv + n;
    const gf2_mat Am{dA, n, n, nw, n}, Lm{dL, n, n, nw, n}, Em{dE, n, n, nw, n};
    float best_ms = 1e30f;
    int best = 0;
    if (launch_fill_bits(dA, words, 0x7a11 + c, s) != hipSuccess) rc = fail(GF2_EHIP, "fill");
    for (int W : {2, 4, 8}) {
      if (rc) break;
      g_panel_words = W;
      float ms = 0.f;
      rc = timed([&]() -> int { return gf2_decompose(&Am, &Lm, &Em, perm, piv, rk, stream); }, &ms);
      if (!rc && ms < best_ms) {
        best_ms = ms;
        best = W;
      }
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(mem);
    g_tuned_W[c] = best;
  }
  g_panel_words = saved_w;
  g_tuned_on = saved_on;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int gf2_autotune_params(int64_t rows, int64_t cols, int32_t *panel_words, int32_t *table_bits,
                        int32_t *analytic_table_bits, int64_t *analytic_strassen) {
  if (rows < 0 || cols < 0) return fail(GF2_EINVAL, "gf2_autotune_params: rows and cols must be >= 0");
  const int W = panel_words_for(rows, cols);
  if (panel_words) *panel_words = W;
  if (table_bits) *table_bits = 8;  // the trailing-update product's tables: 2^8 entries per 8 inner bits
  if (analytic_table_bits) {
    // Section 6: the table size minimising C(b, c, n) = (b / c)(2^c - 1 + n)
    // for the panel's product, b = 64 W inner bits and n = rows output rows
    double best = 1e300;
    int bc = 1;
    for (int c = 1; c <= 24; ++c) {
      const double cost = (64.0 * W / c) * (std::ldexp(1.0, c) - 1.0 + (double)rows);
      if (cost < best) {
        best = cost;
        bc = c;
      }
    }
    *analytic_table_bits = bc;
  }
  // Section 6: Strassen-Winograd pays on the CPU model from n >= 44c + 6(2^c - 1)
  if (analytic_strassen) *analytic_strassen = 44 * 8 + 6 * ((1 << 8) - 1);
  return GF2_OK;
}

int gf2_autotune_table(int32_t *variants, int64_t *strassen_cutoff) {
  if (variants)
    for (int r = 0; r < kTuneRows; ++r)
      for (int c = 0; c < kTuneBlocks; ++c) variants[r * kTuneBlocks + c] = g_tuned_valid ? g_tuned[r][c] : -1;
  if (strassen_cutoff) *strassen_cutoff = g_strassen_cutoff;
  return GF2_OK;
}

int gf2_rref(const gf2_mat *A, const gf2_mat *R, int64_t *pivcols, int64_t *rank, void *stream) {
  int rc;
  if ((rc = check_mat(A, "A"))) return rc;
  const int64_t n = A->rows, m = A->cols, kmin = n < m ? n : m;
  if (kmin == 0) return fail(GF2_EINVAL, "gf2_rref: empty matrices are not supported");
  if (R) {
    if ((rc = check_mat(R, "R"))) return rc;
    if (R->rows != kmin || R->cols != m) return fail(GF2_EINVAL, "gf2_rref: R must be min(n,m) x m");
  }
  hipStream_t s = (hipStream_t)stream;
  RrefWork rw;
  if ((rc = rref_run(A, s, rw))) return rc;
  if (R) HIPCHK(launch_unpack(rw.E, rw.ldE, *R, s));
  if (pivcols) HIPCHK(hipMemcpyAsync(pivcols, rw.piv, (size_t)kmin * 8, hipMemcpyDeviceToDevice, s));
  if (rank) HIPCHK(hipMemcpyAsync(rank, rw.rank, 8, hipMemcpyDeviceToDevice, s));
  return GF2_OK;
}

int gf2_inverse(const gf2_mat *A, const gf2_mat *X, uint64_t *invertible, void *stream) {
  int rc;
  if ((rc = check_mat(A, "A")) || (rc = check_mat(X, "X"))) return rc;
  const int64_t n = A->rows;
  if (n == 0 || A->cols != n) return fail(GF2_EINVAL, "gf2_inverse: A must be square and not empty");
  if (X->rows != n || X->cols != n) return fail(GF2_EINVAL, "gf2_inverse: X must be n x n");
  hipStream_t s = (hipStream_t)stream;
  RrefWork rw;
  if ((rc = rref_run(A, s, rw, true))) return rc;
  HIPCHK(launch_inverse_out(rw.E, rw.ldE, rw.piv, n, *X, invertible, s));
  return GF2_OK;
}

int gf2_nullspace(const gf2_mat *A, const gf2_mat *N, int64_t *nullity, void *stream) {
  int rc;
  if ((rc = check_mat(A, "A")) || (rc = check_mat(N, "N"))) return rc;
  const int64_t n = A->rows, m = A->cols;
  if (n == 0 || m == 0) return fail(GF2_EINVAL, "gf2_nullspace: empty matrices are not supported");
  if (N->rows != m || N->cols != m) return fail(GF2_EINVAL, "gf2_nullspace: N must be m x m");
  if (!nullity) return fail(GF2_EINVAL, "gf2_nullspace: null nullity pointer");
  hipStream_t s = (hipStream_t)stream;
  RrefWork rw;
  if ((rc = rref_run(A, s, rw))) return rc;
  HIPCHK(launch_null_basis(rw.E, rw.ldE, rw.piv, rw.rank, rw.bitmap, rw.tw0, rw.freecols, nullity, *N, s));
  return GF2_OK;
}

}  // extern "C"
