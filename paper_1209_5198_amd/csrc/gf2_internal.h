// gf2_internal.h -- internal layout, device state and launcher declarations of
// libgf2 (gfx950).  Not installed; the public ABI is include/gf2.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gf2.h"

// v_writelane_b32 (lane `lane` of `old` receives the uniform value `val`): an
// LLVM intrinsic that clang does not expose as a builtin.
extern "C" __device__ int gf2_llvm_writelane(int val, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

namespace gf2 {

// ---------------------------------------------------------------- working layout
// The library's working matrices use the paper's column-blocked row-major
// storage (Section 3) with a fixed block of TW = 16 words (1024 columns):
// word (i, q) lives at base[((q / 16) * ldw + i) * 16 + q % 16].  A 16-word
// block row is 128 contiguous bytes, so a 16-lane group of a wave reads or
// writes one block row in a single coalesced 128-byte access, and a 64-row
// tile of one block is 8 KB contiguous.
constexpr int TW = 16;

__host__ __device__ inline size_t widx(int64_t ldw, int64_t i, int64_t q) {
  return ((size_t)(q >> 4) * (size_t)ldw + (size_t)i) * TW + (size_t)(q & 15);
}

// word (i, q) of a caller matrix described by gf2_mat
__host__ __device__ inline size_t uidx(int64_t w, int64_t ld, int64_t i, int64_t q) {
  return ((size_t)(q / w) * (size_t)ld + (size_t)i) * (size_t)w + (size_t)(q % w);
}

__host__ __device__ inline uint64_t pad_mask(int64_t cols, int64_t q) {
  int64_t valid = cols - 64 * q;
  if (valid >= 64) return ~0ull;
  if (valid <= 0) return 0ull;
  return (1ull << valid) - 1ull;
}

__device__ inline uint32_t wrlane(uint32_t val, int lane, uint32_t old) {
  return (uint32_t)gf2_llvm_writelane((int)val, lane, (int)old);
}
__device__ inline int wrlane(int val, int lane, int old) { return gf2_llvm_writelane(val, lane, old); }

__device__ inline uint64_t shfl_xor64(uint64_t x, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, m), hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), m);
  return ((uint64_t)hi << 32) | lo;
}

// 64 x 64 bit transpose across a wave: lane k holds row k of the block (bit j =
// column j); afterwards lane j holds column j.  The step with distance d
// exchanges, between rows k and k + d (bit d of k clear), the d x d sub-blocks
// off the diagonal of each 2d x 2d block.
__device__ inline uint64_t transpose64(uint64_t x, int lane) {
  uint64_t m = 0x00000000FFFFFFFFull;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t y = shfl_xor64(x, d);
    const bool low = (lane & d) == 0;
    const uint64_t t = low ? (((x >> d) ^ y) & m) : (((y >> d) ^ x) & m);
    x ^= low ? (t << d) : t;
    m ^= m << (d >> 1);
  }
  return x;
}

// ---------------------------------------------------------------- decomposition state
// Per 64-column sub-panel q: rank before it (R), its number of pivots (r) and
// the bit positions of its pivot columns inside word q.
struct SubInfo {
  int64_t R;
  int32_t r;
  int32_t pad;
  uint64_t pivmask;
};

struct DecState {
  int64_t R;         // rank found so far
  int32_t bp_count;  // positions listed in bp_list for the current panel
  int32_t pad0;
};

// Everything the decomposition kernels address; all pointers are device memory.
struct DecWork {
  uint64_t *W;       // working matrix, (NB * ldw * 16) words
  int64_t ldw;       // rows per block (>= n, multiple of 256)
  int64_t n, m;      // rows, cols (bits)
  int32_t Mw;        // ceil(m / 64) word columns
  int32_t NB;        // ceil(Mw / 16) blocks
  DecState *st;
  SubInfo *sub;      // [Mw]
  uint64_t *Zc;      // [Mw * 64]  coefficient map of each sub-panel
  uint64_t *Linv;    // [Mw * 64]  inverse of each sub-panel's unit lower block
  int64_t *perm;     // [n]
  int64_t *pivcols;  // [Mw * 64]
  int32_t *bp_src;   // [n]  position at panel start of the row now at position p
  int32_t *bp_mark;  // [n]  1 if p is listed in bp_list
  int32_t *bp_list;  // [kMaxPanelWords * 64 * 2]
  uint32_t *nzflag;  // [Mw]  trailing-update nonzero flag per panel
  int32_t *lvl;      // [n]   16*q0 + L: sub-panels 0..L-1 of the panel at q0 applied to row p
  uint64_t *ptab;    // [kPanelTabWords] 4-bit tables of the current panel (written by its chain)
  // net row permutation of the current super-panel, two buffers (super-panel
  // parity): position p holds the row that was at sp_src[p] when it started;
  // sp_list holds the sp_count positions that changed (sp_mark[p] = 1)
  int32_t *sp_src;   // [2 * n]
  int32_t *sp_mark;  // [2 * n]
  int32_t *sp_list;  // [2 * kSpListMax]
  int32_t *sp_count; // [2]
};

constexpr int kMaxPanelWords = 8;       // s <= 8 sub-panels per trailing-update panel
// A super-panel is at most kSpSubMax sub-panels (whole panels); its far
// update is one product of inner dimension 64 * (sub-panels)
constexpr int kSpSubMax = 32;
constexpr int kSpListMax = 2 * 64 * kSpSubMax;  // positions a super-panel can move
constexpr int kWin = 128;               // window rows examined per sub-panel
// words of one panel's 4-bit tables: Tz (y = x * Zc_c) for 8 sub-panels and Te
// (y * E_c[w]) for the 28 sub-panel / later-word pairs, 16 x 16 entries each
constexpr int kPanelTabWords = (kMaxPanelWords + kMaxPanelWords * (kMaxPanelWords - 1) / 2) * 256;

// ---------------------------------------------------------------- product arguments
struct GemmArgs {
  const uint64_t *A; int64_t ldA; int32_t a_word0;   // A words [a_word0, a_word0 + kwords)
  const uint64_t *B; int64_t ldB; int64_t b_rows;    // plain B: row k for k < b_rows
  const SubInfo *bsub;                               // mapped B: row (kw, t) -> bsub[kw].R + t, t < bsub[kw].r;
                                                     // then also rows >= bsub[kwords-1].R + bsub[kwords-1].r;
                                                     // with bsub, kwords <= kSpSubMax
  uint64_t *C; int64_t ldC;
  int64_t row_tile0;                                 // first row of tile 0
  int64_t row_end;                                   // rows < row_end
  int32_t kwords;
  int32_t qc0, qc1;                                  // C word columns [qc0, qc1)
  int32_t accumulate;
  uint32_t *nzflag;                                  // optional: OR of all written words != 0
  const uint32_t *skip_flag;                         // optional: skip the launch when *skip_flag == 0
  unsigned long long *work;                          // optional: += table lookups performed
  int32_t kparts;                                    // narrow kernels, accumulate only: parts of the inner
                                                     // words (blockIdx.z), each XORed into C atomically;
                                                     // 0 or 1: one part (-1 on entry to run_gemm: may split)
};

// ---------------------------------------------------------------- launchers (one per kernel file)
hipError_t launch_init_state(const DecWork &w, hipStream_t s);
hipError_t launch_pack(const gf2_mat &src, uint64_t *W, int64_t ldw, int64_t n, int64_t m,
                       int32_t NB, hipStream_t s);
hipError_t launch_pack_transposed(const gf2_mat &src, uint64_t *W, int64_t ldw, int32_t NB, hipStream_t s);
hipError_t launch_unpack(const uint64_t *W, int64_t ldw, const gf2_mat &dst, hipStream_t s);
hipError_t launch_extract_E(const DecWork &w, const gf2_mat &E, hipStream_t s);
hipError_t launch_extract_L(const DecWork &w, const gf2_mat &L, hipStream_t s);
hipError_t launch_finish(const DecWork &w, int64_t *perm, int64_t *pivcols, int64_t *rank,
                         hipStream_t s);

constexpr int kGemmVariants = 6;   // product-kernel variants 0 .. kGemmVariants-1
constexpr int kGemmMfma = 6;       // gf2_matmul only: the fp4 matrix-core product (k_mfma.hip)
size_t mfma_ws_bytes(int64_t kwords, int64_t m_words, int64_t rows);  // its workspace
bool mfma_splits_inner(const GemmArgs &a, int ncu);  // the launch splits the inner dimension
hipError_t launch_gemm_mfma(const GemmArgs &a, int64_t bwords, uint64_t *ws, int ncu, hipStream_t s);
// e0, e1: optional timing events the launch records itself (start, end)
hipError_t launch_gemm(const GemmArgs &a, int64_t nrows_max, int variant, hipStream_t s, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
int gemm_auto_variant(int64_t active_rows, int qc0, int qc1, int ncu);  // variant for a launch shape
int gemm_wall_variant(int64_t active_rows, int qc0, int qc1, int ncu);  // ... minimising its wall time
int gemm_tile_rows(int v);                                               // rows of a variant's tile
bool gemm_narrow_ok(int qc0, int qc1);                                   // an 8-aligned range of <= 8 words
extern int g_wide_threads;  // threads of the 2048-row product tile (512 or 1024)

hipError_t launch_panel(const DecWork &w, int q0, int s_eff, int flag_q0, int spb, hipStream_t s);
hipError_t launch_post(const DecWork &w, int q0, int s_eff, int wlo, int whi, int ncu, hipStream_t s);
// closing a super-panel (k_super.hip): net permutation on the words outside
// [lo, hi), list reset, pivot rows in echelon form on the far words [qa, qb)
hipError_t launch_sp_swap(const DecWork &w, int buf, int lo, int hi, hipStream_t s);
hipError_t launch_sp_reset(const DecWork &w, int buf, hipStream_t s);
hipError_t launch_trsm_far(const DecWork &w, int s0, int nsub, int qa, int qb, hipStream_t s);
hipError_t launch_xor(uint64_t *dst, const uint64_t *a, const uint64_t *b, size_t nwords,
                      hipStream_t s);
// dst[0 .. nwords) = 0 by a kernel (no memset node where a caller captures the launches)
hipError_t launch_zero(uint64_t *dst, size_t nwords, hipStream_t s);
// outputs of an empty factorization: perm[i] = i for i < n (perm may be null), *rank = 0 (rank may be null)
hipError_t launch_empty_outputs(int64_t *perm, int64_t n, int64_t *rank, hipStream_t s);
hipError_t launch_fill_bits(uint64_t *dst, size_t nwords, uint64_t seed, hipStream_t s);  // timing operands
// microbenchmarks (k_probe.hip): kinds 0..5, *work = bytes, operations or multiply-accumulates
constexpr int kProbeKinds = 6;
hipError_t launch_probe(int kind, void *buf, size_t bytes, int iters, int ncu, uint32_t *sink, hipStream_t s,
                        double *work);

// A rows x (words) region of a working-layout matrix: word (i, q) at
// p[((q / 16) * ld + i) * 16 + q % 16].  A quadrant of a view whose words are
// a multiple of 32 is again a view (a pointer offset with the same ld).
struct BView {
  uint64_t *p;
  int64_t ld;
  int64_t rows;
  int64_t words;
};
// dst = (acc ? dst : 0) ^ a ^ b ^ (c ? c : 0), all of dst's shape; views may coincide with dst
hipError_t launch_xor_view(const BView &dst, const BView &a, const BView &b, const BView *c, int acc,
                           hipStream_t s);

struct SolveWork {
  uint64_t *Y;       // n x kw words, row-major (right-hand sides after P, then Y)
  int64_t kw;        // words per RHS row
  int64_t k;         // number of right-hand sides
  uint64_t *bad;     // [kw] OR of residual rows
};
hipError_t launch_solve(const DecWork &w, const gf2_mat &B, const gf2_mat &X,
                        const SolveWork &sw, uint64_t *consistent, hipStream_t s);

// ---------------------------------------------------------------- batches
// Many independent matrices of at most kBatchMaxDim rows and columns, each
// factored from start to finish by one workgroup of a persistent launch.
constexpr int kBatchMaxDim = GF2_BATCH_MAX_DIM;
constexpr int kBatchMaxPanels = kBatchMaxDim / 64;
constexpr int kBatchThreads = 256;   // threads per workgroup
constexpr int kBatchWGPerCU = 3;     // resident workgroups per CU (LDS-limited)

// One matrix of a batch, in the order the workers take them (offsets as in
// gf2_batch_item; idx = the item's index in the caller's array).
struct BatchDesc {
  int32_t n, m;
  int32_t idx;
  int32_t pad;
  int64_t a, l, e, p, c, b, x;
};

struct BatchArgs {
  const BatchDesc *d;
  int32_t count;
  uint32_t *counter;     // queue head, zeroed by the launcher
  const uint64_t *A;
  uint64_t *L, *E;       // may be null
  int64_t *perm, *pivcols;  // may be null
  int64_t *rank;
  uint64_t *W;           // worker slots, wslot words each
  int64_t wslot;
};

struct BatchSolveArgs {
  const BatchDesc *d;
  int32_t count;
  const uint64_t *L, *E;
  const int64_t *perm, *pivcols, *rank;
  const uint64_t *B;
  uint64_t *X;
  int32_t *consistent;
};

int batch_workers(int ncu);  // workgroups of one batched launch on a device of ncu CUs
hipError_t launch_batch_dec(const BatchArgs &a, int workers, hipStream_t s);
hipError_t launch_batch_solve(const BatchSolveArgs &a, hipStream_t s);

// ---------------------------------------------------------------- reduced echelon form, null space
hipError_t launch_gather_pivcols(const uint64_t *E, int64_t ldE, const int64_t *pivcols, const int64_t *rankp,
                                 uint64_t *G, int64_t kmin, int64_t Gw, hipStream_t s);
hipError_t launch_rref_diag(uint64_t *E, int64_t ldE, const uint64_t *G, const int64_t *rankp, int J, int64_t Mw,
                            hipStream_t s);
hipError_t launch_copy_block_rows(const uint64_t *E, int64_t ldE, const int64_t *rankp, int64_t R0, uint64_t *B,
                                  int64_t NB, hipStream_t s);
hipError_t launch_null_basis(const uint64_t *R, int64_t ldE, const int64_t *pivcols, const int64_t *rankp,
                             uint64_t *bitmap, int64_t *tw0, int64_t *freecols, int64_t *nullity,
                             const gf2_mat &N, hipStream_t s);
hipError_t launch_set_identity(uint64_t *W, int64_t ldw, int64_t n, int64_t col0, hipStream_t s);
hipError_t launch_inverse_out(const uint64_t *R, int64_t ldE, const int64_t *pivcols, int64_t n, const gf2_mat &X,
                              uint64_t *invertible, hipStream_t s);

}  // namespace gf2
