/*
 * gf2.h -- C ABI of libgf2: dense GF(2) matrix decomposition, rank, product
 * and linear solve on one MI355X (gfx950) GPU.
 *
 * Method: Bertolazzi & Rimoldi, "Fast matrix decomposition in F2".  The
 * decomposition is the column-swap-free P*A = L*E of Lemma 4.1 (Section 4),
 * computed by the block method of Section 4 (panel factorization by the
 * incremental pseudo-inverse of procedure buildZ, Sections 4.1-4.4; trailing
 * Schur complement update eq. (Aj) by the Four-Russians product of Section 6).
 *
 * ---------------------------------------------------------------- storage
 * A matrix is a caller-owned device buffer described by gf2_mat.  Element
 * a_ij is bit (j mod 64) (weight 2^(j mod 64)) of 64-bit word q = j / 64 of
 * row i -- the bit order of Section 3 (a_ij is bit r of word q, j = qb + r,
 * b = 64).  Words are grouped in column blocks of w words (64*w columns);
 * inside a block the words are row-major ("column blocks of row-major
 * matrices", Section 3):
 *
 *     word (i, q)  at  data[(q / w) * ld * w + i * w + (q % w)]
 *
 * w = 1 is the column-major word order the paper prefers; w = ceil(cols/64)
 * is plain row-major.  The buffer holds ceil(ceil(cols/64) / w) blocks of
 * ld * w words.  Input bits at or beyond `cols` (padding) are ignored; on
 * output they are written as zero, and rows in [rows, ld) are not touched.
 *
 * ---------------------------------------------------------------- calls
 * Every call is asynchronous on `stream` (a hipStream_t; NULL = the default
 * stream).  Pointer arguments other than the gf2_mat descriptors themselves
 * are device pointers.  The library never frees caller memory.  The plain
 * calls use a workspace per (device, stream) that the library grows on demand
 * with hipMalloc and releases in gf2_release(); the *_ws forms take a
 * caller-owned workspace instead (sizes from gf2_workspace_bytes) and never
 * allocate.  A factorization of more than two 512-column panels runs on two
 * internal look-ahead streams per (device, stream), ordered after the work
 * already on `stream` and before work enqueued on it later; smaller ones run
 * on `stream` itself.  Calls that share a device must not run concurrently
 * from several host threads.
 *
 * Return value: 0 on success, or a negative GF2_E* code; gf2_last_error()
 * then returns a message (thread-local, valid until the next call).  An
 * inconsistent linear system is not an error.
 */
#ifndef GF2_H
#define GF2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GF2_OK 0
#define GF2_EINVAL (-1) /* bad descriptor, shape mismatch or null pointer   */
#define GF2_ENOMEM (-2) /* workspace allocation failed                      */
#define GF2_EHIP (-3)   /* a HIP runtime call failed                        */

typedef struct gf2_mat {
  uint64_t *data; /* device pointer to the words                        */
  int64_t rows;   /* number of rows (bits)                              */
  int64_t cols;   /* number of columns (bits)                           */
  int64_t w;      /* words per row inside one column block (>= 1)       */
  int64_t ld;     /* rows allocated per block (>= rows)                 */
} gf2_mat;

/*
 * C = A*B (accumulate == 0) or C ^= A*B (accumulate != 0) over GF(2).
 * A: n x k, B: k x m, C: n x m.  C must not overlap A or B.
 * Four-Russians product (Section 6, eq. (M4RM:cost)) with Strassen-Winograd
 * recursion above a size cutoff (Section 6.2).
 */
int gf2_matmul(const gf2_mat *C, const gf2_mat *A, const gf2_mat *B, int accumulate,
               void *stream);

/*
 * Decomposition P*A = L*E of Lemma 4.1, no column exchanges.  A (n x m) is
 * read only.  With kmin = min(n, m) and r = rank:
 *   L       : n x kmin; unit lower trapezoidal in columns [0, r), zero beyond
 *             (may be NULL)
 *   E       : kmin x m; row echelon, E[t][pivcols[t]] = 1 and zero to its
 *             left; rows [r, kmin) zero (may be NULL)
 *   perm    : n int64; perm[i] = row of A that is row i of P*A
 *   pivcols : kmin int64; pivcols[t] = pivot column of row t, -1 for t >= r
 *   rank    : 1 int64
 * The pivot of each column is the first row, in the current order, at or
 * below the next free position whose reduced entry is 1 (procedure buildZ,
 * Section 4.4), exchanged by a transposition; this makes P unique and equal to
 * that of plain elimination (b = 1, Remark after Lemma 4.1).
 */
int gf2_decompose(const gf2_mat *A, const gf2_mat *L, const gf2_mat *E, int64_t *perm,
                  int64_t *pivcols, int64_t *rank, void *stream);

/*
 * rank(A) = number of rows of E = sum of the panel ranks r_j (Lemma 4.1).
 * rank: device int64.  A matrix with more columns than rows is factored as its
 * transpose (rank A = rank A^T), which needs fewer column panels; its column
 * count must then be below 2^31.
 */
int gf2_rank(const gf2_mat *A, int64_t *rank, void *stream);

/*
 * Solve A*X = B for k right-hand sides at once (column c of B is one system).
 * A: n x m (read only), B: n x k, X: m x k (written).
 * consistent: ceil(k/64) uint64 words, bit c set iff system c is solvable.
 * X column c is the solution whose free (non-pivot) variables are zero, or
 * zero when system c is inconsistent.  rank may be NULL.
 * Method: y = L_top^{-1} (P b)_top; consistent iff L_bot y = (P b)_bot;
 * back-substitution with E (uses of the decomposition, Section 1).
 */
int gf2_solve(const gf2_mat *A, const gf2_mat *B, const gf2_mat *X, uint64_t *consistent,
              int64_t *rank, void *stream);

/*
 * Reduced row echelon form: R (min(n,m) x m) = E of gf2_decompose with every
 * pivot column cleared above its pivot (rows >= rank zero).  pivcols
 * (min(n,m) int64, -1 beyond the rank) and rank (1 int64) as in
 * gf2_decompose.  R, pivcols and rank may each be NULL.  A must not be empty.
 * Method: R = U^-1 E with U = E restricted to the pivot columns, bottom-up in
 * blocks of 512 pivot rows (back-substitution inside a block, then one
 * Four-Russians product per block for the rows above it).
 */
int gf2_rref(const gf2_mat *A, const gf2_mat *R, int64_t *pivcols, int64_t *rank, void *stream);

/*
 * Null space of A (n x m), the use of the echelon form named in Section 1.
 * N (m x m, caller allocated): row j < nullity = m - rank is the vector x of
 * the j-th free (non-pivot) column f_j in increasing order -- x_{f_j} = 1,
 * every other free variable 0, x_{p_t} = R[t][f_j] -- so A x = 0; rows from
 * nullity on are written as zero.  nullity: 1 int64.  A must not be empty.
 */
int gf2_nullspace(const gf2_mat *A, const gf2_mat *N, int64_t *nullity, void *stream);

/*
 * Inverse of a square A (n x n, n >= 1) over GF(2): X (n x n, caller
 * allocated) with A*X = X*A = I.  Section 4.2 builds such inverses for the
 * pivot blocks; here the whole matrix is done as the reduced echelon form of
 * [A | I] (the decomposition of the n x 2n matrix, then the upward elimination
 * of gf2_rref), which is [I | A^-1] exactly when A is invertible.
 * invertible: optional device uint64, set to 1 or 0.  A singular A gives X = 0.
 * Errors: GF2_EINVAL for a non-square or empty A or a mis-shaped X.
 */
int gf2_inverse(const gf2_mat *A, const gf2_mat *X, uint64_t *invertible, void *stream);

/*
 * ---------------------------------------------------------------- batches
 * Many independent matrices of at most GF2_BATCH_MAX_DIM rows and columns,
 * each of its own shape, factored (and solved) in one launch.  The matrices
 * and results live in caller-owned device pools; item i of the host array
 * `items` gives matrix i's shape and the offsets of its pieces.  Every piece is
 * plain row-major: a row of c columns is ceil(c/64) words, element j of a row
 * is bit j % 64 of word j / 64 (Section 3's bit order), padding bits are
 * ignored on input and written as zero.  With kmin_i = min(rows, cols):
 */
#define GF2_BATCH_MAX_DIM 2048

typedef struct gf2_batch_item {
  int64_t rows; /* n_i, 0 <= n_i <= GF2_BATCH_MAX_DIM                          */
  int64_t cols; /* m_i, 0 <= m_i <= GF2_BATCH_MAX_DIM                          */
  int64_t a;    /* A_i at A + a: n_i rows of ceil(m_i/64) words                 */
  int64_t l;    /* L_i at L + l: n_i rows of ceil(kmin_i/64) words              */
  int64_t e;    /* E_i at E + e: kmin_i rows of ceil(m_i/64) words              */
  int64_t p;    /* perm_i at perm + p: n_i int64                               */
  int64_t c;    /* pivcols_i at pivcols + c: kmin_i int64                      */
  int64_t b;    /* b_i at B + b: ceil(n_i/64) words, bit i of the vector is     */
                /* bit i % 64 of word i / 64 (gf2_solve_batched only)           */
  int64_t x;    /* x_i at X + x: ceil(m_i/64) words (gf2_solve_batched only)    */
} gf2_batch_item;

/*
 * P_i*A_i = L_i*E_i for every item, with the meaning of gf2_decompose (same
 * pivots, same L, E, perm, pivcols).  rank[i] (int64, caller order) receives
 * the rank of item i.  L, E, perm and pivcols may each be NULL (not written);
 * A and rank are required.  The items are taken largest first by one
 * persistent launch in which each workgroup factors whole matrices (Section 4
 * with 64-column panels, 4-bit Four-Russians trailing updates of Section 6).
 * Errors: GF2_EINVAL for count < 0, a null required pointer, a shape outside
 * [0, GF2_BATCH_MAX_DIM] or a negative offset (checked on the host before any
 * launch; pools are not bounds-checked against the offsets).
 */
int gf2_decompose_batched(const gf2_batch_item *items, int64_t count, const uint64_t *A,
                          uint64_t *L, uint64_t *E, int64_t *perm, int64_t *pivcols,
                          int64_t *rank, void *stream);

/*
 * Solve A_i x = b_i for every item from the outputs of gf2_decompose_batched
 * (L, E, perm, pivcols, rank for the same items and pools): y = L_top^{-1}
 * (P b)_top, consistent iff L_bot y = (P b)_bot, then x by back-substitution
 * with E, free (non-pivot) variables zero (the uses of the decomposition in
 * Section 1).  consistent[i] (int32, caller order) is 1 or 0; x_i is zero when
 * system i is inconsistent.  All pointers are required; errors as above.
 */
int gf2_solve_batched(const gf2_batch_item *items, int64_t count, const uint64_t *L,
                      const uint64_t *E, const int64_t *perm, const int64_t *pivcols,
                      const int64_t *rank, const uint64_t *B, uint64_t *X, int32_t *consistent,
                      void *stream);

/*
 * Autotuner (process-wide, per device of the calling thread).  Times the
 * product-kernel tile variants on synthetic operands for every size class --
 * active rows in [256 * 2^r, 512 * 2^r) (r = 0..8, up to max_size) crossed with
 * 1, 2-3, 4-15 or 16+ column blocks of 1024 bits, at the decomposition's
 * 512-bit inner dimension -- and one Strassen-Winograd level against the plain
 * product at 32768^3 and 65536^3 (up to max_size); afterwards the trailing
 * update and gf2_matmul use the fastest tile of each class and the measured
 * cutoff (the smallest size where one level paid, else twice the largest size
 * compared).  Then it times one decomposition of a random square matrix of
 * 2048, 16384 and 32768 bits (up to max_size) for each panel width W = 2, 4,
 * 8; the fastest becomes the width of the size class (see
 * gf2_autotune_params).  No result of any call depends on it.  Allocates its
 * operands with hipMalloc (up to about 3.5 GB at max_size >= 65536) and
 * synchronises `stream`.  GF2_EINVAL for max_size < 256.
 */
int gf2_autotune(int64_t max_size, void *stream);

/*
 * The tuned tiles, row-major over (row class r, block class c):
 * variants[4 * r + c] for r < 9, c < 4 (-1 everywhere before gf2_autotune),
 * and the Strassen cutoff in use.  Either pointer (host memory) may be NULL.
 */
int gf2_autotune_table(int32_t *variants, int64_t *strassen_cutoff);

/*
 * The parameters an n x m decomposition uses now, beside Section 6's analytic
 * choices (host pointers, each may be NULL):
 *   panel_words          W, sub-panels of 64 columns per trailing-update panel:
 *                        the "panel_words" knob when set, else the width
 *                        gf2_autotune measured for the size class of max(n, m)
 *                        (<= 4096, <= 16384, larger) while "autotuned" is 1,
 *                        else 8;
 *   table_bits           c of the trailing-update product's tables (8: 2^8
 *                        entries per 8 inner bits; the batched kernel uses
 *                        c = 4 and one-word panels);
 *   analytic_table_bits  the c minimising C(b, c, n) = (b/c)(2^c - 1 + n) for
 *                        that product (b = 64 W inner bits, n = rows), the
 *                        paper's choice of table size;
 *   analytic_strassen    44c + 6(2^c - 1) at c = table_bits, the size from
 *                        which the paper's cost model makes one Strassen-
 *                        Winograd level pay (the measured cutoff is reported
 *                        by gf2_autotune_table).
 * GF2_EINVAL for negative sizes.
 */
int gf2_autotune_params(int64_t rows, int64_t cols, int32_t *panel_words, int32_t *table_bits,
                        int32_t *analytic_table_bits, int64_t *analytic_strassen);

/*
 * Tuning knobs, process-wide (no knob changes any result):
 *   "panel_words"        : W, sub-panels of 64 columns per trailing-update panel
 *                          (1..8; 0 = automatic, the default: the width measured by
 *                          gf2_autotune for the size class while "autotuned" is 1,
 *                          else 8)
 *   "strassen_cutoff"    : gf2_matmul recurses with Strassen-Winograd (one level
 *                          per halving) while every dimension of the current
 *                          product is at least this many bits (default 65536; 0 = never)
 *   "gemm_variant"       : product-kernel variant for gf2_matmul (-1 = automatic;
 *                          0..5 Four-Russians kernels -- 0..3 tiles of 2048, 1024,
 *                          512, 256 rows x 16 words, 4..5 tiles of 256, 512 rows x
 *                          8 words --, 6 the fp4 matrix-core product, chosen
 *                          automatically when k >= 1024 and the output has fewer
 *                          1024 x 1024 tiles than the device has CUs)
 *   "panel_gemm_variant" : product-kernel variant for the trailing update (-1 = automatic)
 *   "chain_cus"          : must be 0 (CU-masked chain streams are not supported)
 *   "autotuned"          : 1 = use the table measured by gf2_autotune (its
 *                          default once measured), 0 = the built-in tile rule
 *   "overlap_lookups"    : size of a panel's bulk update (table lookups) from
 *                          which it starts concurrently with the next panel's
 *                          columns rather than after them (default 3e8; 0: always)
 *   "post_follow_lookups": size of a panel's bulk update (table lookups) from
 *                          which the next panel's row exchanges and pivot-row
 *                          solve run on the bulk update's stream right after it
 *                          (default 1.5e9; -1 = never, 0 = always)
 *   "wall_tiles"         : trailing-update tiles that minimise rounds x a fitted
 *                          step time instead of the largest tile filling the CUs:
 *                          0 = never, 1 = always (default), 2 = for launches
 *                          of at most 16384 active rows where that tile fits
 *                          the CUs in one round
 * Returns 0, or GF2_EINVAL for an unknown name or out-of-range value.
 */
int gf2_set_param(const char *name, int64_t value);

/*
 * Timing of the dominant kernel (the trailing-update product, the hot path of
 * Section 6.3).  While enabled, the library brackets each of its launches with
 * HIP events on the launch stream; gf2_profile_read() synchronizes them and
 * returns the summed kernel time (ms), the number of launches and the summed
 * algorithmic work in table lookups (one 64-bit lookup-XOR per 8 bits of the
 * inner dimension per output word).  Enabling resets the counters.
 */
int gf2_profile(int enable);
int gf2_profile_read(double *ms, int64_t *launches, double *lookups);

/*
 * Microbenchmarks of the units the kernels depend on, for comparing measured
 * ceilings with nominal ones (not part of the decomposition path).  kind:
 *   0 HBM read of `bytes` (16-byte loads)   -> *rate in bytes/s
 *   1 HBM copy of bytes/2 into bytes/2      -> bytes/s (read + written)
 *   2 32-bit VALU exclusive-or, `iters`     -> operations/s (one per lane per instruction)
 *   3 LDS 16-byte reads, conflict-free      -> bytes/s
 *   4 int8 matrix cores (32x32x32)          -> multiply-accumulates/s
 *   5 fp4 (e2m1) matrix cores (32x32x64)    -> multiply-accumulates/s
 * bytes (kinds 0, 1): a positive multiple of 65536, allocated and freed by the
 * call; iters (kinds 2..5): 1 .. 2^24 loop trips per thread.  *ms is the mean
 * time of three launches after one warm-up, HIP events on `stream`; the call
 * synchronizes it.  Returns 0, GF2_EINVAL for a bad kind, size or null output
 * (nothing launched), or GF2_EHIP / GF2_ENOMEM.
 */
int gf2_microbench(int kind, int64_t bytes, int iters, double *rate, double *ms, void *stream);

/*
 * ---------------------------------------------------------------- caller workspace
 * Device bytes of workspace a call needs (the working copy of the matrix in
 * the column-blocked layout of Section 3, the per-panel state of the block
 * decomposition of Section 4, product operands and Strassen temporaries):
 *   GF2_OP_MATMUL            C rows x cols, inner dimension k (with the current
 *                            strassen_cutoff and gemm_variant settings)
 *   GF2_OP_DECOMPOSE         A rows x cols (k ignored); also gf2_decompose_noalloc
 *   GF2_OP_RANK              A rows x cols (k ignored)
 *   GF2_OP_SOLVE             A rows x cols, k right-hand sides
 *   GF2_OP_DECOMPOSE_BATCHED rows = number of items, cols and k = the largest
 *                            item's columns and rows (at most GF2_BATCH_MAX_DIM)
 *   GF2_OP_SOLVE_BATCHED     rows = number of items (cols, k ignored)
 * The sizes depend on the current device (its CU count) and knobs only through
 * the choices named above.  Returns SIZE_MAX (and sets gf2_last_error) for an
 * unknown op or a negative or out-of-range size.
 */
#define GF2_OP_MATMUL 0
#define GF2_OP_DECOMPOSE 1
#define GF2_OP_RANK 2
#define GF2_OP_SOLVE 3
#define GF2_OP_DECOMPOSE_BATCHED 4
#define GF2_OP_SOLVE_BATCHED 5
size_t gf2_workspace_bytes(int op, int64_t rows, int64_t cols, int64_t k);

/*
 * The calls above with a caller-owned workspace: `workspace` is device memory,
 * 256-byte aligned, of at least gf2_workspace_bytes(op, ...) bytes; the library
 * neither allocates nor frees it and keeps nothing in it between calls.  These
 * forms never allocate device memory and never synchronise the device (the
 * look-ahead streams and events of a caller stream are created once, on its
 * first call).  Two calls whose work overlaps in time must not share a
 * workspace.  Results are identical to the allocating forms.  Errors as those,
 * plus GF2_EINVAL for a null, misaligned or too small workspace.
 */
int gf2_matmul_ws(const gf2_mat *C, const gf2_mat *A, const gf2_mat *B, int accumulate, void *workspace,
                  size_t workspace_bytes, void *stream);
int gf2_decompose_ws(const gf2_mat *A, const gf2_mat *L, const gf2_mat *E, int64_t *perm, int64_t *pivcols,
                     int64_t *rank, void *workspace, size_t workspace_bytes, void *stream);
int gf2_rank_ws(const gf2_mat *A, int64_t *rank, void *workspace, size_t workspace_bytes, void *stream);
int gf2_solve_ws(const gf2_mat *A, const gf2_mat *B, const gf2_mat *X, uint64_t *consistent, int64_t *rank,
                 void *workspace, size_t workspace_bytes, void *stream);
int gf2_decompose_batched_ws(const gf2_batch_item *items, int64_t count, const uint64_t *A, uint64_t *L, uint64_t *E,
                             int64_t *perm, int64_t *pivcols, int64_t *rank, void *workspace,
                             size_t workspace_bytes, void *stream);
int gf2_solve_batched_ws(const gf2_batch_item *items, int64_t count, const uint64_t *L, const uint64_t *E,
                         const int64_t *perm, const int64_t *pivcols, const int64_t *rank, const uint64_t *B,
                         uint64_t *X, int32_t *consistent, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Allocation-free decomposition, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, outputs and errors as gf2_decompose, but
 * the working state lives in a static device array of GF2_NOALLOC_MAX_BYTES
 * that the library holds on every GPU it runs on until the process ends, and
 * every launch goes in order onto `stream`: the call makes no hipMalloc, no
 * hipFree, creates no stream or event and records no profiling event.
 * GF2_EINVAL if the working state of an n x m decomposition
 * (gf2_workspace_bytes(GF2_OP_DECOMPOSE, n, m)) exceeds GF2_NOALLOC_MAX_BYTES
 * (16384 x 16384 fits).  All calls on one GPU share that GPU's array: calls
 * that overlap in time on one GPU (other streams, other host threads) race
 * and give wrong results; calls ordered on one stream are safe.
 */
#define GF2_NOALLOC_MAX_BYTES ((size_t)36 << 20)
int gf2_decompose_noalloc(const gf2_mat *A, const gf2_mat *L, const gf2_mat *E, int64_t *perm, int64_t *pivcols,
                          int64_t *rank, void *stream);

/*
 * Captured decomposition.  gf2_decompose_graph records one gf2_decompose_ws
 * call with these arguments into a HIP graph (stream capture on `stream`,
 * which must not be the null stream; every launch in order on that stream,
 * without the look-ahead streams) and instantiates it; nothing runs and
 * nothing is allocated on the device.
 * gf2_graph_launch replays the whole decomposition on `stream` with the same
 * pointers: the caller refills A between replays, and every output and the
 * workspace are rewritten by each replay (the workspace must stay allocated
 * and must not be used by other calls while a replay runs).  Errors as
 * gf2_decompose_ws, plus GF2_EHIP when capture or instantiation fails.
 * gf2_graph_destroy releases the graph (NULL is accepted).
 */
typedef struct gf2_graph_s *gf2_graph;
int gf2_decompose_graph(const gf2_mat *A, const gf2_mat *L, const gf2_mat *E, int64_t *perm, int64_t *pivcols,
                        int64_t *rank, void *workspace, size_t workspace_bytes, void *stream, gf2_graph *graph);
int gf2_graph_launch(gf2_graph graph, void *stream);
int gf2_graph_destroy(gf2_graph graph);

/* Free the library-owned workspace, look-ahead streams and events of every
 * device (after synchronising those devices).  Safe to call at any time
 * between calls; later calls create what they need again. */
int gf2_release(void);

/* Message of the last failing call on this thread ("" if none). */
const char *gf2_last_error(void);

/* Library version string. */
const char *gf2_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GF2_H */
