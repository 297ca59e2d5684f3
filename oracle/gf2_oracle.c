/*
 * gf2_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct CPU reference for dense GF(2) linear algebra.
 * Only tests/, the smoke check and the bench's cpu_baseline leg may load it;
 * the GPU library never links, includes or calls anything from this file.
 *
 * Storage here is plain row-major bit rows: row i, word j at A[i*wpr + j],
 * column c is bit (c mod 64) of word c/64 (weight 2^(c mod 64)).  This is the
 * bit order of Section 3 of the paper (element a_ij is bit r of word q where
 * j = q*b + r), with b = 64 and the whole row in one block.
 *
 * What is computed:
 *  - or_ple:    the decomposition P*A = L*E of Lemma 4.1 in the form the
 *               paper's Remark after Lemma 4.1 names for b = 1 (PLE): columns
 *               are taken strictly left to right and never swapped; the pivot
 *               for column k is the first row, in the current order, at or
 *               below the next free position whose (already reduced) bit k is
 *               set (the row search of procedure buildZ, Section 4.4); that
 *               row is exchanged with the free position by a transposition;
 *               every later row with bit k set is reduced by it (the Schur
 *               complement update, eq. (Aj), with b = 1).  L records the
 *               multipliers, E the reduced pivot rows, rank = number of pivots
 *               (rank = sum of r_j, Lemma 4.1).
 *  - or_matmul: C (^)= A*B straight from the definition of the product:
 *               row i of C is the XOR of the rows t of B with A[i][t] = 1.
 *  - or_solve:  A*x = b by the decomposition (uses listed in the paper's
 *               introduction: rank, systems): y = L_top^{-1} (P b)_top,
 *               consistent iff L_bot*y = (P b)_bot, x the solution whose
 *               non-pivot (free) variables are zero.
 *  - or_inverse: the inverse of a square non-singular matrix over F2 (Section
 *               4.2 builds it for the pivot blocks; here for a whole matrix)
 *               from its definition A*X = I, by Gauss-Jordan elimination of
 *               [A | I].
 *
 * No blocking, tables or reordering beyond what those definitions state.
 * The optional OpenMP loop only splits the independent row reductions of one
 * elimination step; it cannot change any result.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static inline int64_t wpr_of(int64_t bits) { return (bits + 63) / 64; }

static inline int getbit(const uint64_t *row, int64_t c) {
  return (int)((row[c >> 6] >> (c & 63)) & 1u);
}

static inline void setbit(uint64_t *row, int64_t c) { row[c >> 6] |= (uint64_t)1 << (c & 63); }

static void swap_rows(uint64_t *M, int64_t wpr, int64_t a, int64_t b) {
  if (a == b) return;
  for (int64_t j = 0; j < wpr; ++j) {
    uint64_t t = M[a * wpr + j];
    M[a * wpr + j] = M[b * wpr + j];
    M[b * wpr + j] = t;
  }
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/*
 * PLE decomposition (b = 1 form of Lemma 4.1).
 *   A       : n x m, row-major, wpr(m) words per row (read only)
 *   E       : out, kmin x m (kmin = min(n,m)), wpr(m) words per row; rows >= rank zero
 *   L       : out, n x kmin, wpr(kmin) words per row; unit lower trapezoidal in
 *             columns < rank, columns >= rank zero
 *   perm    : out, n entries; perm[i] = row of A that is row i of P*A
 *   pivcols : out, kmin entries; pivcols[t] = column of pivot t, -1 for t >= rank
 * Returns rank, or -1 if memory ran out.  E or L may be NULL (rank only).
 */
int64_t or_ple(int64_t n, int64_t m, const uint64_t *A, uint64_t *E, uint64_t *L,
               int64_t *perm, int64_t *pivcols) {
  const int64_t wm = wpr_of(m);
  const int64_t kmin = n < m ? n : m;
  const int64_t wl = wpr_of(n > 0 ? n : 1);
  uint64_t *R = (uint64_t *)malloc((size_t)(n * wm + 1) * sizeof(uint64_t));
  uint64_t *Lr = (uint64_t *)calloc((size_t)(n * wl + 1), sizeof(uint64_t));
  int64_t *pv = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
  if (!R || !Lr || !pv) { free(R); free(Lr); free(pv); return -1; }
  memcpy(R, A, (size_t)(n * wm) * sizeof(uint64_t));
  for (int64_t i = 0; i < n; ++i) pv[i] = i;

  int64_t ib = 0;                                   /* next free pivot position */
  for (int64_t k = 0; k < m && ib < n; ++k) {
    int64_t piv = -1;
    for (int64_t i = ib; i < n; ++i)                /* first row in current order */
      if (getbit(R + i * wm, k)) { piv = i; break; }
    if (piv < 0) continue;                          /* column k has no pivot */
    swap_rows(R, wm, piv, ib);                      /* transposition piv <-> ib */
    swap_rows(Lr, wl, piv, ib);
    { int64_t t = pv[piv]; pv[piv] = pv[ib]; pv[ib] = t; }
    if (pivcols && ib < kmin) pivcols[ib] = k;
    setbit(Lr + ib * wl, ib);                       /* unit diagonal */
    const uint64_t *prow = R + ib * wm;
    const int64_t w0 = k >> 6;                      /* bits left of k are zero in prow */
    const int64_t t = ib;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if (n - ib > 4096)
#endif
    for (int64_t l = ib + 1; l < n; ++l) {
      uint64_t *row = R + l * wm;
      if (getbit(row, k)) {
        for (int64_t j = w0; j < wm; ++j) row[j] ^= prow[j];
        setbit(Lr + l * wl, t);
      }
    }
    ++ib;
  }
  const int64_t rank = ib;

  if (perm) memcpy(perm, pv, (size_t)n * sizeof(int64_t));
  if (pivcols) for (int64_t t = rank; t < kmin; ++t) pivcols[t] = -1;
  if (E) {
    memset(E, 0, (size_t)(kmin * wm) * sizeof(uint64_t));
    memcpy(E, R, (size_t)(rank * wm) * sizeof(uint64_t));
  }
  if (L) {
    const int64_t wk = wpr_of(kmin > 0 ? kmin : 1);
    memset(L, 0, (size_t)(n * wk) * sizeof(uint64_t));
    for (int64_t i = 0; i < n; ++i)
      for (int64_t t = 0; t < rank; ++t)
        if (getbit(Lr + i * wl, t)) setbit(L + i * wk, t);
  }
  free(R); free(Lr); free(pv);
  return rank;
}

/*
 * Null space of A (n x m), the use of the row-echelon form named in Section 1.
 * From the PLE's echelon rows E (rank r, pivot columns p_t): the reduced row
 * echelon form R by back-substitution (pivot row t, from the last to the first,
 * reduced by every later pivot row u whose pivot column p_u it has a 1 in);
 * then, for the j-th free (non-pivot) column f_j in increasing order, the
 * vector x with x_{f_j} = 1, every other free variable 0 and x_{p_t} = R[t][f_j],
 * the unique solution of R x = 0 with that choice of free variables.
 *   N : out, (m - r) rows of wpr(m) words (NULL: not written)
 *   R : out, kmin x m, wpr(m) words per row; rows >= r zero (NULL: not written)
 * Returns the nullity m - r, or -1 on allocation failure.
 */
int64_t or_nullspace(int64_t n, int64_t m, const uint64_t *A, uint64_t *N, uint64_t *R) {
  const int64_t wm = wpr_of(m);
  const int64_t kmin = n < m ? n : m;
  uint64_t *E = (uint64_t *)calloc((size_t)(kmin * wm + 1), sizeof(uint64_t));
  int64_t *piv = (int64_t *)malloc((size_t)(kmin + 1) * sizeof(int64_t));
  uint8_t *is_piv = (uint8_t *)calloc((size_t)(m + 1), 1);
  if (!E || !piv || !is_piv) { free(E); free(piv); free(is_piv); return -1; }
  const int64_t r = or_ple(n, m, A, E, NULL, NULL, piv);
  if (r < 0) { free(E); free(piv); free(is_piv); return -1; }
  for (int64_t t = r - 1; t >= 0; --t) {           /* back-substitution, bottom up */
    uint64_t *row = E + t * wm;
    for (int64_t u = t + 1; u < r; ++u)
      if (getbit(row, piv[u])) {
        const uint64_t *ru = E + u * wm;
        for (int64_t j = 0; j < wm; ++j) row[j] ^= ru[j];
      }
  }
  if (R) memcpy(R, E, (size_t)(kmin * wm) * sizeof(uint64_t));
  for (int64_t t = 0; t < r; ++t) is_piv[piv[t]] = 1;
  if (N) {
    memset(N, 0, (size_t)((m - r) * wm) * sizeof(uint64_t));
    int64_t j = 0;
    for (int64_t f = 0; f < m; ++f) {
      if (is_piv[f]) continue;
      uint64_t *x = N + j * wm;
      setbit(x, f);
      for (int64_t t = 0; t < r; ++t)
        if (getbit(E + t * wm, f)) setbit(x, piv[t]);
      ++j;
    }
  }
  free(E); free(piv); free(is_piv);
  return m - r;
}

/* Inverse of a square A (n x n): X with A*X = I, from its definition by
 * Gauss-Jordan elimination of [A | I]: for each column c in order, the first
 * row at or below c with bit c set is exchanged into row c and every other row
 * with bit c set is reduced by it; A is singular when some column has no such
 * row.  Then [A | I] has become [I | X].
 *   X : out, n x n, wpr(n) words per row; all zero when A is singular
 * Returns 1 (invertible), 0 (singular) or -1 on allocation failure. */
int64_t or_inverse(int64_t n, const uint64_t *A, uint64_t *X) {
  const int64_t wn = wpr_of(n), w2 = wpr_of(2 * n);
  uint64_t *M = (uint64_t *)calloc((size_t)(n * w2 + 1), sizeof(uint64_t));
  if (!M) return -1;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t c = 0; c < n; ++c)
      if (getbit(A + i * wn, c)) setbit(M + i * w2, c);
    setbit(M + i * w2, n + i);
  }
  int64_t ok = 1;
  for (int64_t c = 0; c < n && ok; ++c) {
    int64_t p = c;
    while (p < n && !getbit(M + p * w2, c)) ++p;
    if (p == n) { ok = 0; break; }
    swap_rows(M, w2, c, p);
    const uint64_t *pr = M + c * w2;
    for (int64_t i = 0; i < n; ++i)
      if (i != c && getbit(M + i * w2, c))
        for (int64_t j = 0; j < w2; ++j) M[i * w2 + j] ^= pr[j];
  }
  memset(X, 0, (size_t)(n * wn) * sizeof(uint64_t));
  if (ok)
    for (int64_t i = 0; i < n; ++i)
      for (int64_t c = 0; c < n; ++c)
        if (getbit(M + i * w2, n + c)) setbit(X + i * wn, c);
  free(M);
  return ok;
}

/* C = A*B (accumulate = 0) or C ^= A*B (accumulate != 0).
 * A: n x k (wpr(k) words/row), B: k x m (wpr(m)), C: n x m (wpr(m)). */
void or_matmul(int64_t n, int64_t k, int64_t m, const uint64_t *A, const uint64_t *B,
               uint64_t *C, int accumulate) {
  const int64_t wk = wpr_of(k), wm = wpr_of(m);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if (n * k > (1 << 20))
#endif
  for (int64_t i = 0; i < n; ++i) {
    uint64_t *c = C + i * wm;
    if (!accumulate) memset(c, 0, (size_t)wm * sizeof(uint64_t));
    const uint64_t *a = A + i * wk;
    for (int64_t t = 0; t < k; ++t)
      if (getbit(a, t)) {
        const uint64_t *b = B + t * wm;
        for (int64_t j = 0; j < wm; ++j) c[j] ^= b[j];
      }
  }
}

/*
 * Solve A*X = B for nrhs right-hand sides at once (column c of B is one
 * system).  A: n x m, B: n x nrhs (wpr(nrhs) words/row), X: out m x nrhs,
 * consistent: out wpr(nrhs) words, bit c set iff system c has a solution.
 * Columns of X for inconsistent systems are zero.  Returns rank or -1.
 */
int64_t or_solve(int64_t n, int64_t m, int64_t nrhs, const uint64_t *A, const uint64_t *B,
                 uint64_t *X, uint64_t *consistent) {
  const int64_t kmin = n < m ? n : m;
  const int64_t wm = wpr_of(m), wk = wpr_of(kmin > 0 ? kmin : 1), wr = wpr_of(nrhs);
  uint64_t *E = (uint64_t *)calloc((size_t)(kmin * wm + 1), sizeof(uint64_t));
  uint64_t *L = (uint64_t *)calloc((size_t)(n * wk + 1), sizeof(uint64_t));
  int64_t *perm = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
  int64_t *piv = (int64_t *)malloc((size_t)(kmin + 1) * sizeof(int64_t));
  uint64_t *Y = (uint64_t *)calloc((size_t)(n * wr + 1), sizeof(uint64_t));
  if (!E || !L || !perm || !piv || !Y) {
    free(E); free(L); free(perm); free(piv); free(Y);
    return -1;
  }
  const int64_t r = or_ple(n, m, A, E, L, perm, piv);
  if (r < 0) { free(E); free(L); free(perm); free(piv); free(Y); return -1; }

  /* Y = P*B */
  for (int64_t i = 0; i < n; ++i)
    memcpy(Y + i * wr, B + perm[i] * wr, (size_t)wr * sizeof(uint64_t));
  /* forward substitution with the unit lower triangular L_top (r x r) */
  for (int64_t t = 0; t < r; ++t)
    for (int64_t s = 0; s < t; ++s)
      if (getbit(L + t * wk, s))
        for (int64_t j = 0; j < wr; ++j) Y[t * wr + j] ^= Y[s * wr + j];
  /* consistency: residual of the rows below the rank */
  uint64_t *bad = (uint64_t *)calloc((size_t)(wr + 1), sizeof(uint64_t));
  for (int64_t i = r; i < n; ++i) {
    for (int64_t j = 0; j < wr; ++j) {
      uint64_t v = Y[i * wr + j];
      for (int64_t s = 0; s < r; ++s)
        if (getbit(L + i * wk, s)) v ^= Y[s * wr + j];
      bad[j] |= v;
    }
  }
  for (int64_t j = 0; j < wr; ++j) {
    uint64_t valid = (j == wr - 1 && (nrhs & 63)) ? (((uint64_t)1 << (nrhs & 63)) - 1) : ~(uint64_t)0;
    consistent[j] = ~bad[j] & valid;
  }
  /* back substitution with E (row echelon), free variables zero */
  memset(X, 0, (size_t)(m * wr) * sizeof(uint64_t));
  for (int64_t t = r - 1; t >= 0; --t) {
    uint64_t *xt = X + piv[t] * wr;
    for (int64_t j = 0; j < wr; ++j) xt[j] = Y[t * wr + j];
    for (int64_t s = t + 1; s < r; ++s)
      if (getbit(E + t * wm, piv[s]))
        for (int64_t j = 0; j < wr; ++j) xt[j] ^= X[piv[s] * wr + j];
  }
  /* zero the columns of inconsistent systems */
  for (int64_t c = 0; c < m; ++c)
    for (int64_t j = 0; j < wr; ++j) X[c * wr + j] &= consistent[j];
  free(bad); free(E); free(L); free(perm); free(piv); free(Y);
  return r;
}
