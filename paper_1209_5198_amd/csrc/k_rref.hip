// k_rref.hip -- reduced row echelon form and null space from the decomposition.
//
// The row-echelon form E of P*A = L*E (rank r, pivot columns p_t) gives the
// null space of A, the use named in Section 1: with R the reduced row echelon
// form (E with every pivot column cleared above its pivot), the vector of the
// j-th free column f_j has x_{f_j} = 1, every other free variable 0 and
// x_{p_t} = R[t][f_j].
//
// R = U^-1 E with U = E restricted to the pivot columns (r x r, upper
// unitriangular), computed bottom-up in blocks of 512 pivot rows: the diagonal
// block's rows are solved by back-substitution over its 64-row sub-blocks
// (4-bit tables, one workgroup per 16-word column block), then every row above
// the block gets E_above ^= U_above,J * R_J -- a Four-Russians product with a
// 512-bit inner dimension on the same kernel as the trailing update.
#include "gf2_internal.h"

namespace gf2 {
namespace {

// G[t][u] = E[t][p_u] for t, u < r (zero elsewhere): one thread per (row, word) of G
__global__ void k_gather_pivcols(const uint64_t *E, int64_t ldE, const int64_t *pivcols, const int64_t *rankp,
                                 uint64_t *G, int64_t kmin, int64_t Gw) {
  const int64_t r = *rankp;
  const size_t total = (size_t)kmin * (size_t)Gw;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int64_t t = (int64_t)(e % (size_t)kmin), w = (int64_t)(e / (size_t)kmin);
    uint64_t v = 0ull;
    if (t < r) {
      for (int j = 0; j < 64; ++j) {
        const int64_t u = 64 * w + j;
        if (u >= r) break;
        const int64_t c = pivcols[u];
        v |= ((E[widx(ldE, t, c >> 6)] >> (c & 63)) & 1ull) << j;
      }
    }
    G[widx(ldE, t, w)] = v;
  }
}

constexpr int kRT = 1024;  // threads of the diagonal-block kernel

struct DiagShared {
  uint64_t X[512][TW];     // 64 KB: the block's rows, this column block
  uint64_t T[16][16][TW];  // 32 KB: 4-bit tables
  uint64_t Uo[512][8];     // 32 KB: U_cb = G[rows of c][word of b] (b > c)
  uint64_t Ui[8][64];      // 4 KB: inverse of each 64 x 64 diagonal block
  int rb[8];
};

// Rows [512 J, 512 J + 512) of E (those below rank r excluded), column block
// blk: back-substitution X_b = U_bb^-1 X_b for b = 7 .. 0, each followed by
// X_c ^= U_cb X_b for the sub-blocks c < b.
__global__ __launch_bounds__(kRT) void k_rref_diag(uint64_t *E, int64_t ldE, const uint64_t *G,
                                                   const int64_t *rankp, int J, int64_t Mw) {
  __shared__ DiagShared sh;
  const int64_t r = *rankp, R0 = 512ll * J;
  if (R0 >= r) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, h = lane >> 4, wl = lane & 15;
  const int blk = blockIdx.x + J / 2;  // the block's rows are zero in words < 8 J
  const int64_t qw = (int64_t)blk * TW + wl;
  const bool qok = qw < Mw;
  if (tid < 8) {
    const int64_t left = r - R0 - 64ll * tid;
    sh.rb[tid] = left >= 64 ? 64 : (left > 0 ? (int)left : 0);
  }
  __syncthreads();
  for (int ri = tid >> 4; ri < 512; ri += kRT / 16) {
    const int b = ri >> 6, t = ri & 63;
    sh.X[ri][wl] = (qok && t < sh.rb[b]) ? E[widx(ldE, R0 + ri, qw)] : 0ull;
  }
  for (int e = tid; e < 512 * 8; e += kRT) {
    const int ri = e >> 3, b = e & 7, c = ri >> 6, t = ri & 63;
    sh.Uo[ri][b] = (b > c && t < sh.rb[c]) ? G[widx(ldE, R0 + ri, 8ll * J + b)] : 0ull;
  }
  __syncthreads();
  // inverse of the upper unitriangular diagonal blocks: wave b, lane = row;
  // rows are finished from the last to the first (row t needs rows u > t)
  if (wv < 8) {
    const int b = wv, rbb = sh.rb[b];
    uint64_t urow = 0ull, inv = 0ull;
    if (lane < rbb) {
      urow = G[widx(ldE, R0 + 64 * b + lane, 8ll * J + b)] & ~((2ull << lane) - 1ull);  // bits above the diagonal
      inv = 1ull << lane;
    }
    for (int u = rbb - 1; u >= 0; --u) {
      const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)inv, u);
      const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(inv >> 32), u);
      const uint64_t iu = ((uint64_t)hi << 32) | lo;
      if ((urow >> u) & 1ull) inv ^= iu;
    }
    sh.Ui[b][lane] = inv;
  }
  __syncthreads();
  auto tables = [&](int b) {  // 16 tables of 16 entries over the 64 rows of X_b
    if (tid < 256) {
      const int g = tid >> 4, c = tid & 15;
      uint64_t v[4];
      for (int j = 0; j < 4; ++j) v[j] = sh.X[64 * b + 4 * g + j][c];
      uint64_t cur = 0ull;
      for (int j = 0; j < 16; ++j) {
        sh.T[g][j ^ (j >> 1)][c] = cur;
        if (j < 15) cur ^= v[__builtin_ctz(j + 1)];
      }
    }
    __syncthreads();
  };
  for (int b = 7; b >= 0; --b) {
    const int rbb = sh.rb[b];
    if (rbb == 0) continue;
    tables(b);
    {
      const int t = 4 * wv + h;  // 16 waves x 4 groups = 64 rows
      if (t < rbb) {
        const uint64_t l = sh.Ui[b][t];
        uint64_t v = 0ull;
#pragma unroll
        for (int g = 0; g < 16; ++g) v ^= sh.T[g][(l >> (4 * g)) & 15u][wl];
        sh.X[64 * b + t][wl] = v;
      }
    }
    __syncthreads();
    if (b == 0) break;
    tables(b);
    for (int ri = 4 * wv + h; ri < 64 * b; ri += kRT / 16) {
      const int c = ri >> 6, t = ri & 63;
      if (t < sh.rb[c]) {
        const uint64_t l = sh.Uo[ri][b];
        uint64_t v = 0ull;
#pragma unroll
        for (int g = 0; g < 16; ++g) v ^= sh.T[g][(l >> (4 * g)) & 15u][wl];
        sh.X[ri][wl] ^= v;
      }
    }
    __syncthreads();
  }
  for (int ri = tid >> 4; ri < 512; ri += kRT / 16) {
    const int b = ri >> 6, t = ri & 63;
    if (qok && t < sh.rb[b]) E[widx(ldE, R0 + ri, qw)] = sh.X[ri][wl];
  }
}

// rows [R0, R0 + 512) of E (zero at and beyond rank r) -> a 512-row operand
__global__ void k_copy_block_rows(const uint64_t *E, int64_t ldE, const int64_t *rankp, int64_t R0, uint64_t *B,
                                  int64_t NB) {
  const int64_t r = *rankp;
  const size_t total = (size_t)NB * 512 * TW;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int64_t q = (int64_t)(e % TW), i = (int64_t)((e / TW) % 512), b = (int64_t)(e / (TW * 512));
    const int64_t row = R0 + i;
    B[e] = row < r ? E[((size_t)b * ldE + row) * TW + q] : 0ull;
  }
}

// pivot bitmap of the columns, first pivot index of each 64-column word (tw0),
// free columns in order; one workgroup
constexpr int kNT = 1024;
__global__ __launch_bounds__(kNT) void k_null_prep(const int64_t *pivcols, const int64_t *rankp, int64_t m,
                                                   uint64_t *bitmap, int64_t *tw0, int64_t *freecols,
                                                   int64_t *nullity) {
  __shared__ int64_t part[kNT];
  const int tid = threadIdx.x;
  const int64_t r = *rankp, Mw = (m + 63) >> 6;
  for (int64_t w = tid; w < Mw; w += kNT) bitmap[w] = 0ull;
  __syncthreads();
  for (int64_t u = tid; u < r; u += kNT) {
    const int64_t c = pivcols[u];
    atomicOr((unsigned long long *)&bitmap[c >> 6], 1ull << (c & 63));
  }
  __threadfence_block();
  __syncthreads();
  // each thread owns a contiguous range of words; exclusive scan of the pivot counts
  const int64_t per = (Mw + kNT - 1) / kNT, w0 = tid * per, w1 = w0 + per < Mw ? w0 + per : Mw;
  int64_t cnt = 0;
  for (int64_t w = w0; w < w1; ++w) cnt += __popcll(bitmap[w]);
  part[tid] = cnt;
  __syncthreads();
  for (int off = 1; off < kNT; off <<= 1) {
    const int64_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int64_t piv_before = part[tid] - cnt;
  for (int64_t w = w0; w < w1; ++w) {
    tw0[w] = piv_before;
    const uint64_t valid = (w == Mw - 1 && (m & 63)) ? ((1ull << (m & 63)) - 1ull) : ~0ull;
    uint64_t fr = ~bitmap[w] & valid;
    int64_t fidx = 64 * w - piv_before;  // free columns before word w
    while (fr) {
      const int b = __builtin_ctzll(fr);
      fr &= fr - 1ull;
      freecols[fidx++] = 64 * w + b;
    }
    piv_before += __popcll(bitmap[w]);
  }
  if (tid == 0) {
    tw0[Mw] = r;
    *nullity = m - r;
  }
}

// Row j of N (j < m - r): the vector of free column f_j; rows j >= m - r zero.
__global__ void k_null_rows(const uint64_t *R, int64_t ldE, const int64_t *pivcols, const int64_t *tw0,
                            const int64_t *freecols, const int64_t *rankp, gf2_mat N) {
  const int64_t m = N.cols, Mw = (m + 63) >> 6, nul = m - *rankp;
  const size_t total = (size_t)N.rows * (size_t)Mw;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int64_t w = (int64_t)(e % (size_t)Mw), j = (int64_t)(e / (size_t)Mw);
    uint64_t v = 0ull;
    if (j < nul) {
      const int64_t f = freecols[j], fw = f >> 6;
      const int fb = (int)(f & 63);
      for (int64_t t = tw0[w]; t < tw0[w + 1]; ++t) {
        const int64_t p = pivcols[t];
        v |= ((R[widx(ldE, t, fw)] >> fb) & 1ull) << (p & 63);
      }
      if (fw == w) v |= 1ull << fb;
    }
    N.data[uidx(N.w, N.ld, j, w)] = v;
  }
}

inline unsigned grid_for(size_t total, int threads) {
  size_t b = (total + threads - 1) / threads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// OR the identity into columns col0 .. col0 + n - 1 of rows 0 .. n - 1 of the
// working layout (one bit per row, so no two threads share a word)
__global__ void k_set_identity(uint64_t *W, int64_t ldw, int64_t n, int64_t col0) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = col0 + i;
    W[widx(ldw, i, c >> 6)] |= 1ull << (c & 63);
  }
}

// The reduced echelon form R of [A | I] (n x 2n) is [I | A^-1] exactly when A is
// invertible, i.e. when the last of the n pivots lies left of column n.  Then X
// = columns n .. 2n - 1 of R, else X = 0; *invertible (optional) gets 1 or 0.
__global__ void k_inverse_out(const uint64_t *R, int64_t ldE, const int64_t *pivcols, int64_t n, gf2_mat X,
                              uint64_t *invertible) {
  const bool inv = pivcols[n - 1] < n;
  if (invertible && blockIdx.x == 0 && threadIdx.x == 0) *invertible = inv ? 1ull : 0ull;
  const int64_t Xw = (n + 63) / 64, Rw = (2 * n + 63) / 64, total = n * Xw;
  const int sh = (int)(n & 63);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / Xw, q = e - i * Xw, wd = (n >> 6) + q;
    uint64_t v = 0ull;
    if (inv) {
      v = R[widx(ldE, i, wd)] >> sh;
      if (sh && wd + 1 < Rw) v |= R[widx(ldE, i, wd + 1)] << (64 - sh);
    }
    X.data[uidx(X.w, X.ld, i, q)] = v & pad_mask(n, q);
  }
}

}  // namespace

hipError_t launch_set_identity(uint64_t *W, int64_t ldw, int64_t n, int64_t col0, hipStream_t s) {
  hipLaunchKernelGGL(k_set_identity, dim3(grid_for((size_t)n, 256)), dim3(256), 0, s, W, ldw, n, col0);
  return hipGetLastError();
}

hipError_t launch_inverse_out(const uint64_t *R, int64_t ldE, const int64_t *pivcols, int64_t n, const gf2_mat &X,
                              uint64_t *invertible, hipStream_t s) {
  const size_t total = (size_t)n * (size_t)((n + 63) / 64);
  hipLaunchKernelGGL(k_inverse_out, dim3(grid_for(total, 256)), dim3(256), 0, s, R, ldE, pivcols, n, X, invertible);
  return hipGetLastError();
}

hipError_t launch_gather_pivcols(const uint64_t *E, int64_t ldE, const int64_t *pivcols, const int64_t *rankp,
                                 uint64_t *G, int64_t kmin, int64_t Gw, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_pivcols, dim3(grid_for((size_t)kmin * Gw, 256)), dim3(256), 0, s, E, ldE, pivcols,
                     rankp, G, kmin, Gw);
  return hipGetLastError();
}

hipError_t launch_rref_diag(uint64_t *E, int64_t ldE, const uint64_t *G, const int64_t *rankp, int J, int64_t Mw,
                            hipStream_t s) {
  const int64_t nbe = (Mw + TW - 1) / TW;  // column blocks from J / 2 on (words >= 8 J)
  if (nbe <= J / 2) return hipSuccess;
  const unsigned nb = (unsigned)(nbe - J / 2);
  hipLaunchKernelGGL(k_rref_diag, dim3(nb), dim3(kRT), 0, s, E, ldE, G, rankp, J, Mw);
  return hipGetLastError();
}

hipError_t launch_copy_block_rows(const uint64_t *E, int64_t ldE, const int64_t *rankp, int64_t R0, uint64_t *B,
                                  int64_t NB, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_block_rows, dim3(grid_for((size_t)NB * 512 * TW, 256)), dim3(256), 0, s, E, ldE, rankp,
                     R0, B, NB);
  return hipGetLastError();
}

hipError_t launch_null_basis(const uint64_t *R, int64_t ldE, const int64_t *pivcols, const int64_t *rankp,
                             uint64_t *bitmap, int64_t *tw0, int64_t *freecols, int64_t *nullity,
                             const gf2_mat &N, hipStream_t s) {
  hipLaunchKernelGGL(k_null_prep, dim3(1), dim3(kNT), 0, s, pivcols, rankp, N.cols, bitmap, tw0, freecols, nullity);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t total = (size_t)N.rows * (size_t)((N.cols + 63) / 64);
  hipLaunchKernelGGL(k_null_rows, dim3(grid_for(total, 256)), dim3(256), 0, s, R, ldE, pivcols, tw0, freecols,
                     rankp, N);
  return hipGetLastError();
}

}  // namespace gf2
