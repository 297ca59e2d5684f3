// k_layout.hip -- state initialisation, layout conversion and extraction of
// L and E from the in-place working matrix.
//
// In-place form kept by the decomposition (the L\U picture of Fig. 1, with
// the L part stored compressed per 64-column sub-panel): after sub-panel q
// (rank R_q before it, r_q pivots at bit positions pos_0 < ... inside word q)
//   * pivot row R_q + t holds, in word q, the echelon row E_t restricted to
//     word q (bits >= pos_t) together with its multipliers for the earlier
//     pivots of the same sub-panel in bits [0, t);
//   * every later row holds, in word q, its multipliers for the r_q pivots of
//     the sub-panel in bits [0, r_q).
// So column R_q + t of L is bit t of word q, and row t of E is the working row
// t with the bits left of its pivot cleared.
#include "gf2_internal.h"

namespace gf2 {

__global__ void k_init_state(DecWork w) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = g; i < w.n; i += stride) {
    w.perm[i] = i;
    w.bp_src[i] = (int32_t)i;
    w.bp_mark[i] = 0;
    w.lvl[i] = -1;
    w.sp_src[i] = (int32_t)i;
    w.sp_src[w.n + i] = (int32_t)i;
    w.sp_mark[i] = 0;
    w.sp_mark[w.n + i] = 0;
  }
  for (int64_t i = g; i < (int64_t)w.Mw * 64; i += stride) w.pivcols[i] = -1;
  for (int64_t i = g; i <= w.Mw; i += stride) {
    w.nzflag[i] = 0;
    if (i == w.Mw) continue;
    w.sub[i].R = 0;
    w.sub[i].r = 0;
    w.sub[i].pad = 0;
    w.sub[i].pivmask = 0;
  }
  if (g == 0) {
    w.st->R = 0;
    w.st->bp_count = 0;
    w.st->pad0 = 0;
    w.sp_count[0] = 0;
    w.sp_count[1] = 0;
  }
}

hipError_t launch_init_state(const DecWork &w, hipStream_t s) {
  int64_t work = w.n > (int64_t)w.Mw * 64 + 1 ? w.n : (int64_t)w.Mw * 64 + 1;
  int blocks = (int)((work + 255) / 256);
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_init_state, dim3(blocks), dim3(256), 0, s, w);
  return hipGetLastError();
}

// caller layout -> working layout; pads rows [n, ldw) and words [Mw, 16*NB) with 0
__global__ void k_pack(gf2_mat src, uint64_t *W, int64_t ldw, int64_t n, int64_t m, int32_t NB) {
  const int64_t Mw = (m + 63) / 64;
  const int64_t total = (int64_t)NB * ldw * TW;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t blk = e / (ldw * TW);
    const int64_t rem = e - blk * ldw * TW;
    const int64_t i = rem / TW;
    const int64_t q = blk * TW + (rem % TW);
    uint64_t v = 0;
    if (i < n && q < Mw) v = src.data[uidx(src.w, src.ld, i, q)] & pad_mask(m, q);
    W[e] = v;
  }
}

hipError_t launch_pack(const gf2_mat &src, uint64_t *W, int64_t ldw, int64_t n, int64_t m,
                       int32_t NB, hipStream_t s) {
  int64_t total = (int64_t)NB * ldw * TW;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)blocks), dim3(256), 0, s, src, W, ldw, n, m, NB);
  return hipGetLastError();
}

// src^T (cols x rows of src) -> working layout, every word of W written (zero
// past the transpose).  Wave (q, p): rows 64 q .. 64 q + 63 of src, word p
// (columns 64 p ..), one 64 x 64 bit transpose; lane j then holds row 64 p + j of
// the transpose, word q.
__global__ void k_pack_transposed(gf2_mat src, uint64_t *W, int64_t ldw, int64_t nq, int64_t np) {
  const int lane = threadIdx.x & 63;
  const int64_t srcw = (src.cols + 63) / 64;
  const int64_t waves = nq * np;
  for (int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; b < waves;
       b += ((int64_t)gridDim.x * blockDim.x) >> 6) {
    const int64_t q = b % nq, p = b / nq;  // consecutive waves: consecutive words q of the same W rows
    const int64_t row = 64 * q + lane;
    const uint64_t x = (row < src.rows && p < srcw) ? src.data[uidx(src.w, src.ld, row, p)] & pad_mask(src.cols, p) : 0ull;
    W[widx(ldw, 64 * p + lane, q)] = transpose64(x, lane);
  }
}

hipError_t launch_pack_transposed(const gf2_mat &src, uint64_t *W, int64_t ldw, int32_t NB, hipStream_t s) {
  const int64_t nq = (int64_t)NB * TW, np = ldw / 64;  // every word of W, every 64-row group
  int64_t blocks = (nq * np * 64 + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_pack_transposed, dim3((unsigned)blocks), dim3(256), 0, s, src, W, ldw, nq, np);
  return hipGetLastError();
}

// working layout -> caller layout (rows [0, rows), words [0, ceil(cols/64)))
__global__ void k_unpack(const uint64_t *W, int64_t ldw, gf2_mat dst) {
  const int64_t Mw = (dst.cols + 63) / 64;
  const int64_t total = dst.rows * Mw;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e / Mw;
    const int64_t q = e - i * Mw;
    dst.data[uidx(dst.w, dst.ld, i, q)] = W[widx(ldw, i, q)] & pad_mask(dst.cols, q);
  }
}

hipError_t launch_unpack(const uint64_t *W, int64_t ldw, const gf2_mat &dst, hipStream_t s) {
  int64_t total = dst.rows * ((dst.cols + 63) / 64);
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_unpack, dim3((unsigned)blocks), dim3(256), 0, s, W, ldw, dst);
  return hipGetLastError();
}

// E (kmin x m): row t < rank = working row t with the bits left of its pivot
// cleared.  Thread x of the grid owns word column q and takes the rows
// blockIdx.y + gridDim.y * (4 k + j), four at a time (their loads issued
// before any store): no index division, and each row's pivot column is one
// broadcast read.
__global__ void k_extract_E(DecWork w, gf2_mat E) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= w.Mw) return;
  const int64_t rank = w.st->R, gy = gridDim.y;
  const uint64_t pad = pad_mask(E.cols, q);
  for (int64_t t0 = blockIdx.y; t0 < E.rows; t0 += 4 * gy) {
    uint64_t v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t t = t0 + j * gy;
      v[j] = 0;
      if (t < rank) {
        const int64_t pc = w.pivcols[t];
        const int64_t qt = pc >> 6;
        if (q >= qt) v[j] = w.W[widx(w.ldw, t, q)] & (q > qt ? ~0ull : (~0ull << (pc & 63)));
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t t = t0 + j * gy;
      if (t < E.rows) E.data[uidx(E.w, E.ld, t, q)] = v[j] & pad;
    }
  }
}

// grid for a (words x rows) extraction: 256 word columns per workgroup, rows
// spread over at most 4096 workgroup rows
static dim3 extract_grid(int64_t words, int64_t rows) {
  const int64_t gx = (words + 255) / 256, gy = rows < 4096 ? (rows > 0 ? rows : 1) : 4096;
  return dim3((unsigned)(gx > 0 ? gx : 1), (unsigned)gy);
}

hipError_t launch_extract_E(const DecWork &w, const gf2_mat &E, hipStream_t s) {
  hipLaunchKernelGGL(k_extract_E, extract_grid(w.Mw, E.rows), dim3(256), 0, s, w, E);
  return hipGetLastError();
}

// index of the sub-panel whose pivot range [R_q, R_q + r_q) contains t (t < rank)
__device__ inline int find_sub(const SubInfo *sub, int Mw, int64_t t) {
  int lo = 0, hi = Mw - 1;  // last q with sub[q].R <= t
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (sub[mid].R <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// L (n x kmin): column t < rank of L is bit (t - R_q) of word q of the working
// matrix (q = sub-panel of pivot t), below the diagonal; 1 on it; 0 above.
// Thread x of the grid owns word column u of L.  It lists once the sub-panel
// segments of its 64 columns (columns [cs, ce) are bits cs - R_q .. of word q;
// at most kSeg of them, else the general walk per row), then takes the rows
// blockIdx.y + gridDim.y * (4 k + j), four at a time.
constexpr int kSeg = 4;
__global__ void k_extract_L(DecWork w, gf2_mat L) {
  const int64_t Lw = (L.cols + 63) / 64;
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= Lw) return;
  const int64_t rank = w.st->R, gy = gridDim.y;
  const int64_t t0 = 64 * u;
  const int64_t tcols = t0 + 64 < rank ? t0 + 64 : rank;  // columns of this word that hold pivots
  const int q_first = t0 < tcols ? find_sub(w.sub, w.Mw, t0) : 0;
  const uint64_t pad = pad_mask(L.cols, u);
  int nseg = 0, segq[kSeg];
  int64_t segs[kSeg], sege[kSeg], segR[kSeg];
  {
    int64_t t = t0;
    int q = q_first;
    while (t < tcols) {
      while (q < w.Mw && (w.sub[q].r == 0 || w.sub[q].R + w.sub[q].r <= t)) ++q;
      if (q >= w.Mw) break;
      if (nseg == kSeg) { nseg = -1; break; }
      const int64_t Rq = w.sub[q].R, end = Rq + w.sub[q].r < tcols ? Rq + w.sub[q].r : tcols;
      segq[nseg] = q; segs[nseg] = t; sege[nseg] = end; segR[nseg] = Rq; ++nseg;
      t = end;
      ++q;
    }
  }
  for (int64_t i0 = blockIdx.y; i0 < L.rows; i0 += 4 * gy) {
    uint64_t out[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t i = i0 + j * gy;
      int64_t tend = tcols;
      if (i < rank && tend > i) tend = i;  // strictly below the diagonal
      uint64_t o = 0;
      if (i < L.rows && nseg >= 0) {
#pragma unroll
        for (int k = 0; k < kSeg; ++k) {
          if (k < nseg && segs[k] < tend) {
            const int64_t end = sege[k] < tend ? sege[k] : tend;
            const int nb = (int)(end - segs[k]);
            const uint64_t word = w.W[widx(w.ldw, i, segq[k])] >> (segs[k] - segR[k]);
            const uint64_t mask = nb >= 64 ? ~0ull : ((1ull << nb) - 1ull);
            o |= (word & mask) << (segs[k] - t0);
          }
        }
      } else if (i < L.rows) {  // more segments than kSeg: walk the sub-panels
        int64_t t = t0;
        int q = q_first;
        while (t < tend) {
          while (q < w.Mw && (w.sub[q].r == 0 || w.sub[q].R + w.sub[q].r <= t)) ++q;
          if (q >= w.Mw) break;
          const int64_t Rq = w.sub[q].R;
          const int64_t end = Rq + w.sub[q].r < tend ? Rq + w.sub[q].r : tend;
          const int nb = (int)(end - t);
          const uint64_t word = w.W[widx(w.ldw, i, q)] >> (t - Rq);
          const uint64_t mask = nb >= 64 ? ~0ull : ((1ull << nb) - 1ull);
          o |= (word & mask) << (t - t0);
          t = end;
          ++q;
        }
      }
      if (i < rank && i >= t0 && i < t0 + 64) o |= 1ull << (i - t0);  // unit diagonal
      out[j] = o;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t i = i0 + j * gy;
      if (i < L.rows) L.data[uidx(L.w, L.ld, i, u)] = out[j] & pad;
    }
  }
}

hipError_t launch_extract_L(const DecWork &w, const gf2_mat &L, hipStream_t s) {
  hipLaunchKernelGGL(k_extract_L, extract_grid((L.cols + 63) / 64, L.rows), dim3(256), 0, s, w, L);
  return hipGetLastError();
}

__global__ void k_finish(DecWork w, int64_t *perm, int64_t *pivcols, int64_t *rank, int64_t kmin) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (perm)
    for (int64_t i = g; i < w.n; i += stride) perm[i] = w.perm[i];
  if (pivcols)
    for (int64_t i = g; i < kmin; i += stride) pivcols[i] = w.pivcols[i];
  if (rank && g == 0) *rank = w.st->R;
}

hipError_t launch_finish(const DecWork &w, int64_t *perm, int64_t *pivcols, int64_t *rank,
                         hipStream_t s) {
  int64_t kmin = w.n < w.m ? w.n : w.m;
  int64_t work = w.n > kmin ? w.n : kmin;
  int blocks = (int)((work + 255) / 256);
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_finish, dim3(blocks), dim3(256), 0, s, w, perm, pivcols, rank, kmin);
  return hipGetLastError();
}

__global__ void k_xor(uint64_t *dst, const uint64_t *a, const uint64_t *b, size_t nwords) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nwords; e += stride)
    dst[e] = a[e] ^ b[e];
}

// Words of a timing operand: the SplitMix64 output function of (seed, index),
// a bit pattern for kernels whose run time does not depend on the values.
__global__ void k_fill_bits(uint64_t *dst, size_t nwords, uint64_t seed) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += (size_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    dst[i] = z ^ (z >> 31);
  }
}

__global__ void k_zero(uint64_t *dst, size_t nwords) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = 0ull;
}

hipError_t launch_zero(uint64_t *dst, size_t nwords, hipStream_t s) {
  if (nwords == 0) return hipSuccess;
  size_t blocks = (nwords + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, dst, nwords);
  return hipGetLastError();
}

__global__ void k_empty_outputs(int64_t *perm, int64_t n, int64_t *rank) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (perm)
    for (int64_t i = g; i < n; i += (int64_t)gridDim.x * blockDim.x) perm[i] = i;
  if (rank && g == 0) *rank = 0;
}

hipError_t launch_empty_outputs(int64_t *perm, int64_t n, int64_t *rank, hipStream_t s) {
  if (!rank && (!perm || n <= 0)) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_empty_outputs, dim3((unsigned)blocks), dim3(256), 0, s, perm, n, rank);
  return hipGetLastError();
}

hipError_t launch_fill_bits(uint64_t *dst, size_t nwords, uint64_t seed, hipStream_t s) {
  size_t blocks = (nwords + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_bits, dim3((unsigned)blocks), dim3(256), 0, s, dst, nwords, seed);
  return hipGetLastError();
}

hipError_t launch_xor(uint64_t *dst, const uint64_t *a, const uint64_t *b, size_t nwords,
                      hipStream_t s) {
  size_t blocks = (nwords + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_xor, dim3((unsigned)blocks), dim3(256), 0, s, dst, a, b, nwords);
  return hipGetLastError();
}

__global__ void k_xor_view(BView d, BView a, BView b, BView c, int has_c, int acc) {
  const int64_t nblk = (d.words + TW - 1) / TW;
  const int64_t total = nblk * d.rows * TW;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t w = e % TW;
    const int64_t r = (e / TW) % d.rows;
    const int64_t blk = e / (TW * d.rows);
    if (blk * TW + w >= d.words) continue;
    uint64_t v = a.p[(blk * a.ld + r) * TW + w] ^ b.p[(blk * b.ld + r) * TW + w];
    if (has_c) v ^= c.p[(blk * c.ld + r) * TW + w];
    uint64_t *q = d.p + (blk * d.ld + r) * TW + w;
    *q = acc ? (*q ^ v) : v;
  }
}

hipError_t launch_xor_view(const BView &dst, const BView &a, const BView &b, const BView *c, int acc,
                           hipStream_t s) {
  if (dst.rows <= 0 || dst.words <= 0) return hipSuccess;
  const int64_t total = (dst.words + TW - 1) / TW * dst.rows * TW;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_xor_view, dim3((unsigned)blocks), dim3(256), 0, s, dst, a, b, c ? *c : a, c ? 1 : 0, acc);
  return hipGetLastError();
}

}  // namespace gf2
