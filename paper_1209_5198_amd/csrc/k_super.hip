// k_super.hip -- the two kernels that close a super-panel of the decomposition.
//
// A super-panel is G consecutive trailing-update panels (G * 8 sub-panels of
// 64 columns).  While its panels are factored, their row exchanges are applied
// only to the words of the super-panel and of the next one (the "near" words,
// which also receive each panel's Schur complement update, eq. (Aj)); every
// other word keeps the row order of the super-panel's start and receives the
// whole super-panel's update at once, as one product with an inner dimension
// of up to 64 * G * 8 bits (the block elimination of Section 5 with the split
// on a super-panel boundary: the Schur complement of the left block,
// D xor L_bot * X, with X the top-right block after L_top^{-1}).  Closing a
// super-panel takes:
//   k_sp_swap   the super-panel's net row permutation applied to every word
//               outside the near words (P^(j) applied to the other columns)
//   k_trsm_far  its pivot rows in echelon form on those words right of the
//               near words: X = L_top^{-1} * X by block forward substitution
//               over the super-panel's sub-panels (E_b = Linv_b * X_b, then
//               X_c ^= L_cb * E_b for every later sub-panel c)
// followed by the products of k_gemm (Section 6) for the far words.
#include "gf2_internal.h"

namespace gf2 {

// ---------------------------------------------------------------- net row permutation
// Listed position p (sp_list) receives the row that was at position sp_src[p]
// when the super-panel started.  The listed positions are closed under the
// permutation (every source is listed), so all rows of a word are read before
// any is written.  Workgroup: kSwW word columns x 256 position slots.
constexpr int kSwThreads = 1024;
constexpr int kSwW = 4;
constexpr int kSwPer = kSpListMax / (kSwThreads / kSwW);
static_assert(kSwPer * (kSwThreads / kSwW) == kSpListMax, "position slots");

__global__ __launch_bounds__(kSwThreads) void k_sp_swap(DecWork w, int buf, int lo, int hi) {
  const int cnt = w.sp_count[buf];
  if (cnt == 0) return;
  const int tid = threadIdx.x, wl = tid % kSwW, e0 = tid / kSwW;
  // word u of the words outside [lo, hi): [0, lo) then [hi, Mw)
  const int64_t u = (int64_t)blockIdx.x * kSwW + wl;
  const int64_t qw = u < lo ? u : u - lo + hi;
  const bool act = qw < w.Mw;
  const int32_t *list = w.sp_list + (size_t)buf * kSpListMax;
  const int32_t *src = w.sp_src + (size_t)buf * w.n;
  uint64_t vals[kSwPer];
#pragma unroll
  for (int k = 0; k < kSwPer; ++k) {
    const int e = e0 + (kSwThreads / kSwW) * k;
    vals[k] = (act && e < cnt) ? w.W[widx(w.ldw, src[list[e]], qw)] : 0ull;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSwPer; ++k) {
    const int e = e0 + (kSwThreads / kSwW) * k;
    if (act && e < cnt) w.W[widx(w.ldw, list[e], qw)] = vals[k];
  }
}

hipError_t launch_sp_swap(const DecWork &w, int buf, int lo, int hi, hipStream_t s) {
  const int64_t nout = (int64_t)lo + (w.Mw - hi);
  if (nout <= 0) return hipSuccess;
  const int64_t blocks = (nout + kSwW - 1) / kSwW;
  hipLaunchKernelGGL(k_sp_swap, dim3((unsigned)blocks), dim3(kSwThreads), 0, s, w, buf, lo, hi);
  return hipGetLastError();
}

// After the swap: the list of buffer `buf` is emptied (sp_src back to the
// identity) for the super-panel after next, which uses the same buffer.
__global__ __launch_bounds__(1024) void k_sp_reset(DecWork w, int buf) {
  const int cnt = w.sp_count[buf];
  const int32_t *list = w.sp_list + (size_t)buf * kSpListMax;
  int32_t *src = w.sp_src + (size_t)buf * w.n, *mark = w.sp_mark + (size_t)buf * w.n;
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
    const int p = list[e];
    src[p] = p;
    mark[p] = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) w.sp_count[buf] = 0;
}

hipError_t launch_sp_reset(const DecWork &w, int buf, hipStream_t s) {
  hipLaunchKernelGGL(k_sp_reset, dim3(1), dim3(1024), 0, s, w, buf);
  return hipGetLastError();
}

// ---------------------------------------------------------------- pivot rows, far words
// Workgroup: one word column of [qa, qb) and all pivot rows of the
// super-panel (sub-panels s0 .. s0 + nsub - 1), held in LDS.  Per sub-panel b:
// 4-bit tables of X_b, E_b = Linv_b * X_b (row t: the XOR of the rows of X_b
// named by bit t of Linv_b), then 4-bit tables of E_b and every later pivot row
// XORs in the rows named by its multipliers for sub-panel b (word s0 + b of
// that row).  The multipliers of step b + 1 are loaded into registers during
// step b.  The 32 steps are serial, so a workgroup keeps a single word: its
// latency is the launch's, and the words spread over all CUs.
constexpr int kTfThreads = 512;
constexpr int kTfPre = kSpSubMax * 64 / kTfThreads;  // multipliers per thread and step

struct TrsmFarShared {
  uint64_t X[kSpSubMax * 64];      // 16 KB
  uint64_t Lm[2][kSpSubMax * 64];  // 32 KB: multipliers of the later pivot rows, two steps
  uint64_t T[16][16];              // 2 KB
  uint64_t Li[2][64];
  SubInfo Sb[kSpSubMax];
};

__global__ __launch_bounds__(kTfThreads) void k_trsm_far(DecWork w, int s0, int nsub, int qa) {
  __shared__ TrsmFarShared sh;
  const int tid = threadIdx.x;
  const int64_t qw = (int64_t)qa + blockIdx.x;
  const int64_t ldw = w.ldw;
  uint64_t *W = w.W;
  if (tid < nsub) sh.Sb[tid] = w.sub[s0 + tid];
  __syncthreads();
  int last = -1;  // last sub-panel with pivots
  for (int b = 0; b < nsub; ++b)
    if (sh.Sb[b].r > 0) last = b;
  if (last < 0) return;
  for (int ri = tid; ri < 64 * (last + 1); ri += kTfThreads) {
    const int c = ri >> 6, t = ri & 63;
    sh.X[ri] = t < sh.Sb[c].r ? W[widx(ldw, sh.Sb[c].R + t, qw)] : 0ull;
  }
  __syncthreads();
  // multipliers for sub-panel b of the pivot rows after it, and Linv_b
  uint64_t pre[kTfPre], pli = 0ull;
  auto fetch = [&](int b) {
#pragma unroll
    for (int u = 0; u < kTfPre; ++u) {
      const int ri = tid + kTfThreads * u;
      const int c = ri >> 6, t = ri & 63;
      pre[u] = (c > b && c <= last && t < sh.Sb[c].r) ? W[widx(ldw, sh.Sb[c].R + t, s0 + b)] : 0ull;
    }
    pli = tid < 64 ? w.Linv[(size_t)(s0 + b) * 64 + tid] : 0ull;
  };
  auto stage = [&](int slot) {
#pragma unroll
    for (int u = 0; u < kTfPre; ++u) sh.Lm[slot][tid + kTfThreads * u] = pre[u];
    if (tid < 64) sh.Li[slot][tid] = pli;
  };
  auto tables = [&](int b) {  // 16 tables of 16 entries over the 64 rows of X_b, one entry per thread
    if (tid < 256) {
      const int g = tid >> 4, v = tid & 15;
      uint64_t acc = 0ull;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (v & (1 << j)) acc ^= sh.X[64 * b + 4 * g + j];
      sh.T[g][v] = acc;
    }
  };
  auto lookup = [&](uint64_t l) {
    uint64_t v = 0ull;
#pragma unroll
    for (int g = 0; g < 16; ++g) v ^= sh.T[g][(l >> (4 * g)) & 15u];
    return v;
  };
  fetch(0);
  for (int b = 0; b <= last; ++b) {
    const int slot = b & 1;
    stage(slot);
    if (b < last) fetch(b + 1);  // in flight during this step
    tables(b);
    __syncthreads();
    const int rb = sh.Sb[b].r;
    // (the lookups read only the tables, so rows of X_b are overwritten in place)
    if (tid < rb) sh.X[64 * b + tid] = lookup(sh.Li[slot][tid]);
    __syncthreads();
    if (b == last) break;
    if (rb > 0) {
      tables(b);
      __syncthreads();
      // multipliers have no bits at or beyond rb, so unused tables contribute entry 0 = 0
      for (int ri = 64 * (b + 1) + tid; ri < 64 * (last + 1); ri += kTfThreads) {
        const int c = ri >> 6, t = ri & 63;
        if (t < sh.Sb[c].r) sh.X[ri] ^= lookup(sh.Lm[slot][ri]);
      }
    }
    __syncthreads();
  }
  for (int ri = tid; ri < 64 * (last + 1); ri += kTfThreads) {
    const int c = ri >> 6, t = ri & 63;
    if (t < sh.Sb[c].r) W[widx(ldw, sh.Sb[c].R + t, qw)] = sh.X[ri];
  }
}

hipError_t launch_trsm_far(const DecWork &w, int s0, int nsub, int qa, int qb, hipStream_t s) {
  if (qb <= qa || nsub <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trsm_far, dim3((unsigned)(qb - qa)), dim3(kTfThreads), 0, s, w, s0, nsub, qa);
  return hipGetLastError();
}

}  // namespace gf2
