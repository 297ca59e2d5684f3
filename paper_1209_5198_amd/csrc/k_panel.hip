// k_panel.hip -- the per-panel steps of the block decomposition (Section 4).
//
// A trailing-update panel is s <= 8 consecutive 64-column sub-panels (words
// q0 .. q0+s-1).  Per sub-panel q:
//   k_panel        pivot selection for the 64 columns of word q (procedure
//                  buildZ, Sections 4.2-4.4): for each bit k in order, the
//                  first row at or below the next free position whose reduced
//                  bit k is 1 becomes the pivot and is exchanged with that
//                  position (a transposition).  Produces the pivot columns,
//                  the coefficient map Zc of the sub-panel (row j of Zc gives
//                  the multipliers of bit j, so y = x * Zc are a row's
//                  multipliers -- the role of Z in D*Z = Y, Section 4.1), the
//                  inverse of the sub-panel's unit lower block, and moves the
//                  panel's words of every exchanged row.
//   k_rows_update  every row below the pivots: y = x * Zc is stored in word
//                  q (its L entries) and the other words of the panel are
//                  updated, word q' ^= y * E[.][q'] (eq. (Aj) restricted to
//                  the panel).
// Per panel:
//   k_swap         applies the panel's net row permutation to all words
//                  outside the panel (P^(j) applied to all columns).
//   k_trsm         pivot rows right of the panel: E = L_pp^{-1} * rows
//                  (block forward substitution over the sub-panels).
// The trailing product (Schur complement, eq. (Aj)) is k_gemm_m4rm.
//
// Reduced bit of a row.  The panel kernel keeps, for every pivot found so
// far, its fully reduced row M_j (indexed by the pivot's bit position j; rows
// of M are the identity on pivot positions -- the words M of buildZ).  The
// reduced form of any row x is Proj(x) = x xor sum_{pivot j} x_j M_j; its bit k
// is the parity test popC(c AND x) of buildZ with c = e_k xor sum_j M_j[k] e_j.
// Rows of a window (the first kWin free positions) are kept reduced in
// registers; rows below the window are tested with Proj on demand.
#include "gf2_internal.h"

namespace gf2 {

__device__ inline uint64_t rdl64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// slot s of a 128-slot window held as two registers per lane (slot = 64*g + lane).
// Value selects only (no references or pointer selects), so the window stays in
// registers instead of being lowered to a dynamically indexed private array.
__device__ inline uint64_t rdslot(uint64_t a0, uint64_t a1, int s) {
  const uint64_t u0 = rdl64(a0, s & 63), u1 = rdl64(a1, s & 63);
  return s < 64 ? u0 : u1;
}
__device__ inline int rdslot_i(int a0, int a1, int s) {
  const int u0 = __builtin_amdgcn_readlane(a0, s & 63), u1 = __builtin_amdgcn_readlane(a1, s & 63);
  return s < 64 ? u0 : u1;
}
__device__ inline uint64_t wrslot0(uint64_t a0, int s, uint64_t v, int lane) {
  return (s < 64 && lane == s) ? v : a0;
}
__device__ inline uint64_t wrslot1(uint64_t a1, int s, uint64_t v, int lane) {
  return (s >= 64 && lane == s - 64) ? v : a1;
}
__device__ inline int wrslot0i(int a0, int s, int v, int lane) { return (s < 64 && lane == s) ? v : a0; }
__device__ inline int wrslot1i(int a1, int s, int v, int lane) { return (s >= 64 && lane == s - 64) ? v : a1; }
// lanes l with base + l >= ib
__device__ inline uint64_t geq_mask(int ib, int base) {
  if (ib <= base) return ~0ull;
  if (ib >= base + 64) return 0ull;
  return ~0ull << (ib - base);
}

// One workgroup of 4 waves.  All four waves hold the same window state and
// take the same decisions (no communication on the common path); the
// fallback scan below the window and the final moves use all 256 threads.
__global__ __launch_bounds__(256) void k_panel(DecWork w, int q, int q0, int s_eff, int prev_q0) {
  __shared__ uint64_t Tp[8][256];                 // Proj tables for the scan (16 KB)
  __shared__ uint64_t Ms[64];
  __shared__ int bl_pos[64], bl_tag[64];          // rows moved out of the window
  __shared__ int bl_cnt;
  __shared__ int scan_best;
  __shared__ unsigned long long scan_F;
  __shared__ int mv_dst[kWin + 64], mv_src[kWin + 64];
  __shared__ int mv_cnt;
  __shared__ uint64_t G[kWin + 64][kMaxPanelWords];
  __shared__ uint64_t Praw[64][kMaxPanelWords];
  __shared__ int ptag[64];
  __shared__ int64_t gperm[kWin + 64];
  __shared__ int gbp[kWin + 64];
  __shared__ int wave_new[4];
  __shared__ int list_base;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t n = w.n, ldw = w.ldw;
  uint64_t *W = w.W;

  if (q == q0) {  // first sub-panel of a panel: forget the previous panel's row list
    const int cnt = w.st->bp_count;
    for (int j = tid; j < cnt; j += 256) {
      const int p = w.bp_list[j];
      w.bp_src[p] = p;
      w.bp_mark[p] = 0;
    }
    __syncthreads();
    if (tid == 0) w.st->bp_count = 0;
  }
  const int64_t R = w.st->R;
  int nbits = (int)(w.m - 64ll * q);
  if (nbits > 64) nbits = 64;
  bool skip = R >= n;
  if (prev_q0 >= 0 && w.nzflag[prev_q0] == 0u) skip = true;  // Schur complement already zero
  if (skip) {
    if (tid == 0) {
      w.sub[q].R = R;
      w.sub[q].r = 0;
      w.sub[q].pivmask = 0;
    }
    return;
  }
  if (tid == 0) bl_cnt = 0;
  __syncthreads();

  const int64_t p0 = R + lane, p1 = R + 64 + lane;
  const bool v0 = p0 < n, v1 = p1 < n;
  uint64_t x0 = v0 ? W[widx(ldw, p0, q)] : 0ull;
  uint64_t x1 = v1 ? W[widx(ldw, p1, q)] : 0ull;
  uint64_t xr0 = x0, xr1 = x1;
  int tag0 = (int)p0, tag1 = (int)p1;
  uint64_t Mrow = 0ull, pivmask = 0ull, F = 0ull;
  bool Fknown = false;
  int ib = 0;

  for (int k = 0; k < nbits; ++k) {
    const uint64_t kb = 1ull << k;
    const uint64_t m0 = __ballot(v0 && (xr0 & kb)) & geq_mask(ib, 0);
    const uint64_t m1 = __ballot(v1 && (xr1 & kb)) & geq_mask(ib, 64);
    int sp = -1;
    if (m0) sp = __builtin_ctzll(m0);
    else if (m1) sp = 64 + __builtin_ctzll(m1);
    uint64_t Mnew;
    if (sp >= 0) {
      const uint64_t xs = rdslot(x0, x1, sp), xrs = rdslot(xr0, xr1, sp);
      const int ts = rdslot_i(tag0, tag1, sp);
      if (sp != ib) {
        const uint64_t xi = rdslot(x0, x1, ib), xri = rdslot(xr0, xr1, ib);
        const int ti = rdslot_i(tag0, tag1, ib);
        x0 = wrslot0(x0, sp, xi, lane);
        x1 = wrslot1(x1, sp, xi, lane);
        xr0 = wrslot0(xr0, sp, xri, lane);
        xr1 = wrslot1(xr1, sp, xri, lane);
        tag0 = wrslot0i(tag0, sp, ti, lane);
        tag1 = wrslot1i(tag1, sp, ti, lane);
        x0 = wrslot0(x0, ib, xs, lane);
        x1 = wrslot1(x1, ib, xs, lane);
        xr0 = wrslot0(xr0, ib, xrs, lane);
        xr1 = wrslot1(xr1, ib, xrs, lane);
        tag0 = wrslot0i(tag0, ib, ts, lane);
        tag1 = wrslot1i(tag1, ib, ts, lane);
      }
      Mnew = xrs;
    } else {
      if (Fknown && !(F & kb)) continue;  // no row below the window can have bit k
      // ---- scan the rows below the window (all threads)
      __syncthreads();
      if (wv == 0) Ms[lane] = Mrow;
      if (tid == 0) {
        scan_best = 0x7fffffff;
        scan_F = 0ull;
      }
      __syncthreads();
      for (int e = tid; e < 8 * 256; e += 256) {
        const int g = e >> 8, idx = e & 255;
        uint64_t v = 0ull;
#pragma unroll
        for (int b = 0; b < 8; ++b)
          if (idx & (1 << b)) v ^= Ms[8 * g + b];
        Tp[g][idx] = v;
      }
      __syncthreads();
      int best = 0x7fffffff;
      uint64_t Floc = 0ull;
      for (int64_t p = R + kWin + tid; p < n; p += 256) {
        const uint64_t x = W[widx(ldw, p, q)];
        uint64_t pr = x;
#pragma unroll
        for (int g = 0; g < 8; ++g) pr ^= Tp[g][(x >> (8 * g)) & 255u];
        Floc |= pr;
        if ((pr & kb) && (int)p < best) best = (int)p;
      }
      if (best != 0x7fffffff) atomicMin(&scan_best, best);
      if (Floc) atomicOr(&scan_F, (unsigned long long)Floc);
      __syncthreads();
      best = scan_best;
      F = scan_F;
      Fknown = true;
      if (best == 0x7fffffff) continue;
      // ---- bring row `best` into slot ib; the slot's row goes to position `best`
      const uint64_t xp = W[widx(ldw, best, q)];
      int tp = best;
      for (int j = 0; j < bl_cnt; ++j)
        if (bl_pos[j] == best) tp = bl_tag[j];
      uint64_t xrp = xp;
#pragma unroll
      for (int g = 0; g < 8; ++g) xrp ^= Tp[g][(xp >> (8 * g)) & 255u];
      const uint64_t xo = rdslot(x0, x1, ib), xro = rdslot(xr0, xr1, ib);
      const int to = rdslot_i(tag0, tag1, ib);
      __syncthreads();
      if (tid == 0) {
        W[widx(ldw, best, q)] = xo;
        int j = 0;
        while (j < bl_cnt && bl_pos[j] != best) ++j;
        if (j == bl_cnt) {
          bl_pos[j] = best;
          bl_cnt = j + 1;
        }
        bl_tag[j] = to;
      }
      __syncthreads();
      x0 = wrslot0(x0, ib, xp, lane);
      x1 = wrslot1(x1, ib, xp, lane);
      xr0 = wrslot0(xr0, ib, xrp, lane);
      xr1 = wrslot1(xr1, ib, xrp, lane);
      tag0 = wrslot0i(tag0, ib, tp, lane);
      tag1 = wrslot1i(tag1, ib, tp, lane);
      F |= xro;
      Mnew = xrp;
    }
    // ---- pivot for bit k at slot ib: reduce the bookkeeping rows and the window
    pivmask |= kb;
    if (Mrow & kb) Mrow ^= Mnew;
    if (lane == k) Mrow = Mnew;
    if (v0 && lane > ib && (xr0 & kb)) xr0 ^= Mnew;
    if (v1 && 64 + lane > ib && (xr1 & kb)) xr1 ^= Mnew;
    if (Fknown) {
      if (F & kb) F |= Mnew;
      F &= ~kb;
    }
    ++ib;
  }
  const int r = ib;

  // ---- coefficient map Zc, multipliers of the pivot rows, inverse block
  // E_t = reduced pivot row t = xr0 of lane t.  y(M_j) gives row j of Zc; the
  // raw pivot rows reduce to their rows of the unit lower block L_pp.
  uint64_t Mcur = Mrow, yM = 0ull;
  uint64_t xred = lane < r ? x0 : 0ull, yx = 0ull;
  {
    uint64_t pm = pivmask;
    int t = 0;
    while (pm) {
      const int p = __builtin_ctzll(pm);
      pm &= pm - 1;
      const uint64_t e = rdl64(xr0, t);
      if ((Mcur >> p) & 1ull) { Mcur ^= e; yM |= 1ull << t; }
      if ((xred >> p) & 1ull) { xred ^= e; yx |= 1ull << t; }
      ++t;
    }
  }
  uint64_t li = lane < r ? (1ull << lane) : 0ull;
  for (int t = 0; t < r; ++t) {
    const uint64_t row = rdl64(li, t);
    if (lane > t && lane < r && ((yx >> t) & 1ull)) li ^= row;
  }

  // ---- move list: window slots whose row changed, then rows moved out
  if (wv == 0) {
    const int64_t pos0 = R + lane, pos1 = R + 64 + lane;
    const bool mv0 = v0 && tag0 != (int)pos0, mv1 = v1 && tag1 != (int)pos1;
    const uint64_t b0 = __ballot(mv0), b1 = __ballot(mv1);
    const uint64_t lt = (1ull << lane) - 1ull;
    if (mv0) {
      const int o = __popcll(b0 & lt);
      mv_dst[o] = (int)pos0;
      mv_src[o] = tag0;
    }
    const int c0 = __popcll(b0);
    if (mv1) {
      const int o = c0 + __popcll(b1 & lt);
      mv_dst[o] = (int)pos1;
      mv_src[o] = tag1;
    }
    const int c1 = c0 + __popcll(b1);
    for (int j = lane; j < bl_cnt; j += 64) {
      mv_dst[c1 + j] = bl_pos[j];
      mv_src[c1 + j] = bl_tag[j];
    }
    if (lane == 0) mv_cnt = c1 + bl_cnt;
    if (lane < r) ptag[lane] = tag0;
    // outputs of the pivot selection
    w.Zc[(size_t)q * 64 + lane] = yM;
    w.Linv[(size_t)q * 64 + lane] = li;
    if ((pivmask >> lane) & 1ull) {
      const int t = __popcll(pivmask & lt);
      w.pivcols[R + t] = 64ll * q + lane;
    }
  }
  __syncthreads();
  const int cnt = mv_cnt;
  const int jq = q - q0;
  // ---- gather (nothing is written before every read is done)
  for (int e = tid; e < cnt * s_eff; e += 256) {
    const int mvi = e / s_eff, j = e - mvi * s_eff;
    if (j != jq) G[mvi][j] = W[widx(ldw, mv_src[mvi], q0 + j)];
  }
  for (int e = tid; e < cnt; e += 256) {
    gperm[e] = w.perm[mv_src[e]];
    gbp[e] = w.bp_src[mv_src[e]];
  }
  for (int e = tid; e < r * s_eff; e += 256) {
    const int t = e / s_eff, j = e - t * s_eff;
    if (j > jq) Praw[t][j] = W[widx(ldw, ptag[t], q0 + j)];
  }
  __syncthreads();
  // ---- scatter
  for (int e = tid; e < cnt * s_eff; e += 256) {
    const int mvi = e / s_eff, j = e - mvi * s_eff;
    const int dst = mv_dst[mvi];
    if (j == jq) continue;
    if (j > jq && dst - R < r) continue;  // pivot rows right of q: written below
    W[widx(ldw, dst, q0 + j)] = G[mvi][j];
  }
  {
    // cnt <= 128 (two positions per transposition, at most 64 of them)
    int dst = 0;
    bool fresh = false;
    if (tid < cnt) {
      dst = mv_dst[tid];
      w.perm[dst] = gperm[tid];
      w.bp_src[dst] = gbp[tid];
      fresh = w.bp_mark[dst] == 0;
      if (fresh) w.bp_mark[dst] = 1;
    }
    const uint64_t fm = __ballot(fresh);
    if (lane == 0) wave_new[wv] = __popcll(fm);
    __syncthreads();
    if (tid == 0) list_base = atomicAdd(&w.st->bp_count, wave_new[0] + wave_new[1] + wave_new[2] + wave_new[3]);
    __syncthreads();
    int at = list_base + __popcll(fm & ((1ull << lane) - 1ull));
    for (int v = 0; v < wv; ++v) at += wave_new[v];
    if (fresh) w.bp_list[at] = dst;
  }
  if (wv == 0) {
    // word q: pivot rows get E_t | multipliers of earlier pivots; moved rows their raw word
    const int64_t pos0 = R + lane, pos1 = R + 64 + lane;
    if (lane < r) W[widx(ldw, pos0, q)] = xr0 | (yx & ((1ull << lane) - 1ull));
    else if (v0 && tag0 != (int)pos0) W[widx(ldw, pos0, q)] = x0;
    if (v1 && tag1 != (int)pos1) W[widx(ldw, pos1, q)] = x1;
  }
  // pivot rows, panel words right of q: E = L_pp^{-1} * rows
  for (int j = jq + 1 + wv; j < s_eff; j += 4) {
    uint64_t acc = 0ull;
    for (int t = 0; t < r; ++t)
      if ((li >> t) & 1ull) acc ^= Praw[t][j];
    if (lane < r) W[widx(ldw, R + lane, q0 + j)] = acc;
  }
  if (tid == 0) {
    w.sub[q].R = R;
    w.sub[q].r = r;
    w.sub[q].pivmask = pivmask;
    w.st->R = R + r;
  }
}

hipError_t launch_panel(const DecWork &w, int q, int q0, int s_eff, int prev_q0, hipStream_t s) {
  hipLaunchKernelGGL(k_panel, dim3(1), dim3(256), 0, s, w, q, q0, s_eff, prev_q0);
  return hipGetLastError();
}

// Rows below the pivots of sub-panel q: multipliers y = x * Zc into word q,
// then the panel's later words: word q' ^= y * E[.][q'].  Four-Russians with
// 4-bit tables (16 tables of 16 entries per word).
constexpr int kRowsPerThread = 2;
__global__ __launch_bounds__(256) void k_rows_update(DecWork w, int q, int q0, int s_eff) {
  __shared__ uint64_t Tz[16][16];
  __shared__ uint64_t Te[kMaxPanelWords - 1][16][16];
  const SubInfo si = w.sub[q];
  const int r = si.r;
  if (r == 0) return;
  const int tid = threadIdx.x;
  const int64_t ldw = w.ldw;
  uint64_t *W = w.W;
  const int nq = q0 + s_eff - 1 - q;  // words right of q inside the panel
  {
    const int g = tid >> 4, e = tid & 15;
    uint64_t v = 0ull;
    for (int b = 0; b < 4; ++b)
      if (e & (1 << b)) v ^= w.Zc[(size_t)q * 64 + 4 * g + b];
    Tz[g][e] = v;
    for (int j = 0; j < nq; ++j) {
      uint64_t u = 0ull;
      for (int b = 0; b < 4; ++b) {
        const int t = 4 * g + b;
        if ((e & (1 << b)) && t < r) u ^= W[widx(ldw, si.R + t, q + 1 + j)];
      }
      Te[j][g][e] = u;
    }
  }
  __syncthreads();
  const int ng = (r + 3) >> 2;
  const int64_t rowbeg = si.R + r;
  for (int u = 0; u < kRowsPerThread; ++u) {
    const int64_t i = ((int64_t)blockIdx.x * kRowsPerThread + u) * 256 + tid;
    if (i < rowbeg || i >= w.n) continue;
    const uint64_t x = W[widx(ldw, i, q)];
    uint64_t y = 0ull;
#pragma unroll
    for (int g = 0; g < 16; ++g) y ^= Tz[g][(x >> (4 * g)) & 15u];
    W[widx(ldw, i, q)] = y;
    for (int j = 0; j < nq; ++j) {
      uint64_t v = W[widx(ldw, i, q + 1 + j)];
      for (int g = 0; g < ng; ++g) v ^= Te[j][g][(y >> (4 * g)) & 15u];
      W[widx(ldw, i, q + 1 + j)] = v;
    }
  }
}

hipError_t launch_rows_update(const DecWork &w, int q, int q0, int s_eff, hipStream_t s) {
  const int64_t per = 256ll * kRowsPerThread;
  const int64_t blocks = (w.n + per - 1) / per;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_update, dim3((unsigned)blocks), dim3(256), 0, s, w, q, q0, s_eff);
  return hipGetLastError();
}

// Net row permutation of the panel on all words outside the panel: the row now
// at listed position p comes from position bp_src[p] at the panel start.
__global__ __launch_bounds__(1024) void k_swap(DecWork w, int q0, int s_eff) {
  const int cnt = w.st->bp_count;
  if (cnt == 0) return;
  const int tid = threadIdx.x, wl = tid & 15, e0 = tid >> 4;
  const int64_t qw = (int64_t)blockIdx.x * TW + wl;
  const bool act = qw < w.Mw && !(qw >= q0 && qw < q0 + s_eff);
  constexpr int PER = (kMaxPanelWords * 64 * 2) / 64;
  uint64_t vals[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = e0 + 64 * u;
    vals[u] = (act && e < cnt) ? w.W[widx(w.ldw, w.bp_src[w.bp_list[e]], qw)] : 0ull;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = e0 + 64 * u;
    if (act && e < cnt) w.W[widx(w.ldw, w.bp_list[e], qw)] = vals[u];
  }
}

hipError_t launch_swap(const DecWork &w, int q0, int s_eff, hipStream_t s) {
  hipLaunchKernelGGL(k_swap, dim3((unsigned)w.NB), dim3(1024), 0, s, w, q0, s_eff);
  return hipGetLastError();
}

// Pivot rows of the panel, words right of the panel:
//   E_b = Linv_b * X_b, then X_c ^= L_cb * E_b for later sub-panels c,
// with L_cb = word q0+b of the pivot rows of sub-panel c (their multipliers for
// the pivots of sub-panel b).  16-lane groups over a 16-word block, 4-bit tables.
constexpr int kTrsmThreads = 1024;
__global__ __launch_bounds__(kTrsmThreads) void k_trsm(DecWork w, int q0, int s_eff) {
  __shared__ uint64_t X[kMaxPanelWords * 64][TW];           // 64 KB: pivot rows, this block
  __shared__ uint64_t T[16][16][TW];                        // 32 KB: 4-bit tables
  __shared__ uint64_t Cf[kMaxPanelWords * 64][kMaxPanelWords];  // 32 KB: multipliers L_cb
  __shared__ uint64_t Li[kMaxPanelWords][64];               // 4 KB: Linv_b
  __shared__ SubInfo Sb[kMaxPanelWords];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, h = lane >> 4, wl = lane & 15;
  const int qc0 = q0 + s_eff;
  const int blk = blockIdx.x + (qc0 >> 4);
  const int64_t qw = (int64_t)blk * TW + wl;
  const bool qok = qw >= qc0 && qw < w.Mw;
  const int64_t ldw = w.ldw;
  uint64_t *W = w.W;
  if (tid < s_eff) Sb[tid] = w.sub[q0 + tid];
  __syncthreads();
  int rtot = 0;
  for (int b = 0; b < s_eff; ++b) rtot += Sb[b].r;
  if (rtot == 0) return;
  for (int ri = tid >> 4; ri < 64 * s_eff; ri += kTrsmThreads / 16) {
    const int b = ri >> 6, t = ri & 63;
    X[ri][wl] = (qok && t < Sb[b].r) ? W[widx(ldw, Sb[b].R + t, qw)] : 0ull;
  }
  for (int e = tid; e < 64 * s_eff * s_eff; e += kTrsmThreads) {
    const int ri = e / s_eff, b = e - ri * s_eff;
    const int c = ri >> 6, t = ri & 63;
    Cf[ri][b] = (b < c && t < Sb[c].r) ? W[widx(ldw, Sb[c].R + t, q0 + b)] : 0ull;
  }
  for (int e = tid; e < 64 * s_eff; e += kTrsmThreads) Li[e >> 6][e & 63] = w.Linv[(size_t)(q0 + (e >> 6)) * 64 + (e & 63)];
  __syncthreads();
  for (int b = 0; b < s_eff; ++b) {
    const int rb = Sb[b].r;
    if (rb == 0) continue;
    // tables over the rows of X_b
    if (tid < 256) {
      const int g = tid >> 4, c = tid & 15;
      uint64_t v[4];
      for (int j = 0; j < 4; ++j) v[j] = X[64 * b + 4 * g + j][c];
      uint64_t cur = 0ull;
      for (int j = 0; j < 16; ++j) {
        T[g][j ^ (j >> 1)][c] = cur;
        if (j < 15) cur ^= v[__builtin_ctz(j + 1)];
      }
    }
    __syncthreads();
    {
      const int t = 4 * wv + h;  // 16 waves x 4 groups = 64 rows
      if (t < rb) {
        const uint64_t l = Li[b][t];
        uint64_t v = 0ull;
#pragma unroll
        for (int g = 0; g < 16; ++g) v ^= T[g][(l >> (4 * g)) & 15u][wl];
        X[64 * b + t][wl] = v;
      }
    }
    __syncthreads();
    if (b == s_eff - 1) break;
    if (tid < 256) {
      const int g = tid >> 4, c = tid & 15;
      uint64_t v[4];
      for (int j = 0; j < 4; ++j) v[j] = X[64 * b + 4 * g + j][c];
      uint64_t cur = 0ull;
      for (int j = 0; j < 16; ++j) {
        T[g][j ^ (j >> 1)][c] = cur;
        if (j < 15) cur ^= v[__builtin_ctz(j + 1)];
      }
    }
    __syncthreads();
    // multipliers have no bits at or beyond rb, so unused tables contribute entry 0 = 0
    for (int ri = 64 * (b + 1) + 4 * wv + h; ri < 64 * s_eff; ri += kTrsmThreads / 16) {
      const int c = ri >> 6, t = ri & 63;
      if (t < Sb[c].r) {
        const uint64_t l = Cf[ri][b];
        uint64_t v = 0ull;
#pragma unroll
        for (int g = 0; g < 16; ++g) v ^= T[g][(l >> (4 * g)) & 15u][wl];
        X[ri][wl] ^= v;
      }
    }
    __syncthreads();
  }
  for (int ri = tid >> 4; ri < 64 * s_eff; ri += kTrsmThreads / 16) {
    const int b = ri >> 6, t = ri & 63;
    if (qok && t < Sb[b].r) W[widx(ldw, Sb[b].R + t, qw)] = X[ri][wl];
  }
}

hipError_t launch_trsm(const DecWork &w, int q0, int s_eff, hipStream_t s) {
  const int qc0 = q0 + s_eff;
  if (qc0 >= w.Mw) return hipSuccess;
  const int blocks = ((w.Mw - 1) >> 4) - (qc0 >> 4) + 1;
  hipLaunchKernelGGL(k_trsm, dim3((unsigned)blocks), dim3(kTrsmThreads), 0, s, w, q0, s_eff);
  return hipGetLastError();
}

}  // namespace gf2
