// k_batch.hip -- many independent decompositions (and solves) in one launch.
//
// A batch holds up to thousands of matrices of at most kBatchMaxDim rows and
// columns, each of its own shape.  One persistent launch factors all of them:
// every workgroup takes the next matrix from a queue (the host orders the queue
// by decreasing work, so the largest matrices start first and the small ones
// fill the tail) and runs the whole decomposition of Section 4 on it, with the
// matrix's working copy in a slot of its own (L2-resident for the sizes here).
//
// Per 64-column panel (word q of every row; the b = 64 panel of Section 4):
//   * pivot search, procedure buildZ (Sections 4.2-4.4) in its b = 1 reading:
//     for each bit k, the first position at or below the next free one whose
//     reduced bit k is 1 is exchanged with it (a transposition of the
//     position -> row map; rows never move in memory).  The panel words of the
//     rows at or below R live in registers (8 per thread) while the search
//     runs; every later row with bit k set is reduced in the bits above k and
//     keeps its bit k as the multiplier (the compressed L of Fig. 1).
//   * canonical multipliers: with T the unit lower matrix of the pivot rows'
//     multipliers (U = T * E for the panel's pivot rows U and echelon rows E),
//     every row at or below R gets c = y * T^-1 (its multipliers y applied to
//     the unreduced pivot rows), and pivot row t gets row t of T^-1 without its
//     diagonal.  Everything is indexed by bit position inside word q.
//   * trailing update (the Schur complement, eq. (Aj)): for each chunk of 8
//     later words, sixteen 4-bit Four-Russians tables (Section 6, c = 4) of
//     the pivot rows' chunk words are built in LDS, and each row XORs in
//     sixteen 64-byte table entries selected by the nibbles of its c; rows of
//     the panel's pivots get their echelon form by the same product.
// At the end L, E, the permutation, the pivot columns and the rank are written
// in the caller's row-major formats.
#include <limits.h>

#include "gf2_internal.h"

namespace gf2 {
namespace {

constexpr int NT = kBatchThreads;          // threads per workgroup
constexpr int NW = NT / 64;                // waves per workgroup
constexpr int kWin = 128;                  // window rows of the pivot search, two per lane of wave 0
constexpr int RB = (kBatchMaxDim - kWin + NT - 1) / NT;  // rows beyond the window per thread
constexpr int kChunk = 8;                  // later words per table build (one 64-byte segment)
constexpr int kRU = 2;                     // rows per thread in each stage of the row update
constexpr int kCp = 8;                     // rows per thread in flight in the working copy

__device__ inline uint64_t rdl64b(uint64_t v, int l) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
// Values every lane of a wave holds alike (LDS words read at one address), made
// scalar so that the compiler keeps the loops they control uniform.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline uint64_t uni64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint64_t wrl64b(uint64_t old, uint64_t v, int l) {
  const uint32_t lo = wrlane((uint32_t)v, l, (uint32_t)old);
  const uint32_t hi = wrlane((uint32_t)(v >> 32), l, (uint32_t)(old >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint64_t wave_or64(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    lo |= (uint32_t)__shfl_xor((int)lo, o);
    hi |= (uint32_t)__shfl_xor((int)hi, o);
  }
  return ((uint64_t)hi << 32) | lo;
}
// x times the 64 x 64 matrix whose sixteen 4-bit tables are tab (Section 6, c = 4)
__device__ inline uint64_t apply16(const uint64_t (&tab)[16][16], uint64_t x) {
  uint64_t acc = 0ull;
#pragma unroll
  for (int g = 0; g < 16; ++g) acc ^= tab[g][(x >> (4 * g)) & 15u];
  return acc;
}

// Bit compression (gather the bits of x selected by mask into the low bits, in
// order): the parallel-suffix method of H. S. Warren, "Hacker's Delight",
// Section 7-4.  The six move masks depend on the mask only and are computed
// once per panel; compressing a word then costs six and/xor/shift/or steps.
__device__ inline void compress_masks(uint64_t m, uint64_t (&mv)[6]) {
  uint64_t mk = ~m << 1;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    uint64_t mp = mk ^ (mk << 1);
    mp ^= mp << 2;
    mp ^= mp << 4;
    mp ^= mp << 8;
    mp ^= mp << 16;
    mp ^= mp << 32;
    const uint64_t v = mp & m;
    mv[i] = v;
    m = (m ^ v) | (v >> (1 << i));
    mk &= ~mp;
  }
}
__device__ inline uint64_t compress(uint64_t x, uint64_t m, const uint64_t *mv) {
  x &= m;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const uint64_t t = x & mv[i];
    x = (x ^ t) | (t >> (1 << i));
  }
  return x;
}

struct BatchShared {
  int32_t map[kBatchMaxDim];          // position -> row of the working copy
  uint64_t cvec[kBatchMaxDim];        // canonical multipliers of positions R.. (then pivot columns)
  union {
    struct {
      uint64_t T[16][16][kChunk + 1]; // 4-bit tables of the current chunk (rows padded: fewer bank conflicts)
    } up;
    uint64_t rowq[NT / 8][kBatchMaxPanels];  // outputs: panel words of the rows in flight
    struct {
      uint64_t ninv[64];              // row k of (I + N)^-1 (bit-position space)
      uint64_t Nt[16][16];            // its 4-bit tables
    } fin;
  } tr;
  uint64_t Tt[16][16];                // 4-bit tables of the rows of T^-1
  uint64_t tinv[64];                  // row k of T^-1 (bit-position space)
  uint64_t pivw[64];                  // panel words of the panel's pivot rows, as found
  uint64_t pK[kBatchMaxPanels];       // pivot mask of each panel
  uint64_t pmv[kBatchMaxPanels][6];   // compress masks of each panel's pivot mask
  int32_t pR[kBatchMaxPanels];        // rank before each panel
  int32_t pr[kBatchMaxPanels];        // pivots of each panel
  int32_t prow[64];                   // pivot t of the current panel -> bit position
  uint64_t fb[NW];                    // per-wave OR of the rows' words
  int32_t cand[NW];                   // per-wave first beyond row with the requested bit
  uint64_t candw[NW];                 // ... its word
  int32_t cando[NW];                  // ... its row
  uint64_t kmask;                     // pivot mask so far
  uint64_t xfer_x;                    // word of the row leaving the window
  int32_t xfer_o;                     // ... its row
  int32_t cmd;                        // bit the window has no candidate for, or -1 when done
  int32_t tcnt;                       // pivots so far
  int32_t lj0[kBatchMaxPanels];       // first panel whose pivots reach L word lw
  int32_t job;
};

__global__ __launch_bounds__(NT, kBatchWGPerCU) void k_batch_dec(BatchArgs a) {
  __shared__ BatchShared sh;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  uint64_t *W = a.W + (size_t)blockIdx.x * (size_t)a.wslot;

  for (;;) {
    __syncthreads();  // the previous matrix is finished with the shared state
    if (tid == 0) sh.job = (int)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int job = uni(sh.job);
    if (job >= a.count) return;
    const BatchDesc d = a.d[job];
    const int n = d.n, m = d.m, Mw = (m + 63) >> 6, kmin = n < m ? n : m;

    // ---- working copy (row stride ld words, a multiple of one 64-byte
    // segment, so that a chunk of kChunk words is one aligned segment; padding
    // bits cleared) and identity map.  A row is read by the next power of two
    // lanes at or above Mw; each thread moves kCp rows at a time.  The input is
    // read once, with non-temporal loads, and the E and L rows below are written
    // with non-temporal stores: the working slots keep the cache (on the
    // 4096-matrix batch this took the decomposition from 5.05 to 4.76 ms).
    const int ld = (Mw + kChunk - 1) & ~(kChunk - 1);
    {
      const uint64_t *A = a.A + d.a;
      const int lsh = Mw <= 1 ? 0 : 32 - __builtin_clz(Mw - 1);
      const int rows_it = NT >> lsh, w = tid & ((1 << lsh) - 1);
      const uint64_t pm = pad_mask(m, w);
      for (int i0 = tid >> lsh; i0 < n; i0 += kCp * rows_it) {
        uint64_t v[kCp];
#pragma unroll
        for (int j = 0; j < kCp; ++j) {
          const int i = i0 + j * rows_it;
          v[j] = (i < n && w < Mw) ? __builtin_nontemporal_load(&A[(size_t)i * Mw + w]) : 0ull;
        }
#pragma unroll
        for (int j = 0; j < kCp; ++j) {
          const int i = i0 + j * rows_it;
          if (i < n && w < Mw) W[(uint32_t)(i * ld + w)] = v[j] & pm;
        }
      }
      for (int i = tid; i < n; i += NT) sh.map[i] = i;
    }
    __syncthreads();
    auto rd = [&](int row, int w) -> uint64_t { return W[(uint32_t)(row * ld + w)]; };

    int R = 0, nq = 0;
    for (int q = 0; q < Mw && R < n; ++q) {
      nq = q + 1;
      const int nbits = (m - 64 * q) < 64 ? (m - 64 * q) : 64;

      const int nrest = n - R;  // rows at or below the next free position
      // Positions R .. R + kWin - 1 form the window: position R + 64 * s + l is
      // slot s of lane l of wave 0.  Position R + kWin + NT * u + tid is slot u
      // of thread tid ("beyond" rows); slots at or beyond nslb hold no row.
      const int nslb = nrest > kWin ? (nrest - kWin + NT - 1) / NT : 0;
      uint64_t xw0 = 0ull, xw1 = 0ull;
      int ow0 = 0, ow1 = 0;
      uint64_t f = 0ull;
      if (wv == 0) {
        if (lane < nrest) {
          ow0 = sh.map[R + lane];
          xw0 = rd(ow0, q);
        }
        if (64 + lane < nrest) {
          ow1 = sh.map[R + 64 + lane];
          xw1 = rd(ow1, q);
        }
        f = xw0 | xw1;
      }
      uint64_t xb[RB];
      int ob[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        xb[u] = 0ull;
        ob[u] = 0;
        const int pos = R + kWin + NT * u + tid;
        if (u < nslb && pos < n) {
          ob[u] = sh.map[pos];
          xb[u] = rd(ob[u], q);
        }
        f |= xb[u];
      }
      // F: the bits some row at or below the next free position has.  A bit
      // that no such row has cannot become a pivot later in this word: every
      // reduction XORs one of these rows into another.
      f = wave_or64(f);
      if (lane == 0) sh.fb[wv] = f;
      __syncthreads();
      uint64_t F = 0ull;
#pragma unroll
      for (int w = 0; w < NW; ++w) F |= uni64(sh.fb[w]);

      // ---- pivot search over the bits of word q.  Wave 0 decides from the
      // window alone while it holds a candidate for the current bit; the beyond
      // rows are reduced lazily, by the pivots logged since their last catch-up,
      // only when the window has none (then the whole workgroup takes part).
      int t = 0, k = 0, lstart = 0, xfer = -1;
      uint64_t K = 0ull;
      // pivot log of wave 0, lane i = pivot i: its word as found and its row
      uint64_t lgw = 0ull;
      int lgo = 0;
      const int tmax = nrest < 64 ? nrest : 64;
      const uint64_t wbits = nbits == 64 ? ~0ull : ((1ull << nbits) - 1ull);
      for (;;) {
        if (wv == 0) {
          int need = -1;
          // bits still to examine, in increasing order
          uint64_t Fr = F & wbits & (k >= 64 ? 0ull : (~0ull << k));
          while (Fr && t < tmax) {
            t = uni(t);
            k = (int)__builtin_ctzll(Fr);
            Fr &= Fr - 1ull;
            const uint64_t kb = 1ull << k;
            // all ones in the lanes whose row has bit k: the one-bit field of
            // the word half holding bit k, sign-extended
            const int ks = 31 - (k & 31);
            auto bitmask = [&](uint64_t x) -> uint64_t {
              const uint32_t h = k < 32 ? (uint32_t)x : (uint32_t)(x >> 32);
              const uint32_t mk = (uint32_t)((int32_t)(h << ks) >> 31);
              return ((uint64_t)mk << 32) | mk;
            };
            uint64_t m0 = bitmask(xw0), m1 = bitmask(xw1);
            bool c0 = (uint32_t)m0 != 0u, c1 = (uint32_t)m1 != 0u;
            const uint64_t bal0 = __ballot(c0) & (~0ull << t);  // positions t.. of slot 0
            int p = (int)__builtin_ctzll(bal0);
            if (__builtin_expect(bal0 == 0ull, 0)) {
              const uint64_t bal1 = __ballot(c1);
              if (!bal1) {
                if (nslb > 0) {
                  need = k;
                  break;
                }
                continue;  // the window is every remaining row: not a pivot column
              }
              // the first candidate is in slot 1: exchange it with position t
              const int p1 = (int)__builtin_ctzll(bal1);
              const uint64_t xp = rdl64b(xw1, p1), xt = rdl64b(xw0, t);
              const int op = __builtin_amdgcn_readlane(ow1, p1), ot = __builtin_amdgcn_readlane(ow0, t);
              xw1 = wrl64b(xw1, xt, p1);
              ow1 = wrlane(ot, p1, ow1);
              xw0 = wrl64b(xw0, xp, t);
              ow0 = wrlane(op, t, ow0);
              m0 = bitmask(xw0);
              m1 = bitmask(xw1);
              p = t;
            }
            p = uni(p);
            const uint64_t pw = rdl64b(xw0, p);
            const int porg = __builtin_amdgcn_readlane(ow0, p);
            // every row with bit k is reduced in the bits above k.  Lanes
            // before t are finished positions (their rows are in the log) and
            // lane p is the pivot, overwritten below or finished itself.
            const uint64_t ph = pw & ~((kb << 1) - 1ull);  // zero for k = 63
            xw0 ^= ph & m0;
            xw1 ^= ph & m1;
            if (p != t) {  // the row at position t moves to position p
              const uint64_t xt = rdl64b(xw0, t);
              const int ot = __builtin_amdgcn_readlane(ow0, t);
              xw0 = wrl64b(xw0, xt, p);
              ow0 = wrlane(ot, p, ow0);
            }
            lgw = wrl64b(lgw, pw, t);
            lgo = wrlane(porg, t, lgo);
            K |= kb;
            ++t;
          }
          k = need >= 0 ? need : 64;
          if (lane < t) sh.pivw[lane] = lgw;
          // pivot i sits at the i-th set bit of K (bits are taken in order)
          if ((K >> lane) & 1ull) sh.prow[__popcll(K & ((1ull << lane) - 1ull))] = lane;
          if (lane == 0) {
            sh.cmd = need;
            sh.tcnt = t;
            sh.kmask = K;
          }
        }
        __syncthreads();
        const int cmd = uni(sh.cmd), tt = uni(sh.tcnt);
        if (xfer >= 0) {  // the row that left the window for beyond position xfer
          const int j = xfer - R - kWin, jt = j % NT, ju = j / NT;
          if (tid == jt) {
#pragma unroll
            for (int u = 0; u < RB; ++u)
              if (u == ju) {
                xb[u] = sh.xfer_x;
                ob[u] = sh.xfer_o;
              }
          }
          xfer = -1;
        }
        if (cmd < 0) break;
        // catch the beyond rows up with the pivots found since their last one
        for (int i = lstart; i < tt; ++i) {
          const int kk = uni(sh.prow[i]);
          const uint64_t P = (kk == 63) ? 0ull : (uni64(sh.pivw[i]) & (~0ull << (kk + 1)));
#pragma unroll
          for (int u = 0; u < RB; ++u)
            if (u < nslb) xb[u] ^= P & (0ull - ((xb[u] >> kk) & 1ull));
        }
        lstart = tt;
        // first beyond row with bit cmd, and the bits the beyond rows still have
        int first = INT_MAX, co = 0;
        uint64_t cw = 0ull, fo = 0ull;
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          if (u < nslb) {
            fo |= xb[u];
            const uint64_t bal = __ballot((xb[u] >> cmd) & 1ull);
            if (first == INT_MAX && bal) {
              const int l = (int)__builtin_ctzll(bal);
              first = R + kWin + NT * u + 64 * wv + l;
              cw = rdl64b(xb[u], l);
              co = __builtin_amdgcn_readlane(ob[u], l);
            }
          }
        }
        fo = wave_or64(fo);
        if (lane == 0) {
          sh.cand[wv] = first;
          sh.candw[wv] = cw;
          sh.cando[wv] = co;
          sh.fb[wv] = fo;
        }
        __syncthreads();
        int p = uni(sh.cand[0]), wb = 0;
#pragma unroll
        for (int w = 1; w < NW; ++w) {
          const int c = uni(sh.cand[w]);
          if (c < p) {
            p = c;
            wb = w;
          }
        }
        if (p != INT_MAX) xfer = p;
        if (wv == 0) {
          uint64_t fw = uni64(wave_or64((lane >= t ? xw0 : 0ull) | xw1));
#pragma unroll
          for (int w = 0; w < NW; ++w) fw |= uni64(sh.fb[w]);
          F = (cmd == 63) ? 0ull : (fw & (~0ull << (cmd + 1)));
          k = cmd + 1;
          if (p != INT_MAX) {  // the candidate enters the window at position t
            const uint64_t xt = rdl64b(xw0, t);
            const int ot = __builtin_amdgcn_readlane(ow0, t);
            if (lane == 0) {
              sh.xfer_x = xt;
              sh.xfer_o = ot;
            }
            xw0 = wrl64b(xw0, uni64(sh.candw[wb]), t);
            ow0 = wrlane(uni(sh.cando[wb]), t, ow0);
            F |= 1ull << cmd;
            k = cmd;
          }
        }
      }
      const int r = uni(sh.tcnt);
      K = uni64(sh.kmask);
      if (tid == 0) {
        sh.pK[q] = K;
        sh.pR[q] = R;
        sh.pr[q] = r;
      }
      if (tid == 64) {
        uint64_t mv[6];
        compress_masks(K, mv);
#pragma unroll
        for (int i = 0; i < 6; ++i) sh.pmv[q][i] = mv[i];
      }
      if (r == 0) {  // no row has a bit of this word: nothing moved or changed
        __syncthreads();
        continue;
      }

      // ---- T^-1 (wave 0) and the inverse of I + N (wave 1), in bit-position
      // space (lane = bit position).  T is the unit lower matrix of the pivot
      // rows' multipliers; N holds, for each pivot the beyond rows still owe,
      // its row's bits at the later pivot positions, so a beyond row's
      // multipliers are its pivot-position bits times (I + N)^-1.
      if (wv == 0) {
        uint64_t trow = 0ull, tv = 0ull;
        const uint64_t below = (1ull << lane) - 1ull;
        if ((K >> lane) & 1ull) {
          trow = sh.pivw[__popcll(K & below)] & K & below;
          tv = 1ull << lane;
        }
        uint64_t Kr = K;
        while (Kr) {
          const int kk = (int)__builtin_ctzll(Kr);
          Kr &= Kr - 1ull;
          const uint64_t v = rdl64b(tv, kk);
          if ((trow >> kk) & 1ull) tv ^= v;
        }
        sh.tinv[lane] = tv;
      } else if (wv == 1) {
        uint64_t nrow = 0ull, nv = 0ull;
        const uint64_t below = (1ull << lane) - 1ull;
        if ((K >> lane) & 1ull) {
          const int i = __popcll(K & below);
          nv = 1ull << lane;
          if (i >= lstart) nrow = sh.pivw[i] & K & ~below & ~(1ull << lane);
        }
        uint64_t Kp = K;  // pivots lstart .. r-1
        for (int i = 0; i < lstart; ++i) Kp &= Kp - 1ull;
        while (Kp) {
          const int kk = 63 - (int)__builtin_clzll(Kp);
          Kp &= ~(1ull << kk);
          const uint64_t v = rdl64b(nv, kk);
          if ((nrow >> kk) & 1ull) nv ^= v;
        }
        sh.tr.fin.ninv[lane] = nv;
      }
      __syncthreads();
      {
        const int g = tid >> 4, v = tid & 15;
        uint64_t a0 = 0ull, a1 = 0ull;
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if ((v >> b) & 1) {
            a0 ^= sh.tinv[4 * g + b];
            a1 ^= sh.tr.fin.ninv[4 * g + b];
          }
        sh.Tt[g][v] = a0;
        sh.tr.fin.Nt[g][v] = a1;
      }
      __syncthreads();
      // ---- canonical multipliers c (the trailing update applies c to the
      // unreduced pivot rows); words, positions written back
      auto put_q = [&](int row, uint64_t v) { W[(size_t)row * ld + q] = v; };
      if (wv == 0) {
        if (lane < nrest) {
          uint64_t c, xo = xw0;
          int oo = ow0;
          if (lane < r) {  // pivot lane: its row as found, from the log
            const int kk = sh.prow[lane];
            c = sh.tinv[kk] & ~(1ull << kk);
            xo = lgw;
            oo = lgo;
          } else {
            c = apply16(sh.Tt, xw0 & K);
          }
          sh.cvec[lane] = c;
          sh.map[R + lane] = oo;
          put_q(oo, xo);
        }
        if (64 + lane < nrest) {
          sh.cvec[64 + lane] = apply16(sh.Tt, xw1 & K);
          sh.map[R + 64 + lane] = ow1;
          put_q(ow1, xw1);
        }
      }
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int pos = R + kWin + NT * u + tid;
        if (u < nslb && pos < n) {
          const uint64_t mm = apply16(sh.tr.fin.Nt, xb[u] & K);
          sh.cvec[pos - R] = apply16(sh.Tt, mm);
          sh.map[pos] = ob[u];
          put_q(ob[u], mm);
        }
      }

      // ---- trailing update (eq. (Aj)) over 64-byte aligned chunks of kChunk
      // words.  Thread (g, w, h) builds entries v = 8h .. 8h+7 of table g for
      // chunk word w from the four pivot rows of bit positions 4g .. 4g+3,
      // whose words it loads one chunk ahead; the row update keeps two stages
      // of kRU rows per thread in flight.
      {
        const int tg = tid >> 4, tw = (tid >> 1) & 7, th = tid & 1;
        const int c_first = (q + 1) & ~(kChunk - 1);
        __syncthreads();  // positions, multipliers and panel words written above
        // offsets of the pivot rows of bit positions 4 tg .. 4 tg + 3 (-1: no pivot)
        int urow[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int kp = 4 * tg + b;
          urow[b] = ((K >> kp) & 1ull) ? sh.map[R + __popcll(K & ((1ull << kp) - 1ull))] : -1;
        }
        auto load_u = [&](int c0, uint64_t (&u)[4]) {
          const int cw = c0 + tw;
#pragma unroll
          for (int b = 0; b < 4; ++b) u[b] = (urow[b] >= 0 && cw > q && cw < Mw) ? rd(urow[b], cw) : 0ull;
        };
        uint64_t u[4];
        if (c_first < Mw) load_u(c_first, u);
        const int grp = tid >> 3, w = tid & 7;
        constexpr int G = NT / kChunk;  // row groups
        const int nst = (n - R + G * kRU - 1) / (G * kRU);
        for (int c0 = c_first; c0 < Mw; c0 += kChunk) {
          if (c0 != c_first) __syncthreads();  // the previous chunk's tables are no longer read
          {
            const uint64_t base = th ? u[3] : 0ull;
#pragma unroll
            for (int j = 0; j < 8; ++j)
              sh.tr.up.T[tg][8 * th + j][tw] =
                  base ^ ((j & 1) ? u[0] : 0ull) ^ ((j & 2) ? u[1] : 0ull) ^ ((j & 4) ? u[2] : 0ull);
          }
          __syncthreads();
          if (c0 + kChunk < Mw) load_u(c0 + kChunk, u);
          const int cw = c0 + w;
          if (cw > q && cw < Mw) {
            int rowA[kRU], rowB[kRU];
            uint64_t oldA[kRU], oldB[kRU];
            auto load_stage = [&](int st, int (&rw)[kRU], uint64_t (&old)[kRU]) {
#pragma unroll
              for (int j = 0; j < kRU; ++j) {
                const int i = R + grp + G * (kRU * st + j);
                rw[j] = 0;
                old[j] = 0ull;
                if (i < n) {
                  rw[j] = sh.map[i];
                  old[j] = rd(rw[j], cw);
                }
              }
            };
            auto update_stage = [&](int st, const int (&rw)[kRU], const uint64_t (&old)[kRU]) {
              uint64_t acc[kRU], cc[kRU];
#pragma unroll
              for (int j = 0; j < kRU; ++j) {
                const int i = R + grp + G * (kRU * st + j);
                cc[j] = i < n ? sh.cvec[i - R] : 0ull;
                acc[j] = old[j];
              }
#pragma unroll 4
              for (int g = 0; g < 16; ++g)
#pragma unroll
                for (int j = 0; j < kRU; ++j) acc[j] ^= sh.tr.up.T[g][(cc[j] >> (4 * g)) & 15u][w];
#pragma unroll
              for (int j = 0; j < kRU; ++j) {
                const int i = R + grp + G * (kRU * st + j);
                if (i < n) W[(size_t)rw[j] * ld + cw] = acc[j];
              }
            };
            load_stage(0, rowA, oldA);
            for (int st = 0; st < nst; st += 2) {
              if (st + 1 < nst) load_stage(st + 1, rowB, oldB);
              update_stage(st, rowA, oldA);
              if (st + 1 < nst) {
                if (st + 2 < nst) load_stage(st + 2, rowA, oldA);
                update_stage(st + 1, rowB, oldB);
              }
            }
          }
        }
      }
      R += r;
      __syncthreads();  // the next panel reads words written above
    }

    // ---- outputs
    const int rank = R;
    int32_t *pcol = (int32_t *)sh.cvec;  // pivot column of pivot t
    for (int t = tid; t < rank; t += NT) {
      int j = 0;
      for (int jj = 0; jj < nq; ++jj)
        if (t >= sh.pR[jj] && t < sh.pR[jj] + sh.pr[jj]) j = jj;
      uint64_t Kj = sh.pK[j];
      for (int s = t - sh.pR[j]; s > 0; --s) Kj &= Kj - 1ull;
      pcol[t] = 64 * j + (int)__builtin_ctzll(Kj);
    }
    __syncthreads();
    if (tid == 0) a.rank[d.idx] = rank;
    if (a.pivcols)
      for (int t = tid; t < kmin; t += NT) a.pivcols[d.c + t] = t < rank ? pcol[t] : -1;
    if (a.perm)
      for (int i = tid; i < n; i += NT) a.perm[d.p + i] = sh.map[i];
    // One pass over the positions, 8 lanes per row (lane w8 holds words w8,
    // w8 + 8, ...): each row's words are read once (the next rows' while the
    // current ones are written); position t < kmin writes its E row, and the
    // row's panel words are staged in LDS so that each lane forms its L words.
    const int w8 = tid & 7, rg = tid >> 3;
    constexpr int kOW = kBatchMaxPanels / 8;  // words per lane
    const int Lw = (kmin + 63) >> 6;
    if (a.L && tid < Lw) {  // first panel whose pivot range reaches past column 64 * lw
      int j = 0;
      while (j < nq && sh.pR[j] + sh.pr[j] <= 64 * tid) ++j;
      sh.lj0[tid] = j;
    }
    __syncthreads();
    if (a.E || a.L) {
      uint64_t *E = a.E ? a.E + d.e : nullptr;
      uint64_t *L = a.L ? a.L + d.l : nullptr;
      auto load_row = [&](int i, uint64_t (&x)[kOW]) {
        const size_t src = i < n ? (size_t)sh.map[i] * ld : 0;
#pragma unroll
        for (int jj = 0; jj < kOW; ++jj) {
          const int w = w8 + 8 * jj;
          x[jj] = (i < n && w < Mw) ? W[src + w] : 0ull;
        }
      };
      uint64_t x[kOW], xn[kOW];
      load_row(rg, x);
      for (int i0 = 0; i0 < n; i0 += NT / 8) {
        const int i = i0 + rg;
        load_row(i + NT / 8, xn);
        if (E && i < kmin) {
          const int pc = i < rank ? pcol[i] : 0, qt = pc >> 6;
#pragma unroll
          for (int jj = 0; jj < kOW; ++jj) {
            const int w = w8 + 8 * jj;
            if (w < Mw) {
              uint64_t v = (i < rank && w >= qt) ? x[jj] : 0ull;
              if (w == qt) v &= ~0ull << (pc & 63);
              if (w == Mw - 1) v &= pad_mask(m, w);
              __builtin_nontemporal_store(v, &E[(size_t)i * Mw + w]);
            }
          }
        }
        if (L) {
#pragma unroll
          for (int jj = 0; jj < kOW; ++jj) {
            const int w = w8 + 8 * jj;
            if (w < nq) sh.tr.rowq[rg][w] = x[jj];
          }
          __syncthreads();
          if (i < n) {
#pragma unroll
            for (int jj = 0; jj < kOW; ++jj) {
              const int lw = w8 + 8 * jj;
              if (lw < Lw) {
                const int c_lo = 64 * lw;
                uint64_t v = 0ull;
                for (int j = sh.lj0[lw]; j < nq && sh.pR[j] < c_lo + 64; ++j) {
                  const int Rj = sh.pR[j], rj = sh.pr[j];
                  if (rj == 0 || i < Rj) continue;
                  const uint64_t xw = sh.tr.rowq[rg][j];
                  const uint64_t Kj = sh.pK[j];
                  uint64_t bits;
                  if (i < Rj + rj) {
                    const int s = i - Rj, kk = pcol[i] & 63;
                    const uint64_t lo = xw & ((1ull << kk) - 1ull);
                    bits = (Kj == ~0ull ? lo : compress(lo, Kj, sh.pmv[j])) | (1ull << s);
                  } else {
                    bits = Kj == ~0ull ? xw : compress(xw, Kj, sh.pmv[j]);  // a full panel needs no compression
                  }
                  const int shf = Rj - c_lo;
                  v |= shf >= 0 ? (bits << shf) : (bits >> (-shf));
                }
                __builtin_nontemporal_store(v, &L[(size_t)i * Lw + lw]);
              }
            }
          }
          __syncthreads();
        }
#pragma unroll
        for (int jj = 0; jj < kOW; ++jj) x[jj] = xn[jj];
      }
    }
  }
}

__global__ void k_batch_reset(uint32_t *counter) {
  if (threadIdx.x == 0) *counter = 0u;
}

// ---------------------------------------------------------------- solve
// One wave per system A x = b from the factors P*A = L*E (the use of the
// decomposition named in Section 1): y = L_top^-1 (P b)_top by blocks of 64
// pivots, consistency L_bot y = (P b)_bot, then x from E by back-substitution
// with the free (non-pivot) variables zero.  Within a block of 64 the
// triangular recurrences run on lane-indexed registers; across blocks they are
// parities of staged rows against the finished part.
constexpr int kSolveNT = 64;
constexpr int kSolveU = 8;  // words (or row groups) whose loads one lane issues together

__global__ __launch_bounds__(kSolveNT) void k_batch_solve(BatchSolveArgs a) {
  __shared__ uint64_t pb[kBatchMaxDim / 64], y[kBatchMaxDim / 64], xs[kBatchMaxDim / 64];
  __shared__ uint64_t blk[64][kBatchMaxDim / 64 + 1];
  const int lane = threadIdx.x;
  const BatchDesc d = a.d[blockIdx.x];
  const int n = d.n, m = d.m, kmin = n < m ? n : m;
  const int Mw = (m + 63) >> 6, Lw = (kmin + 63) >> 6, nbw = (n + 63) >> 6;
  int64_t rr = a.rank[d.idx];
  const int r = rr < 0 ? 0 : (rr > kmin ? kmin : (int)rr);
  const uint64_t *L = a.L + d.l, *E = a.E + d.e, *B = a.B + d.b;
  const int64_t *perm = a.perm + d.p, *pivcols = a.pivcols + d.c;

  if (lane < kBatchMaxDim / 64) {
    y[lane] = 0ull;
    xs[lane] = 0ull;
    pb[lane] = 0ull;
  }
  __syncthreads();
  // (P b): bit i is bit perm[i] of b; eight 64-row groups per round, their
  // loads issued together
  for (int c0 = 0; c0 < nbw; c0 += kSolveU) {
    int64_t pi[kSolveU];
#pragma unroll
    for (int j = 0; j < kSolveU; ++j) {
      const int i = 64 * (c0 + j) + lane;
      pi[j] = i < n ? perm[i] : 0;
    }
    uint64_t bw[kSolveU];
#pragma unroll
    for (int j = 0; j < kSolveU; ++j) {
      pi[j] = pi[j] < 0 ? 0 : (pi[j] >= n ? n - 1 : pi[j]);
      bw[j] = (64 * (c0 + j) + lane < n) ? B[pi[j] >> 6] : 0ull;
    }
#pragma unroll
    for (int j = 0; j < kSolveU; ++j) {
      const uint64_t wbits = __ballot((bw[j] >> (pi[j] & 63)) & 1ull);
      if (lane == 0 && c0 + j < nbw) pb[c0 + j] = wbits;
    }
  }
  __syncthreads();

  // ---- forward substitution with L's unit lower r x r block
  const int nblk = (r + 63) >> 6;
  for (int b = 0; b < nblk; ++b) {
    const int t0 = 64 * b, nb = (r - t0) < 64 ? (r - t0) : 64;
    // lane = row t0 + lane: the parity of its words before b with y, and its
    // diagonal word b, read kSolveU words at a time
    uint32_t acc = (uint32_t)((pb[b] >> lane) & 1ull);
    uint64_t dw = 0ull;
    const uint64_t *Lrow = L + (size_t)(t0 + lane) * Lw;
    for (int w0 = 0; w0 <= b; w0 += kSolveU) {
      uint64_t v[kSolveU];
#pragma unroll
      for (int j = 0; j < kSolveU; ++j) v[j] = (lane < nb && w0 + j <= b) ? Lrow[w0 + j] : 0ull;
#pragma unroll
      for (int j = 0; j < kSolveU; ++j) {
        if (w0 + j < b) acc ^= (uint32_t)__popcll(v[j] & y[w0 + j]) & 1u;
        if (w0 + j == b) dw = v[j] & ((1ull << lane) - 1ull);
      }
    }
    uint64_t yb = 0ull;
    for (int s = 0; s < nb; ++s) {
      const uint64_t ds = rdl64b(dw, s);
      const uint32_t as = __builtin_amdgcn_readlane(acc, s);
      yb |= (uint64_t)((as ^ (uint32_t)__popcll(ds & yb)) & 1u) << s;
    }
    __syncthreads();
    if (lane == 0) y[b] = yb;
    __syncthreads();
  }

  // ---- consistency of the rows below the pivots
  uint64_t bad = 0ull;
  for (int i0 = r; i0 < n; i0 += 64) {
    const int i = i0 + lane;
    uint32_t v = 0u;
    if (i < n) {
      v = (uint32_t)((pb[i >> 6] >> (i & 63)) & 1ull);
      const uint64_t *Lrow = L + (size_t)i * Lw;
      for (int w0 = 0; w0 < nblk; w0 += kSolveU) {
        uint64_t lv[kSolveU];
#pragma unroll
        for (int j = 0; j < kSolveU; ++j) lv[j] = w0 + j < nblk ? Lrow[w0 + j] : 0ull;
#pragma unroll
        for (int j = 0; j < kSolveU; ++j)
          if (w0 + j < nblk) v ^= (uint32_t)__popcll(lv[j] & y[w0 + j]) & 1u;
      }
    }
    bad |= __ballot(v);
  }
  const bool ok = bad == 0ull;

  // ---- back-substitution with E, free variables zero
  if (ok) {
    for (int b = nblk - 1; b >= 0; --b) {
      const int t0 = 64 * b, nb = (r - t0) < 64 ? (r - t0) : 64;
      __syncthreads();  // xs holds the solved blocks after b
      const bool valid = lane < nb;
      int pc = 0;
      if (valid) {
        const int64_t v = pivcols[t0 + lane];
        pc = v < 0 ? 0 : (v >= m ? m - 1 : (int)v);
      }
      // lane = row t0 + lane of E: its parity with the solved part, and the row
      // itself staged in the lane's own slot of blk for the bits at this
      // block's pivot columns
      uint32_t acc = valid ? (uint32_t)((y[b] >> lane) & 1ull) : 0u;
      const uint64_t *Erow = E + (size_t)(t0 + lane) * Mw;
      for (int w0 = 0; w0 < Mw; w0 += kSolveU) {
        uint64_t v[kSolveU];
#pragma unroll
        for (int j = 0; j < kSolveU; ++j) v[j] = (valid && w0 + j < Mw) ? Erow[w0 + j] : 0ull;
#pragma unroll
        for (int j = 0; j < kSolveU; ++j)
          if (w0 + j < Mw) {
            acc ^= (uint32_t)__popcll(v[j] & xs[w0 + j]) & 1u;
            blk[lane][w0 + j] = v[j];
          }
      }
      uint64_t dm = 0ull;
      for (int u = 0; u < nb; ++u) {
        const int pu = __builtin_amdgcn_readlane(pc, u);
        dm |= ((blk[lane][pu >> 6] >> (pu & 63)) & 1ull) << u;
      }
      dm &= lane >= 63 ? 0ull : (~0ull << (lane + 1));
      uint64_t xb = 0ull;
      for (int u = nb - 1; u >= 0; --u) {
        const uint64_t du = rdl64b(dm, u);
        const uint32_t au = __builtin_amdgcn_readlane(acc, u);
        xb |= (uint64_t)((au ^ (uint32_t)__popcll(du & xb)) & 1u) << u;
      }
      __syncthreads();
      if (valid && ((xb >> lane) & 1ull)) atomicOr((unsigned long long *)&xs[pc >> 6], 1ull << (pc & 63));
    }
  }
  __syncthreads();
  uint64_t *X = a.X + d.x;
  for (int w = lane; w < Mw; w += kSolveNT) X[w] = ok ? xs[w] : 0ull;
  if (lane == 0) a.consistent[d.idx] = ok ? 1 : 0;
}

}  // namespace

int batch_workers(int ncu) { return kBatchWGPerCU * ncu; }

hipError_t launch_batch_dec(const BatchArgs &a, int workers, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, a.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_dec, dim3(workers), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_batch_solve(const BatchSolveArgs &a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_solve, dim3(a.count), dim3(kSolveNT), 0, s, a);
  return hipGetLastError();
}

}  // namespace gf2
