// k_panel.hip -- the per-panel steps of the block decomposition (Section 4).
//
// A trailing-update panel is s <= 8 consecutive 64-column sub-panels (words
// q0 .. q0+s-1):
//   k_chain   one workgroup per panel: for each sub-panel q in order it selects
//             the pivots of the 64 columns of word q (procedure buildZ,
//             Sections 4.2-4.4): for each bit k in order, the first row at or
//             below the next free position whose reduced bit k is 1 becomes the
//             pivot and is exchanged with that position (a transposition).  It
//             produces the pivot columns, the coefficient map Zc (row j of Zc
//             gives the multipliers of bit j, so y = x * Zc are a row's
//             multipliers -- the role of Z in D*Z = Y, Section 4.1), the
//             inverse of the sub-panel's unit lower block and the pivot rows in
//             final form, and applies the sub-panel to the rows it holds in LDS.
//   k_post    one launch per panel after its chain: the panel's net row
//             permutation on all words outside the panel (P^(j) applied to all
//             columns), the pivot rows right of the panel in echelon form
//             (E = L_pp^{-1} * rows, block forward substitution over the
//             sub-panels), and every row below the pivots brought to the
//             panel's last sub-panel so its panel words hold its multipliers
//             (eq. (Aj) restricted to the panel).
// The trailing product (Schur complement, eq. (Aj)) is k_gemm.
//
// Reduced bit of a row.  The chain kernel keeps, for every pivot found so
// far, its fully reduced row M_j (indexed by the pivot's bit position j; rows
// of M are the identity on pivot positions -- the words M of buildZ).  The
// reduced form of any row x is Proj(x) = x xor sum_{pivot j} x_j M_j; its bit k
// is the parity test popC(c AND x) of buildZ with c = e_k xor sum_j M_j[k] e_j.
// Rows of a window (the first kWin free positions) are kept reduced in
// registers; rows below the window are tested with Proj on demand.
#include <type_traits>

#include "gf2_internal.h"

namespace gf2 {

__device__ inline uint64_t rdl64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// lane l's value of the 64-bit pair (lo, hi), as a wave-uniform value
__device__ inline uint64_t rdl64p(uint32_t lo, uint32_t hi, int l) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)hi, l) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)lo, l);
}

// bit s (uniform, 0..63) of the 64-bit pair (lo, hi): 0 or all ones
__device__ inline uint32_t lanebit(uint32_t lo, uint32_t hi, int s) {
  const uint64_t v = (((uint64_t)hi << 32) | lo) >> s;
  return (uint32_t)__builtin_amdgcn_sbfe((int)(uint32_t)v, 0, 1);
}

// ---------------------------------------------------------------- panel-local update
// Inside a panel, rows are updated lazily ("left-looking"): row p carries a
// level lvl[p] = 16*q0 + L meaning sub-panels 0..L-1 of the panel starting at
// word q0 have been applied to its panel words (words q0..q0+L-1 then hold its
// multipliers y_c, the later words the updated entries).  Applying sub-panel c
// to a row: y = word_c * Zc_c (its multipliers), word_c = y, and every later
// panel word w gets word_w ^= y * E_c[w] (E_c[w] = word w of the pivot rows of
// sub-panel c) -- eq. (Aj) restricted to the panel, one sub-panel at a time.
// Four-Russians with 4-bit tables: 16 tables of 16 entries per word.
constexpr int kPairs = kMaxPanelWords * (kMaxPanelWords - 1) / 2;
__host__ __device__ inline int pidx(int c, int wd) { return c * (2 * kMaxPanelWords - c - 1) / 2 + (wd - c - 1); }

struct PanelTables {
  uint64_t Tz[kMaxPanelWords][16][16];  // y = x * Zc_c
  uint64_t Te[kPairs][16][16];          // y * E_c[w]
};
static_assert(sizeof(PanelTables) == (size_t)kPanelTabWords * 8, "table buffer size");

// Apply sub-panels [from, to) to the panel words x[], touching words <= wmax.
__device__ inline void panel_update(uint64_t (&x)[kMaxPanelWords], int from, int to, int wmax,
                                    const PanelTables &pt) {
#pragma unroll
  for (int c = 0; c < kMaxPanelWords - 1; ++c) {
    if (c >= from && c < to) {
      uint64_t y = 0ull;
#pragma unroll
      for (int g = 0; g < 16; ++g) y ^= pt.Tz[c][g][(x[c] >> (4 * g)) & 15u];
      x[c] = y;
#pragma unroll
      for (int wd = c + 1; wd < kMaxPanelWords; ++wd) {
        if (wd <= wmax) {
          uint64_t v = 0ull;
#pragma unroll
          for (int g = 0; g < 16; ++g) v ^= pt.Te[pidx(c, wd)][g][(y >> (4 * g)) & 15u];
          x[wd] ^= v;
        }
      }
    }
  }
  if (kMaxPanelWords - 1 >= from && kMaxPanelWords - 1 < to) {  // last sub-panel: multipliers only
    constexpr int c = kMaxPanelWords - 1;
    uint64_t y = 0ull;
#pragma unroll
    for (int g = 0; g < 16; ++g) y ^= pt.Tz[c][g][(x[c] >> (4 * g)) & 15u];
    x[c] = y;
  }
}

__device__ inline int row_level(const DecWork &w, int64_t p, int q0) {
  const int v = w.lvl[p];
  return (v >> 4) == q0 ? (v & 15) : 0;
}

// ---------------------------------------------------------------- pivot selection
// One workgroup of 8 waves factors a whole panel (s <= 8 sub-panels).  The rows
// at positions [R0, R0 + 64 s + kWin) -- every position a window of this panel
// can reach -- are held in LDS ("block") with their panel words, and are
// brought up to date right-looking after each sub-panel by all waves (eq. (Aj)
// restricted to the panel).  Rows further down stay in HBM at their level and
// are only read by the rare scan below the window.
//
// Per sub-panel b (word q = q0 + b, rank Rb before it): the window is the kWin
// positions from Rb, slot s = position Rb + s.  Wave 0 alone takes the pivot
// decisions with lane-indexed registers: the first 64 slots are kept reduced by
// every pivot; the second 64 are reduced on demand (Proj, 4-bit tables) only
// when the first half has no candidate.  For each bit k the candidates are one
// ballot ANDed with the scalar mask of free slots; the first candidate becomes
// the pivot of position Rb + ib (a transposition of slots), and every other
// candidate is reduced by it.  The fully reduced pivot rows M_j (lane j) and
// their coefficient map Zc are updated in the same step.  When no window row
// has bit k, all threads scan the rows below the window with
// Proj(x) = x xor sum_j x_j M_j and keep an over-approximation F of the bits
// such rows can still have, so a zero tail costs one scan per sub-panel.
constexpr int kBlkMax = 64 * kMaxPanelWords + kWin;  // block rows
constexpr int kMbMax = 64 * kMaxPanelWords;          // rows moved below the block per panel
constexpr int kChainThreads = 512;

struct ChainShared {
  PanelTables pt;                            // tables of the panel's finished sub-panels
  uint64_t blk[kBlkMax][kMaxPanelWords];     // block rows: panel words, level = current sub-panel
  int bsrc[kBlkMax];                         // panel-start position of the row at block index i
  uint64_t win[kWin][kMaxPanelWords];        // staging for window permutations
  uint64_t Pt[kMaxPanelWords - 1][16][16];   // 4-bit tables of the pivot rows before the solve
  int wsrc[kWin];
  int sorg[kWin];
  uint64_t Tp[16][16];                       // 4-bit tables of M: Proj during a scan
  uint64_t Tw[16][16];                       // Proj tables private to the pivot wave
  uint64_t Ms[64];
  uint64_t Li[64];
  uint64_t ynext[kWin];                      // y = (word b) * Zc of the next window's rows
  int mb_pos[kMbMax], mb_src[kMbMax];        // positions below the block that received a block row
  int mb_n;
  int scan_best;
  unsigned long long scan_F;
  int nmv;
  int ctl_need, ctl_k, ctl_ib;
  int sp_new, sp_base;
};
// end-of-panel staging, placed over the (then dead) tables
struct ChainMoved {
  int64_t perm[kBlkMax + kMbMax];
  int pos[kBlkMax + kMbMax];
  int src[kBlkMax + kMbMax];
  int sps[kBlkMax + kMbMax];
  int spi[kBlkMax + kMbMax];
};
static_assert(sizeof(ChainMoved) <= sizeof(PanelTables), "staging fits in the table area");

__device__ inline uint64_t proj4(const uint64_t (&T)[16][16], uint64_t x) {
  uint64_t r = 0ull;
#pragma unroll
  for (int g = 0; g < 16; ++g) r ^= T[g][(x >> (4 * g)) & 15u];
  return r;
}

// 16 tables of 16 entries over the 64 words src[0..63] (entry v of table g = XOR
// of src[4g + bit] for the set bits of v); one entry per thread of the range.
__device__ inline uint64_t table4_entry(const uint64_t *src, int e) {
  const int g = e >> 4, v = e & 15;
  uint64_t acc = 0ull;
#pragma unroll
  for (int bb = 0; bb < 4; ++bb)
    if (v & (1 << bb)) acc ^= src[4 * g + bb];
  return acc;
}

__global__ __launch_bounds__(kChainThreads) void k_chain(DecWork w, int q0, int s_eff, int flag_q0, int spb) {
  constexpr int NT = kChainThreads;
  __shared__ ChainShared sh;
  // (wave index made visibly uniform, so the pivot wave's loop stays scalar)
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t n = w.n, ldw = w.ldw;
  uint64_t *W = w.W;

  const int64_t R0 = w.st->R;
  const int cnt = w.st->bp_count;
  const uint32_t nz = flag_q0 >= 0 ? w.nzflag[flag_q0] : 1u;
  // forget the previous panel's row list
  for (int j = tid; j < cnt; j += NT) {
    const int p = w.bp_list[j];
    w.bp_src[p] = p;
    w.bp_mark[p] = 0;
  }
  if (R0 >= n || nz == 0u) {  // no rows left, or the Schur complement is already zero
    __syncthreads();
    if (tid == 0) w.st->bp_count = 0;
    for (int b = 0; b < s_eff; ++b) {
      if (tid < 64) {
        w.Zc[(size_t)(q0 + b) * 64 + tid] = 0ull;
        w.Linv[(size_t)(q0 + b) * 64 + tid] = 0ull;
      }
      if (tid == 0) {
        w.sub[q0 + b].R = R0;
        w.sub[q0 + b].r = 0;
        w.sub[q0 + b].pivmask = 0ull;
      }
    }
    return;
  }
  const int nblk = (int)((n - R0) < (int64_t)(64 * s_eff + kWin) ? (n - R0) : (int64_t)(64 * s_eff + kWin));
  {
    constexpr int PER = kBlkMax * kMaxPanelWords / NT;
    uint64_t v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NT, i = e >> 3, j = e & 7;
      v[u] = (i < nblk && j < s_eff) ? W[widx(ldw, R0 + i, q0 + j)] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NT, i = e >> 3, j = e & 7;
      if (i < nblk) sh.blk[i][j] = v[u];
    }
  }
  for (int i = tid; i < nblk; i += NT) sh.bsrc[i] = (int)(R0 + i);
  if (tid == 0) sh.mb_n = 0;
  __syncthreads();
  if (tid == 0) w.st->bp_count = 0;

  // window permutation (sorg, written by the pivot wave) applied to the block rows
  auto materialize = [&](int wb) {
    for (int e = tid; e < kWin * kMaxPanelWords; e += NT) {
      const int s = e >> 3, j = e & 7;
      if (wb + s < nblk) {
        sh.win[s][j] = sh.blk[wb + sh.sorg[s]][j];
        if (j == 0) sh.wsrc[s] = sh.bsrc[wb + sh.sorg[s]];
      }
    }
    __syncthreads();
    for (int e = tid; e < kWin * kMaxPanelWords; e += NT) {
      const int s = e >> 3, j = e & 7;
      if (wb + s < nblk) {
        sh.blk[wb + s][j] = sh.win[s][j];
        if (j == 0) sh.bsrc[wb + s] = sh.wsrc[s];
      }
    }
    __syncthreads();
  };

  int wb = 0;  // block index of position Rb
  // The update of the block rows by sub-panel b runs in two parts: the next
  // window's word b + 1 (all the next search reads) right away, the rest by
  // waves 1..7 while wave 0 searches the pivots of sub-panel b + 1.
  int def_b = -1, def_win = 0;  // deferred sub-panel; rows [wb, def_win) hold word b + 1 already
  for (int b = 0; b < s_eff; ++b) {
    const int q = q0 + b;
    const int64_t Rb = R0 + wb;
    int nbits = (int)(w.m - 64ll * q);
    if (nbits > 64) nbits = 64;

    // ---- pivot-wave state.  Slot s of the window is position Rb + s; the
    // first half (slots 0..63) is kept reduced by every pivot, the second half
    // holds rows that are reduced on demand (Proj) when the first half has no
    // candidate.  A pivot leaves the first half: its slot reads zero there
    // (so it is never a candidate again) and lane t of e holds pivot t.
    uint32_t a_lo = 0u, a_hi = 0u, b_lo = 0u, b_hi = 0u, e_lo = 0u, e_hi = 0u;
    int org0 = lane, org1 = 64 + lane;
    uint64_t act1 = 0ull;
    uint32_t m_lo = 0u, m_hi = 0u, y_lo = 0u, y_hi = 0u;  // M_j and Zc row j (lane j)
    uint64_t pivmask = 0ull, F = 0ull;
    bool Fknown = false;
    uint64_t Fdone = 0ull;  // pivots (their bits) already folded into F
    int ib = 0;
    if (wv == 0) {
      const bool v0 = wb + lane < nblk, v1 = wb + 64 + lane < nblk;
      if (v0) { const uint64_t x = sh.blk[wb + lane][b]; a_lo = (uint32_t)x; a_hi = (uint32_t)(x >> 32); }
      if (v1) { const uint64_t x = sh.blk[wb + 64 + lane][b]; b_lo = (uint32_t)x; b_hi = (uint32_t)(x >> 32); }
      act1 = __ballot(v1);
    }

    // all ones in the lanes whose x has bit s (s < 32), zero elsewhere
    auto bit_lanes = [](uint32_t x, int s) -> uint32_t { return (uint32_t)__builtin_amdgcn_sbfe((int)x, s, 1); };
    // pivot t = ib for bit k with reduced row (p_lo, p_hi): bookkeeping rows M
    // (RREF of the pivots so far), the coefficient map and the pivot row.
    // mm: all ones in the lanes j of earlier pivots whose M_j has bit k.
    auto commit = [&](int k, uint32_t p_lo, uint32_t p_hi, uint32_t mm) {
      const uint64_t tb = 1ull << ib;
      const uint32_t t_lo = (uint32_t)tb, t_hi = (uint32_t)(tb >> 32);
      m_lo ^= p_lo & mm;
      m_hi ^= p_hi & mm;
      y_lo ^= t_lo & mm;
      y_hi ^= t_hi & mm;
      m_lo = wrlane(p_lo, k, m_lo);
      m_hi = wrlane(p_hi, k, m_hi);
      y_lo = wrlane(t_lo, k, y_lo);
      y_hi = wrlane(t_hi, k, y_hi);
      e_lo = wrlane(p_lo, ib, e_lo);
      e_hi = wrlane(p_hi, ib, e_hi);
      const uint64_t kb = 1ull << k;
      pivmask |= kb;
      ++ib;
    };

    // Bits [k, kend) whose word half is fixed, while the first half of the
    // window has a candidate (the common case); returns at the first bit where
    // it has none.  Every candidate is reduced by the pivot (which empties the
    // pivot's own slot), then the row of slot ib moves to the pivot's slot.
    // The next bit's candidates are taken before the pivot's bookkeeping, so
    // that the ballot's latency overlaps it.
    auto run_bits = [&](auto hi_tag, int &k, int kend) {
      constexpr bool HI = decltype(hi_tag)::value;
      uint32_t vc = bit_lanes(HI ? a_hi : a_lo, k & 31);  // candidates of bit k (lane masks)
      uint64_t c0 = __ballot(vc != 0u);
      // bit kk; false when the first half has no candidate for it
      auto step = [&](int kk) __attribute__((always_inline)) -> bool {
        if (__builtin_expect(c0 == 0ull, 0)) return false;
        const int sp = __builtin_ctzll(c0);
        const uint32_t p_lo = __builtin_amdgcn_readlane(a_lo, sp), p_hi = __builtin_amdgcn_readlane(a_hi, sp);
        a_lo ^= p_lo & vc;
        a_hi ^= p_hi & vc;
        if (sp != ib) {  // slot ib holds no candidate: its row moves to slot sp
          const uint32_t i_lo = __builtin_amdgcn_readlane(a_lo, ib), i_hi = __builtin_amdgcn_readlane(a_hi, ib);
          const int p_org = __builtin_amdgcn_readlane(org0, sp), i_org = __builtin_amdgcn_readlane(org0, ib);
          a_lo = wrlane(i_lo, sp, a_lo);
          a_hi = wrlane(i_hi, sp, a_hi);
          org0 = wrlane(i_org, sp, org0);
          a_lo = wrlane(0u, ib, a_lo);
          a_hi = wrlane(0u, ib, a_hi);
          org0 = wrlane(p_org, ib, org0);
        }
        if ((kk & 31) != 31) {
          vc = bit_lanes(HI ? a_hi : a_lo, (kk & 31) + 1);
          c0 = __ballot(vc != 0u);
        }
        commit(kk, p_lo, p_hi, bit_lanes(HI ? m_hi : m_lo, kk & 31));
        return true;
      };
      constexpr int k0 = HI ? 32 : 0;
      if (k == k0 && kend == k0 + 32) {  // a whole half from its first bit: constant bit positions
#pragma unroll
        for (int i = 0; i < 32; ++i)
          if (!step(k0 + i)) {
            k = k0 + i;
            return;
          }
        k = kend;
        return;
      }
      for (; k < kend; ++k)
        if (!step(k)) return;
    };

    // Pivot wave: bits from k on, until the end of the sub-panel or a bit that
    // needs the scan below the window (returned true).
    auto pivot_wave = [&](int &k) -> bool {
      while (true) {
        if (k < 32) run_bits(std::false_type{}, k, nbits < 32 ? nbits : 32);
        if (k >= 32 && k < nbits) run_bits(std::true_type{}, k, nbits);
        if (k >= nbits) return false;
        // bit k: no candidate in the first half; reduce the second half (Proj)
        const uint32_t bit = 1u << (k & 31);
        sh.Ms[lane] = ((uint64_t)m_hi << 32) | m_lo;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int u = 0; u < 4; ++u) sh.Tw[(lane >> 4) + 4 * u][lane & 15] = table4_entry(sh.Ms, lane + 64 * u);
        __builtin_amdgcn_wave_barrier();
        {
          const uint64_t x = ((uint64_t)b_hi << 32) | b_lo;
          const uint64_t xr = x ^ proj4(sh.Tw, x);
          b_lo = (uint32_t)xr;
          b_hi = (uint32_t)(xr >> 32);
        }
        __builtin_amdgcn_wave_barrier();
        const uint64_t c1 = __ballot(((k < 32 ? b_lo : b_hi) & bit) != 0u) & act1;
        if (c1) {  // pivot from the second half; the row of slot ib takes its slot
          const int sp = __builtin_ctzll(c1);
          const uint32_t p_lo = __builtin_amdgcn_readlane(b_lo, sp), p_hi = __builtin_amdgcn_readlane(b_hi, sp);
          const int p_org = __builtin_amdgcn_readlane(org1, sp);
          const uint32_t i_lo = __builtin_amdgcn_readlane(a_lo, ib), i_hi = __builtin_amdgcn_readlane(a_hi, ib);
          const int i_org = __builtin_amdgcn_readlane(org0, ib);
          b_lo = wrlane(i_lo, sp, b_lo);
          b_hi = wrlane(i_hi, sp, b_hi);
          org1 = wrlane(i_org, sp, org1);
          a_lo = wrlane(0u, ib, a_lo);
          a_hi = wrlane(0u, ib, a_hi);
          org0 = wrlane(p_org, ib, org0);
          commit(k, p_lo, p_hi, bit_lanes(k < 32 ? m_lo : m_hi, k & 31));
          ++k;
          continue;
        }
        if (Fknown) {
          // F is brought up to date only here, where it is read: the pivots
          // taken since, in order, from their rows in e (pivot t is the t-th
          // set bit of pivmask)
          for (uint64_t todo = pivmask & ~Fdone; todo; todo &= todo - 1ull) {
            const int kf = __builtin_ctzll(todo);
            const uint64_t fb = 1ull << kf;
            if (F & fb) {
              const int t = __popcll(pivmask & (fb - 1ull));
              F |= ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(e_hi, t) << 32) |
                   (uint32_t)__builtin_amdgcn_readlane(e_lo, t);
            }
            F &= ~fb;
          }
          Fdone = pivmask;
          if (!((F >> k) & 1ull)) {  // no row below the window can have bit k
            ++k;
            continue;
          }
        }
        return true;
      }
    };

    int k = 0;
    if (wv != 0 && def_b >= 0) {  // the rest of sub-panel def_b's block-row update
      for (int i = wb + tid - 64; i < nblk; i += NT - 64) {
        uint64_t x[kMaxPanelWords];
#pragma unroll
        for (int j = 0; j < kMaxPanelWords; ++j) x[j] = sh.blk[i][j];
        panel_update(x, def_b, def_b + 1, s_eff - 1, sh.pt);
#pragma unroll
        for (int j = 0; j < kMaxPanelWords; ++j)
          if (j != def_b + 1 || i >= def_win) sh.blk[i][j] = x[j];
      }
    }
    def_b = -1;
    while (true) {
      if (wv == 0) {
        const bool need = pivot_wave(k);
        if (lane == 0) {
          sh.ctl_need = need ? 1 : 0;
          sh.ctl_k = k;
          sh.ctl_ib = ib;
        }
        sh.sorg[lane] = org0;
        sh.sorg[64 + lane] = org1;
        // M for a scan below the window; at the end the coefficient map
        sh.Ms[lane] = need ? ((uint64_t)m_hi << 32) | m_lo : ((uint64_t)y_hi << 32) | y_lo;
      }
      __syncthreads();
      if (!sh.ctl_need) break;
      // ---- bit kk: no window row has it; scan the rows below the window (all threads)
      const int kk = sh.ctl_k, ibs = sh.ctl_ib;
      const uint64_t kb = 1ull << kk;
      materialize(wb);
      if (tid < 256) sh.Tp[tid >> 4][tid & 15] = table4_entry(sh.Ms, tid);
      if (tid == 0) {
        sh.scan_best = 0x7fffffff;
        sh.scan_F = 0ull;
      }
      __syncthreads();
      int best = 0x7fffffff;
      uint64_t Floc = 0ull;
      for (int64_t p = Rb + kWin + tid; p < n; p += NT) {
        uint64_t xq;
        if (p - R0 < nblk) {
          xq = sh.blk[p - R0][b];
        } else {
          uint64_t x[kMaxPanelWords];
#pragma unroll
          for (int j = 0; j < kMaxPanelWords; ++j) x[j] = j <= b ? W[widx(ldw, p, q0 + j)] : 0ull;
          panel_update(x, row_level(w, p, q0), b, b, sh.pt);
          xq = x[0];
#pragma unroll
          for (int j = 1; j < kMaxPanelWords; ++j)
            if (j == b) xq = x[j];
        }
        const uint64_t pr = xq ^ proj4(sh.Tp, xq);
        Floc |= pr;
        if ((pr & kb) && (int)p < best) best = (int)p;
      }
      if (best != 0x7fffffff) atomicMin(&sh.scan_best, best);
      if (Floc) atomicOr(&sh.scan_F, (unsigned long long)Floc);
      __syncthreads();
      best = __builtin_amdgcn_readfirstlane(sh.scan_best);
      const int si = wb + ibs;
      if (best != 0x7fffffff) {
        // position `best` and slot ib (position Rb + ib) exchange their rows
        if (best - R0 < nblk) {
          const int bi = (int)(best - R0);
          if (tid < kMaxPanelWords) {
            const uint64_t t0 = sh.blk[bi][tid], t1 = sh.blk[si][tid];
            sh.blk[bi][tid] = t1;
            sh.blk[si][tid] = t0;
          }
          if (tid == 0) {
            const int s0 = sh.bsrc[bi];
            sh.bsrc[bi] = sh.bsrc[si];
            sh.bsrc[si] = s0;
          }
        } else if (tid == 0) {
          // a row below the block: bring it to level b; the slot's row takes its
          // place in HBM at level b
          uint64_t x[kMaxPanelWords];
#pragma unroll
          for (int j = 0; j < kMaxPanelWords; ++j) x[j] = j < s_eff ? W[widx(ldw, best, q0 + j)] : 0ull;
          panel_update(x, row_level(w, best, q0), b, s_eff - 1, sh.pt);
          for (int j = 0; j < s_eff; ++j) W[widx(ldw, best, q0 + j)] = sh.blk[si][j];
          w.lvl[best] = (q0 << 4) | b;
          int e = 0;
          while (e < sh.mb_n && sh.mb_pos[e] != best) ++e;
          const int src_in = e < sh.mb_n ? sh.mb_src[e] : best;
          if (e == sh.mb_n) {
            sh.mb_pos[e] = best;
            sh.mb_n = e + 1;
          }
          sh.mb_src[e] = sh.bsrc[si];
#pragma unroll
          for (int j = 0; j < kMaxPanelWords; ++j) sh.blk[si][j] = x[j];
          sh.bsrc[si] = src_in;
        }
        __syncthreads();
      }
      if (wv == 0) {
        org0 = lane;
        org1 = 64 + lane;
        {
          const unsigned long long fv = sh.scan_F;
          F = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(fv >> 32)) << 32) |
              (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)fv);
        }
        Fknown = true;
        Fdone = pivmask;  // (F is the rows' state now)
        if (best != 0x7fffffff) {
          const uint64_t xro = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(a_hi, ib) << 32) |
                               (uint32_t)__builtin_amdgcn_readlane(a_lo, ib);
          const uint64_t xin = sh.blk[si][b];
          const uint64_t xrp = xin ^ proj4(sh.Tp, xin);
          a_lo = wrlane(0u, ib, a_lo);
          a_hi = wrlane(0u, ib, a_hi);
          F |= xro;
          commit(k, (uint32_t)xrp, (uint32_t)(xrp >> 32), bit_lanes(k < 32 ? m_lo : m_hi, k & 31));
        }
        ++k;
      }
      __syncthreads();
    }
    const int r = sh.ctl_ib;
    // (pivot wave) lane t < r: word q of E_t, the coefficient map yM
    const uint64_t yM = ((uint64_t)y_hi << 32) | y_lo;
    const uint64_t xr0 = ((uint64_t)e_hi << 32) | e_lo;
    materialize(wb);

    // ---- multipliers of the pivot rows (unit lower block L_pp) from the
    // coefficient map (in Ms since the search ended): word q of pivot row t
    // at level b lies in the span of E_0..E_t, so y = word * Zc lists its
    // multipliers (bit t set).  Then the block's inverse.  The pivot rows'
    // later words get 4-bit tables.
    if (tid < 256) sh.pt.Tz[b][tid >> 4][tid & 15] = table4_entry(sh.Ms, tid);
    for (int e = tid; e < (s_eff - 1 - b) * 256; e += NT) {
      const int wd = b + 1 + (e >> 8), g = (e >> 4) & 15, v = e & 15;
      uint64_t acc = 0ull;
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
        if ((v & (1 << bb)) && 4 * g + bb < r) acc ^= sh.blk[wb + 4 * g + bb][wd];
      sh.Pt[wd - b - 1][g][v] = acc;
    }
    __syncthreads();
    uint64_t yx = 0ull;
    const int we = wb + r + kWin < nblk ? wb + r + kWin : nblk;  // end of the next window
    if (wv != 0 && b + 1 < s_eff) {
      // meanwhile, the first half of the next window's word b + 1: y = (word b) * Zc
      for (int i = wb + r + tid - 64; i < we; i += NT - 64) sh.ynext[i - wb - r] = proj4(sh.pt.Tz[b], sh.blk[i][b]);
    }
    if (wv == 0) {
      if (lane < r) yx = proj4(sh.pt.Tz[b], sh.blk[wb + lane][b]);
      // Linv = L_pp^{-1} by forward substitution over t: every row s > t whose
      // multipliers include pivot t XORs in the finished row t (a lane read
      // and a masked XOR per step).  Rows and multipliers past r are zero, so
      // all 64 steps run; rows t < 32 have no bits in the high half.
      const uint64_t ylow = lane < r ? (yx & ((1ull << lane) - 1ull)) : 0ull;
      const uint32_t yl_lo = (uint32_t)ylow, yl_hi = (uint32_t)(ylow >> 32);
      uint32_t li_lo = lane < r && lane < 32 ? 1u << lane : 0u;
      uint32_t li_hi = lane < r && lane >= 32 ? 1u << (lane - 32) : 0u;
#pragma unroll
      for (int t = 0; t < 32; ++t) li_lo ^= (uint32_t)__builtin_amdgcn_readlane(li_lo, t) & bit_lanes(yl_lo, t);
#pragma unroll
      for (int t = 32; t < 64; ++t) {
        const uint32_t mt = bit_lanes(yl_hi, t - 32);
        const uint32_t r_lo = __builtin_amdgcn_readlane(li_lo, t), r_hi = __builtin_amdgcn_readlane(li_hi, t);
        li_lo ^= r_lo & mt;
        li_hi ^= r_hi & mt;
      }
      const uint64_t li = ((uint64_t)li_hi << 32) | li_lo;
      sh.Li[lane] = li;
      w.Zc[(size_t)q * 64 + lane] = yM;
      w.Linv[(size_t)q * 64 + lane] = li;
      if ((pivmask >> lane) & 1ull) {
        const int t = __popcll(pivmask & ((1ull << lane) - 1ull));
        w.pivcols[Rb + t] = 64ll * q + lane;
      }
      if (lane == 0) {
        w.sub[q].R = Rb;
        w.sub[q].r = r;
        w.sub[q].pivmask = pivmask;
      }
    }
    __syncthreads();
    // ---- pivot rows in final form: word q = E_t | L_pp bits left of t; later
    // panel words = L_pp^{-1} * (pivot rows at level b), from the tables of
    // those words built before the last barrier
    {
      const int nw = s_eff - 1 - b;
      for (int e = tid; e < r * nw; e += NT) {
        const int t = e / nw, wd = b + 1 + (e - t * nw);
        sh.blk[wb + t][wd] = proj4(sh.Pt[wd - b - 1], sh.Li[t]);
      }
    }
    if (wv == 0 && lane < r) sh.blk[wb + lane][b] = xr0 | (yx & ((1ull << lane) - 1ull));
    __syncthreads();
    // ---- tables of sub-panel b (Tz built above), then every block row below
    // its pivots gets it
    for (int e = tid; e < (s_eff - 1 - b) * 256; e += NT) {
      const int wd = b + 1 + (e >> 8), g = (e >> 4) & 15, v = e & 15;
      uint64_t acc = 0ull;
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
        if ((v & (1 << bb)) && 4 * g + bb < r) acc ^= sh.blk[wb + 4 * g + bb][wd];
      sh.pt.Te[pidx(b, wd)][g][v] = acc;
    }
    __syncthreads();
    if (b + 1 < s_eff) {
      // word b + 1 of the next window's rows: word b + 1 ^= y * E_b[b + 1]
      // (4-bit tables; y = (word b) * Zc_b was formed beside the inverse);
      // the rest is deferred
      for (int i = wb + r + tid; i < we; i += NT) {
        const uint64_t y = sh.ynext[i - wb - r];
        uint64_t v = 0ull;
#pragma unroll
        for (int g = 0; g < 16; ++g) v ^= sh.pt.Te[pidx(b, b + 1)][g][(y >> (4 * g)) & 15u];
        sh.blk[i][b + 1] ^= v;
      }
      def_b = b;
      def_win = we;
    } else {
      for (int i = wb + r + tid; i < nblk; i += NT) {
        uint64_t x[kMaxPanelWords];
#pragma unroll
        for (int j = 0; j < kMaxPanelWords; ++j) x[j] = sh.blk[i][j];
        panel_update(x, b, b + 1, s_eff - 1, sh.pt);
#pragma unroll
        for (int j = 0; j < kMaxPanelWords; ++j) sh.blk[i][j] = x[j];
      }
    }
    __syncthreads();
    wb += r;
  }

  // ---- block rows back to HBM; every row below the pivots is at level s
  {
    constexpr int PER = kBlkMax * kMaxPanelWords / NT;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NT, i = e >> 3, j = e & 7;
      if (i < nblk && j < s_eff) W[widx(ldw, R0 + i, q0 + j)] = sh.blk[i][j];
    }
  }
  for (int i = tid; i < nblk; i += NT) w.lvl[R0 + i] = i < wb ? (q0 << 4) | 15 : (q0 << 4) | s_eff;
  // ---- the panel's tables for the row update after the chain (before the
  // staging below reuses their LDS); sub-panels never reached stay zero there
  {
    const uint64_t *src = &sh.pt.Tz[0][0][0];
    for (int e = tid; e < kPanelTabWords; e += NT) w.ptab[e] = src[e];
  }
  __syncthreads();
  // ---- permutation bookkeeping of every position whose row changed
  ChainMoved &mv = *reinterpret_cast<ChainMoved *>(&sh.pt);
  if (tid == 0) sh.nmv = 0;
  __syncthreads();
  for (int i = tid; i < nblk + sh.mb_n; i += NT) {
    int pos, src;
    if (i < nblk) {
      pos = (int)(R0 + i);
      src = sh.bsrc[i];
    } else {
      pos = sh.mb_pos[i - nblk];
      src = sh.mb_src[i - nblk];
    }
    if (pos != src) {
      const int e = atomicAdd(&sh.nmv, 1);
      mv.pos[e] = pos;
      mv.src[e] = src;
      mv.perm[e] = w.perm[src];
      mv.sps[e] = spb >= 0 ? w.sp_src[(size_t)spb * n + src] : 0;
    }
  }
  __syncthreads();
  const int nmv = sh.nmv;
  // the super-panel's net permutation (spb >= 0: its buffer): the row now at
  // pos was at position sp_src[pos] when the super-panel started; pos joins
  // its list once
  const int spv = spb >= 0 ? spb : 0;
  int32_t *sp_src = w.sp_src + (size_t)spv * n, *sp_mark = w.sp_mark + (size_t)spv * n;
  int32_t *sp_list = w.sp_list + (size_t)spv * kSpListMax;
  if (tid == 0) sh.sp_new = 0;
  __syncthreads();
  for (int e = tid; e < nmv; e += NT) {
    const int pos = mv.pos[e];
    w.perm[pos] = mv.perm[e];
    w.bp_src[pos] = mv.src[e];
    w.bp_mark[pos] = 1;
    w.bp_list[e] = pos;
    mv.spi[e] = -1;
    if (spb < 0) continue;
    sp_src[pos] = mv.sps[e];
    if (!sp_mark[pos]) {
      sp_mark[pos] = 1;
      mv.spi[e] = atomicAdd(&sh.sp_new, 1);
    }
  }
  __syncthreads();
  if (tid == 0) {
    w.st->bp_count = nmv;
    w.st->R = R0 + wb;
    if (spb >= 0) {
      const int base = w.sp_count[spb];
      sh.sp_base = base;
      w.sp_count[spb] = base + sh.sp_new;
    }
  }
  __syncthreads();
  for (int e = tid; e < nmv; e += NT)
    if (mv.spi[e] >= 0) sp_list[sh.sp_base + mv.spi[e]] = mv.pos[e];
}

hipError_t launch_panel(const DecWork &w, int q0, int s_eff, int flag_q0, int spb, hipStream_t s) {
  hipLaunchKernelGGL(k_chain, dim3(1), dim3(kChainThreads), 0, s, w, q0, s_eff, flag_q0, spb);
  return hipGetLastError();
}

// ---------------------------------------------------------------- after the chain
// One launch per panel, two kinds of workgroups (1024 threads each):
//   * one per part (2, 4 or 8 words) of a 16-word column block: the panel's net row
//     permutation applied to its words outside the panel (P^(j) applied to all
//     columns), then, for trailing words, the pivot rows in echelon form
//     E = L_pp^{-1} * rows (block forward substitution over the sub-panels).
//     Both touch only the workgroup's own words, so the permutation finishes
//     before the solve reads.
//   * one per 512 rows: every row below the pivots gets the sub-panels it still
//     lacks, so its panel words hold its multipliers y_c (the Y of D*Z = Y,
//     eq. (Aj) restricted to the panel).  These touch only panel words.
constexpr int kPostThreads = 1024;
constexpr int kRowsPerWG = kPostThreads / 2;

// PW: words per column workgroup (2, 4 or 8 of a 16-word block)
template <int PW>
struct TrsmShared {
  uint64_t X[kMaxPanelWords * 64][PW];              // up to 32 KB: pivot rows, this part of the block
  uint64_t T[16][16][PW];                           // up to 16 KB: 4-bit tables
  uint64_t Cf[kMaxPanelWords * 64][kMaxPanelWords]; // 32 KB: multipliers L_cb
  uint64_t Li[kMaxPanelWords][64];                  // 4 KB: Linv_b
  SubInfo Sb[kMaxPanelWords];
};
template <int PW>
union PostShared {
  TrsmShared<PW> t;
  PanelTables pt;
};

// the row now at listed position p comes from position bp_src[p] at the panel start
template <int PW>
__device__ void post_swap(const DecWork &w, int q0, int s_eff, int blk, int half, int wlo, int whi) {
  constexpr int kPW = PW;
  const int cnt = w.st->bp_count;
  if (cnt == 0) return;
  const int tid = threadIdx.x, wl = tid % kPW, e0 = tid / kPW;
  const int64_t qw = (int64_t)blk * TW + kPW * half + wl;
  const bool act = qw < w.Mw && qw >= wlo && qw < whi && !(qw >= q0 && qw < q0 + s_eff);
  constexpr int PER = (kMaxPanelWords * 64 * 2) / (kPostThreads / kPW);
  uint64_t vals[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = e0 + (kPostThreads / kPW) * u;
    vals[u] = (act && e < cnt) ? w.W[widx(w.ldw, w.bp_src[w.bp_list[e]], qw)] : 0ull;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = e0 + (kPostThreads / kPW) * u;
    if (act && e < cnt) w.W[widx(w.ldw, w.bp_list[e], qw)] = vals[u];
  }
  __syncthreads();
}

// Pivot rows of the panel, words of part `half` (PW words) of column block blk
// right of the panel:
//   E_b = Linv_b * X_b, then X_c ^= L_cb * E_b for later sub-panels c,
// with L_cb = word q0+b of the pivot rows of sub-panel c (their multipliers for
// the pivots of sub-panel b).  PW-lane groups over the part, 4-bit tables.
template <int PW>
__device__ void post_trsm(const DecWork &w, int q0, int s_eff, int blk, int half, int whi, TrsmShared<PW> &sh) {
  constexpr int kPW = PW;
  constexpr int G = kPostThreads / kPW;  // row groups
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, h = lane / kPW, wl = lane % kPW;
  const int qc0 = q0 + s_eff;
  const int64_t qw = (int64_t)blk * TW + kPW * half + wl;
  const bool qok = qw >= qc0 && qw < whi;
  const int64_t ldw = w.ldw;
  uint64_t *W = w.W;
  if (tid < s_eff) sh.Sb[tid] = w.sub[q0 + tid];
  __syncthreads();
  int rtot = 0;
  for (int b = 0; b < s_eff; ++b) rtot += sh.Sb[b].r;
  if (rtot == 0) return;
  for (int ri = tid / kPW; ri < 64 * s_eff; ri += G) {
    const int b = ri >> 6, t = ri & 63;
    sh.X[ri][wl] = (qok && t < sh.Sb[b].r) ? W[widx(ldw, sh.Sb[b].R + t, qw)] : 0ull;
  }
  for (int e = tid; e < 64 * s_eff * s_eff; e += kPostThreads) {
    const int ri = e / s_eff, b = e - ri * s_eff;
    const int c = ri >> 6, t = ri & 63;
    sh.Cf[ri][b] = (b < c && t < sh.Sb[c].r) ? W[widx(ldw, sh.Sb[c].R + t, q0 + b)] : 0ull;
  }
  for (int e = tid; e < 64 * s_eff; e += kPostThreads)
    sh.Li[e >> 6][e & 63] = w.Linv[(size_t)(q0 + (e >> 6)) * 64 + (e & 63)];
  __syncthreads();
  auto tables = [&](int b) {  // 16 tables of 16 entries over the 64 rows of X_b
    if (tid < 16 * kPW) {
      const int g = tid / kPW, c = tid % kPW;
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
  for (int b = 0; b < s_eff; ++b) {
    const int rb = sh.Sb[b].r;
    if (rb == 0) continue;
    tables(b);
    {
      const int t = (64 / kPW) * wv + h;  // the first kPW waves, 64 / kPW groups each: 64 rows
      if (t < rb) {
        const uint64_t l = sh.Li[b][t];
        uint64_t v = 0ull;
#pragma unroll
        for (int g = 0; g < 16; ++g) v ^= sh.T[g][(l >> (4 * g)) & 15u][wl];
        sh.X[64 * b + t][wl] = v;
      }
    }
    __syncthreads();
    if (b == s_eff - 1) break;
    tables(b);
    // multipliers have no bits at or beyond rb, so unused tables contribute entry 0 = 0
    for (int ri = 64 * (b + 1) + (64 / kPW) * wv + h; ri < 64 * s_eff; ri += G) {
      const int c = ri >> 6, t = ri & 63;
      if (t < sh.Sb[c].r) {
        const uint64_t l = sh.Cf[ri][b];
        uint64_t v = 0ull;
#pragma unroll
        for (int g = 0; g < 16; ++g) v ^= sh.T[g][(l >> (4 * g)) & 15u][wl];
        sh.X[ri][wl] ^= v;
      }
    }
    __syncthreads();
  }
  for (int ri = tid / kPW; ri < 64 * s_eff; ri += G) {
    const int b = ri >> 6, t = ri & 63;
    if (qok && t < sh.Sb[b].r) W[widx(ldw, sh.Sb[b].R + t, qw)] = sh.X[ri][wl];
  }
}

__device__ void post_rows(const DecWork &w, int q0, int s_eff, int64_t blk0, PanelTables &pt) {
  int rtot = 0;
  for (int b = 0; b < s_eff; ++b) rtot += w.sub[q0 + b].r;
  if (rtot == 0) return;  // no pivots: the rows below are zero in the panel (and stay so)
  const SubInfo last = w.sub[q0 + s_eff - 1];
  const int64_t rowbeg = last.R + last.r;
  if (blk0 + kRowsPerWG <= rowbeg || blk0 >= w.n) return;
  // the chain kernel left the panel's tables in w.ptab
  {
    uint64_t *dst = &pt.Tz[0][0][0];
    for (int e = threadIdx.x; e < kPanelTabWords; e += kPostThreads) dst[e] = w.ptab[e];
  }
  __syncthreads();
  const int64_t i = blk0 + threadIdx.x;
  if (threadIdx.x >= kRowsPerWG || i < rowbeg || i >= w.n) return;
  const int L = row_level(w, i, q0);
  if (L >= s_eff) return;  // already at the panel's last level (held by the chain kernel)
  uint64_t x[kMaxPanelWords];
#pragma unroll
  for (int j = 0; j < kMaxPanelWords; ++j) x[j] = j < s_eff ? w.W[widx(w.ldw, i, q0 + j)] : 0ull;
  panel_update(x, L, s_eff, s_eff - 1, pt);
#pragma unroll
  for (int j = 0; j < kMaxPanelWords; ++j)
    if (j >= L && j < s_eff) w.W[widx(w.ldw, i, q0 + j)] = x[j];
}

// Words [wlo, whi) (wlo <= q0, whi <= Mw): the column workgroups cover the
// blocks that meet them.
template <int PW>
__global__ __launch_bounds__(kPostThreads) void k_post(DecWork w, int q0, int s_eff, int wlo, int whi) {
  __shared__ PostShared<PW> sh;
  constexpr int kPW = PW, kParts = TW / kPW;
  const int blk0 = wlo / TW;
  const int nc = kParts * ((whi - 1) / TW - blk0 + 1);  // column workgroups: kParts per 16-word block
  if ((int)blockIdx.x < nc) {
    const int blk = blk0 + (int)blockIdx.x / kParts, half = blockIdx.x % kParts;
    post_swap<PW>(w, q0, s_eff, blk, half, wlo, whi);
    const int qc0 = q0 + s_eff;
    if (qc0 < whi && blk * TW + kPW * half + kPW - 1 >= qc0) post_trsm<PW>(w, q0, s_eff, blk, half, whi, sh.t);
  } else {
    post_rows(w, q0, s_eff, (int64_t)(blockIdx.x - nc) * kRowsPerWG, sh.pt);
  }
}

// The column workgroups take the narrowest part of a block (2, 4 or 8 words)
// for which the whole launch still fits the device's CUs in one round: each
// workgroup's solve is a chain of dependent steps, so narrower parts finish
// sooner, until a second round of workgroups costs more (2048^2 and 16384^2
// take 2 words, 32768^2 4, 65536^2 8).
hipError_t launch_post(const DecWork &w, int q0, int s_eff, int wlo, int whi, int ncu, hipStream_t s) {
  const int64_t rows_wg = (w.n + kRowsPerWG - 1) / kRowsPerWG;
  const int64_t nblk = (whi - 1) / TW - wlo / TW + 1;
  if ((TW / 2) * nblk + rows_wg <= ncu) {
    hipLaunchKernelGGL(k_post<2>, dim3((unsigned)((TW / 2) * nblk + rows_wg)), dim3(kPostThreads), 0, s, w, q0,
                       s_eff, wlo, whi);
  } else if ((TW / 4) * nblk + rows_wg <= ncu) {
    hipLaunchKernelGGL(k_post<4>, dim3((unsigned)((TW / 4) * nblk + rows_wg)), dim3(kPostThreads), 0, s, w, q0,
                       s_eff, wlo, whi);
  } else {
    hipLaunchKernelGGL(k_post<8>, dim3((unsigned)((TW / 8) * nblk + rows_wg)), dim3(kPostThreads), 0, s, w, q0,
                       s_eff, wlo, whi);
  }
  return hipGetLastError();
}

}  // namespace gf2
