// k_panel.hip -- the per-panel steps of the block decomposition (Section 4).
//
// A trailing-update panel is s <= 8 consecutive 64-column sub-panels (words
// q0 .. q0+s-1), factored left-looking:
//   k_panel        per sub-panel q: brings the window rows up to date for the
//                  panel's earlier sub-panels, then selects the pivots of the
//                  64 columns of word q (procedure buildZ, Sections 4.2-4.4):
//                  for each bit k in order, the first row at or below the next
//                  free position whose reduced bit k is 1 becomes the pivot and
//                  is exchanged with that position (a transposition).  It
//                  produces the pivot columns, the coefficient map Zc (row j of
//                  Zc gives the multipliers of bit j, so y = x * Zc are a row's
//                  multipliers -- the role of Z in D*Z = Y, Section 4.1), the
//                  inverse of the sub-panel's unit lower block, and writes back
//                  the window rows (pivot rows in final form).
//   k_rows_panel   once per panel: every row below the pivots gets the
//                  sub-panels it still lacks, so its panel words hold its
//                  multipliers (eq. (Aj) restricted to the panel).
//   k_swap         applies the panel's net row permutation to all words
//                  outside the panel (P^(j) applied to all columns).
//   k_trsm         pivot rows right of the panel: E = L_pp^{-1} * rows
//                  (block forward substitution over the sub-panels).
// The trailing product (Schur complement, eq. (Aj)) is k_gemm.
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
  uint64_t Src[kPairs + kMaxPanelWords][64];  // staged Zc_c rows and E_c[w] words
};

// Tables of sub-panels c in [0, cend) of the panel starting at q0 (all threads).
__device__ void build_panel_tables(PanelTables &pt, const DecWork &w, int q0, int s_eff, int cend,
                                   int tid, int nthr) {
  // stage: slot c*64+t of Src for Zc_c; slot (kMaxPanelWords + pidx)*64 + t for E_c[w]
  for (int e = tid; e < cend * 64; e += nthr) {
    const int c = e >> 6, t = e & 63;
    pt.Src[c][t] = w.Zc[(size_t)(q0 + c) * 64 + t];
  }
  for (int c = 0; c < cend; ++c) {
    const SubInfo sc = w.sub[q0 + c];
    const int nwd = s_eff - 1 - c;
    for (int e = tid; e < nwd * 64; e += nthr) {
      const int wd = c + 1 + (e >> 6), t = e & 63;
      pt.Src[kMaxPanelWords + pidx(c, wd)][t] = t < sc.r ? w.W[widx(w.ldw, sc.R + t, q0 + wd)] : 0ull;
    }
  }
  __syncthreads();
  for (int e = tid; e < cend * 256; e += nthr) {
    const int c = e >> 8, g = (e >> 4) & 15, v = e & 15;
    uint64_t acc = 0ull;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (v & (1 << b)) acc ^= pt.Src[c][4 * g + b];
    pt.Tz[c][g][v] = acc;
  }
  for (int c = 0; c < cend; ++c) {
    const int nwd = s_eff - 1 - c;
    for (int e = tid; e < nwd * 256; e += nthr) {
      const int wd = c + 1 + (e >> 8), g = (e >> 4) & 15, v = e & 15;
      const int pi = pidx(c, wd);
      uint64_t acc = 0ull;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (v & (1 << b)) acc ^= pt.Src[kMaxPanelWords + pi][4 * g + b];
      pt.Te[pi][g][v] = acc;
    }
  }
  __syncthreads();
}

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
// One workgroup of 4 waves.  The window (the first kWin free positions) is
// brought up to date for the panel's earlier sub-panels, then all four waves
// hold the same reduced words of word q and take the same decisions (no
// communication on the common path); the scan below the window and the
// write-back use all 256 threads.  A slot carries an origin code: o < kWin is
// the row that sat at window position o, o >= kWin the row kept in Xr[o-kWin]
// (brought up from below the window).
__global__ __launch_bounds__(256) void k_panel(DecWork w, int q, int q0, int s_eff, int flag_q0) {
  __shared__ PanelTables pt;
  __shared__ uint64_t Wl[kWin][kMaxPanelWords];  // window rows, panel words at level b
  __shared__ uint64_t Xr[64][kMaxPanelWords];    // rows brought up from below the window
  __shared__ int Xsrc[64];
  __shared__ int nX;
  __shared__ uint64_t Tp[8][256];                // Proj tables for the scan
  __shared__ uint64_t Ms[64];
  __shared__ int po_pos[64], po_org[64];         // positions below the window now holding a window row
  __shared__ int npo;
  __shared__ uint32_t po_bloom[128];
  __shared__ int scan_best;
  __shared__ unsigned long long scan_F;
  __shared__ int sorg[kWin];
  __shared__ uint64_t Praw[64][kMaxPanelWords];
  __shared__ int wr_pos[kWin + 64], wr_org[kWin + 64];
  __shared__ int nwr;
  __shared__ int64_t gperm[kWin + 64];
  __shared__ int gbp[kWin + 64];
  __shared__ int wave_new[4];
  __shared__ int list_base;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t n = w.n, ldw = w.ldw;
  uint64_t *W = w.W;
  const int b = q - q0;

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
  if (flag_q0 >= 0 && w.nzflag[flag_q0] == 0u) skip = true;  // Schur complement already zero
  if (skip) {
    if (tid < 64) {
      w.Zc[(size_t)q * 64 + tid] = 0ull;
      w.Linv[(size_t)q * 64 + tid] = 0ull;
    }
    if (tid == 0) {
      w.sub[q].R = R;
      w.sub[q].r = 0;
      w.sub[q].pivmask = 0;
    }
    return;
  }

  // ---- tables of the earlier sub-panels, window rows brought to level b
  build_panel_tables(pt, w, q0, s_eff, b, tid, 256);
  if (tid == 0) {
    nX = 0;
    npo = 0;
  }
  if (tid < 128) po_bloom[tid] = 0u;
  if (tid < kWin) {
    const int64_t p = R + tid;
    uint64_t x[kMaxPanelWords];
#pragma unroll
    for (int j = 0; j < kMaxPanelWords; ++j) x[j] = (p < n && j < s_eff) ? W[widx(ldw, p, q0 + j)] : 0ull;
    if (p < n) panel_update(x, row_level(w, p, q0), b, s_eff - 1, pt);
#pragma unroll
    for (int j = 0; j < kMaxPanelWords; ++j) Wl[tid][j] = x[j];
  }
  __syncthreads();

  const bool v0 = R + lane < n, v1 = R + 64 + lane < n;
  // Window state of this wave: slot 64g + lane holds reduced word (lo, hi) and origin.
  uint32_t a_lo = (uint32_t)Wl[lane][b], a_hi = (uint32_t)(Wl[lane][b] >> 32);
  uint32_t b_lo = (uint32_t)Wl[64 + lane][b], b_hi = (uint32_t)(Wl[64 + lane][b] >> 32);
  int org0 = lane, org1 = 64 + lane;
  // Slots still free (at or after the next pivot position), as scalar lane masks.
  uint64_t act0 = __ballot(v0), act1 = __ballot(v1);
  uint64_t Mrow = 0ull, yM = 0ull, pivmask = 0ull, F = 0ull;
  bool Fknown = false;
  int ib = 0;

  for (int k = 0; k < nbits; ++k) {
    const uint64_t kb = 1ull << k;
    const uint32_t bit = 1u << (k & 31);
    uint64_t c0, c1;
    if (k < 32) {
      c0 = __ballot((a_lo & bit) != 0u) & act0;
      c1 = __ballot((b_lo & bit) != 0u) & act1;
    } else {
      c0 = __ballot((a_hi & bit) != 0u) & act0;
      c1 = __ballot((b_hi & bit) != 0u) & act1;
    }
    int sp = -1;
    if (c0) sp = __builtin_ctzll(c0);
    else if (c1) sp = 64 + __builtin_ctzll(c1);
    uint64_t Mnew;
    uint64_t rs0 = 0ull, rs1 = 0ull;  // slots to reduce by the new pivot row
    if (sp >= 0) {
      uint32_t p_lo, p_hi;
      int p_org;
      if (sp < 64) {
        p_lo = __builtin_amdgcn_readlane(a_lo, sp);
        p_hi = __builtin_amdgcn_readlane(a_hi, sp);
        p_org = __builtin_amdgcn_readlane(org0, sp);
      } else {
        p_lo = __builtin_amdgcn_readlane(b_lo, sp - 64);
        p_hi = __builtin_amdgcn_readlane(b_hi, sp - 64);
        p_org = __builtin_amdgcn_readlane(org1, sp - 64);
      }
      if (sp != ib) {  // transposition: the row at ib moves to sp, the pivot to ib
        uint32_t i_lo, i_hi;
        int i_org;
        if (ib < 64) {
          i_lo = __builtin_amdgcn_readlane(a_lo, ib);
          i_hi = __builtin_amdgcn_readlane(a_hi, ib);
          i_org = __builtin_amdgcn_readlane(org0, ib);
        } else {
          i_lo = __builtin_amdgcn_readlane(b_lo, ib - 64);
          i_hi = __builtin_amdgcn_readlane(b_hi, ib - 64);
          i_org = __builtin_amdgcn_readlane(org1, ib - 64);
        }
        const uint64_t msp0 = sp < 64 ? 1ull << sp : 0ull, msp1 = sp >= 64 ? 1ull << (sp - 64) : 0ull;
        const uint64_t mib0 = ib < 64 ? 1ull << ib : 0ull, mib1 = ib >= 64 ? 1ull << (ib - 64) : 0ull;
        if (msp0 | mib0) {
          const bool ws = __builtin_amdgcn_inverse_ballot_w64(msp0), wi = __builtin_amdgcn_inverse_ballot_w64(mib0);
          a_lo = ws ? i_lo : (wi ? p_lo : a_lo);
          a_hi = ws ? i_hi : (wi ? p_hi : a_hi);
          org0 = ws ? i_org : (wi ? p_org : org0);
        }
        if (msp1 | mib1) {
          const bool ws = __builtin_amdgcn_inverse_ballot_w64(msp1), wi = __builtin_amdgcn_inverse_ballot_w64(mib1);
          b_lo = ws ? i_lo : (wi ? p_lo : b_lo);
          b_hi = ws ? i_hi : (wi ? p_hi : b_hi);
          org1 = ws ? i_org : (wi ? p_org : org1);
        }
      }
      Mnew = ((uint64_t)p_hi << 32) | p_lo;
      // candidates other than the pivot itself (the row now at sp has bit k clear)
      rs0 = c0 & ~(sp < 64 ? 1ull << sp : 0ull);
      rs1 = c1 & ~(sp >= 64 ? 1ull << (sp - 64) : 0ull);
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
        for (int bb = 0; bb < 8; ++bb)
          if (idx & (1 << bb)) v ^= Ms[8 * g + bb];
        Tp[g][idx] = v;
      }
      __syncthreads();
      int best = 0x7fffffff;
      uint64_t Floc = 0ull;
      for (int64_t p = R + kWin + tid; p < n; p += 256) {
        uint64_t xq;
        int o = -1;
        if ((po_bloom[(p >> 5) & 127] >> (p & 31)) & 1u)
          for (int j = 0; j < npo; ++j)
            if (po_pos[j] == (int)p) o = po_org[j];
        if (o >= 0) {
          xq = o < kWin ? Wl[o][b] : Xr[o - kWin][b];
        } else {
          uint64_t x[kMaxPanelWords];
#pragma unroll
          for (int j = 0; j < kMaxPanelWords; ++j) x[j] = j <= b ? W[widx(ldw, p, q0 + j)] : 0ull;
          panel_update(x, row_level(w, p, q0), b, b, pt);
          xq = x[0];
#pragma unroll
          for (int j = 1; j < kMaxPanelWords; ++j)
            if (j == b) xq = x[j];
        }
        uint64_t pr = xq;
#pragma unroll
        for (int g = 0; g < 8; ++g) pr ^= Tp[g][(xq >> (8 * g)) & 255u];
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
      // ---- bring the row at `best` into slot ib; the slot's row goes to position `best`
      int oin = -1;
      for (int j = 0; j < npo; ++j)
        if (po_pos[j] == best) oin = po_org[j];
      int oout;
      uint64_t xro;
      if (ib < 64) {
        oout = __builtin_amdgcn_readlane(org0, ib);
        xro = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(a_hi, ib) << 32) | (uint32_t)__builtin_amdgcn_readlane(a_lo, ib);
      } else {
        oout = __builtin_amdgcn_readlane(org1, ib - 64);
        xro = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(b_hi, ib - 64) << 32) |
              (uint32_t)__builtin_amdgcn_readlane(b_lo, ib - 64);
      }
      __syncthreads();
      if (oin < 0 && tid == 0) {  // a row never seen: load it and bring it to level b
        const int j = nX;
        uint64_t x[kMaxPanelWords];
#pragma unroll
        for (int jj = 0; jj < kMaxPanelWords; ++jj) x[jj] = jj < s_eff ? W[widx(ldw, best, q0 + jj)] : 0ull;
        panel_update(x, row_level(w, best, q0), b, s_eff - 1, pt);
#pragma unroll
        for (int jj = 0; jj < kMaxPanelWords; ++jj) Xr[j][jj] = x[jj];
        Xsrc[j] = best;
        nX = j + 1;
      }
      if (tid == 0) {
        int j = 0;
        while (j < npo && po_pos[j] != best) ++j;
        if (j == npo) {
          po_pos[j] = best;
          npo = j + 1;
          po_bloom[(best >> 5) & 127] |= 1u << (best & 31);
        }
        po_org[j] = oout;
      }
      __syncthreads();
      if (oin < 0) oin = kWin + nX - 1;
      const uint64_t xin = oin < kWin ? Wl[oin][b] : Xr[oin - kWin][b];
      uint64_t xrp = xin;
#pragma unroll
      for (int g = 0; g < 8; ++g) xrp ^= Tp[g][(xin >> (8 * g)) & 255u];
      if (ib < 64) {
        if (lane == ib) { a_lo = (uint32_t)xrp; a_hi = (uint32_t)(xrp >> 32); org0 = oin; }
      } else {
        if (lane == ib - 64) { b_lo = (uint32_t)xrp; b_hi = (uint32_t)(xrp >> 32); org1 = oin; }
      }
      F |= xro;
      Mnew = xrp;
    }
    // ---- pivot t = ib for bit k: bookkeeping rows (RREF), their multipliers, the window
    pivmask |= kb;
    const uint64_t tb = 1ull << ib;
    {
      const uint64_t mm = __ballot((Mrow & kb) != 0ull);  // earlier pivots with bit k set
      const bool upd = __builtin_amdgcn_inverse_ballot_w64(mm);
      const bool me = __builtin_amdgcn_inverse_ballot_w64(kb);  // lane k
      Mrow = me ? Mnew : (upd ? Mrow ^ Mnew : Mrow);
      yM = me ? tb : (upd ? yM ^ tb : yM);
    }
    {
      const uint32_t n_lo = (uint32_t)Mnew, n_hi = (uint32_t)(Mnew >> 32);
      if (rs0) {
        const bool r0 = __builtin_amdgcn_inverse_ballot_w64(rs0);
        a_lo = r0 ? a_lo ^ n_lo : a_lo;
        a_hi = r0 ? a_hi ^ n_hi : a_hi;
      }
      if (rs1) {
        const bool r1 = __builtin_amdgcn_inverse_ballot_w64(rs1);
        b_lo = r1 ? b_lo ^ n_lo : b_lo;
        b_hi = r1 ? b_hi ^ n_hi : b_hi;
      }
    }
    if (ib < 64) act0 &= ~(1ull << ib);
    else act1 &= ~(1ull << (ib - 64));
    if (Fknown) {
      if (F & kb) F |= Mnew;
      F &= ~kb;
    }
    ++ib;
  }
  const int r = ib;
  const uint64_t xr0 = ((uint64_t)a_hi << 32) | a_lo;  // lane t < r: E_t

  // ---- multipliers of the pivot rows (unit lower block L_pp) from the coefficient
  // map: the current word b of pivot row t is in the span of E_0..E_t, so
  // y = word * Zc lists its multipliers (bit t set).  Then the block's inverse.
  if (wv == 0) Ms[lane] = yM;
  __syncthreads();
  {
    const int g = tid >> 4, v = tid & 15;
    uint64_t acc = 0ull;
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
      if (v & (1 << bb)) acc ^= Ms[4 * g + bb];
    Tp[0][tid] = acc;  // table g = tid >> 4 of 16 entries
  }
  __syncthreads();
  const int myorg = org0;
  uint64_t yx = 0ull;
  if (lane < r) {
    const uint64_t xb = myorg < kWin ? Wl[myorg][b] : Xr[myorg - kWin][b];
#pragma unroll
    for (int g = 0; g < 16; ++g) yx ^= Tp[0][16 * g + ((xb >> (4 * g)) & 15u)];
  }
  uint64_t li = lane < r ? (1ull << lane) : 0ull;
  for (int t = 0; t < r; ++t) {
    const uint64_t row = rdl64(li, t);
    if (lane > t && lane < r && ((yx >> t) & 1ull)) li ^= row;
  }

  // ---- rows to write back: every window position, then positions below it now
  // holding a window row
  if (wv == 0) {
    if (v0) sorg[lane] = org0;
    if (v1) sorg[64 + lane] = org1;
    w.Zc[(size_t)q * 64 + lane] = yM;
    w.Linv[(size_t)q * 64 + lane] = li;
    if ((pivmask >> lane) & 1ull) {
      const int t = __popcll(pivmask & ((1ull << lane) - 1ull));
      w.pivcols[R + t] = 64ll * q + lane;
    }
  }
  __syncthreads();
  {
    const int nvalid = (n - R) < kWin ? (int)(n - R) : kWin;
    if (tid < nvalid) {
      wr_pos[tid] = (int)(R + tid);
      wr_org[tid] = sorg[tid];
    }
    if (tid < npo) {
      wr_pos[nvalid + tid] = po_pos[tid];
      wr_org[nvalid + tid] = po_org[tid];
    }
    if (tid == 0) nwr = nvalid + npo;
  }
  for (int e = tid; e < r * kMaxPanelWords; e += 256) {
    const int t = e / kMaxPanelWords, j = e % kMaxPanelWords;
    const int o = sorg[t];
    Praw[t][j] = o < kWin ? Wl[o][j] : Xr[o - kWin][j];
  }
  __syncthreads();
  const int nw = nwr;
  // perm / panel-start positions of the rows that moved (gather, then scatter)
  for (int e = tid; e < nw; e += 256) {
    const int o = wr_org[e];
    const int src = o < kWin ? (int)(R + o) : Xsrc[o - kWin];
    gperm[e] = w.perm[src];
    gbp[e] = w.bp_src[src];
  }
  __syncthreads();
  {
    int dst = 0;
    bool fresh = false;
    if (tid < nw) {
      const int o = wr_org[tid];
      const int src = o < kWin ? (int)(R + o) : Xsrc[o - kWin];
      dst = wr_pos[tid];
      if (src != dst) {
        w.perm[dst] = gperm[tid];
        w.bp_src[dst] = gbp[tid];
        fresh = w.bp_mark[dst] == 0;
        if (fresh) w.bp_mark[dst] = 1;
      }
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
  // panel words of every written row; pivot rows: multipliers left of b, E | L_pp at b,
  // echelon words right of b
  for (int e = tid; e < nw * s_eff; e += 256) {
    const int i = e / s_eff, j = e - i * s_eff;
    const int dst = wr_pos[i];
    const int o = wr_org[i];
    if (dst - R < r && j >= b) continue;  // pivot rows, words b.. written below
    W[widx(ldw, dst, q0 + j)] = o < kWin ? Wl[o][j] : Xr[o - kWin][j];
  }
  for (int e = tid; e < nw; e += 256) {
    const int dst = wr_pos[e];
    w.lvl[dst] = dst - R < r ? (q0 << 4) | 15 : (q0 << 4) | b;
  }
  if (wv == 0 && lane < r) W[widx(ldw, R + lane, q)] = xr0 | (yx & ((1ull << lane) - 1ull));
  for (int j = b + 1 + wv; j < s_eff; j += 4) {
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

hipError_t launch_panel(const DecWork &w, int q, int q0, int s_eff, int flag_q0, hipStream_t s) {
  hipLaunchKernelGGL(k_panel, dim3(1), dim3(256), 0, s, w, q, q0, s_eff, flag_q0);
  return hipGetLastError();
}

// All rows below the panel's pivots: apply the sub-panels each row still lacks
// (from its level to the end of the panel), so every panel word holds the
// row's multipliers y_c -- the Y of the paper's D*Z = Y, per sub-panel.
constexpr int kRowsThreads = 256;
constexpr int kRowsPerThread = 2;
__global__ __launch_bounds__(kRowsThreads) void k_rows_panel(DecWork w, int q0, int s_eff) {
  __shared__ PanelTables pt;
  const SubInfo last = w.sub[q0 + s_eff - 1];
  const int64_t rowbeg = last.R + last.r;
  const int64_t blk0 = (int64_t)blockIdx.x * kRowsThreads * kRowsPerThread;
  if (blk0 + kRowsThreads * kRowsPerThread <= rowbeg || blk0 >= w.n) return;
  build_panel_tables(pt, w, q0, s_eff, s_eff, threadIdx.x, kRowsThreads);
  for (int u = 0; u < kRowsPerThread; ++u) {
    const int64_t i = blk0 + (int64_t)u * kRowsThreads + threadIdx.x;
    if (i < rowbeg || i >= w.n) continue;
    const int L = row_level(w, i, q0);
    uint64_t x[kMaxPanelWords];
#pragma unroll
    for (int j = 0; j < kMaxPanelWords; ++j) x[j] = j < s_eff ? w.W[widx(w.ldw, i, q0 + j)] : 0ull;
    panel_update(x, L, s_eff, s_eff - 1, pt);
#pragma unroll
    for (int j = 0; j < kMaxPanelWords; ++j)
      if (j >= L && j < s_eff) w.W[widx(w.ldw, i, q0 + j)] = x[j];
  }
}

hipError_t launch_rows_panel(const DecWork &w, int q0, int s_eff, hipStream_t s) {
  const int64_t per = (int64_t)kRowsThreads * kRowsPerThread;
  const int64_t blocks = (w.n + per - 1) / per;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_panel, dim3((unsigned)blocks), dim3(kRowsThreads), 0, s, w, q0, s_eff);
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
