// k_gemm.hip -- Four-Russians GF(2) product C (^)= A*B on gfx950.
//
// Section 6 of the paper: for each group of c = 8 consecutive bits of the
// inner dimension, a table of the 2^c XOR combinations of the matching 8 rows
// of B is built once (one XOR per entry, Gray-code order), and each output row
// then needs a single table lookup and one XOR per group (eq. (M4RM:cost):
// T = (b/c)(2^c - 1) XORs for the tables plus R = b/c XORs per row).
//
// gfx950 mapping.  A workgroup owns a tile of TM rows x one 16-word column
// block of C (1024 columns); four tables (32 inner bits) are built per step in
// LDS (128 KB) and every row of the tile then does its four lookups, with two
// barriers per step.  B rows and A words of the next step are prefetched during
// the lookups, and the accumulators stay in registers for the whole inner loop,
// so C is read and written once per launch.
//   k_gemm_wide    eight 8-lane groups per wave; lane w2 of a group owns words
//                  2*w2, 2*w2+1 of its group's row and one 16-byte read fetches
//                  them from a 128-byte table entry.  Adjacent groups read the
//                  two interleaved tables of a pair in the same instruction, so
//                  16 lanes cover 256 contiguous bytes (no bank conflicts at the
//                  full 16-byte read rate).
//   k_gemm_narrow  the next panel's 8 words: 64-byte entries, eight tables (a
//                  whole 64-bit A word) per step.
// The byte address of a table entry is formed by one byte permute of (A bits,
// lane base), and the XORs use the three-input bitwise instruction.
#include <hip/hip_ext.h>

#include "gf2_internal.h"

namespace gf2 {

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

// Rows owned by one lane of a product tile: tile0 + l0 + S*u for u in [0, RPL)
// (l0 = the lane's group index in the workgroup, S = groups per workgroup).
// [ulo, uhi) are the u whose row lies in [rb, re).
template <int RPL, int S>
__device__ inline void lane_rows(int64_t tile0, int l0, int64_t rb, int64_t re, int &ulo, int &uhi) {
  const int64_t b = tile0 + l0;
  int64_t lo = rb - b, hi = re - b;
  lo = lo <= 0 ? 0 : (lo + S - 1) / S;
  hi = hi <= 0 ? 0 : (hi + S - 1) / S;
  ulo = (int)(lo < RPL ? lo : RPL);
  uhi = (int)(hi < RPL ? hi : RPL);
}

// Accumulators of a lane that owns words 2*w2, 2*w2+1 of its rows: C is read
// (accumulate) and written as one 16-byte access per row where both words lie
// in the written column range.  Both are non-temporal, as a launch touches each
// C word once: in the 65536^2 decomposition this cut the HBM bytes fetched per
// product launch by 12% and the bulk launches' time by about 2%.
template <int RPL, int S>
__device__ inline void load_acc2(uint64_t (&acc)[RPL][2], const uint64_t *Cl, bool ok0, bool ok1, int ulo,
                                 int uhi) {
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    acc[u][0] = 0ull;
    acc[u][1] = 0ull;
    if (u >= ulo && u < uhi) {
      const uint64_t *p = Cl + (int64_t)u * S * TW;
      if (ok0 && ok1) {
        const u64x2 v = __builtin_nontemporal_load((const u64x2 *)p);
        acc[u][0] = v.x;
        acc[u][1] = v.y;
      } else {
        if (ok0) acc[u][0] = p[0];
        if (ok1) acc[u][1] = p[1];
      }
    }
  }
}

template <int RPL, int S>
__device__ inline uint64_t store_acc2(const uint64_t (&acc)[RPL][2], uint64_t *Cl, bool ok0, bool ok1, int ulo,
                                      int uhi) {
  uint64_t any = 0;
#pragma unroll
  for (int u = 0; u < RPL; ++u)
    if (u >= ulo && u < uhi) {
      uint64_t *p = Cl + (int64_t)u * S * TW;
      if (ok0 && ok1) {
        __builtin_nontemporal_store((u64x2){acc[u][0], acc[u][1]}, (u64x2 *)p);
      } else {
        if (ok0) p[0] = acc[u][0];
        if (ok1) p[1] = acc[u][1];
      }
      any |= (ok0 ? acc[u][0] : 0ull) | (ok1 ? acc[u][1] : 0ull);
    }
  return any;
}

// The same rows XORed into C with 64-bit atomics (one part of a product split
// over its inner dimension).  Every word gets its atomic, a zero one included,
// so that the last part to reach a word sees its final value: `any` is then
// nonzero whenever some written word ends nonzero (it may also be nonzero when
// none does, which only costs a zero-tail exit).
template <int RPL, int S>
__device__ inline uint64_t xor_acc2(const uint64_t (&acc)[RPL][2], uint64_t *Cl, bool ok0, bool ok1, int ulo,
                                    int uhi) {
  uint64_t any = 0;
#pragma unroll
  for (int u = 0; u < RPL; ++u)
    if (u >= ulo && u < uhi) {
      unsigned long long *p = (unsigned long long *)(Cl + (int64_t)u * S * TW);
      if (ok0) any |= atomicXor(p, (unsigned long long)acc[u][0]) ^ acc[u][0];
      if (ok1) any |= atomicXor(p + 1, (unsigned long long)acc[u][1]) ^ acc[u][1];
    }
  return any;
}

// Four tables (32 inner bits) per step.  The B rows of a step are staged
// through LDS (two 4 KB buffers): 256 threads load the 32 rows x 16 words of a
// later step with one 16-byte load each, store them (masked) into the free
// buffer while the tables are built, and every thread reads its eight rows back
// from LDS for the build.  The registers this leaves free hold a second set of
// lookups: the loads of the next row pair are in flight while the current pair
// is combined, so the table reads of a wave never wait for its own XORs.
template <int NT, int TM>
__global__ __launch_bounds__(NT) void k_gemm_wide(GemmArgs a) {
  constexpr int UB = NT >= 1024 ? 1 : 2;  // rows per lane looked up together (registers: 4 waves per SIMD at 1024)
  constexpr int NW = NT / 64;          // waves
  constexpr int RPL = TM / (8 * NW);   // rows per lane
  // Table builds: jobs of 8 threads (one word pair per thread).  At 1024
  // threads half of them build, 16 entries each: the staged B rows are then
  // read half as often (512 build threads measured faster than 1024, 256 or 128).
  constexpr int BT = NT >= 1024 ? 512 : NT;
  constexpr int JOBS = BT / 8;
  constexpr int EPJ = 4 * 256 / JOBS;  // entries per job
  constexpr int LOGE = EPJ == 8 ? 3 : (EPJ == 16 ? 4 : (EPJ == 32 ? 5 : 6));
  static_assert(RPL * 8 * NW == TM && RPL % (2 * UB) == 0, "tile");
  static_assert(EPJ == 8 || EPJ == 16 || EPJ == 32 || EPJ == 64, "build split");
  static_assert(TM % NT == 0 && NT >= 256, "A staging, B staging");
  // Tables g = 2p + s stored as T[p][idx][s][word], as in k_gemm_wide.
  __shared__ uint64_t T[2][256][2][TW];
  __shared__ uint32_t As[2 * TM];         // the tile's A word for the current 64 inner bits
  __shared__ ulonglong2 Bs[2][32][TW / 2];  // B rows of a step (zero past the operand), two buffers
  __shared__ int64_t sR[kSpSubMax];  // pivot-row ranges of a mapped B (at most one super-panel)
  __shared__ int sr[kSpSubMax];

  if (a.skip_flag && *a.skip_flag == 0u) return;  // the Schur complement is already zero
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, G = lane >> 3, w2 = lane & 7;
  // A trailing update (mapped B) has its grid as (column block, tile), the
  // tiles counted from the one holding d, the first row below the panel's
  // pivots: the grid still has a tile for every row of the matrix, and the
  // workgroups past the last row, one row of tiles per tile of pivots so far,
  // come last in dispatch order (a 1024-thread workgroup takes a whole CU even
  // to find it has no rows).  A plain product keeps (tile, column block).
  const bool mapped = a.bsub != nullptr;
  const int blk = (mapped ? blockIdx.x : blockIdx.y) + (a.qc0 >> 4);
  const int64_t qw = (int64_t)blk * TW + 2 * w2;
  const bool ok0 = qw >= a.qc0 && qw < a.qc1, ok1 = qw + 1 >= a.qc0 && qw + 1 < a.qc1;

  int64_t d = a.row_tile0;
  if (mapped) {
    const int64_t dd = a.bsub[a.kwords - 1].R + a.bsub[a.kwords - 1].r;
    if (dd > d) d = dd;
  }
  const int64_t tile0 =
      a.row_tile0 + (mapped ? (d - a.row_tile0) / TM + (int64_t)blockIdx.y : (int64_t)blockIdx.x) * TM;
  int64_t rb = d > tile0 ? d : tile0;
  int64_t re = tile0 + TM < a.row_end ? tile0 + TM : a.row_end;
  if (rb >= re) return;

  // rows of this lane: tile0 + 8*wv + G + 8*NW*u
  int ulo, uhi;
  lane_rows<RPL, 8 * NW>(tile0, 8 * wv + G, rb, re, ulo, uhi);
  uint64_t acc[RPL][2];
  {
    uint64_t *C = a.C;
    asm volatile("" : "+s"(C));
    const uint64_t *Cl = C + (((int64_t)blk * a.ldC + tile0 + 8 * wv + G) * TW + 2 * w2);
    load_acc2<RPL, 8 * NW>(acc, Cl, a.accumulate && ok0, a.accumulate && ok1, ulo, uhi);
  }

  const int job = tid >> 3;
  const int g_b = job / (256 / EPJ), uu = job % (256 / EPJ);
  const int64_t bq = (int64_t)blk * TW + 2 * w2;  // this thread's word pair of B (= qw)
  const bool bok0 = ok0, bok1 = ok1;

  // B staging: thread tid < 256 loads row srow of a step, words 2*w2, 2*w2+1,
  // from a clamped (always valid) row; the row limit is applied when it is
  // stored into LDS, a step later.
  const int srow = tid >> 3;
  ulonglong2 bnext = make_ulonglong2(0ull, 0ull);
  bool bnext_ok = false;
  auto load_b = [&](int hh) {
    if (tid >= 256) return;
    const int kw = hh >> 1;
    int64_t browR = 64ll * kw;
    int blim;
    if (a.bsub) {
      browR = sR[kw];
      blim = sr[kw];
    } else {
      const int64_t left = a.b_rows - 64ll * kw;
      blim = left >= 64 ? 64 : (left > 0 ? (int)left : 0);
    }
    const int r = 32 * (hh & 1) + srow;
    bnext_ok = r < blim;
    int64_t row = browR + r;
    row = row < a.ldB ? row : a.ldB - 1;
    bnext = *(const ulonglong2 *)(a.B + widx(a.ldB, row, bq));
  };
  auto stage_b = [&](int buf) {
    if (tid >= 256) return;
    Bs[buf][srow][w2] = make_ulonglong2((bnext_ok && bok0) ? bnext.x : 0ull, (bnext_ok && bok1) ? bnext.y : 0ull);
  };
  constexpr int APT = TM / NT;
  auto load_a = [&](int kw, uint64_t (&av)[APT]) {
#pragma unroll
    for (int j = 0; j < APT; ++j) {
      const int64_t i = tile0 + tid + (int64_t)j * NT;
      av[j] = a.A[widx(a.ldA, i < a.ldA ? i : a.ldA - 1, a.a_word0 + kw)];  // masked when staged
    }
  };

  if (a.bsub) {
    if (tid < a.kwords) {
      sR[tid] = a.bsub[tid].R;
      sr[tid] = a.bsub[tid].r;
    }
    __syncthreads();
  }
  const int nh = 2 * a.kwords;
  uint64_t av[APT];
  load_b(0);
  load_a(0, av);
  stage_b(0);
  if (nh > 1) load_b(1);
  const char *Tb = (const char *)&T[0][0][0][0];
  // Read g of a row: odd groups read table g ^ 1 (the other table of the
  // pair), so their A words are staged with the bytes of each half swapped
  // (byte g of the staged word is then byte g ^ 1 of A) and one selector per
  // g serves every lane.  The entry address is [half offset | A byte | pair |
  // 0]: the half offset is byte 0 of lb for even g and byte 3 for odd g, and
  // the pair is byte 2 of lb (1) for g >= 2 and zero otherwise.
  const uint32_t h_even = ((uint32_t)(G & 1) << 7) | ((uint32_t)w2 << 4);
  const uint32_t h_odd = ((uint32_t)((G & 1) ^ 1) << 7) | ((uint32_t)w2 << 4);
  const uint32_t lb = h_even | (1u << 16) | (h_odd << 24);
  constexpr uint32_t kSel[4] = {0x0C0C0400u, 0x0C0C0503u, 0x0C020600u, 0x0C020703u};
  for (int hh = 0; hh < nh; ++hh) {
    const int half = hh & 1;
    __syncthreads();  // previous lookups finished: T and As are free; B rows of step hh staged
    if (half == 0) {
#pragma unroll
      for (int j = 0; j < APT; ++j) {
        const int64_t i = tile0 + tid + (int64_t)j * NT;
        const uint64_t v = (i >= rb && i < re) ? av[j] : 0ull;
        uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
        if (tid & 1) {  // the row is read by an odd group: bytes 0,1 and 2,3 swapped
          lo = __builtin_amdgcn_perm(lo, lo, 0x02030001u);
          hi = __builtin_amdgcn_perm(hi, hi, 0x02030001u);
        }
        As[2 * (tid + j * NT)] = lo;
        As[2 * (tid + j * NT) + 1] = hi;
      }
    }
    if (tid < BT) {
      ulonglong2 bv[8];
#pragma unroll
      for (int b = 0; b < 8; ++b) bv[b] = Bs[half][8 * g_b + b][w2];
      uint64_t c0 = 0ull, c1 = 0ull;
#pragma unroll
      for (int b = LOGE; b < 8; ++b)
        if ((uu >> (b - LOGE)) & 1) {
          c0 ^= bv[b].x;
          c1 ^= bv[b].y;
        }
#pragma unroll
      for (int j = 0; j < EPJ; ++j) {
        const int gj = j ^ (j >> 1);
        *(ulonglong2 *)&T[g_b >> 1][EPJ * uu + gj][g_b & 1][2 * w2] = make_ulonglong2(c0, c1);
        if (j < EPJ - 1) {
          c0 ^= bv[__builtin_ctz(j + 1)].x;
          c1 ^= bv[__builtin_ctz(j + 1)].y;
        }
      }
    }
    if (hh + 1 < nh) stage_b(half ^ 1);  // buffer half ^ 1 was last read before the previous barrier
    if (hh + 2 < nh) load_b(hh + 2);     // in flight during the lookups
    if (half == 0 && (hh >> 1) + 1 < a.kwords) load_a((hh >> 1) + 1, av);
    __syncthreads();
    // A words of a row pair are read two pairs ahead and the table reads of
    // the next pair are issued before the current pair is combined: LDS reads
    // complete in order, so every wait leaves the nine later reads in flight.
    auto read_a = [&](int u0, uint32_t (&a32)[UB]) {
#pragma unroll
      for (int v = 0; v < UB; ++v) a32[v] = As[2 * (8 * (wv + NW * (u0 + v)) + G) + half];
    };
    auto issue = [&](const uint32_t (&a32)[UB], uint4 (&t)[UB][4]) {
#pragma unroll
      for (int v = 0; v < UB; ++v)
#pragma unroll
        for (int g = 0; g < 4; ++g) t[v][g] = *(const uint4 *)(Tb + __builtin_amdgcn_perm(a32[v], lb, kSel[g]));
    };
    auto combine = [&](int u0, const uint4 (&t)[UB][4]) {
#pragma unroll
      for (int v = 0; v < UB; ++v) {
        uint32_t x0 = (uint32_t)acc[u0 + v][0], x1 = (uint32_t)(acc[u0 + v][0] >> 32);
        uint32_t x2 = (uint32_t)acc[u0 + v][1], x3 = (uint32_t)(acc[u0 + v][1] >> 32);
        x0 = __builtin_amdgcn_bitop3_b32(x0, t[v][0].x, t[v][1].x, 0x96);
        x1 = __builtin_amdgcn_bitop3_b32(x1, t[v][0].y, t[v][1].y, 0x96);
        x2 = __builtin_amdgcn_bitop3_b32(x2, t[v][0].z, t[v][1].z, 0x96);
        x3 = __builtin_amdgcn_bitop3_b32(x3, t[v][0].w, t[v][1].w, 0x96);
        x0 = __builtin_amdgcn_bitop3_b32(x0, t[v][2].x, t[v][3].x, 0x96);
        x1 = __builtin_amdgcn_bitop3_b32(x1, t[v][2].y, t[v][3].y, 0x96);
        x2 = __builtin_amdgcn_bitop3_b32(x2, t[v][2].z, t[v][3].z, 0x96);
        x3 = __builtin_amdgcn_bitop3_b32(x3, t[v][2].w, t[v][3].w, 0x96);
        acc[u0 + v][0] = ((uint64_t)x1 << 32) | x0;
        acc[u0 + v][1] = ((uint64_t)x3 << 32) | x2;
      }
    };
    uint32_t aA[UB], aB[UB];
    uint4 tA[UB][4], tB[UB][4];
    read_a(0, aA);
    read_a(UB, aB);
    issue(aA, tA);
#pragma unroll
    for (int u0 = 0; u0 < RPL; u0 += 2 * UB) {
      if (u0 + 2 * UB < RPL) read_a(u0 + 2 * UB, aA);
      issue(aB, tB);
      combine(u0, tA);
      if (u0 + 3 * UB < RPL) read_a(u0 + 3 * UB, aB);
      if (u0 + 2 * UB < RPL) issue(aA, tA);
      combine(u0 + UB, tB);
    }
  }

  uint64_t any;
  {
    uint64_t *C = a.C;
    asm volatile("" : "+s"(C));
    uint64_t *Cl = C + (((int64_t)blk * a.ldC + tile0 + 8 * wv + G) * TW + 2 * w2);
    any = store_acc2<RPL, 8 * NW>(acc, Cl, ok0, ok1, ulo, uhi);
  }
  if (a.nzflag) {
    if (__ballot(any != 0ull) != 0ull && lane == 0) atomicOr(a.nzflag, 1u);
  }
  if (a.work && tid == 0) {
    int64_t lo = (int64_t)blk * TW, hi = lo + TW;
    if (lo < a.qc0) lo = a.qc0;
    if (hi > a.qc1) hi = a.qc1;
    const unsigned long long words = hi > lo ? (unsigned long long)(hi - lo) : 0ull;
    atomicAdd(a.work, (unsigned long long)(re - rb) * words * (unsigned long long)a.kwords * 8ull);
  }
}


// Narrow product (the next panel's columns): column tiles of 8 words (chunk
// blockIdx.y of the 8-aligned chunks covering [qc0, qc1)), 64-byte entries
// (8 words), and a step takes a whole 64-bit A word: eight tables of 256
// entries (128 KB), so K = 512 takes 8 barrier-separated steps instead of 16.
// Tables g = 4p + s at byte p*65536 + idx*256 + s*64 + word*8.
// A wave is 16 groups of 4 lanes; lane w4 owns words 2*w4, 2*w4+1 and a 16-byte
// read fetches them.  In read i of a row, group G uses table (i + G) mod 4 of
// half p, so the four groups of every 16 lanes cover 256 distinct bytes.
template <int NT, int TM>
__global__ __launch_bounds__(NT) void k_gemm_narrow(GemmArgs a) {
  constexpr int TPS = 8;                 // tables per step
  constexpr int NW = NT / 64;            // waves
  constexpr int RPL = TM / (16 * NW);    // rows per lane
  constexpr int JOBS = NT / 4;           // table-build jobs (4 threads each, one word pair per thread)
  constexpr int EPJ = TPS * 256 / JOBS;  // entries per job
  constexpr int LOGE = EPJ == 4 ? 2 : (EPJ == 8 ? 3 : (EPJ == 16 ? 4 : (EPJ == 32 ? 5 : 6)));
  static_assert(RPL * 16 * NW == TM && RPL >= 1, "tile");
  static_assert(EPJ == 4 || EPJ == 8 || EPJ == 16 || EPJ == 32 || EPJ == 64, "build split");
  static_assert(TM % NT == 0, "A staging");
  __shared__ uint64_t T[2][256][4][8];
  __shared__ uint64_t As[TM];            // the tile's A word for the current 64 inner bits

  if (a.skip_flag && *a.skip_flag == 0u) return;  // the Schur complement is already zero
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, G = lane >> 2, w4 = lane & 3;
  const int64_t q8 = (int64_t)(a.qc0 & ~7) + 8ll * blockIdx.y;  // first word of this chunk
  const int64_t qw = q8 + 2 * w4;
  const bool ok0 = qw >= a.qc0 && qw < a.qc1, ok1 = qw + 1 >= a.qc0 && qw + 1 < a.qc1;

  const int64_t tile0 = a.row_tile0 + (int64_t)blockIdx.x * TM;
  int64_t rb = tile0;
  if (a.bsub) {
    const int64_t d = a.bsub[a.kwords - 1].R + a.bsub[a.kwords - 1].r;
    if (d > rb) rb = d;
  }
  int64_t re = tile0 + TM < a.row_end ? tile0 + TM : a.row_end;
  if (rb >= re) return;

  // rows of this lane: tile0 + 16*wv + G + 16*NW*u
  int ulo, uhi;
  lane_rows<RPL, 16 * NW>(tile0, 16 * wv + G, rb, re, ulo, uhi);
  const size_t cbase = widx(a.ldC, tile0 + 16 * wv + G, q8) + 2 * w4;  // (q8 % 16) + 2*w4 stays in the block
  // inner words [kw0, kw1) of part blockIdx.z; with several parts each one
  // starts from zero and XORs its partial product into C
  const int nparts = a.kparts > 1 ? a.kparts : 1;
  const int kw0 = (int)(((int64_t)blockIdx.z * a.kwords) / nparts);
  const int kw1 = (int)(((int64_t)(blockIdx.z + 1) * a.kwords) / nparts);
  uint64_t acc[RPL][2];
  {
    uint64_t *C = a.C;
    asm volatile("" : "+s"(C));
    const bool ld = a.accumulate && nparts == 1;
    load_acc2<RPL, 16 * NW>(acc, C + cbase, ld && ok0, ld && ok1, ulo, uhi);
  }

  const int bw4 = tid & 3;
  const int job = tid >> 2;
  const int gb = job / (256 / EPJ), uu = job % (256 / EPJ);  // table of the step, entry block
  const int64_t bq = q8 + 2 * bw4;
  const bool bok0 = bq >= a.qc0 && bq < a.qc1, bok1 = bq + 1 >= a.qc0 && bq + 1 < a.qc1;

  // B rows of table gb of inner word kw (bits [64 kw + 8 gb, +8))
  auto load_b = [&](int kw, uint64_t (&bv)[8][2]) {
    int64_t browR = 64ll * kw;
    int blim;
    if (a.bsub) {
      browR = a.bsub[kw].R;
      blim = a.bsub[kw].r;
    } else {
      const int64_t left = a.b_rows - 64ll * kw;
      blim = left >= 64 ? 64 : (left > 0 ? (int)left : 0);
    }
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int t = 8 * gb + b;
      const uint64_t *p = a.B + widx(a.ldB, browR + t, bq);
      bv[b][0] = (bok0 && t < blim) ? p[0] : 0ull;
      bv[b][1] = (bok1 && t < blim) ? p[1] : 0ull;
    }
  };
  constexpr int APT = TM / NT;
  auto load_a = [&](int kw, uint64_t (&av)[APT]) {
#pragma unroll
    for (int j = 0; j < APT; ++j) {
      const int64_t i = tile0 + tid + (int64_t)j * NT;
      av[j] = (i >= rb && i < re) ? a.A[widx(a.ldA, i, a.a_word0 + kw)] : 0ull;
    }
  };

  uint64_t bv[8][2], av[APT];
  load_b(kw0, bv);
  load_a(kw0, av);
  const char *Tb = (const char *)&T[0][0][0][0];
  uint32_t lbase[4], sel[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int s = (i + G) & 3;
    lbase[i] = ((uint32_t)s << 6) | ((uint32_t)w4 << 4);
    sel[i] = 0x0C0C0000u | ((4u + (uint32_t)s) << 8);  // [lane base | byte s of the A half | 0 | 0]
  }
  for (int kw = kw0; kw < kw1; ++kw) {
    __syncthreads();  // previous lookups finished: T and As are free
#pragma unroll
    for (int j = 0; j < APT; ++j) As[tid + j * NT] = av[j];
    {
      uint64_t c0 = 0ull, c1 = 0ull;
#pragma unroll
      for (int b = LOGE; b < 8; ++b)
        if ((uu >> (b - LOGE)) & 1) {
          c0 ^= bv[b][0];
          c1 ^= bv[b][1];
        }
#pragma unroll
      for (int j = 0; j < EPJ; ++j) {
        const int gj = j ^ (j >> 1);
        *(ulonglong2 *)&T[gb >> 2][EPJ * uu + gj][gb & 3][2 * bw4] = make_ulonglong2(c0, c1);
        if (j < EPJ - 1) {
          c0 ^= bv[__builtin_ctz(j + 1)][0];
          c1 ^= bv[__builtin_ctz(j + 1)][1];
        }
      }
    }
    if (kw + 1 < kw1) {  // in flight during the lookups
      load_b(kw + 1, bv);
      load_a(kw + 1, av);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const uint64_t aw = As[16 * (wv + NW * u) + G];
      const uint32_t alo = (uint32_t)aw, ahi = (uint32_t)(aw >> 32);
      uint4 t[TPS];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        t[i] = *(const uint4 *)(Tb + __builtin_amdgcn_perm(alo, lbase[i], sel[i]));
        t[4 + i] = *(const uint4 *)(Tb + (__builtin_amdgcn_perm(ahi, lbase[i], sel[i]) | 0x10000u));
      }
      uint32_t x0 = (uint32_t)acc[u][0], x1 = (uint32_t)(acc[u][0] >> 32);
      uint32_t x2 = (uint32_t)acc[u][1], x3 = (uint32_t)(acc[u][1] >> 32);
#pragma unroll
      for (int i = 0; i < TPS; i += 2) {
        x0 = __builtin_amdgcn_bitop3_b32(x0, t[i].x, t[i + 1].x, 0x96);
        x1 = __builtin_amdgcn_bitop3_b32(x1, t[i].y, t[i + 1].y, 0x96);
        x2 = __builtin_amdgcn_bitop3_b32(x2, t[i].z, t[i + 1].z, 0x96);
        x3 = __builtin_amdgcn_bitop3_b32(x3, t[i].w, t[i + 1].w, 0x96);
      }
      acc[u][0] = ((uint64_t)x1 << 32) | x0;
      acc[u][1] = ((uint64_t)x3 << 32) | x2;
    }
  }

  uint64_t any;
  {
    uint64_t *C = a.C;
    asm volatile("" : "+s"(C));
    any = nparts == 1 ? store_acc2<RPL, 16 * NW>(acc, C + cbase, ok0, ok1, ulo, uhi)
                      : xor_acc2<RPL, 16 * NW>(acc, C + cbase, ok0, ok1, ulo, uhi);
  }
  if (a.nzflag) {
    if (__ballot(any != 0ull) != 0ull && lane == 0) atomicOr(a.nzflag, 1u);
  }
  if (a.work && tid == 0) {
    int64_t lo = q8, hi = q8 + 8;
    if (lo < a.qc0) lo = a.qc0;
    if (hi > a.qc1) hi = a.qc1;
    const unsigned long long words = hi > lo ? (unsigned long long)(hi - lo) : 0ull;
    atomicAdd(a.work, (unsigned long long)(re - rb) * words * (unsigned long long)(kw1 - kw0) * 8ull);
  }
}

// Product-kernel variants (same results; chosen per call by a tuning knob, or
// automatically when the knob is -1):
//   0: k_gemm_wide, 512 threads, 2048-row tiles
//   1: k_gemm_wide, 512 threads, 1024-row tiles
//   2: k_gemm_wide, 256 threads, 512-row tiles
//   3: k_gemm_wide, 256 threads, 256-row tiles
//   4: k_gemm_narrow, 256 threads, 256 rows x 8 words
//   5: k_gemm_narrow, 256 threads, 512 rows x 8 words
// Automatic choice: the largest tile that still gives at least one workgroup
// per CU for the rows expected to be active; small launches get small tiles.
// threads of the 2048-row tile (variant 0): 512 (8 waves, two rows per
// lookup group) or 1024 (16 waves, one row per lookup group: 128 registers,
// four waves per SIMD).  Measured on MI355X: 65536^2 decomposition 55.7-56.1
// against 57.1-57.3 ms; 16384^3 product on this tile 1.80 against 1.88 ms.
int g_wide_threads = 1024;

int gemm_tile_rows(int v) {
  switch (v) {
    case 0: return 2048;
    case 1: return 1024;
    case 2: case 5: return 512;
    default: return 256;
  }
}

// An 8-word column range starting at a multiple of 8 (the next panel's
// columns) fits the narrow kernel.
bool gemm_narrow_ok(int qc0, int qc1) { return qc0 % 8 == 0 && qc1 > qc0 && qc1 - qc0 <= 8; }

int gemm_auto_variant(int64_t active_rows, int qc0, int qc1, int ncu) {
  const int64_t want = ncu;
  if (gemm_narrow_ok(qc0, qc1)) return (active_rows + 511) / 512 >= want ? 5 : 4;
  const int blocks_y = ((qc1 - 1) >> 4) - (qc0 >> 4) + 1;
  for (int v = 0; v < 4; ++v) {
    const int tm = gemm_tile_rows(v);
    if (((active_rows + tm - 1) / tm) * (int64_t)blocks_y >= want) return v;
  }
  return 3;
}

// Tile for a product whose wall time matters (a decomposition's updates run
// between two dependent launches): the tile minimising rounds x (time of one
// 32-bit step of a workgroup), with the step time alpha * TM + beta fitted to
// MI355X measurements of the wide kernel (0.00212 us per row: the lookups;
// 1.66 us: the table build, barriers and staging), one workgroup per CU.
int gemm_wall_variant(int64_t active_rows, int qc0, int qc1, int ncu) {
  if (gemm_narrow_ok(qc0, qc1)) return gemm_auto_variant(active_rows, qc0, qc1, ncu);
  const int blocks_y = ((qc1 - 1) >> 4) - (qc0 >> 4) + 1;
  int best = 0;
  double best_t = 1e300;
  for (int v = 0; v < 4; ++v) {
    const int tm = gemm_tile_rows(v);
    const int64_t wgs = ((active_rows + tm - 1) / tm) * (int64_t)blocks_y;
    const double rounds = (double)((wgs + ncu - 1) / ncu);
    const double t = rounds * (0.00212 * tm + 1.66);
    if (t < best_t) {
      best_t = t;
      best = v;
    }
  }
  return best;
}

// With timing events (e0, e1 both set) the launch itself records the kernel's
// start and end, instead of two marker packets around it on the stream.
hipError_t launch_gemm(const GemmArgs &a, int64_t nrows_max, int v, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (nrows_max <= 0 || a.qc1 <= a.qc0) {
    if (e0 && e1) {  // an empty interval, so the pair stays valid
      hipError_t r = hipEventRecord(e0, s);
      return r != hipSuccess ? r : hipEventRecord(e1, s);
    }
    return hipSuccess;
  }

  const int TM = gemm_tile_rows(v);
  const int64_t tiles = (nrows_max + TM - 1) / TM;
  const int blocks_y = ((a.qc1 - 1) >> 4) - (a.qc0 >> 4) + 1;
  const dim3 grid = a.bsub ? dim3((unsigned)blocks_y, (unsigned)tiles) : dim3((unsigned)tiles, (unsigned)blocks_y);
  const int chunks = ((a.qc1 - 1) >> 3) - (a.qc0 >> 3) + 1;  // 8-word chunks (narrow kernels)
  const dim3 gridn((unsigned)tiles, (unsigned)chunks, (unsigned)(a.kparts > 1 ? a.kparts : 1));
#define GF2_LAUNCH(K, GRID, NT)                                              \
  do {                                                                       \
    if (e0 && e1)                                                            \
      hipExtLaunchKernelGGL(K, GRID, dim3(NT), 0, s, e0, e1, 0, a);          \
    else                                                                     \
      hipLaunchKernelGGL(K, GRID, dim3(NT), 0, s, a);                        \
  } while (0)
  switch (v) {
    case 0:
      if (g_wide_threads == 1024)
        GF2_LAUNCH((k_gemm_wide<1024, 2048>), grid, 1024);
      else
        GF2_LAUNCH((k_gemm_wide<512, 2048>), grid, 512);
      break;
    case 1: GF2_LAUNCH((k_gemm_wide<512, 1024>), grid, 512); break;
    case 2: GF2_LAUNCH((k_gemm_wide<256, 512>), grid, 256); break;
    case 4: GF2_LAUNCH((k_gemm_narrow<256, 256>), gridn, 256); break;
    case 5: GF2_LAUNCH((k_gemm_narrow<256, 512>), gridn, 256); break;
    default: GF2_LAUNCH((k_gemm_wide<256, 256>), grid, 256); break;
  }
#undef GF2_LAUNCH
  return hipGetLastError();
}

}  // namespace gf2
