// k_gemm.hip -- Four-Russians GF(2) product C (^)= A*B on gfx950.
//
// Section 6 of the paper: for each group of c = 8 consecutive bits of the
// inner dimension, a table of the 2^c XOR combinations of the matching 8 rows
// of B is built once (one XOR per entry, Gray-code order), and each output row
// then needs a single table lookup and one XOR per group (eq. (M4RM:cost):
// T = (b/c)(2^c - 1) XORs for the tables plus R = b/c XORs per row).
//
// gfx950 mapping.  A workgroup owns a tile of TM rows x one 16-word column
// block of C (1024 columns).  A wave is four 16-lane groups; each group works
// on one row at a time and lane l of the group owns word l of the block row,
// so the table index (a byte of the row's A word) is uniform in the group and
// every lookup reads one contiguous 128-byte table entry: 512 bytes per wave
// instruction with no LDS bank conflicts.  Four tables (32 inner bits, 128 KB
// of LDS) are live at a time.  Accumulators stay in registers for the whole
// inner loop, so C is read and written once per launch.
#include "gf2_internal.h"

namespace gf2 {

template <int NT, int TM>
__global__ __launch_bounds__(NT) void k_gemm_m4rm(GemmArgs a) {
  constexpr int NW = NT / 64;          // waves
  constexpr int RPL = TM / (4 * NW);   // rows per lane
  static_assert(RPL * 4 * NW == TM, "tile");
  __shared__ uint64_t T[4][256][TW];   // 4 tables x 256 entries x 16 words = 128 KB
  __shared__ uint64_t As[TM];          // the tile's A word for the current 64 inner bits

  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, h = lane >> 4, wl = lane & 15;
  const int blk = blockIdx.y + (a.qc0 >> 4);
  const int64_t q = (int64_t)blk * TW + wl;
  const bool qok = q >= a.qc0 && q < a.qc1;

  if (a.skip_flag && *a.skip_flag == 0u) return;  // the Schur complement is already zero
  const int64_t tile0 = a.row_tile0 + (int64_t)blockIdx.x * TM;
  int64_t rb = tile0;
  if (a.row_begin_dev) {
    int64_t d = *a.row_begin_dev;
    if (d > rb) rb = d;
  }
  int64_t re = tile0 + TM < a.row_end ? tile0 + TM : a.row_end;
  if (rb >= re) return;

  uint64_t acc[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int64_t i = tile0 + 4 * (wv + NW * u) + h;
    acc[u] = 0;
    if (a.accumulate && qok && i >= rb && i < re) acc[u] = a.C[widx(a.ldC, i, q)];
  }

  // table-build role of this thread: word bw of the block, tables g, entries [32*uu, 32*uu+32)
  const int bw = tid & 15;
  const int64_t bq = (int64_t)blk * TW + bw;
  const bool bq_ok = bq >= a.qc0 && bq < a.qc1;

  for (int kw = 0; kw < a.kwords; ++kw) {
    __syncthreads();
    for (int j = tid; j < TM; j += NT) {
      const int64_t i = tile0 + j;
      As[j] = (i >= rb && i < re) ? a.A[widx(a.ldA, i, a.a_word0 + kw)] : 0ull;
    }
    int64_t browR = 64ll * kw;  // B row of inner bit 64*kw + t is browR + t when t < blim
    int blim;
    if (a.bsub) {
      browR = a.bsub[kw].R;
      blim = a.bsub[kw].r;
    } else {
      int64_t left = a.b_rows - 64ll * kw;
      blim = left >= 64 ? 64 : (left > 0 ? (int)left : 0);
    }
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
      if (half) __syncthreads();
      // ---- build 4 tables for inner bits [64kw + 32half, +32)
      for (int job = tid >> 4; job < 32; job += NT / 16) {
        const int g = job >> 3, uu = job & 7;
        uint64_t bv[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const int t = 32 * half + 8 * g + b;
          bv[b] = (bq_ok && t < blim) ? a.B[widx(a.ldB, browR + t, bq)] : 0ull;
        }
        uint64_t cur = ((uu & 1) ? bv[5] : 0ull) ^ ((uu & 2) ? bv[6] : 0ull) ^ ((uu & 4) ? bv[7] : 0ull);
#pragma unroll
        for (int j = 0; j < 32; ++j) {
          const int gj = j ^ (j >> 1);
          T[g][32 * uu + gj][bw] = cur;
          if (j < 31) cur ^= bv[__builtin_ctz(j + 1)];
        }
      }
      __syncthreads();
      // ---- lookups: one 8-byte read and one XOR per 8 inner bits per output word
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const uint32_t a32 = (uint32_t)(As[4 * (wv + NW * u) + h] >> (32 * half));
        acc[u] ^= T[0][a32 & 255u][wl] ^ T[1][(a32 >> 8) & 255u][wl] ^
                  T[2][(a32 >> 16) & 255u][wl] ^ T[3][a32 >> 24][wl];
      }
    }
  }

  uint64_t any = 0;
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int64_t i = tile0 + 4 * (wv + NW * u) + h;
    if (qok && i >= rb && i < re) {
      a.C[widx(a.ldC, i, q)] = acc[u];
      any |= acc[u];
    }
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

hipError_t launch_gemm(const GemmArgs &a, int64_t nrows_max, hipStream_t s) {
  constexpr int NT = 512, TM = 1024;
  if (nrows_max <= 0 || a.qc1 <= a.qc0) return hipSuccess;
  const int64_t tiles = (nrows_max + TM - 1) / TM;
  const int blocks_y = ((a.qc1 - 1) >> 4) - (a.qc0 >> 4) + 1;
  hipLaunchKernelGGL((k_gemm_m4rm<NT, TM>), dim3((unsigned)tiles, (unsigned)blocks_y), dim3(NT), 0,
                     s, a);
  return hipGetLastError();
}

}  // namespace gf2
