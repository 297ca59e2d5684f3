// k_mfma.hip -- the GF(2) product C (^)= A*B on the fp4 matrix cores of gfx950.
//
// Over the integers, (A*B)[i][j] = popcount(A_i AND B^T_j) and the GF(2) entry is
// its parity (Section 6 computes the same sum with tables instead).  Each bit
// becomes an e2m1 value, 1.0 or 0.0, so one v_mfma_scale_f32_32x32x64_f8f6f4
// (unit scales) adds 64 products per output exactly in fp32 (sums stay far below
// 2^24), and the parity of the integer-valued result is the output bit.
//
// Operand layout of the instruction: lane l holds row (or column) l % 32 and 32
// of the 64 inner indices (half l / 32 of a word), eight per register as
// nibbles; output register r of lane l is row 8 (r / 4) + 4 (l / 32) + r % 4,
// column l % 32.
//
// Both operands are first repacked into "quad" layout: for every group of four
// inner words, entry (row, half) holds that half of the four words as one
// 16-byte vector, and the 32 rows x 2 halves a wave needs for one fragment are
// 1 KB of consecutive bytes.
//   k_at_pack   A (column-blocked)          -> At4[kq][row][half]
//   k_bt_pack   B (column-blocked, K x m)   -> Bt4[kq][column][half]: one 64 x 64
//               bit transpose per inner word (a butterfly of six exchange steps
//               across lanes), four words per wave.
//   k_gemm_mfma every wave owns 128 rows x one output word (4 x 2 MFMAs per
//               inner word) and builds its own fragments: one 16-byte load per
//               fragment and quad, spread into four registers per word, loads
//               kQuadsAhead quads ahead.  No LDS and no workgroup barrier.
//               At the end a ballot of the low bit of each register yields 32
//               columns of two rows at once, already bit-packed.
#include "gf2_internal.h"

namespace gf2 {

// v_writelane_b32 (lane `lane` of `old` receives the uniform value `val`)
extern "C" __device__ int gf2_mfma_writelane(int val, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

namespace {

typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// The 32 bits of x -> four registers of eight e2m1 nibbles (0b0010 = 1.0 or
// 0.0): register r, nibble j holds bit 4 j + r.  The inner sum runs over all
// indices of a word in any order, so rows of A and columns of B need only share
// the placement.
__device__ inline uint4 spread32(uint32_t x) {
  return make_uint4((x << 1) & 0x22222222u, x & 0x22222222u, (x >> 1) & 0x22222222u, (x >> 2) & 0x22222222u);
}

constexpr int kQuadsAhead = 2;  // raw quads in flight per fragment (loads run this many quads ahead)
constexpr int kWR = 2, kWC = 2;   // waves per workgroup: row groups x output words
constexpr int kMThreads = 64 * kWR * kWC, kMRows = 128 * kWR;

// Wave (kq, q): words 4 kq .. 4 kq + 3 of the 64 rows 64 w .. of B (column word
// q), transposed; lane j then holds column 64 q + j and writes its two halves
// of the four words.  Rows past the operand and words past bwords are zero.
__global__ __launch_bounds__(256) void k_bt_pack(const uint64_t *B, int64_t ldB, int64_t b_rows, int64_t bwords,
                                                 uint4 *Bt4, int64_t mpad, int kqp) {
  const int lane = threadIdx.x & 63;
  const int64_t nq = mpad / 64;
  const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (blk >= (int64_t)kqp * nq) return;  // whole waves
  const int64_t kq = blk / nq, q = blk % nq;
  uint32_t lo[4], hi[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t row = 64 * (4 * kq + u) + lane;
    const uint64_t x = (row < b_rows && q < bwords) ? B[widx(ldB, row, q)] : 0ull;
    const uint64_t t = transpose64(x, lane);
    lo[u] = (uint32_t)t;
    hi[u] = (uint32_t)(t >> 32);
  }
  uint4 *dst = Bt4 + 2 * (kq * mpad + 64 * q + lane);
  dst[0] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
  dst[1] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
}

// Thread (kq, r): words 4 kq .. 4 kq + 3 of row row0 + r of A into At4, for
// kq < kqp and r < npad.  Four consecutive threads take four consecutive quads
// of one row (128 contiguous bytes of a column block).  Rows past the operand
// repeat its last row (their results are never stored); words from kwords on
// are zero.
__global__ __launch_bounds__(256) void k_at_pack(const uint64_t *A, int64_t ldA, int64_t a_word0, int64_t row0,
                                                 int kwords, uint4 *At4, int64_t npad, int kqp) {
  const int64_t nb = (kqp + 3) / 4, total = 4 * nb * npad;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t rest = e >> 2, r = rest % npad, kq = 4 * (rest / npad) + (e & 3);
    if (kq >= kqp) continue;
    int64_t row = row0 + r;
    row = row < ldA ? row : ldA - 1;
    uint32_t lo[4], hi[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t kw = 4 * kq + u;
      const uint64_t x = kw < kwords ? A[widx(ldA, row, a_word0 + kw)] : 0ull;
      lo[u] = (uint32_t)x;
      hi[u] = (uint32_t)(x >> 32);
    }
    uint4 *dst = At4 + 2 * (kq * npad + r);
    dst[0] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
    dst[1] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
  }
}

// Wave w of a workgroup: rows 128 (w / kWC) .. +127 of its kMRows, output word
// w % kWC of its kWC.  kqp (a multiple of kQuadsAhead) quads of At4 and Bt4 are
// valid, npad and mpad their row and column extents.  Two waves per SIMD (the
// 128 accumulators stay in ordinary registers).
// Split inner dimension: workgroup z takes quads [z * per, (z + 1) * per) (per a
// multiple of kQuadsAhead) and, when gridDim.z > 1, XORs its parity words into
// C with atomics -- the parity of a sum is the XOR of the parities of its parts.
// C then has to hold its initial value (zero for a plain product) and nzflag
// is not supported.
__global__ __launch_bounds__(kMThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_gemm_mfma(
    GemmArgs a, const uint4 *At4, int64_t npad, const uint4 *Bt4, int64_t mpad, int kqp, int per) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int h = lane >> 5, li = lane & 31;
  const int64_t rw = a.row_tile0 + (int64_t)blockIdx.x * kMRows + 128 * (wv / kWC);            // first row
  const int64_t q = (int64_t)(a.qc0 / kWC) * kWC + (int64_t)kWC * blockIdx.y + (wv % kWC);  // output word
  const int kq0 = (int)blockIdx.z * per, kq1 = kq0 + per < kqp ? kq0 + per : kqp;
  const bool split = gridDim.z > 1;
  const uint4 *ap = At4 + 2 * (rw - a.row_tile0 + li) + h, *bp = Bt4 + 2 * (64 * q + li) + h;
  auto load = [&](int kq, uint4 (&ra)[4], uint4 (&rb)[2]) {
    const int64_t kc = kq < kqp ? kq : kqp - 1;  // (past the end: a valid quad nobody uses)
#pragma unroll
    for (int i = 0; i < 4; ++i) ra[i] = ap[2 * kc * npad + 64 * i];
#pragma unroll
    for (int j = 0; j < 2; ++j) rb[j] = bp[2 * kc * mpad + 64 * j];
  };
  auto frag = [](uint32_t x) -> v8i {
    const uint4 v = spread32(x);
    return v8i{(int)v.x, (int)v.y, (int)v.z, (int)v.w, 0, 0, 0, 0};
  };
  auto comp = [](const uint4 &v, int u) -> uint32_t { return u == 0 ? v.x : u == 1 ? v.y : u == 2 ? v.z : v.w; };

  v16f acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v16f{};

  uint4 ra[kQuadsAhead][4], rb[kQuadsAhead][2];
#pragma unroll
  for (int d = 0; d < kQuadsAhead; ++d) {
    load(kq0 + d, ra[d], rb[d]);
    __builtin_amdgcn_sched_barrier(0);  // issue in the loop's order, so the waits at its head stay partial
  }
  for (int g0 = kq0; g0 < kq1; g0 += kQuadsAhead) {
#pragma unroll
    for (int d = 0; d < kQuadsAhead; ++d) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        v8i fa[4], fb[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) fa[i] = frag(comp(ra[d][i], u));
#pragma unroll
        for (int k = 0; k < 2; ++k) fb[k] = frag(comp(rb[d][k], u));
        if (u == 3) load(g0 + d + kQuadsAhead, ra[d], rb[d]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < 2; ++k)
            acc[i][k] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[i], fb[k], acc[i][k], 4, 4, 0, 127, 0, 127);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }

  // parity bits: register r of block (i, k) holds rows 8 (r / 4) + r % 4 (lanes
  // 0..31) and + 4 (lanes 32..63) of rows 32 i.., columns 32 k + lane % 32.
  // Row t of this wave's 128 rows goes to lane t % 64 of word pair t / 64.
  int wlo[2] = {0, 0}, whi[2] = {0, 0};
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint64_t b0 = __ballot(((uint32_t)acc[i][0][r] & 1u) != 0u);
      const uint64_t b1 = __ballot(((uint32_t)acc[i][1][r] & 1u) != 0u);
      const int ta = 32 * i + 8 * (r >> 2) + (r & 3), tb = ta + 4;
      wlo[ta >> 6] = gf2_mfma_writelane((int)(uint32_t)b0, ta & 63, wlo[ta >> 6]);
      whi[ta >> 6] = gf2_mfma_writelane((int)(uint32_t)b1, ta & 63, whi[ta >> 6]);
      wlo[tb >> 6] = gf2_mfma_writelane((int)(uint32_t)(b0 >> 32), tb & 63, wlo[tb >> 6]);
      whi[tb >> 6] = gf2_mfma_writelane((int)(uint32_t)(b1 >> 32), tb & 63, whi[tb >> 6]);
    }
  uint64_t any = 0ull;
  if (q >= a.qc0 && q < a.qc1) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int64_t row = rw + 64 * p + lane;
      if (row < a.row_end) {
        uint64_t v = ((uint64_t)(uint32_t)whi[p] << 32) | (uint32_t)wlo[p];
        uint64_t *cp = a.C + widx(a.ldC, row, q);
        if (split) {
          atomicXor((unsigned long long *)cp, (unsigned long long)v);
        } else {
          if (a.accumulate) v ^= *cp;
          *cp = v;
          any |= v;
        }
      }
    }
  }
  if (a.nzflag) {
    if (__ballot(any != 0ull) != 0ull && lane == 0) atomicOr(a.nzflag, 1u);
  }
  if (a.work && lane == 0 && q >= a.qc0 && q < a.qc1) {
    const int64_t re = rw + 128 < a.row_end ? rw + 128 : a.row_end;
    const int w1 = 4 * kq1 < a.kwords ? 4 * kq1 : a.kwords, words = w1 - 4 * kq0;
    if (re > rw && words > 0) atomicAdd(a.work, (unsigned long long)(re - rw) * (unsigned long long)words * 8ull);
  }
}

int64_t quads_padded(int64_t kwords) {
  const int64_t kq = (kwords > 0 ? kwords + 3 : 4) / 4;
  return (kq + kQuadsAhead - 1) / kQuadsAhead * kQuadsAhead;
}
int64_t cols_padded(int64_t words) { return (words + kWC - 1) / kWC * kWC * 64; }
int64_t rows_padded(int64_t rows) { return (rows + kMRows - 1) / kMRows * kMRows; }

// Quads per split of the inner dimension (== kqp: no split).  Split while the
// tiles fill fewer than the device's two resident workgroups per CU, down to
// four quads (16 inner words) per split.
int64_t split_quads(const GemmArgs &a, int ncu) {
  const int64_t kqp = quads_padded(a.kwords);
  if (a.nzflag || ncu <= 0) return kqp;
  const int64_t tiles = (rows_padded(a.row_end - a.row_tile0) / kMRows) * (((a.qc1 - 1) / kWC) - (a.qc0 / kWC) + 1);
  int64_t splits = 2ll * ncu / (tiles > 0 ? tiles : 1);
  if (splits > kqp / 4) splits = kqp / 4;
  if (splits < 2) return kqp;
  const int64_t per = (kqp + splits - 1) / splits;
  return (per + kQuadsAhead - 1) / kQuadsAhead * kQuadsAhead;
}

}  // namespace

bool mfma_splits_inner(const GemmArgs &a, int ncu) {
  if (a.bsub || a.qc1 <= a.qc0 || a.row_end <= a.row_tile0) return false;
  return split_quads(a, ncu) < quads_padded(a.kwords);
}

size_t mfma_ws_bytes(int64_t kwords, int64_t m_words, int64_t rows) {
  const int64_t kqp = quads_padded(kwords);
  return (size_t)kqp * (size_t)(cols_padded(m_words) + rows_padded(rows)) * 32;
}

// C (^)= A * B with plain B (a.bsub == nullptr) on the matrix cores; ws is a
// workspace of mfma_ws_bytes(a.kwords, bwords, a.row_end - a.row_tile0) bytes
// (Bt4 first, then At4; both are whole multiples of 32 bytes per quad row).
// When mfma_splits_inner(a, ncu) holds, the inner dimension is split and C must
// already hold its initial value: a plain product needs a zeroed C and
// a.accumulate set.
hipError_t launch_gemm_mfma(const GemmArgs &a, int64_t bwords, uint64_t *ws, int ncu, hipStream_t s) {
  if (a.bsub || a.qc1 <= a.qc0 || a.row_end <= a.row_tile0) return a.bsub ? hipErrorInvalidValue : hipSuccess;
  const int64_t mp_c = cols_padded(a.qc1), mp_b = cols_padded(bwords);
  const int64_t mp = mp_c > mp_b ? mp_c : mp_b;
  const int64_t kqp = quads_padded(a.kwords);
  const int64_t rows = a.row_end - a.row_tile0, npad = rows_padded(rows);
  uint4 *Bt4 = (uint4 *)ws, *At4 = Bt4 + 2 * kqp * mp;
  const int64_t tw = (kqp * (mp / 64) + 3) / 4;
  hipLaunchKernelGGL(k_bt_pack, dim3((unsigned)tw), dim3(256), 0, s, a.B, a.ldB, a.b_rows, bwords, Bt4, mp, (int)kqp);
  const int64_t ta = ((kqp + 3) / 4 * 4 * npad + 255) / 256;
  hipLaunchKernelGGL(k_at_pack, dim3((unsigned)(ta < 16384 ? ta : 16384)), dim3(256), 0, s, a.A, a.ldA,
                     (int64_t)a.a_word0, a.row_tile0, a.kwords, At4, npad, (int)kqp);
  const int64_t tiles_c = ((a.qc1 - 1) / kWC) - (a.qc0 / kWC) + 1;
  const int64_t per = split_quads(a, ncu), nz = (kqp + per - 1) / per;
  hipLaunchKernelGGL(k_gemm_mfma, dim3((unsigned)(npad / kMRows), (unsigned)tiles_c, (unsigned)nz), dim3(kMThreads), 0,
                     s, a, (const uint4 *)At4, npad, (const uint4 *)Bt4, mp, (int)kqp, (int)per);
  return hipGetLastError();
}

}  // namespace gf2
