// k_mfma.hip -- the GF(2) product C (^)= A*B on the fp4 matrix cores of gfx950.
//
// Over the integers, (A*B)[i][j] = popcount(A_i AND B^T_j) and the GF(2) entry is
// its parity (Section 6 computes the same sum with tables instead).  Each bit
// becomes an e2m1 value, 1.0 or 0.0, so one v_mfma_scale_f32_32x32x64_f8f6f4
// (unit scales) adds 64 products per output exactly in fp32 (sums stay far below
// 2^24), and the parity of the integer-valued result is the output bit.
//   k_bt_transpose  B (K x m, column-blocked) -> Bt[kw][j]: word kw of column j
//                   of B, i.e. one 64 x 64 bit transpose per wave (a butterfly
//                   of six exchange steps across lanes).
//   k_gemm_mfma     512 threads own 256 rows x 4 output words.  Per stage of two
//                   64-bit inner words each thread expands one A row or one Bt
//                   column into 2 x 32 bytes of fp4 in LDS (two buffers, one
//                   barrier per stage); wave w runs 2 x 4 x 2 MFMAs of
//                   32 x 32 x 64 on rows 128 (w / 4) .. +127, output word w % 4,
//                   and expands the next stage while they execute.
//                   Operand layout of the instruction: lane l holds row (or
//                   column) l % 32 and inner indices 32 (l / 32) .. +31, one
//                   nibble each in order; output register r of lane l is row
//                   8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
//                   At the end a ballot of the low bit of each register yields
//                   32 columns of two rows at once, already bit-packed.
#include "gf2_internal.h"

namespace gf2 {

// v_writelane_b32 (lane `lane` of `old` receives the uniform value `val`)
extern "C" __device__ int gf2_mfma_writelane(int val, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

namespace {

typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Bits 0..7 of x -> nibbles 0..7 holding e2m1 1.0 (0b0010) or 0.0.
__device__ inline uint32_t spread8(uint32_t x) {
  x &= 0xFFu;
  x = (x | (x << 12)) & 0x000F000Fu;
  x = (x | (x << 6)) & 0x03030303u;
  x = (x | (x << 3)) & 0x11111111u;
  return x << 1;
}

__device__ inline uint64_t shfl_xor64(uint64_t x, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, m), hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), m);
  return ((uint64_t)hi << 32) | lo;
}

// Lane k holds row k of a 64 x 64 bit block (bit j = column j); afterwards lane
// j holds column j.  Step with distance d exchanges, between rows k and k + d
// (bit d of k clear), the d x d sub-blocks off the diagonal of each 2d x 2d block.
__device__ inline uint64_t transpose64(uint64_t x, int lane) {
  uint64_t m = 0x00000000FFFFFFFFull;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t y = shfl_xor64(x, d);
    const bool low = (lane & d) == 0;
    const uint64_t t = low ? (((x >> d) ^ y) & m) : (((y >> d) ^ x) & m);
    x ^= low ? (t << d) : t;
    m ^= m << (d >> 1);
  }
  return x;
}

__global__ __launch_bounds__(256) void k_bt_transpose(const uint64_t *B, int64_t ldB, int64_t b_rows, int64_t bwords,
                                                      uint64_t *Bt, int64_t mpad, int kwords) {
  const int lane = threadIdx.x & 63;
  const int64_t nq = mpad / 64;
  const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (blk >= (int64_t)kwords * nq) return;  // whole waves
  const int64_t kw = blk / nq, q = blk % nq;
  const int64_t row = 64 * kw + lane;
  const uint64_t x = (row < b_rows && q < bwords) ? B[widx(ldB, row, q)] : 0ull;
  Bt[kw * mpad + 64 * q + lane] = transpose64(x, lane);
}

constexpr int kMT = 512;   // threads
constexpr int kMRows = 256;  // rows per tile
constexpr int kMWords = 4;   // output words per tile

__global__ __launch_bounds__(kMT) void k_gemm_mfma(GemmArgs a, const uint64_t *Bt, int64_t mpad) {
  constexpr int KS = 2;                   // inner words per stage (one barrier each)
  __shared__ uint4 As[2][KS][kMRows][2];  // fp4 rows of A: 32 bytes per row and inner word
  __shared__ uint4 Bs[2][KS][kMRows][2];  // fp4 columns of B
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 2, wc = wv & 3, h = lane >> 5, li = lane & 31;
  const int hs = h ^ ((li >> 3) & 1);  // the slot of half h in this lane's rows (row bit 3 = li bit 3)
  const int64_t r0 = a.row_tile0 + (int64_t)blockIdx.x * kMRows;
  const int64_t w0 = (int64_t)(a.qc0 & ~(kMWords - 1)) + (int64_t)kMWords * blockIdx.y;  // first output word
  const int nk = a.kwords, ns = (nk + KS - 1) / KS;

  // the words this thread expands: A row r0 + tid (tid < 256) or column
  // 64 w0 + tid - 256 of B (rows past the operand read a clamped row; their
  // results are never stored; inner words past the operand are zero)
  const bool isA = tid < kMRows;
  const int item = tid & (kMRows - 1);
  int64_t arow = r0 + item;
  arow = arow < a.ldA ? arow : a.ldA - 1;
  const uint64_t *bsrc = Bt + 64 * w0 + item;
  // (inner words past the operand read the last word and are zeroed, without a branch)
  auto load = [&](int st, uint64_t (&x)[KS]) {
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int kw = KS * st + u, kc = kw < nk ? kw : nk - 1;
      const uint64_t v = isA ? a.A[widx(a.ldA, arow, a.a_word0 + kc)] : bsrc[(int64_t)kc * mpad];
      x[u] = kw < nk ? v : 0ull;
    }
  };
  // Half h (inner indices 32 h .. 32 h + 31) of row t sits in slot h ^ ((t >> 3) & 1):
  // rows t and t + 8 then use opposite 16-byte halves, so the sixteen lanes of
  // every 16-byte access (sixteen consecutive rows, one half) cover all 64 banks.
  const int sw = (item >> 3) & 1;
  auto expand = [&](const uint64_t (&x)[KS], int buf) {
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const uint32_t lo = (uint32_t)x[u], hi = (uint32_t)(x[u] >> 32);
      uint4 *dst = isA ? &As[buf][u][item][0] : &Bs[buf][u][item][0];
      dst[sw] = make_uint4(spread8(lo), spread8(lo >> 8), spread8(lo >> 16), spread8(lo >> 24));
      dst[sw ^ 1] = make_uint4(spread8(hi), spread8(hi >> 8), spread8(hi >> 16), spread8(hi >> 24));
    }
  };

  v16f acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v16f{};

  uint64_t xa[KS], xb[KS];  // stages st + 1 and st + 2
  {
    uint64_t x0[KS];
    load(0, x0);
    load(1, xa);
    load(2, xb);
    expand(x0, 0);
  }
  __syncthreads();
  for (int st = 0; st < ns; ++st) {
    const int cur = st & 1;
    // fragments of stage st (complete since the last barrier), their MFMAs, and
    // then, while the matrix cores work, the next stage's expansion into the
    // other buffer (last read before the previous barrier)
    v8i fa[KS][4], fb[KS][2];
#pragma unroll
    for (int u = 0; u < KS; ++u) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint4 v = As[cur][u][128 * wr + 32 * i + li][hs];
        fa[u][i] = v8i{(int)v.x, (int)v.y, (int)v.z, (int)v.w, 0, 0, 0, 0};
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const uint4 v = Bs[cur][u][64 * wc + 32 * j + li][hs];
        fb[u][j] = v8i{(int)v.x, (int)v.y, (int)v.z, (int)v.w, 0, 0, 0, 0};
      }
    }
#pragma unroll
    for (int u = 0; u < KS; ++u)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[u][i], fb[u][j], acc[i][j], 4, 4, 0, 127, 0,
                                                                      127);
    expand(xa, cur ^ 1);  // (after the last stage: zeros nobody reads)
#pragma unroll
    for (int u = 0; u < KS; ++u) xa[u] = xb[u];
    load(st + 3, xb);
    __syncthreads();
  }

  // parity bits: register r of block (i, j) holds rows 8 (r / 4) + r % 4 (lanes
  // 0..31) and + 4 (lanes 32..63) of rows 32 i.., columns 32 j + lane % 32.
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
  const int64_t q = w0 + wc;
  uint64_t any = 0ull;
  if (q >= a.qc0 && q < a.qc1) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int64_t row = r0 + 128 * wr + 64 * p + lane;
      if (row < a.row_end) {
        uint64_t v = ((uint64_t)(uint32_t)whi[p] << 32) | (uint32_t)wlo[p];
        uint64_t *cp = a.C + widx(a.ldC, row, q);
        if (a.accumulate) v ^= *cp;
        *cp = v;
        any |= v;
      }
    }
  }
  if (a.nzflag) {
    if (__ballot(any != 0ull) != 0ull && lane == 0) atomicOr(a.nzflag, 1u);
  }
  if (a.work && tid == 0) {
    int64_t re = r0 + kMRows < a.row_end ? r0 + kMRows : a.row_end;
    int64_t lo = w0, hi = w0 + kMWords;
    if (lo < a.qc0) lo = a.qc0;
    if (hi > a.qc1) hi = a.qc1;
    const unsigned long long words = hi > lo ? (unsigned long long)(hi - lo) : 0ull;
    if (re > r0) atomicAdd(a.work, (unsigned long long)(re - r0) * words * (unsigned long long)nk * 8ull);
  }
}

}  // namespace

size_t mfma_bt_bytes(int64_t kwords, int64_t m_words) {
  const int64_t mpad = ((m_words + kMWords - 1) / kMWords) * kMWords * 64;
  return (size_t)(kwords > 0 ? kwords : 1) * (size_t)mpad * 8;
}

// C (^)= A * B with plain B (a.bsub == nullptr), Bt a workspace of
// mfma_bt_bytes(a.kwords, words of B) bytes.
hipError_t launch_gemm_mfma(const GemmArgs &a, int64_t bwords, uint64_t *Bt, hipStream_t s) {
  if (a.bsub || a.qc1 <= a.qc0 || a.row_end <= a.row_tile0) return a.bsub ? hipErrorInvalidValue : hipSuccess;
  const int64_t mpad = ((int64_t)((a.qc1 + kMWords - 1) / kMWords) * kMWords) * 64;
  const int64_t mpad_b = ((bwords + kMWords - 1) / kMWords) * kMWords * 64;
  const int64_t mp = mpad > mpad_b ? mpad : mpad_b;
  const int64_t blocks = ((int64_t)(a.kwords > 0 ? a.kwords : 1) * (mp / 64) + 3) / 4;
  if (a.kwords > 0)
    hipLaunchKernelGGL(k_bt_transpose, dim3((unsigned)blocks), dim3(256), 0, s, a.B, a.ldB, a.b_rows, bwords, Bt, mp,
                       a.kwords);
  const int64_t rows = a.row_end - a.row_tile0;
  const int64_t tiles_r = (rows + kMRows - 1) / kMRows;
  const int64_t tiles_c = ((a.qc1 - 1) / kMWords) - (a.qc0 / kMWords) + 1;
  hipLaunchKernelGGL(k_gemm_mfma, dim3((unsigned)tiles_r, (unsigned)tiles_c), dim3(kMT), 0, s, a, (const uint64_t *)Bt, mp);
  return hipGetLastError();
}

}  // namespace gf2
