// k_solve.hip -- A*X = B through the decomposition P*A = L*E (uses of the
// decomposition listed in Section 1: rank, systems).
//
//   Y = P*B;  forward substitution with the unit lower L_top (sub-panel by
//   sub-panel: the pivot rows of sub-panel q are solved with their own unit
//   lower block, then every later row is updated with its multipliers, which
//   sit in word q of the working matrix);  rows of Y at or below the rank are
//   then the residuals L_bot*y xor (P b)_bot, so system c is consistent iff
//   column c of those rows is zero;  back substitution with E restricted to the
//   pivot columns (free variables zero), sub-panel by sub-panel from the last.
// The substitution kernels run in one workgroup: they are O(n*r/64) word
// operations per 64 right-hand sides, small next to the decomposition.
#include "gf2_internal.h"

namespace gf2 {

__device__ inline uint64_t rdl64s(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

__global__ void k_solve_prep(DecWork w, gf2_mat B, SolveWork sw) {
  const int64_t total = w.n * sw.kw;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e / sw.kw, c = e - i * sw.kw;
    sw.Y[e] = B.data[uidx(B.w, B.ld, w.perm[i], c)] & pad_mask(B.cols, c);
  }
  if (blockIdx.x == 0)
    for (int64_t c = threadIdx.x; c < sw.kw; c += blockDim.x) sw.bad[c] = 0ull;
}

constexpr int kSolveThreads = 1024;

__global__ __launch_bounds__(kSolveThreads) void k_solve_fwd(DecWork w, SolveWork sw) {
  __shared__ uint64_t T[16][16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t ldw = w.ldw;
  for (int q = 0; q < w.Mw; ++q) {
    const SubInfo si = w.sub[q];
    const int r = si.r;
    if (r == 0) continue;
    for (int64_t c = 0; c < sw.kw; ++c) {
      if (wv == 0) {
        const uint64_t lpp = lane < r ? (w.W[widx(ldw, si.R + lane, q)] & ((1ull << lane) - 1ull)) : 0ull;
        uint64_t yv = lane < r ? sw.Y[(si.R + lane) * sw.kw + c] : 0ull;
        for (int t = 0; t < r; ++t) {
          const uint64_t v = rdl64s(yv, t);
          if (lane > t && lane < r && ((lpp >> t) & 1ull)) yv ^= v;
        }
        if (lane < r) sw.Y[(si.R + lane) * sw.kw + c] = yv;
      }
      __syncthreads();
      if (tid < 256) {
        const int g = tid >> 4, e = tid & 15;
        uint64_t v = 0ull;
        for (int b = 0; b < 4; ++b) {
          const int t = 4 * g + b;
          if ((e & (1 << b)) && t < r) v ^= sw.Y[(si.R + t) * sw.kw + c];
        }
        T[g][e] = v;
      }
      __syncthreads();
      const int ng = (r + 3) >> 2;
      for (int64_t i = si.R + r + tid; i < w.n; i += kSolveThreads) {
        const uint64_t l = w.W[widx(ldw, i, q)];
        uint64_t v = 0ull;
        for (int g = 0; g < ng; ++g) v ^= T[g][(l >> (4 * g)) & 15u];
        sw.Y[i * sw.kw + c] ^= v;
      }
      __syncthreads();
    }
  }
}

__global__ void k_solve_check(DecWork w, SolveWork sw) {
  const int64_t rank = w.st->R;
  const int64_t total = (w.n - rank) * sw.kw;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t c = e % sw.kw;
    const uint64_t v = sw.Y[rank * sw.kw + e];
    if (v) atomicOr((unsigned long long *)&sw.bad[c], (unsigned long long)v);
  }
}

__global__ __launch_bounds__(kSolveThreads) void k_solve_back(DecWork w, SolveWork sw) {
  __shared__ uint64_t T[16][16];
  __shared__ uint64_t Xpos[64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t ldw = w.ldw;
  for (int q = w.Mw - 1; q >= 0; --q) {
    const SubInfo si = w.sub[q];
    const int r = si.r;
    if (r == 0) continue;
    for (int64_t c = 0; c < sw.kw; ++c) {
      if (wv == 0) {
        const uint64_t er = lane < r ? w.W[widx(ldw, si.R + lane, q)] : 0ull;
        uint64_t yv = lane < r ? sw.Y[(si.R + lane) * sw.kw + c] : 0ull;
        // positions of the pivots, highest first
        uint64_t pm = si.pivmask;
        for (int t = r - 1; t >= 0; --t) {
          const int p = 63 - __builtin_clzll(pm);
          pm &= ~(1ull << p);
          const uint64_t v = rdl64s(yv, t);
          if (lane < t && ((er >> p) & 1ull)) yv ^= v;
        }
        if (lane < r) sw.Y[(si.R + lane) * sw.kw + c] = yv;
        // value of the variable at bit position `lane` of word q (0 if not a pivot)
        uint64_t xp = 0ull;
        uint64_t pm2 = si.pivmask;
        int t2 = 0;
        while (pm2) {
          const int p = __builtin_ctzll(pm2);
          pm2 &= pm2 - 1;
          const uint64_t v = rdl64s(yv, t2);
          if (lane == p) xp = v;
          ++t2;
        }
        Xpos[lane] = xp;
      }
      __syncthreads();
      if (tid < 256) {
        const int g = tid >> 4, e = tid & 15;
        uint64_t v = 0ull;
        for (int b = 0; b < 4; ++b)
          if (e & (1 << b)) v ^= Xpos[4 * g + b];
        T[g][e] = v;
      }
      __syncthreads();
      for (int64_t t = tid; t < si.R; t += kSolveThreads) {
        const uint64_t er = w.W[widx(ldw, t, q)];
        uint64_t v = 0ull;
#pragma unroll
        for (int g = 0; g < 16; ++g) v ^= T[g][(er >> (4 * g)) & 15u];
        sw.Y[t * sw.kw + c] ^= v;
      }
      __syncthreads();
    }
  }
}

// X (m x k): variable v = 64q + j takes Y[t] if bit j of word q is pivot t, else 0
__global__ void k_solve_write(DecWork w, gf2_mat X, SolveWork sw, uint64_t *consistent) {
  const int64_t total = X.rows * sw.kw;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t v = e / sw.kw, c = e - v * sw.kw;
    const int q = (int)(v >> 6), j = (int)(v & 63);
    const SubInfo si = w.sub[q];
    uint64_t val = 0ull;
    const uint64_t valid = pad_mask(sw.k, c);
    const uint64_t ok = ~sw.bad[c] & valid;
    if ((si.pivmask >> j) & 1ull) {
      const int64_t t = si.R + __popcll(si.pivmask & ((1ull << j) - 1ull));
      val = sw.Y[t * sw.kw + c] & ok;
    }
    X.data[uidx(X.w, X.ld, v, c)] = val;
  }
  if (blockIdx.x == 0)
    for (int64_t c = threadIdx.x; c < sw.kw; c += blockDim.x) consistent[c] = ~sw.bad[c] & pad_mask(sw.k, c);
}

hipError_t launch_solve(const DecWork &w, const gf2_mat &B, const gf2_mat &X,
                        const SolveWork &sw, uint64_t *consistent, hipStream_t s) {
  int64_t total = w.n * sw.kw;
  int64_t blocks = (total + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_solve_prep, dim3((unsigned)blocks), dim3(256), 0, s, w, B, sw);
  hipLaunchKernelGGL(k_solve_fwd, dim3(1), dim3(kSolveThreads), 0, s, w, sw);
  hipLaunchKernelGGL(k_solve_check, dim3((unsigned)blocks), dim3(256), 0, s, w, sw);
  hipLaunchKernelGGL(k_solve_back, dim3(1), dim3(kSolveThreads), 0, s, w, sw);
  int64_t totx = X.rows * sw.kw;
  int64_t bx = (totx + 255) / 256;
  if (bx < 1) bx = 1;
  if (bx > 65536) bx = 65536;
  hipLaunchKernelGGL(k_solve_write, dim3((unsigned)bx), dim3(256), 0, s, w, X, sw, consistent);
  return hipGetLastError();
}

}  // namespace gf2
