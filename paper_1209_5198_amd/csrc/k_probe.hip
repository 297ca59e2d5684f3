// k_probe.hip -- microbenchmarks of the MI355X units the kernels here lean on,
// so that measured ceilings can be reported beside the nominal ones:
//   0  HBM read (16-byte loads, grid-stride)
//   1  HBM copy (16-byte loads and stores; bytes counted once each way)
//   2  32-bit VALU bitwise throughput (v_xor_b32, eight independent chains)
//   3  LDS 16-byte reads in the conflict-free pattern of the product kernels
//      (every wave reads 1 KB of consecutive bytes per instruction)
//   4  matrix cores, int8 (v_mfma_i32_32x32x32_i8)
//   5  matrix cores, fp4 (v_mfma_scale_f32_32x32x64_f8f6f4 with e2m1 operands
//      and unit scales) -- the contraction a GF(2) product could use instead of
//      Four-Russians tables: 0/1 operands are exact and so are the fp32 sums.
// Every kernel keeps its results live through a store behind a test on the
// data that does not hold, so nothing is optimised away and nothing is written.
#include "gf2_internal.h"

namespace gf2 {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
constexpr uint32_t kNever = 0x9E3779B9u;
constexpr int kProbeNT = 256;

// Four 16-byte loads in flight per thread: vector i + j * stride, j < 4.
__global__ __launch_bounds__(kProbeNT) void k_probe_read(const uint4 *src, size_t n16, uint32_t *sink) {
  uint32_t acc = 0u;
  const size_t stride = (size_t)gridDim.x * kProbeNT;
  for (size_t i = (size_t)blockIdx.x * kProbeNT + threadIdx.x; i < n16; i += 4 * stride) {
    uint4 v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = i + j * stride < n16 ? src[i + j * stride] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int j = 0; j < 4; ++j) acc ^= __builtin_amdgcn_bitop3_b32(v[j].x, v[j].y, v[j].z, 0x96) ^ v[j].w;
  }
  if (acc == kNever) sink[0] = acc;
}

__global__ __launch_bounds__(kProbeNT) void k_probe_copy(const uint4 *src, uint4 *dst, size_t n16) {
  const size_t stride = (size_t)gridDim.x * kProbeNT;
  for (size_t i = (size_t)blockIdx.x * kProbeNT + threadIdx.x; i < n16; i += 4 * stride) {
    uint4 v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (i + j * stride < n16) v[j] = src[i + j * stride];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (i + j * stride < n16) dst[i + j * stride] = v[j];
  }
}

// 128 v_xor_b32 per thread and iteration; each instruction's inputs were
// written at least seven instructions earlier.
__global__ __launch_bounds__(kProbeNT) void k_probe_valu(uint32_t seed, int iters, uint32_t *sink) {
  uint32_t a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = (seed * (2u * j + 1u)) ^ threadIdx.x;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 16; ++r)
#pragma unroll
      for (int j = 0; j < 8; ++j) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[j]) : "v"(a[(j + 1) & 7]));
  }
  uint32_t x = 0u;
#pragma unroll
  for (int j = 0; j < 8; ++j) x ^= a[j];
  if (x == kNever) sink[0] = x;
}

// 32 KB of LDS per workgroup (four resident per CU); eight 16-byte reads per
// thread and iteration, two reads folded per three-input XOR.
__global__ __launch_bounds__(kProbeNT) void k_probe_lds(int iters, uint32_t *sink) {
  __shared__ uint4 buf[2048];
  for (int i = threadIdx.x; i < 2048; i += kProbeNT) buf[i] = make_uint4(i, 3u * i, 5u * i, 7u * i);
  __syncthreads();
  const int base = (int)threadIdx.x;  // wave w reads entries [64 w, 64 w + 64) of each 256-entry row
  uint32_t x = 0u, y = 0u, z = 0u, w = 0u;
  for (int i = 0; i < iters; ++i) {
    const int rot = 256 * (i & 7);
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
      const uint4 p = buf[(base + 256 * j + rot) & 2047];
      const uint4 q = buf[(base + 256 * (j + 1) + rot) & 2047];
      x = __builtin_amdgcn_bitop3_b32(x, p.x, q.x, 0x96);
      y = __builtin_amdgcn_bitop3_b32(y, p.y, q.y, 0x96);
      z = __builtin_amdgcn_bitop3_b32(z, p.z, q.z, 0x96);
      w = __builtin_amdgcn_bitop3_b32(w, p.w, q.w, 0x96);
    }
  }
  if ((x ^ y ^ z ^ w) == kNever) sink[0] = x;
}

// Four independent accumulator chains per wave.
__global__ __launch_bounds__(kProbeNT) void k_probe_mfma_i8(int iters, uint32_t *sink) {
  const int t = (int)threadIdx.x;
  const v4i a = {t, t + 1, t + 2, t + 3}, b = {t ^ 5, t ^ 6, t ^ 7, t ^ 9};
  v16i c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c3, 0, 0, 0);
  }
  int s = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) s ^= c0[j] ^ c1[j] ^ c2[j] ^ c3[j];
  if ((uint32_t)s == kNever) sink[0] = (uint32_t)s;
}

// e2m1 operands (format code 4 for both), scale exponents 127 (= 1.0).
__global__ __launch_bounds__(kProbeNT) void k_probe_mfma_fp4(int iters, uint32_t *sink) {
  const int t = (int)threadIdx.x;
  const v8i a = {t & 0x22222222, 0x22220000, 0x00002222, 0x20202020, 0, 0, 0, 0};
  const v8i b = {0x02020202, t & 0x22222222, 0x22002200, 0x00220022, 0, 0, 0, 0};
  v16f c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c0, 4, 4, 0, 127, 0, 127);
    c1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c1, 4, 4, 0, 127, 0, 127);
    c2 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c2, 4, 4, 0, 127, 0, 127);
    c3 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c3, 4, 4, 0, 127, 0, 127);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 16; ++j) s += c0[j] + c1[j] + c2[j] + c3[j];
  if (s == -1.0f) sink[0] = kNever;
}

}  // namespace

// Launch probe `kind` once; *work receives its bytes (kinds 0, 1, 3), 32-bit
// operations (2) or multiply-accumulates (4, 5).  buf holds `bytes` bytes for
// kinds 0 and 1; sink is a device word that is never written in practice.
hipError_t launch_probe(int kind, void *buf, size_t bytes, int iters, int ncu, uint32_t *sink, hipStream_t s,
                        double *work) {
  const int grid8 = 8 * ncu, grid4 = 4 * ncu;
  const double waves4 = (double)grid4 * (kProbeNT / 64);
  switch (kind) {
    case 0: {
      const size_t n16 = bytes / 16;
      hipLaunchKernelGGL(k_probe_read, dim3(grid8), dim3(kProbeNT), 0, s, (const uint4 *)buf, n16, sink);
      *work = (double)n16 * 16.0;
      break;
    }
    case 1: {
      const size_t n16 = bytes / 32;
      const uint4 *src = (const uint4 *)buf;
      hipLaunchKernelGGL(k_probe_copy, dim3(grid8), dim3(kProbeNT), 0, s, src, (uint4 *)buf + n16, n16);
      *work = (double)n16 * 32.0;
      break;
    }
    case 2:
      hipLaunchKernelGGL(k_probe_valu, dim3(grid8), dim3(kProbeNT), 0, s, 0x2545F491u, iters, sink);
      *work = (double)grid8 * kProbeNT * (double)iters * 128.0;
      break;
    case 3:
      hipLaunchKernelGGL(k_probe_lds, dim3(grid8), dim3(kProbeNT), 0, s, iters, sink);
      *work = (double)grid8 * kProbeNT * (double)iters * 8.0 * 16.0;
      break;
    case 4:
      hipLaunchKernelGGL(k_probe_mfma_i8, dim3(grid4), dim3(kProbeNT), 0, s, iters, sink);
      *work = waves4 * (double)iters * 4.0 * 32.0 * 32.0 * 32.0;
      break;
    case 5:
      hipLaunchKernelGGL(k_probe_mfma_fp4, dim3(grid4), dim3(kProbeNT), 0, s, iters, sink);
      *work = waves4 * (double)iters * 4.0 * 32.0 * 32.0 * 64.0;
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gf2
