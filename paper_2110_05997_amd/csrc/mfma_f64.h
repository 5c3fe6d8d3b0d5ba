// FP64 matrix-core tile product shared by the single-workgroup kernels (dGN, eigensolver).
#pragma once
#include "common.h"

namespace cpd {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// One 16x16 output tile C[m0.., n0..] = sum_k A(m, k) B(k, n) on v_mfma_f64_16x16x4f64.
// Lane layout: A fragment A[lane%16][lane/16], B fragment B[lane/16][lane%16], result
// D[4v + lane/16][lane%16] in acc[v].  fa / fb return 0 outside the operands.
template <class FA, class FB>
__device__ __forceinline__ dbl4 mfma_tile(int m0, int n0, int K, FA fa, FB fb) {
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  // fragments of four k-steps are loaded before their MFMAs, which alternate between two
  // accumulators, so LDS latency and the MFMA dependency chain overlap
  for (int k0 = 0; k0 < K; k0 += 16) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * u + kq;
      a[u] = fa(m0 + r16, k);
      b[u] = fb(k, n0 + r16);
    }
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], b[2], acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], b[3], acc1, 0, 0, 0);
  }
  return acc0 + acc1;
}

// The same tile product for operands in global memory: every fragment of a 64-deep slice of the
// contraction is loaded before its 16 MFMAs, so a slice costs one memory latency instead of four.
// fa / fb must return 0 for k >= K (the slice is padded to 64).
template <class FA, class FB>
__device__ __forceinline__ dbl4 mfma_tile_wide(int m0, int n0, int K, FA fa, FB fb) {
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 64) {
    double a[16], b[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = k0 + 4 * u + kq;
      a[u] = fa(m0 + r16, k);
      b[u] = fb(k, n0 + r16);
    }
#pragma unroll
    for (int u = 0; u < 16; u += 2) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u + 1], b[u + 1], acc1, 0, 0, 0);
    }
  }
  return acc0 + acc1;
}

__device__ __forceinline__ int tiles16(int n) { return (n + 15) >> 4; }

}  // namespace
}  // namespace cpd
