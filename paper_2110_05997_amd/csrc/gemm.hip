// Batched FP64 GEMM with LDS tiling (vector FMA).  Serves the small and skinny products of the
// path: the core projection S = T x1 U1^T x2 U2^T x3 U3^T (ch.2 multilinear multiplication), the
// subspace iteration of the eigensolver, and uncompression W~ = U W (ch.4 "Uncompression").
#include "common.h"

namespace cpd {
namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

template <class TB>
__device__ __forceinline__ double loadB(const TB* p) { return (double)*p; }
template <>
__device__ __forceinline__ double loadB<uint16_t>(const uint16_t* p) { return bf16_bits_to_f64(*p); }

template <class TB>
__global__ __launch_bounds__(NT) void gemm_kernel(int M, int N, int K, double alpha,
                                                  const double* __restrict__ A, int lda,
                                                  long long sA, int ta,
                                                  const TB* __restrict__ B, long long ldb,
                                                  long long sB, int tb, double beta,
                                                  double* __restrict__ C, long long ldc,
                                                  long long sC, int tc) {
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const long long b = blockIdx.z;
  A += b * sA;
  B += b * sB;
  C += b * sC;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int t = 0; t < (BM * BK) / NT; ++t) {
      const int e = tid + t * NT;
      int m, k;
      if (ta) { m = e % BM; k = e / BM; } else { k = e % BK; m = e / BK; }
      const int gm = m0 + m, gk = k0 + k;
      double v = 0.0;
      if (gm < M && gk < K) v = ta ? A[(long long)gk * lda + gm] : A[(long long)gm * lda + gk];
      As[k][m] = v;
    }
#pragma unroll
    for (int t = 0; t < (BN * BK) / NT; ++t) {
      const int e = tid + t * NT;
      int n, k;
      if (tb) { k = e % BK; n = e / BK; } else { n = e % BN; k = e / BN; }
      const int gn = n0 + n, gk = k0 + k;
      double v = 0.0;
      if (gn < N && gk < K) v = tb ? loadB(B + (long long)gn * ldb + gk) : loadB(B + (long long)gk * ldb + gn);
      Bs[k][n] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      double a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + ty + 16 * i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + tx + 16 * j;
      if (gn >= N) continue;
      double* c = tc ? C + (long long)gn * ldc + gm : C + (long long)gm * ldc + gn;
      *c = (beta == 0.0) ? alpha * acc[i][j] : alpha * acc[i][j] + beta * *c;
    }
  }
}

}  // namespace

cpd_status gemm_f64(int M, int N, int K, double alpha, const double* A, int lda, long long sA,
                    bool ta, const void* B, int bdtype, long long ldb, long long sB, bool tb,
                    double beta, double* C, long long ldc, long long sC, int batch,
                    hipStream_t s, bool tc) {
  if (M <= 0 || N <= 0 || batch <= 0) return CPD_OK;
  if (K < 0 || A == nullptr || B == nullptr || C == nullptr) {
    set_error("gemm_f64: bad arguments");
    return CPD_E_INVALID;
  }
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, batch);
  if (grid.y > 65535 || grid.z > 65535) {
    set_error("gemm_f64: grid too large (M=%d batch=%d)", M, batch);
    return CPD_E_UNSUPPORTED;
  }
  switch (bdtype) {
    case CPD_F64:
      hipLaunchKernelGGL(gemm_kernel<double>, grid, dim3(NT), 0, s, M, N, K, alpha, A, lda, sA,
                         (int)ta, (const double*)B, ldb, sB, (int)tb, beta, C, ldc, sC, (int)tc);
      break;
    case CPD_F32:
      hipLaunchKernelGGL(gemm_kernel<float>, grid, dim3(NT), 0, s, M, N, K, alpha, A, lda, sA,
                         (int)ta, (const float*)B, ldb, sB, (int)tb, beta, C, ldc, sC, (int)tc);
      break;
    case CPD_BF16:
      hipLaunchKernelGGL(gemm_kernel<uint16_t>, grid, dim3(NT), 0, s, M, N, K, alpha, A, lda, sA,
                         (int)ta, (const uint16_t*)B, ldb, sB, (int)tb, beta, C, ldc, sC, (int)tc);
      break;
    default:
      set_error("gemm_f64: bad dtype %d", bdtype);
      return CPD_E_INVALID;
  }
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

}  // namespace cpd
