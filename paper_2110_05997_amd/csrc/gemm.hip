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

typedef double sdbl4 __attribute__((ext_vector_type(4)));

// v where ok, else +0.0, by a bit mask: the load of v stays unconditional (a select on a loaded
// value may be turned into a branch around the load, which serialises the loads of a batch).
__device__ __forceinline__ double keep_if(bool ok, double v) {
  const unsigned long long m = ok ? ~0ull : 0ull;
  return __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, v) & m);
}

// C = alpha A B + beta C for row-major A (M x K) and B (K x N), N <= 64, on the FP64 matrix cores
// (tall-skinny products: a subspace block times the Gram, the last mode product of the core
// projection, the uncompression).  A workgroup owns 16 rows and all N columns; wave w takes the
// 4-deep contraction slices w, w + 4, ..., with SK_U slices of loads in flight before their MFMAs;
// the four partial tiles are added in LDS in a fixed order.  Fragments: A[row r16][k kq],
// B[k kq][col r16], result row 4 v + kq, column r16 in acc[v].
constexpr int SK_NT = 256;
constexpr int SK_U = 8;
__global__ __launch_bounds__(SK_NT) void skinny_mfma_kernel(int M, int N, int K, double alpha,
                                                            const double* __restrict__ A, int lda,
                                                            const double* __restrict__ B, long long ldb, double beta,
                                                            double* __restrict__ C, long long ldc) {
  constexpr int NWV = SK_NT / 64;
  __shared__ double part[NWV][16][65];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r16 = lane & 15, kq = lane >> 4;
  const int m0 = blockIdx.x * 16;
  const int nt = (N + 15) >> 4;
  const int row = m0 + r16;
  const bool rok = row < M;
  const double* ar = A + (long long)(rok ? row : 0) * lda;
  sdbl4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = sdbl4{0.0, 0.0, 0.0, 0.0};
  const int nsl = (K + 3) >> 2;
  for (int s0 = w; s0 < nsl; s0 += NWV * SK_U) {
    double a[SK_U], b[SK_U][4];
#pragma unroll
    for (int u = 0; u < SK_U; ++u) {
      const int k = (s0 + NWV * u) * 4 + kq;
      const bool kok = k < K;
      const long long kc = kok ? k : 0;
      a[u] = keep_if(rok && kok, ar[kc]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = t * 16 + r16;
        b[u][t] = keep_if(kok && col < N, B[kc * ldb + (col < N ? col : 0)]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);   // every load of the batch is issued before its MFMAs
#pragma unroll
    for (int u = 0; u < SK_U; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < nt) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u][t], acc[t], 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) part[w][4 * v + kq][t * 16 + r16] = acc[t][v];
  __syncthreads();
  for (int e = threadIdx.x; e < 16 * 64; e += SK_NT) {
    const int r = e >> 6, c = e & 63, gm = m0 + r;
    if (gm < M && c < N) {
      double v = part[0][r][c];
#pragma unroll
      for (int q = 1; q < NWV; ++q) v += part[q][r][c];
      double* cp = C + (long long)gm * ldc + c;
      *cp = (beta == 0.0) ? alpha * v : alpha * v + beta * *cp;
    }
  }
}

// C = alpha A^T B + beta C for A (K x M) and B (K x N), M, N <= 64 (Grams of subspace blocks) on
// the FP64 matrix cores: workgroup (x, y) owns output tile (16 x, 16 y); its four waves take
// interleaved 4-deep slices of the contraction (SK_U in flight) and add their tiles in LDS in a
// fixed order.  Fragments: A^T[m r16][k kq] = A[k][m], B[k kq][n r16].
__global__ __launch_bounds__(SK_NT) void atb_mfma_kernel(int M, int N, int K, double alpha,
                                                         const double* __restrict__ A, int lda,
                                                         const double* __restrict__ B, long long ldb, double beta,
                                                         double* __restrict__ C, long long ldc) {
  constexpr int NWV = SK_NT / 64;
  __shared__ double part[NWV][16][17];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r16 = lane & 15, kq = lane >> 4;
  const int m = blockIdx.x * 16 + r16, n = blockIdx.y * 16 + r16;
  const bool mok = m < M, nok = n < N;
  const int mc = mok ? m : 0, nc = nok ? n : 0;
  sdbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  const int nsl = (K + 3) >> 2;
  for (int s0 = w; s0 < nsl; s0 += NWV * SK_U) {
    double a[SK_U], b[SK_U];
#pragma unroll
    for (int u = 0; u < SK_U; ++u) {
      const int k = (s0 + NWV * u) * 4 + kq;
      const bool kok = k < K;
      const long long kc = kok ? k : 0;
      a[u] = keep_if(kok && mok, A[kc * lda + mc]);
      b[u] = keep_if(kok && nok, B[kc * ldb + nc]);
    }
    __builtin_amdgcn_sched_barrier(0);   // every load of the batch is issued before its MFMAs
#pragma unroll
    for (int u = 0; u < SK_U; u += 2) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u + 1], b[u + 1], acc1, 0, 0, 0);
    }
  }
  const sdbl4 acc = acc0 + acc1;
#pragma unroll
  for (int v = 0; v < 4; ++v) part[w][4 * v + kq][r16] = acc[v];
  __syncthreads();
  if (threadIdx.x < 256) {
    const int r = threadIdx.x >> 4, c = threadIdx.x & 15;
    const int gm = blockIdx.x * 16 + r, gn = blockIdx.y * 16 + c;
    if (gm < M && gn < N) {
      double v = part[0][r][c];
#pragma unroll
      for (int q = 1; q < NWV; ++q) v += part[q][r][c];
      double* cp = C + (long long)gm * ldc + gn;
      *cp = (beta == 0.0) ? alpha * v : alpha * v + beta * *cp;
    }
  }
}

// One thread per output element, for small products where 64x64 tiles would leave the chip idle.
template <class TB>
__global__ void gemm_small_kernel(int M, int N, int K, double alpha, const double* __restrict__ A, int lda,
                                  long long sA, int ta, const TB* __restrict__ B, long long ldb, long long sB,
                                  int tb, double beta, double* __restrict__ C, long long ldc, long long sC,
                                  int tc) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)M * N) return;
  const int m = (int)(e / N), n = (int)(e % N);
  const long long b = blockIdx.y;
  A += b * sA;
  B += b * sB;
  C += b * sC;
  double acc = 0.0;
  if (!ta && !tb) {
    for (int k = 0; k < K; ++k) acc = fma(A[(long long)m * lda + k], loadB(B + (long long)k * ldb + n), acc);
  } else {
    for (int k = 0; k < K; ++k) {
      const double a = ta ? A[(long long)k * lda + m] : A[(long long)m * lda + k];
      const double bv = tb ? loadB(B + (long long)n * ldb + k) : loadB(B + (long long)k * ldb + n);
      acc = fma(a, bv, acc);
    }
  }
  double* c = tc ? C + (long long)n * ldc + m : C + (long long)m * ldc + n;
  *c = (beta == 0.0) ? alpha * acc : alpha * acc + beta * *c;
}

// Mode product along a middle index: Y[a][b][k] = sum_j U[j][b] X[a][j][k] for a < A, b < nb,
// k < K (k contiguous).  The first two factor products of the core projection S = T x1 U1^T x2 U2^T
// x3 U3^T are of this form (a = 1, j = i1, k = (i2, i3); then a = row of the first product, j = i2,
// k = i3).  Lane = k, so every load of X is coalesced and X is read once; U is the same for the
// whole wave and is staged once in LDS (each read a broadcast, off the X loads' wait counter); NB
// accumulators per lane; the four waves split j and are added in a fixed order through LDS.
constexpr int MP_NB = 20;                  // outputs per pass
constexpr size_t MP_LDS = 64 * 1024;   // LDS for the staged rows of U and the reduction: beyond it (J > 217 at
                                       // 20 outputs) one 4-wave workgroup per CU is too little to hide the
                                       // serial j loop; measured slower than the tiled GEMM at J = 600

template <class TX, int NB>
__global__ __launch_bounds__(256) void mprod_kernel(const TX* __restrict__ X, int J, long long K,
                                                    const double* __restrict__ U, int ldu, int b0, int nb,
                                                    double* __restrict__ Y, long long ldy) {
  __shared__ double red[3][NB][64];
  extern __shared__ double us[];   // [J][NB]: columns b0 .. b0 + NB - 1 of U, zero past nb
  for (int e = threadIdx.x; e < J * NB; e += 256) {
    const int jj = e / NB, b = e - jj * NB;
    us[e] = b0 + b < nb ? U[(long long)jj * ldu + b0 + b] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long k = (long long)blockIdx.x * 64 + lane;
  const long long a = blockIdx.y;
  const TX* x = X + a * (long long)J * K + (k < K ? k : 0);
  const int jb = (int)((long long)J * w / 4), je = (int)((long long)J * (w + 1) / 4);
  double acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = 0.0;
  // X values of the next four j in flight (ring, refilled in range: a load past je reloads je - 1)
  double xr[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) xr[u] = loadB(x + (long long)min(jb + u, je - 1 < jb ? jb : je - 1) * K);
  // branch-free steps (a step past je adds 0 times row je - 1): a branch per step would make the
  // wait-count bookkeeping drain the ring at every join
  for (int j = jb; j < je; j += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool ok = j + u < je;
      const double xv = ok ? xr[u] : 0.0;
      xr[u] = loadB(x + (long long)min(j + u + 4, je - 1) * K);
      const double* ur = us + min(j + u, je - 1) * NB;
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = fma(ur[b], xv, acc[b]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if (w > 0) {
#pragma unroll
    for (int b = 0; b < NB; ++b) red[w - 1][b][lane] = acc[b];
  }
  __syncthreads();
  if (w == 0 && k < K) {
    double* y = Y + a * (long long)nb * ldy + k;
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (b0 + b < nb) y[(long long)(b0 + b) * ldy] = ((acc[b] + red[0][b][lane]) + red[1][b][lane]) + red[2][b][lane];
  }
}

template <class TX>
void mprod_launch(const TX* X, int A, int J, long long K, const double* U, int nb, double* Y, hipStream_t s) {
  const dim3 grid((unsigned)((K + 63) / 64), (unsigned)A);
  for (int b0 = 0; b0 < nb; b0 += MP_NB) {
    const int left = nb - b0;
    const int w = left <= 8 ? 8 : left <= 12 ? 12 : left <= 16 ? 16 : 20;
    const size_t lds = (size_t)J * w * sizeof(double);
    if (w == 8) hipLaunchKernelGGL((mprod_kernel<TX, 8>), grid, dim3(256), lds, s, X, J, K, U, nb, b0, nb, Y, K);
    else if (w == 12) hipLaunchKernelGGL((mprod_kernel<TX, 12>), grid, dim3(256), lds, s, X, J, K, U, nb, b0, nb, Y, K);
    else if (w == 16) hipLaunchKernelGGL((mprod_kernel<TX, 16>), grid, dim3(256), lds, s, X, J, K, U, nb, b0, nb, Y, K);
    else hipLaunchKernelGGL((mprod_kernel<TX, 20>), grid, dim3(256), lds, s, X, J, K, U, nb, b0, nb, Y, K);
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
  const long long mn = (long long)M * N;
  if (bdtype == CPD_F64 && batch == 1 && !tc && !tb && N <= 64) {
    if (ta && M <= 64 && K >= 128) {
      hipLaunchKernelGGL(atb_mfma_kernel, dim3((M + 15) / 16, (N + 15) / 16), dim3(SK_NT), 0, s, M, N, K, alpha, A,
                         lda, (const double*)B, ldb, beta, C, ldc);
      CPD_LAUNCH_CHECK();
      return CPD_OK;
    }
    if (!ta && M <= 0x7fffffff - 15) {
      hipLaunchKernelGGL(skinny_mfma_kernel, dim3((unsigned)((M + 15) / 16)), dim3(SK_NT), 0, s, M, N, K, alpha, A,
                         lda, (const double*)B, ldb, beta, C, ldc);
      CPD_LAUNCH_CHECK();
      return CPD_OK;
    }
  }
  // one thread per output element while the whole batch's output is small or the contraction
  // short; a large batch of long contractions (e.g. the second mode product of a 600^3 core
  // projection: 50 products of 50 x 600 x 600) goes to the LDS-tiled kernel
  const bool big_batch = (long long)mn * batch >= (1LL << 20) && K >= 256;
  if (mn <= 65536 && K <= 4096 && batch <= 65535 && (mn < 16384 || K <= 1024) && !big_batch) {
    dim3 g2((unsigned)((mn + 255) / 256), batch);
    switch (bdtype) {
      case CPD_F64:
        hipLaunchKernelGGL(gemm_small_kernel<double>, g2, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, (int)ta,
                           (const double*)B, ldb, sB, (int)tb, beta, C, ldc, sC, (int)tc);
        break;
      case CPD_F32:
        hipLaunchKernelGGL(gemm_small_kernel<float>, g2, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, (int)ta,
                           (const float*)B, ldb, sB, (int)tb, beta, C, ldc, sC, (int)tc);
        break;
      case CPD_BF16:
        hipLaunchKernelGGL(gemm_small_kernel<uint16_t>, g2, dim3(256), 0, s, M, N, K, alpha, A, lda, sA,
                           (int)ta, (const uint16_t*)B, ldb, sB, (int)tb, beta, C, ldc, sC, (int)tc);
        break;
      default:
        set_error("gemm_f64: bad dtype %d", bdtype);
        return CPD_E_INVALID;
    }
    CPD_LAUNCH_CHECK();
    return CPD_OK;
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

// Mode product Y[b] (r x N) = U^T (r x K) X[b] (K x N) for a tall-skinny U (K x r, r <= 64) and
// row-major X (the unfolding whose contraction index is the slowest: the first mode product of the
// core projection, ch.2 multilinear multiplication): FP64 matrix cores, X promoted exactly.  A wave
// owns 16 columns and all r rows (up to four 16-row tiles); the contraction advances four rows of X
// per step, U fragments come from L1/L2 and each element of X is read once.
typedef double pdbl4 __attribute__((ext_vector_type(4)));

template <class TB>
__device__ __forceinline__ double tod(TB x) { return (double)x; }
template <>
__device__ __forceinline__ double tod<uint16_t>(uint16_t x) { return bf16_bits_to_f64(x); }

template <class TB>
__global__ __launch_bounds__(256) void proj_mfma_kernel(const TB* __restrict__ X, int K, long long N, long long sX,
                                                        const double* __restrict__ U, int r,
                                                        double* __restrict__ Y, long long sY) {
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4, w = threadIdx.x >> 6;
  const long long n0 = ((long long)blockIdx.x * 4 + w) * 16;
  if (n0 >= N) return;
  X += (long long)blockIdx.y * sX;
  Y += (long long)blockIdx.y * sY;
  const long long n = n0 + r16;
  const bool nok = n < N;
  const long long nc = nok ? n : N - 1;
  const int mt = (r + 15) / 16;
  pdbl4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = pdbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + kq;
    const bool kok = k < K;
    const int kc = kok ? k : K - 1;
    const double xv = loadB(X + (long long)kc * N + nc);
    const double b = (kok && nok) ? xv : 0.0;   // B[k][n]
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < mt) {
        const int m = t * 16 + r16;
        const double uv = U[(long long)kc * r + (m < r ? m : r - 1)];
        const double a = (kok && m < r) ? uv : 0.0;   // A[m][k] = U[k][m]
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
      }
    }
  }
  // acc[t][v] = Y[t 16 + 4 v + kq][n0 + r16]
  if (!nok) return;
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (t < mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = t * 16 + 4 * v + kq;
        if (m < r) Y[(long long)m * N + n] = acc[t][v];
      }
}

// The same product for long rows: a workgroup owns 256 columns and all r <= 64 rows of Y and
// streams X through LDS sixteen rows at a time (each row of a stage one contiguous 16-byte-vector
// run, so X is read in long bursts), U^T alongside; four waves, each 64 x 64 of the tile as sixteen
// 16x16 FP64 matrix-core accumulators.  Needs N and the batch stride to be multiples of the
// vector width and X 16-byte aligned.
constexpr int PB_N = 256, PB_KC = 16, PB_LD = PB_KC + 1;

template <class TB>
__global__ __launch_bounds__(256) void proj_big_kernel(const TB* __restrict__ X, int K, long long N, long long sX,
                                                       const double* __restrict__ U, int r,
                                                       double* __restrict__ Y, long long sY) {
  constexpr int VW = 16 / (int)sizeof(TB);
  constexpr int NVX = PB_KC * PB_N / VW / 256;   // X vectors per thread and stage
  typedef TB vec_t __attribute__((ext_vector_type(VW)));
  __shared__ double Xm[64][PB_LD];      // U^T: row m, stage index k
  __shared__ double Xn[PB_N][PB_LD];    // X^T: column n, stage index k
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r16 = lane & 15, kq = lane >> 4;
  const long long n0 = (long long)blockIdx.x * PB_N;
  X += (long long)blockIdx.y * sX;
  Y += (long long)blockIdx.y * sY;
  const int wn = w * 64;
  pdbl4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = pdbl4{0.0, 0.0, 0.0, 0.0};
  const int mt = (r + 15) / 16;
  vec_t rx[NVX];
  double ru[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int v = 0; v < NVX; ++v) {
      const int e = tid + v * 256;
      const int kk = e / (PB_N / VW), nq = (e % (PB_N / VW)) * VW;
      const int k = k0 + kk;
      const long long n = n0 + nq;
      const bool ok = k < K && n < N;
      rx[v] = *(const vec_t*)(X + (ok ? (long long)k * N + n : 0ll));
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int e = tid + v * 256, kk = e / 64, m = e % 64, k = k0 + kk;
      const bool ok = k < K && m < r;
      ru[v] = U[ok ? (long long)k * r + m : 0ll];
    }
  };
  auto store = [&](int k0) {
#pragma unroll
    for (int v = 0; v < NVX; ++v) {
      const int e = tid + v * 256;
      const int kk = e / (PB_N / VW), nq = (e % (PB_N / VW)) * VW;
      const bool okk = k0 + kk < K;
#pragma unroll
      for (int u = 0; u < VW; ++u) Xn[nq + u][kk] = (okk && n0 + nq + u < N) ? tod<TB>(rx[v][u]) : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int e = tid + v * 256, kk = e / 64, m = e % 64;
      Xm[m][kk] = (k0 + kk < K && m < r) ? ru[v] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += PB_KC) {
    store(k0);
    __syncthreads();
    if (k0 + PB_KC < K) fetch(k0 + PB_KC);
#pragma unroll
    for (int kk = 0; kk < PB_KC; kk += 4) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = Xm[16 * i + r16][kk + kq];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Xn[wn + 16 * j + r16][kk + kq];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < mt)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // acc[i][j][v] = Y[16 i + 4 v + kq][n0 + wn + 16 j + r16]
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (i < mt)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * i + 4 * v + kq;
          const long long n = n0 + wn + 16 * j + r16;
          if (m < r && n < N) Y[(long long)m * N + n] = acc[i][j][v];
        }
}


// The same product with the operands straight from memory into registers: no LDS and no barrier.
// A workgroup owns all r <= 64 rows of Y and 256 columns, a wave 64 of them.  Lane (p, q) loads
// four consecutive columns 4p .. 4p + 3 of row k of X in one vector load; element b of the four
// feeds the MFMA of column block b, which therefore holds the columns 4p + b (p = 0..15) of the
// wave's 64, and the lane ends up with four consecutive columns of Y per accumulator row, written
// as one 32-byte store.  Within a stage of 16 contraction indices, lane group q holds index
// k0 + 4t + q at MFMA step t in both operands; U^T's fragments are loaded per step (U is small and
// stays in the caches).  The next stage's loads are in flight in a second register set while the
// current one is multiplied; full stages carry no masks.
template <class TB>
__device__ __forceinline__ void load4(const TB* p, TB (&v)[4]) {
  typedef TB v4 __attribute__((ext_vector_type(4)));
  const v4 x = *(const v4*)p;
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = x[u];
}

template <class TB>
constexpr int pd_waves() { return sizeof(TB) <= 4 ? 2 : 1; }

// MT4: r > 48, all four row blocks of U^T in use (no per-block test)
template <class TB, bool MT4>
__global__ __launch_bounds__(256, (pd_waves<TB>())) void proj_direct_kernel(const TB* __restrict__ X, int K, long long N,
                                                                            long long sX, const double* __restrict__ U,
                                                                            int r, double* __restrict__ Y, long long sY) {
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int p16 = lane & 15, q = lane >> 4;
  X += (long long)blockIdx.y * sX;
  Y += (long long)blockIdx.y * sY;
  const long long nc = (long long)blockIdx.x * PB_N + w * 64 + 4 * p16;   // this lane's first column
  const long long ncl = nc < N ? nc : N - 4;                             // clamped for the loads
  const int mt = MT4 ? 4 : (r + 15) / 16;
  pdbl4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[i][b] = pdbl4{0.0, 0.0, 0.0, 0.0};
  // one stage at k0: xb[t][b] = X[k0 + 4t + q][nc + b], ua[t][i] = U[k0 + 4t + q][16 i + p16]
  // (indices clamped into the matrices; with `mask`, values past K or r are zero)
  auto load = [&](TB (&xb)[4][4], double (&ua)[4][4], int k0, bool mask) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + 4 * t + q, kc = k < K ? k : K - 1;
      load4<TB>(X + (long long)kc * N + ncl, xb[t]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = 16 * i + p16;
        const double u = U[(long long)kc * r + (m < r ? m : r - 1)];
        ua[t][i] = (mask && (k >= K || m >= r)) ? 0.0 : u;
      }
      if (mask && k >= K) {
#pragma unroll
        for (int b = 0; b < 4; ++b) xb[t][b] = (TB)0;
      }
    }
  };
  auto stage = [&](const TB (&xb)[4][4], const double (&ua)[4][4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      double bv[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = tod<TB>(xb[t][b]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < mt)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[i][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[t][i], bv[b], acc[i][b], 0, 0, 0);
    }
  };
  // rows m >= r of U only feed rows of Y that are not written, so full stages need no masks
  TB x0[4][4], x1[4][4];
  double u0[4][4], u1[4][4];
  const int nst = K / PB_KC, kfull = nst * PB_KC;
  if (nst > 0) load(x0, u0, 0, false);
  int st = 0;
  for (; st + 2 <= nst; st += 2) {
    const int k0 = st * PB_KC;
    load(x1, u1, k0 + PB_KC, false);
    __builtin_amdgcn_sched_barrier(0);
    stage(x0, u0);
    __builtin_amdgcn_sched_barrier(0);
    load(x0, u0, k0 + 2 * PB_KC, false);   // clamped and unused when the last full stage was st + 1
    __builtin_amdgcn_sched_barrier(0);
    stage(x1, u1);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (st < nst) stage(x0, u0);
  if (kfull < K) {
    load(x1, u1, kfull, true);
    stage(x1, u1);
  }
  // acc[i][b][v] = Y[16 i + 4 v + q][nc + b]
  if (nc < N) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i < mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * i + 4 * v + q;
          if (m < r) {
            pdbl4 o;
#pragma unroll
            for (int b = 0; b < 4; ++b) o[b] = acc[i][b][v];
            *(pdbl4*)(Y + (long long)m * N + nc) = o;
          }
        }
  }
}
}  // namespace cpd

namespace cpd {

// U rows staged in LDS (plus the reduction buffer of up to 30 KB) must fit MP_LDS
bool mode_product_mid_fits(int J, int nb) {
  const int w = nb <= 8 ? 8 : nb <= 12 ? 12 : nb <= 16 ? 16 : MP_NB;
  return J >= 1 && (size_t)J * w * sizeof(double) + 3 * MP_NB * 64 * sizeof(double) <= MP_LDS;
}

cpd_status mode_product_mid(const void* X, int xdtype, int A, int J, long long K, const double* U, int nb,
                            double* Y, hipStream_t s) {
  if (A <= 0 || nb <= 0 || K <= 0) return CPD_OK;
  if (!mode_product_mid_fits(J, nb)) {
    set_error("mode_product_mid: %d rows of U exceed the staging buffer", J);
    return CPD_E_UNSUPPORTED;
  }
  if (X == nullptr || U == nullptr || Y == nullptr || J < 1 || A > 65535 || (K + 63) / 64 > 0x7fffffffLL) {
    set_error("mode_product_mid: bad arguments");
    return CPD_E_INVALID;
  }
  switch (xdtype) {
    case CPD_F64: mprod_launch<double>((const double*)X, A, J, K, U, nb, Y, s); break;
    case CPD_F32: mprod_launch<float>((const float*)X, A, J, K, U, nb, Y, s); break;
    case CPD_BF16: mprod_launch<uint16_t>((const uint16_t*)X, A, J, K, U, nb, Y, s); break;
    default: set_error("mode_product_mid: bad dtype %d", xdtype); return CPD_E_INVALID;
  }
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

cpd_status project_mfma(const void* X, int xdtype, int K, long long N, int batch, long long sX, const double* U,
                        int r, double* Y, long long sY, hipStream_t s) {
  if (K <= 0 || N <= 0 || batch <= 0) return CPD_OK;
  if (X == nullptr || U == nullptr || Y == nullptr || r < 1 || r > 64 || batch > 65535 ||
      (N + 63) / 64 > 0x7fffffffLL || (xdtype != CPD_F64 && xdtype != CPD_F32 && xdtype != CPD_BF16)) {
    set_error("project_mfma: bad arguments");
    return CPD_E_INVALID;
  }
  const int vw = xdtype == CPD_F64 ? 2 : (xdtype == CPD_F32 ? 4 : 8);
  const size_t esz = xdtype == CPD_F64 ? 8 : (xdtype == CPD_F32 ? 4 : 2);
  if (xdtype != CPD_BF16 && N % 4 == 0 && sX % 4 == 0 && sY % 4 == 0 && ((uintptr_t)X & (4 * esz - 1)) == 0 &&
      ((uintptr_t)Y & 31) == 0 && (N + PB_N - 1) / PB_N <= 0x7fffffffLL) {
    // four consecutive columns per lane: rows of X and Y aligned to four elements
    const dim3 gb((unsigned)((N + PB_N - 1) / PB_N), (unsigned)batch);
    if (xdtype == CPD_F64) {
      auto kd = r > 48 ? proj_direct_kernel<double, true> : proj_direct_kernel<double, false>;
      hipLaunchKernelGGL(kd, gb, dim3(256), 0, s, (const double*)X, K, N, sX, U, r, Y, sY);
    } else {
      auto kf = r > 48 ? proj_direct_kernel<float, true> : proj_direct_kernel<float, false>;
      hipLaunchKernelGGL(kf, gb, dim3(256), 0, s, (const float*)X, K, N, sX, U, r, Y, sY);
    }
    CPD_LAUNCH_CHECK();
    return CPD_OK;
  }
  if (N % vw == 0 && sX % vw == 0 && ((uintptr_t)X & 15) == 0 && (N + PB_N - 1) / PB_N <= 0x7fffffffLL) {
    const dim3 gb((unsigned)((N + PB_N - 1) / PB_N), (unsigned)batch);
    switch (xdtype) {
      case CPD_F64:
        hipLaunchKernelGGL(proj_big_kernel<double>, gb, dim3(256), 0, s, (const double*)X, K, N, sX, U, r, Y, sY);
        break;
      case CPD_F32:
        hipLaunchKernelGGL(proj_big_kernel<float>, gb, dim3(256), 0, s, (const float*)X, K, N, sX, U, r, Y, sY);
        break;
      default:
        hipLaunchKernelGGL(proj_big_kernel<uint16_t>, gb, dim3(256), 0, s, (const uint16_t*)X, K, N, sX, U, r, Y,
                           sY);
        break;
    }
    CPD_LAUNCH_CHECK();
    return CPD_OK;
  }
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)batch);
  switch (xdtype) {
    case CPD_F64:
      hipLaunchKernelGGL(proj_mfma_kernel<double>, grid, dim3(256), 0, s, (const double*)X, K, N, sX, U, r, Y, sY);
      break;
    case CPD_F32:
      hipLaunchKernelGGL(proj_mfma_kernel<float>, grid, dim3(256), 0, s, (const float*)X, K, N, sX, U, r, Y, sY);
      break;
    case CPD_BF16:
      hipLaunchKernelGGL(proj_mfma_kernel<uint16_t>, grid, dim3(256), 0, s, (const uint16_t*)X, K, N, sX, U, r, Y,
                         sY);
      break;
    default:
      set_error("project_mfma: bad dtype %d", xdtype);
      return CPD_E_INVALID;
  }
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

}  // namespace cpd
