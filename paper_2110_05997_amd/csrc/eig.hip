// Leading eigenpairs of the symmetric unfolding Gram G_l = T_(l) T_(l)^T.  Its eigenvectors are
// the mode-l left singular vectors and sigma = sqrt(lambda) (App. B lemma relating the SVD of M to
// the eigendecomposition of M M^T); only the P_l = min(I_l, R) leading ones are needed (ch.4
// Alg. Compression, truncated SVD).
//
//  n <= 64 : cyclic Jacobi with the round-robin parallel ordering, the whole matrix in LDS of one
//            workgroup (exact to rounding, no spectral-gap assumption).
//  n  > 64 : subspace iteration on k = min(n, P + max(4, P/8), 64) vectors (four power steps,
//            then Rayleigh-Ritz every step)
//            (Jacobi on the k x k projection), stopped when every wanted Ritz pair has residual
//            ||G u - theta u|| <= 1e-13 theta_1 (at most 200 iterations).
// Eigenvectors are signed so that each one's largest-magnitude entry is positive (ties: lowest
// index), the convention the oracle applies to its singular vectors.
#include "common.h"
#include "jacobi.h"
#include "mfma_f64.h"

#include <string.h>

#include <vector>

namespace cpd {
namespace {

// Jacobi eigendecomposition of an n x n symmetric matrix (row-major, leading dim lda, n <= 64).
// Outputs: lam[n] descending, Vout[n*n] row-major with eigenvector j in column j (ldv = n).
__global__ __launch_bounds__(JNT) void jacobi_kernel(const double* __restrict__ Ag, int n, int lda,
                                                     double* __restrict__ lam,
                                                     double* __restrict__ Vout) {
  __shared__ JacobiLds L;
  jacobi_block<JNT, true>(L, Ag, n, lda, lam, Vout);
}

// The direct path for up to three problems (the modes of one tensor, n <= 64), one workgroup
// each: Jacobi eigendecomposition, the leading P eigenvalues, and the first P eigenvectors signed
// as sign_columns_kernel signs them (one wave per column).
struct DirectArgs {
  const double* G;
  int n, P;
  double *V, *lall, *U, *lam;
};

// The problem descriptors of a multi-problem launch live in a small workspace array (one slot per
// problem); put_args_kernel writes them in stream order from three separate by-value arguments
// (fixed indices only), and each workgroup of the solver then reads slot blockIdx.x from global
// memory.
template <class A>
__global__ void put_args_kernel(const A a0, const A a1, const A a2, int nprob, A* __restrict__ out) {
  if (threadIdx.x == 0 && nprob > 0) out[0] = a0;
  if (threadIdx.x == 1 && nprob > 1) out[1] = a1;
  if (threadIdx.x == 2 && nprob > 2) out[2] = a2;
}

__global__ __launch_bounds__(JNT) void direct_kernel(const DirectArgs* __restrict__ set) {
  __shared__ JacobiLds L;
  const DirectArgs a = set[blockIdx.x];
  const int n = a.n, P = a.P;
  const double* __restrict__ V = a.V;
  double* __restrict__ U = a.U;
  jacobi_block<JNT, true>(L, a.G, n, n, a.lall, a.V);
  __syncthreads();
  const int tid = threadIdx.x, lane = tid & 63, w = wave_id();
  for (int j = tid; j < P; j += JNT) a.lam[j] = a.lall[j];
  for (int j = w; j < P; j += JNT / 64) {
    double best = -1.0;
    int bi = 0;   // stays a valid index if every entry is NaN
    for (int i = lane; i < n; i += 64) {
      const double v = fabs(V[i * n + j]);
      if (v > best || (v == best && i < bi)) { best = v; bi = i; }
    }
    for (int off = 32; off >= 1; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const double sgn = (V[bi * n + j] < 0.0) ? -1.0 : 1.0;
    for (int i = lane; i < n; i += 64) U[i * P + j] = sgn * V[i * n + j];
  }
}

// Copies the first P columns of X (n x ldx) into U (n x P) and signs each column so its
// largest-|.| entry is positive (ties: lowest index).  One workgroup per column.
__global__ void sign_columns_kernel(const double* __restrict__ X, int n, int ldx, int P,
                                    double* __restrict__ U) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  double best = -1.0;
  int besti = 0;   // stays a valid index if every entry is NaN
  for (int i = tid; i < n; i += blockDim.x) {
    const double a = fabs(X[(long long)i * ldx + j]);
    if (a > best || (a == best && i < besti)) { best = a; besti = i; }
  }
  bv[tid] = best; bi[tid] = besti;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) {
      const double a = bv[tid + s];
      const int ia = bi[tid + s];
      if (a > bv[tid] || (a == bv[tid] && ia < bi[tid])) { bv[tid] = a; bi[tid] = ia; }
    }
    __syncthreads();
  }
  const double sgn = (X[(long long)bi[0] * ldx + j] < 0.0) ? -1.0 : 1.0;
  for (int i = tid; i < n; i += blockDim.x) U[(long long)i * P + j] = sgn * X[(long long)i * ldx + j];
}

// Deterministic start block for the subspace iteration.
__global__ void init_block_kernel(double* Q, int n, int k, uint64_t seed) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * k) return;
  Q[e] = 2.0 * u01_from_bits(splitmix64(seed ^ (0x51ED2701ull * (uint64_t)(e + 1)))) - 1.0;
}

// Orthonormalises the k columns of Z (n x k, row-major) in place by classical Gram-Schmidt with
// one re-orthogonalisation pass ("twice is enough").  A column whose norm collapses below 1e-12 of
// its original norm is replaced by a fresh pseudo-random vector and orthogonalised again.
constexpr int ONT = 512;
__global__ __launch_bounds__(ONT) void orth_kernel(double* __restrict__ Z, int n, int k, uint64_t seed,
                                                   const int* __restrict__ only_if,
                                                   const double* __restrict__ src) {
  if (only_if != nullptr && *only_if == 0) return;
  if (src != nullptr) {
    for (long long e = threadIdx.x; e < (long long)n * k; e += ONT) Z[e] = src[e];
    __syncthreads();
  }
  __shared__ double coef[JMAX];
  __shared__ double red[2][ONT / 64];
  __shared__ double nrm0;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = ONT / 64;
  int flip = 0;
  for (int j = 0; j < k; ++j) {
    for (int attempt = 0; attempt < 3; ++attempt) {
      // original norm
      double s = 0.0;
      for (int i = tid; i < n; i += ONT) s += Z[(long long)i * k + j] * Z[(long long)i * k + j];
      s = block_sum(s, red[flip]); flip ^= 1;
      if (tid == 0) nrm0 = sqrt(s);
      for (int pass = 0; pass < 2 && j > 0; ++pass) {
        // coef[c] = <Z[:,c], Z[:,j]>, c < j: wave w handles c = w, w + nw, ...
        for (int c = w; c < j; c += nw) {
          double d = 0.0;
          for (int i = lane; i < n; i += 64) d += Z[(long long)i * k + c] * Z[(long long)i * k + j];
          d = wave_sum(d);
          if (lane == 0) coef[c] = d;
        }
        __syncthreads();
        for (int i = tid; i < n; i += ONT) {
          double v = Z[(long long)i * k + j];
          for (int c = 0; c < j; ++c) v -= coef[c] * Z[(long long)i * k + c];
          Z[(long long)i * k + j] = v;
        }
        __syncthreads();
      }
      s = 0.0;
      for (int i = tid; i < n; i += ONT) s += Z[(long long)i * k + j] * Z[(long long)i * k + j];
      s = block_sum(s, red[flip]); flip ^= 1;
      const double nrm = sqrt(s);
      if (nrm > 1e-12 * nrm0 && nrm > 1e-300) {
        const double inv = 1.0 / nrm;
        for (int i = tid; i < n; i += ONT) Z[(long long)i * k + j] *= inv;
        __syncthreads();
        break;
      }
      // deficient column: restart it from a pseudo-random vector
      for (int i = tid; i < n; i += ONT)
        Z[(long long)i * k + j] =
            2.0 * u01_from_bits(splitmix64(seed + 0x9E37ull * (uint64_t)(j + 1) +
                                           0x1000193ull * (uint64_t)(attempt + 1) + (uint64_t)i * 0x85EBCA6Bull)) - 1.0;
      __syncthreads();
    }
  }
}

// Cholesky of the column-scaled Gram D C D = R^T R, D = diag(C)^{-1/2}, of a k x k SPD matrix
// (k <= 64).  Four wavefronts, lane = column, waves interleaved over rows; right-looking without
// forming the pivot row first: at step j row j is final, and every thread subtracts
// a_jr a_jc / a_jj from its entries of the rows below (one barrier per step).  At the end row r is
// scaled by a_rr^{-1/2}.  Writes R (upper triangular, row-major k x k) and D.  A pivot below 1e-13
// sets *bad = 1 (or-ed with *prev when given).
constexpr int CH_NT = 256;
__global__ __launch_bounds__(CH_NT) void chol_scaled_kernel(const double* __restrict__ C, int k,
                                                            double* __restrict__ Rout, double* __restrict__ Dout,
                                                            const int* __restrict__ prev, int* __restrict__ bad) {
  __shared__ double A[JMAX][JMAX + 1];   // A[row][col], upper triangle used
  __shared__ double dsc[JMAX];
  constexpr int CW = CH_NT / 64;
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x < k) {
    const double cc = C[c * k + c];
    dsc[c] = (cc > 0.0) ? 1.0 / sqrt(cc) : 1.0;
  }
  __syncthreads();
  if (c < k)
    for (int r = w; r <= c; r += CW) A[r][c] = dsc[r] * C[r * k + c] * dsc[c];
  __syncthreads();
  for (int j = 0; j + 1 < k; ++j) {
    if (c > j && c < k) {
      const double t = A[j][c] / fmax(A[j][j], 1e-300);
      for (int r = j + 1 + w; r <= c; r += CW) A[r][c] -= A[j][r] * t;
    }
    __syncthreads();
  }
  int fail = 0;
  if (c < k) {
    for (int r = w; r < k; r += CW) {
      const double piv = A[r][r];
      if (c == r && !(piv > 1e-13)) fail = 1;
      Rout[r * k + c] = (r <= c) ? A[r][c] / sqrt(fmax(piv, 1e-300)) : 0.0;
    }
    if (w == 0) Dout[c] = dsc[c];
  }
  fail = __syncthreads_or(fail);
  if (threadIdx.x == 0) *bad = (fail ? 1 : 0) | (prev ? *prev : 0);
}

// Q[i, :] = (Y[i, :] D) R^{-1} by forward substitution along the row (thread per row, R, D and
// 1 / diag(R) staged in LDS).  Entry c subtracts its c earlier terms in four interleaved partial
// sums (loops unrolled at compile time, so the loads of R run ahead of the arithmetic).  Skipped
// when the factorisation failed.
__global__ __launch_bounds__(128) void rowsolve_kernel(const double* __restrict__ Y, const double* __restrict__ Rm,
                                                       const double* __restrict__ D, int n, int k,
                                                       const int* __restrict__ bad, double* __restrict__ Q) {
  __shared__ double Rs[JMAX * JMAX];
  __shared__ double Ds[JMAX], Ri[JMAX];
  if (*bad) return;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) Rs[e] = Rm[e];
  for (int e = threadIdx.x; e < k; e += blockDim.x) {
    Ds[e] = D[e];
    Ri[e] = 1.0 / Rm[e * k + e];
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* y = Y + (long long)i * k;
  double* q = Q + (long long)i * k;
  double qv[JMAX];
#pragma unroll
  for (int c = 0; c < JMAX; ++c) {
    if (c < k) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
      for (int t = 0; t + 3 < c; t += 4) {
        s0 = fma(qv[t], Rs[t * k + c], s0);
        s1 = fma(qv[t + 1], Rs[(t + 1) * k + c], s1);
        s2 = fma(qv[t + 2], Rs[(t + 2) * k + c], s2);
        s3 = fma(qv[t + 3], Rs[(t + 3) * k + c], s3);
      }
#pragma unroll
      for (int t = c & ~3; t < c; ++t) s0 = fma(qv[t], Rs[t * k + c], s0);
      qv[c] = (y[c] * Ds[c] - ((s0 + s1) + (s2 + s3))) * Ri[c];
      q[c] = qv[c];
    }
  }
}

// max_j ||ZV[:,j] - theta_j U[:,j]|| / |theta_0| over the P <= 64 wanted pairs (one workgroup):
// lane = column (coalesced along the rows), waves interleaved over rows, the waves' column sums
// added in a fixed order.
constexpr int RR_NT = 1024;
__global__ __launch_bounds__(RR_NT) void ritz_residual_kernel(const double* __restrict__ ZV, int ldz,
                                                              const double* __restrict__ U,
                                                              const double* __restrict__ theta, int n, int P,
                                                              double* __restrict__ out) {
  constexpr int RW = RR_NT / 64;
  __shared__ double part[RW][64];
  const int j = threadIdx.x & 63, w = threadIdx.x >> 6;
  double s = 0.0;
  if (j < P) {
    const double th = theta[j];
    for (int i = w; i < n; i += RW) {
      const double r = ZV[(long long)i * ldz + j] - th * U[(long long)i * P + j];
      s += r * r;
    }
  }
  part[w][j] = s;
  __syncthreads();
  if (w == 0) {
    double t = 0.0;
    for (int q = 0; q < RW; ++q) t += part[q][j];
    double worst = (j < P) ? sqrt(t) : 0.0;
    for (int off = 32; off > 0; off >>= 1) worst = fmax(worst, __shfl_xor(worst, off));
    if (j == 0) {
      const double t0 = fabs(theta[0]);
      *out = (t0 > 0.0) ? worst / t0 : 0.0;
    }
  }
}

// ---- whole subspace iteration in one workgroup -------------------------------------------------
// For moderate n the iteration above is a chain of small dependent launches.  The kernel below
// runs the same algorithm (start block, Cholesky-QR, four power steps, Rayleigh-Ritz until the
// Ritz residual test passes, signs) inside one workgroup per problem: the n x k blocks live in
// the workspace (L2-resident), the k x k matrices in LDS, products on the FP64 matrix cores.
constexpr int FNT = 1024;           // threads of the fused solver
constexpr int FNW = FNT / 64;
constexpr int FUSED_NMAX = 320;      // largest order handled by one workgroup

struct FusedLds {
  union {
    JacobiLds jac;
    struct {
      double C[JMAX][JMAX + 1];      // Gram of the block, then the working matrix of the factorisation
      double R[JMAX][JMAX + 1];      // Cholesky factor (upper)
      double M[JMAX][JMAX + 1];      // D R^{-1}
      double dsc[JMAX];              // D = diag(C)^{-1/2}
    } qr;
  } u;
  double coef[JMAX];
  double red[2][FNW];
  double colmax[FNW];
  int bad;
};

// out(m, c) = sum_t A(m, t) B(t, c) over 16 x 16 tiles spread over the waves; fa / fb return 0
// outside the operands (clamped indices), st stores an in-range entry.
template <class FA, class FB, class FS>
__device__ __forceinline__ void wg_gemm(int M, int N, int K, FA fa, FB fb, FS st) {
  const int lane = threadIdx.x & 63, w = wave_id();
  const int tm = tiles16(M), tn = tiles16(N);
  for (int t = w; t < tm * tn; t += FNW) {
    const int bm = t / tn, bn = t - bm * tn;
    const dbl4 acc = mfma_tile(bm * 16, bn * 16, K, fa, fb);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = bm * 16 + 4 * v + (lane >> 4), c = bn * 16 + (lane & 15);
      if (r < M && c < N) st(r, c, acc[v]);
    }
  }
}

// Small product with a long contraction (k x k outputs, K = n): the output tiles times K slices
// are spread over all waves, each slice's tile goes to LDS scratch (ns x tiles x 256 doubles) and
// the slices are summed in a fixed order.
template <class FA, class FB, class FS>
__device__ __forceinline__ void wg_gemm_ksplit(int M, int N, int K, FA fa, FB fb, FS st, double* scratch) {
  const int lane = threadIdx.x & 63, w = wave_id();
  const int tm = tiles16(M), tn = tiles16(N), nt = tm * tn;
  const int ns = max(1, FNW / nt);
  const int ks = (((K + ns - 1) / ns) + 15) & ~15;
  for (int job = w; job < nt * ns; job += FNW) {
    const int t = job % nt, sl = job / nt;
    const int bm = t / tn, bn = t - bm * tn;
    const int k0 = sl * ks, kn = max(0, min(K, k0 + ks) - k0);
    const dbl4 acc = mfma_tile(bm * 16, bn * 16, kn,
        [&](int m, int kk) { return (kk < kn) ? fa(m, k0 + kk) : 0.0; },
        [&](int kk, int c) { return (kk < kn) ? fb(k0 + kk, c) : 0.0; });
#pragma unroll
    for (int v = 0; v < 4; ++v) scratch[(sl * nt + t) * 256 + v * 64 + lane] = acc[v];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nt * 256; e += FNT) {
    const int t = e >> 8, q = e & 255, v = q >> 6, ln = q & 63;
    const int bm = t / tn, bn = t - bm * tn;
    const int r = bm * 16 + 4 * v + (ln >> 4), c = bn * 16 + (ln & 15);
    double sum = 0.0;
    for (int sl = 0; sl < ns; ++sl) sum += scratch[(sl * nt + t) * 256 + q];
    if (r < M && c < N) st(r, c, sum);
  }
}

// Out = G Q (n x k) for symmetric G, formed as (Q^T G)^T: the tiles of Q^T G read rows of Q and
// rows of G, sixteen consecutive doubles per fragment row, where G Q would read sixteen rows of G
// per fragment.
__device__ __forceinline__ void gq_product(const double* G, const double* Q, int n, int k, double* Out) {
  const int n1 = n - 1, k1 = k - 1;
  wg_gemm(k, n, n,
      [&](int c, int t) { return (c < k && t < n) ? Q[min(t, n1) * k + min(c, k1)] : 0.0; },
      [&](int t, int i) { return (t < n && i < n) ? G[min(t, n1) * n + min(i, n1)] : 0.0; },
      [&](int c, int i, double v) { Out[i * k + c] = v; });
}

// One Cholesky-QR pass Out = X D R^{-1}, D C D = R^T R, C = X^T X, D = diag(C)^{-1/2} (n x k, row
// major).  Returns (uniformly) whether a pivot fell below 1e-13; Out is then not written.
__device__ bool cholqr_pass(FusedLds& S, const double* X, int n, int k, double* Out) {
  const int tid = threadIdx.x, lane = tid & 63, w = wave_id();
  const int n1 = n - 1, k1 = k - 1;
  wg_gemm_ksplit(k, k, n,
      [&](int r, int i) { return (r < k && i < n) ? X[min(i, n1) * k + min(r, k1)] : 0.0; },
      [&](int i, int c) { return (c < k && i < n) ? X[min(i, n1) * k + min(c, k1)] : 0.0; },
      [&](int r, int c, double v) { S.u.qr.C[r][c] = v; }, &S.u.qr.M[0][0]);
  __syncthreads();
  double (*A)[JMAX + 1] = S.u.qr.C;
  double (*Rf)[JMAX + 1] = S.u.qr.R;
  double (*Mi)[JMAX + 1] = S.u.qr.M;
  if (tid < k) {
    const double cc = A[tid][tid];
    S.u.qr.dsc[tid] = (cc > 0.0) ? 1.0 / sqrt(cc) : 1.0;
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += FNT) {
    const int r = e / k, c = e - r * k;
    if (r <= c) A[r][c] = S.u.qr.dsc[r] * A[r][c] * S.u.qr.dsc[c];
  }
  __syncthreads();
  // D C D = R^T R by the whole workgroup, one barrier per column: row j of R (row j of the working
  // matrix over sqrt(a_jj)) goes to Rf while the trailing part is updated from the unchanged row j,
  // so the two never touch the same entries.
  int fail = 0;
  for (int j = 0; j < k; ++j) {
    const double piv = A[j][j];
    if (!(piv > 1e-13)) fail = 1;
    const double d = sqrt(fmax(piv, 1e-300));
    for (int c = j + tid; c < k; c += FNT) Rf[j][c] = (c == j) ? d : A[j][c] / d;
    const int m = k - 1 - j;
    for (int e = tid; e < m * m; e += FNT) {
      const int r = j + 1 + e / m, c = j + 1 + (e - (e / m) * m);
      if (r <= c) A[r][c] -= (A[j][r] / d) * (A[j][c] / d);
    }
    __syncthreads();
  }
  if (w == 0) {
    // lane c: column c of R^{-1} by back substitution, scaled by D
    const int c = lane;
    if (c < k) {
      Mi[c][c] = 1.0 / Rf[c][c];
      for (int i = c - 1; i >= 0; --i) {
        // four interleaved partial sums, so four LDS reads are in flight instead of one
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int t = i + 1;
        for (; t + 3 <= c; t += 4) {
          a0 += Rf[i][t] * Mi[t][c];
          a1 += Rf[i][t + 1] * Mi[t + 1][c];
          a2 += Rf[i][t + 2] * Mi[t + 2][c];
          a3 += Rf[i][t + 3] * Mi[t + 3][c];
        }
        for (; t <= c; ++t) a0 += Rf[i][t] * Mi[t][c];
        Mi[i][c] = -((a0 + a1) + (a2 + a3)) / Rf[i][i];
      }
      for (int i = 0; i <= c; ++i) Mi[i][c] *= S.u.qr.dsc[i];
      for (int i = c + 1; i < k; ++i) Mi[i][c] = 0.0;
    }
    if (lane == 0) S.bad = fail;
  }
  __syncthreads();
  const bool bad = S.bad != 0;
  if (!bad) {
    wg_gemm(n, k, k,
        [&](int i, int t) { return (i < n && t < k) ? X[min(i, n1) * k + min(t, k1)] : 0.0; },
        [&](int t, int c) { return (t < k && c < k) ? S.u.qr.M[min(t, k1)][min(c, k1)] : 0.0; },
        [&](int i, int c, double v) { Out[i * k + c] = v; });
  }
  __syncthreads();
  return bad;
}

// Classical Gram-Schmidt with one re-orthogonalisation pass on the k columns of Z (n x k) in
// place; a column whose norm collapses below 1e-12 of its original norm restarts from a
// pseudo-random vector (the breakdown fallback of the Cholesky-QR).
__device__ void cgs2(FusedLds& S, double* Z, int n, int k, uint64_t seed) {
  const int tid = threadIdx.x, lane = tid & 63, w = wave_id();
  int flip = 0;
  for (int j = 0; j < k; ++j) {
    for (int attempt = 0; attempt < 3; ++attempt) {
      double s = 0.0;
      for (int i = tid; i < n; i += FNT) s += Z[i * k + j] * Z[i * k + j];
      const double nrm0 = sqrt(block_sum(s, S.red[flip])); flip ^= 1;
      for (int pass = 0; pass < 2 && j > 0; ++pass) {
        for (int c = w; c < j; c += FNW) {
          double d = 0.0;
          for (int i = lane; i < n; i += 64) d += Z[i * k + c] * Z[i * k + j];
          d = wave_sum(d);
          if (lane == 0) S.coef[c] = d;
        }
        __syncthreads();
        for (int i = tid; i < n; i += FNT) {
          double v = Z[i * k + j];
          for (int c = 0; c < j; ++c) v -= S.coef[c] * Z[i * k + c];
          Z[i * k + j] = v;
        }
        __syncthreads();
      }
      s = 0.0;
      for (int i = tid; i < n; i += FNT) s += Z[i * k + j] * Z[i * k + j];
      const double nrm = sqrt(block_sum(s, S.red[flip])); flip ^= 1;
      if (nrm > 1e-12 * nrm0 && nrm > 1e-300) {
        const double inv = 1.0 / nrm;
        for (int i = tid; i < n; i += FNT) Z[i * k + j] *= inv;
        __syncthreads();
        break;
      }
      for (int i = tid; i < n; i += FNT)
        Z[i * k + j] = 2.0 * u01_from_bits(splitmix64(seed + 0x9E37ull * (uint64_t)(j + 1) +
                                                      0x1000193ull * (uint64_t)(attempt + 1) +
                                                      (uint64_t)i * 0x85EBCA6Bull)) - 1.0;
      __syncthreads();
    }
  }
}

// Orthonormal basis Q of the columns of Y: one or two Cholesky-QR passes, CGS2 on Y's copy when a
// pass breaks down.  Y is left unchanged.
__device__ void cholqr(FusedLds& S, const double* Y, int n, int k, double* Q, double* Qt, bool twice,
                       uint64_t seed) {
  bool bad = cholqr_pass(S, Y, n, k, twice ? Qt : Q);
  if (twice && !bad) bad = cholqr_pass(S, Qt, n, k, Q);
  if (bad) {
    for (int e = threadIdx.x; e < n * k; e += FNT) Q[e] = Y[e];
    __syncthreads();
    cgs2(S, Q, n, k, seed);
  }
}

struct FusedBufs {
  double *Q, *Y, *Z, *Qt, *B, *Vb, *theta, *Uw;
};

// Rayleigh-Ritz on span(Q): Z = G Q, B = Q^T Z, (theta, Vb) = eig(B), Uw = Q Vb[:, :P],
// Y = Z Vb; returns max_j<P ||Y[:, j] - theta_j Uw[:, j]|| / |theta_0|.
__device__ double rayleigh_ritz(FusedLds& S, const double* G, int n, int P, int k, const FusedBufs& b) {
  const int lane = threadIdx.x & 63, w = wave_id();
  const int n1 = n - 1, k1 = k - 1;
  const double* Q = b.Q;
  double* Z = b.Z;
  gq_product(G, Q, n, k, Z);
  __syncthreads();
  double* B = b.B;
  wg_gemm_ksplit(k, k, n,
      [&](int r, int i) { return (r < k && i < n) ? Q[min(i, n1) * k + min(r, k1)] : 0.0; },
      [&](int i, int c) { return (c < k && i < n) ? Z[min(i, n1) * k + min(c, k1)] : 0.0; },
      [&](int r, int c, double v) { B[r * k + c] = v; }, &S.u.qr.M[0][0]);
  __syncthreads();
  jacobi_block<FNT, true>(S.u.jac, B, k, k, b.theta, b.Vb);
  __syncthreads();
  const double* Vb = b.Vb;
  double* Uw = b.Uw;
  double* Y = b.Y;
  const int P1 = P - 1;
  wg_gemm(n, P, k,
      [&](int i, int t) { return (i < n && t < k) ? Q[min(i, n1) * k + min(t, k1)] : 0.0; },
      [&](int t, int c) { return (t < k && c < P) ? Vb[min(t, k1) * k + min(c, P1)] : 0.0; },
      [&](int i, int c, double v) { Uw[i * P + c] = v; });
  wg_gemm(n, k, k,
      [&](int i, int t) { return (i < n && t < k) ? Z[min(i, n1) * k + min(t, k1)] : 0.0; },
      [&](int t, int c) { return (t < k && c < k) ? Vb[min(t, k1) * k + min(c, k1)] : 0.0; },
      [&](int i, int c, double v) { Y[i * k + c] = v; });
  __syncthreads();
  // one wave per wanted column
  double worst = 0.0;
  for (int j = w; j < P; j += FNW) {
    const double th = b.theta[j];
    double s = 0.0;
    for (int i = lane; i < n; i += 64) {
      const double r = Y[i * k + j] - th * Uw[i * P + j];
      s += r * r;
    }
    worst = fmax(worst, sqrt(wave_sum(s)));
  }
  if (lane == 0) S.colmax[w] = worst;
  __syncthreads();
  double m = 0.0;
  for (int i = 0; i < FNW; ++i) m = fmax(m, S.colmax[i]);
  const double t0 = fabs(b.theta[0]);
  __syncthreads();
  return (t0 > 0.0) ? m / t0 : 0.0;
}

// One problem of the fused solver: its Gram, sizes, work blocks and outputs.
struct SubspaceArgs {
  const double* G;
  int n, P, k;
  double *Q, *Y, *Z, *Qt, *B, *Vb, *theta, *Uw;
  uint64_t seed;
  double *U, *lam;
  double *V, *lall;   // orders n <= 64: the full Jacobi's outputs, used when the iteration stalls
};
// Up to three problems per launch, one workgroup each (the modes of one tensor); descriptors in a
// workspace array written by put_args_kernel.
__global__ __launch_bounds__(FNT) void subspace_kernel(const SubspaceArgs* __restrict__ set) {
  __shared__ FusedLds S;
  const SubspaceArgs a = set[blockIdx.x];
  const double* __restrict__ G = a.G;
  const int n = a.n, P = a.P, k = a.k;
  const uint64_t seed = a.seed;
  double* __restrict__ U = a.U;
  double* __restrict__ lam = a.lam;
  const FusedBufs b = {a.Q, a.Y, a.Z, a.Qt, a.B, a.Vb, a.theta, a.Uw};
  const int tid = threadIdx.x, lane = tid & 63, w = wave_id();
  // start block and one Cholesky-QR pass
  for (int e = tid; e < n * k; e += FNT)
    b.Y[e] = 2.0 * u01_from_bits(splitmix64(seed ^ (0x51ED2701ull * (uint64_t)(e + 1)))) - 1.0;
  __syncthreads();
  cholqr(S, b.Y, n, k, b.Q, b.Qt, false, seed + 1);
  // four power steps, the last with two passes
  for (int it = 0; it < 4; ++it) {
    const double* Q = b.Q;
    double* Y = b.Y;
    gq_product(G, Q, n, k, Y);
    __syncthreads();
    cholqr(S, b.Y, n, k, b.Q, b.Qt, it == 3, seed + 100 + it);
  }
  // orders n <= 64 (few wanted pairs) give the iteration eight Rayleigh-Ritz steps, then fall back
  // to the full Jacobi of G (a spectrum without a gap after the P-th eigenvalue converges slowly)
  const int max_rr = (a.V != nullptr) ? 8 : 199;
  double ratio = rayleigh_ritz(S, G, n, P, k, b);
  for (int it = 0; ratio > 1e-13 && it < max_rr; ++it) {
    cholqr(S, b.Y, n, k, b.Q, b.Qt, true, seed + 2 + it);
    ratio = rayleigh_ritz(S, G, n, P, k, b);
  }
  const bool full = a.V != nullptr && ratio > 1e-13;
  if (full) {
    __syncthreads();
    jacobi_block<FNT, true>(S.u.jac, G, n, n, a.lall, a.V);
    __syncthreads();
  }
  const double* X = full ? a.V : b.Uw;
  const int ldx = full ? n : P;
  // eigenvalues and signed eigenvectors (largest-|.| entry positive, ties: lowest index)
  for (int j = tid; j < P; j += FNT) lam[j] = full ? a.lall[j] : b.theta[j];
  for (int j = w; j < P; j += FNW) {
    double best = -1.0;
    int bi = 0;
    for (int i = lane; i < n; i += 64) {
      const double a = fabs(X[i * ldx + j]);
      if (a > best || (a == best && i < bi)) { best = a; bi = i; }
    }
    for (int off = 32; off >= 1; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const double sgn = (X[bi * ldx + j] < 0.0) ? -1.0 : 1.0;
    for (int i = lane; i < n; i += 64) U[i * P + j] = sgn * X[i * ldx + j];
  }
}

int subspace_k(int n, int P) {
  int k = P + (P / 8 > 4 ? P / 8 : 4);
  if (k > JMAX) k = JMAX;
  if (k > n) k = n;
  return k;
}

}  // namespace

// Orthonormal basis Q of the columns of Y (n x k, k <= 64) by Cholesky-QR of the column-scaled
// Gram (one pass, or two when `twice`); if a pivot breaks down the block is orthonormalised by
// CGS2 instead (decided on the device, no synchronisation).  Y is left unchanged.
cpd_status chol_qr(const double* Y, int n, int k, double* Q, double* C, double* Rm, double* D, double* Qtmp,
                   int* flags, bool twice, uint64_t seed, hipStream_t s) {
  cpd_status st;
  const unsigned nb = (unsigned)((n + 127) / 128);
  if ((st = gemm_f64(k, k, n, 1.0, Y, k, 0, true, Y, CPD_F64, k, 0, false, 0.0, C, k, 0, 1, s))) return st;
  hipLaunchKernelGGL(chol_scaled_kernel, dim3(1), dim3(CH_NT), 0, s, C, k, Rm, D, (const int*)nullptr, flags);
  CPD_LAUNCH_CHECK();
  double* out1 = twice ? Qtmp : Q;
  hipLaunchKernelGGL(rowsolve_kernel, dim3(nb), dim3(128), 0, s, Y, Rm, D, n, k, flags, out1);
  CPD_LAUNCH_CHECK();
  int* last = flags;
  if (twice) {
    if ((st = gemm_f64(k, k, n, 1.0, Qtmp, k, 0, true, Qtmp, CPD_F64, k, 0, false, 0.0, C, k, 0, 1, s))) return st;
    hipLaunchKernelGGL(chol_scaled_kernel, dim3(1), dim3(CH_NT), 0, s, C, k, Rm, D, flags, flags + 1);
    CPD_LAUNCH_CHECK();
    hipLaunchKernelGGL(rowsolve_kernel, dim3(nb), dim3(128), 0, s, Qtmp, Rm, D, n, k, flags + 1, Q);
    CPD_LAUNCH_CHECK();
    last = flags + 1;
  }
  hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(ONT), 0, s, Q, n, k, seed, last, Y);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

namespace {

// One eigenproblem, advanced step by step so that several can share the host loop while their
// kernels run on different streams.
struct SubProblem {
  const double* G;
  int n, P, k, it;
  bool direct, done;
  double *U, *lam;
  double *V, *lall;                                              // direct (n <= 64)
  double *Q, *Z, *Y, *Qt, *B, *Vb, *Ri, *Dv, *theta, *Uw, *ratio;   // subspace iteration
  int* flags;
  SubspaceArgs* desc;   // this problem's descriptor slot (single-problem launches)
  uint64_t seed;
  double* r_host;   // the Ritz residual ratio read back by the host (pinned when possible)
  double r_own;     // pageable fallback for r_host
};

// Descriptor slots of one eigensolver call: NSIDE of the larger descriptor type, carved first.
union EigDesc {
  DirectArgs d;
  SubspaceArgs s;
};
constexpr int NSIDE = 3;
template <class Carver>
EigDesc* carve_desc(Carver& ar) { return ar.template take<EigDesc>(NSIDE); }

// Writes up to three descriptors into `out` on stream s.
template <class A>
cpd_status put_args(const A* a, int nprob, A* out, hipStream_t s) {
  A z[3];
  memset((void*)z, 0, sizeof(z));
  for (int i = 0; i < nprob; ++i) z[i] = a[i];
  hipLaunchKernelGGL(put_args_kernel<A>, dim3(1), dim3(64), 0, s, z[0], z[1], z[2], nprob, out);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

bool sp_fused(const SubProblem& q) { return !q.direct && q.n <= FUSED_NMAX; }

SubspaceArgs subspace_args(const SubProblem& q) {
  SubspaceArgs a;
  a.G = q.G; a.n = q.n; a.P = q.P; a.k = q.k;
  a.Q = q.Q; a.Y = q.Y; a.Z = q.Z; a.Qt = q.Qt; a.B = q.B; a.Vb = q.Vb; a.theta = q.theta; a.Uw = q.Uw;
  a.seed = q.seed; a.U = q.U; a.lam = q.lam;
  a.V = q.n <= JMAX ? q.V : nullptr;
  a.lall = q.n <= JMAX ? q.lall : nullptr;
  return a;
}

template <class Carver>
void sp_carve(Carver& ar, SubProblem& q) {
  if (q.direct) {
    q.V = ar.template take<double>((size_t)q.n * q.n);
    q.lall = ar.template take<double>(q.n);
    return;
  }
  if (q.n <= JMAX) {   // the fused iteration's fallback
    q.V = ar.template take<double>((size_t)q.n * q.n);
    q.lall = ar.template take<double>(q.n);
  }
  const size_t nk = (size_t)q.n * q.k, kk = (size_t)q.k * q.k;
  q.Q = ar.template take<double>(nk);
  q.Z = ar.template take<double>(nk);
  q.Y = ar.template take<double>(nk);
  q.Qt = ar.template take<double>(nk);
  q.B = ar.template take<double>(kk);
  q.Vb = ar.template take<double>(kk);
  q.Ri = ar.template take<double>(kk);
  q.Dv = ar.template take<double>(q.k);
  q.theta = ar.template take<double>(q.k);
  q.Uw = ar.template take<double>((size_t)q.n * q.P);
  q.ratio = ar.template take<double>(1);
  q.flags = ar.template take<int>(4);
}

void sp_describe(SubProblem& q, const double* G, int n, int P, double* U, double* lam) {
  memset(&q, 0, sizeof(q));
  q.G = G; q.n = n; q.P = P; q.U = U; q.lam = lam;
  // orders up to 64: the full Jacobi unless few pairs are wanted (subspace block at most n / 2)
  q.direct = n <= JMAX && 2 * subspace_k(n, P) > n;
  q.k = q.direct ? n : subspace_k(n, P);
  q.seed = 0xC0FFEEull + (uint64_t)n * 131 + (uint64_t)P;
}

cpd_status sp_check(int n, int P, const double* G, const double* U, const double* lam) {
  if (n < 1 || P < 1 || P > n || G == nullptr || U == nullptr || lam == nullptr) {
    set_error("eig_top: bad arguments n=%d P=%d", n, P);
    return CPD_E_INVALID;
  }
  if (n > JMAX && P > JMAX - 8) {
    set_error("eig_top: P=%d exceeds %d for n=%d > %d", P, JMAX - 8, n, JMAX);
    return CPD_E_UNSUPPORTED;
  }
  return CPD_OK;
}

// Writes the current pairs (eigenvalues, signed vectors) into the outputs.
cpd_status sp_emit(SubProblem& q, hipStream_t s) {
  const double* X = q.direct ? q.V : q.Uw;
  const int ldx = q.direct ? q.n : q.P;
  CPD_HIP_CHECK(hipMemcpyAsync(q.lam, q.direct ? q.lall : q.theta, sizeof(double) * q.P, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(sign_columns_kernel, dim3(q.P), dim3(256), 0, s, X, q.n, ldx, q.P, q.U);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

cpd_status sp_finish(SubProblem& q, hipStream_t s) {
  q.done = true;
  return sp_emit(q, s);
}

// One Rayleigh-Ritz step; the Ritz residual ratio is copied to *q.r_host (valid after the stream
// has been synchronised).  The Ritz pairs are written to the outputs right away: if the ratio passes
// the test they are the result and the host launches nothing more; otherwise the next step
// overwrites them.
cpd_status sp_rr(SubProblem& q, hipStream_t s) {
  const int n = q.n, k = q.k, P = q.P;
  cpd_status st;
  // Z = G Q ; B = Q^T Z ; Ritz pairs (theta, Vb) of B
  if ((st = gemm_f64(n, k, n, 1.0, q.G, n, 0, false, q.Q, CPD_F64, k, 0, false, 0.0, q.Z, k, 0, 1, s))) return st;
  if ((st = gemm_f64(k, k, n, 1.0, q.Q, k, 0, true, q.Z, CPD_F64, k, 0, false, 0.0, q.B, k, 0, 1, s))) return st;
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(JNT), 0, s, q.B, k, k, q.theta, q.Vb);
  CPD_LAUNCH_CHECK();
  // Ritz vectors U = Q Vb[:, :P]; Y = Z Vb = G (Q Vb) (its first P columns give the residuals)
  if ((st = gemm_f64(n, P, k, 1.0, q.Q, k, 0, false, q.Vb, CPD_F64, k, 0, false, 0.0, q.Uw, P, 0, 1, s))) return st;
  if ((st = gemm_f64(n, k, k, 1.0, q.Z, k, 0, false, q.Vb, CPD_F64, k, 0, false, 0.0, q.Y, k, 0, 1, s))) return st;
  hipLaunchKernelGGL(ritz_residual_kernel, dim3(1), dim3(RR_NT), 0, s, q.Y, k, q.Uw, q.theta, n, P, q.ratio);
  CPD_LAUNCH_CHECK();
  CPD_HIP_CHECK(hipMemcpyAsync(q.r_host, q.ratio, sizeof(double), hipMemcpyDeviceToHost, s));
  return sp_emit(q, s);
}

// Enqueues phase `ph` (0..5) of the first part of the problem: 0 the whole direct solve, or the
// start block; 1..4 the power steps; 5 the first Rayleigh-Ritz step.  Problems that share the host
// loop are enqueued phase by phase so that every stream has work early.
constexpr int START_PHASES = 6;
cpd_status sp_start_phase(SubProblem& q, int ph, hipStream_t s) {
  if (q.direct) {
    if (ph != 0) return CPD_OK;
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(JNT), 0, s, q.G, q.n, q.n, q.lall, q.V);
    CPD_LAUNCH_CHECK();
    return sp_finish(q, s);
  }
  const int n = q.n, k = q.k;
  if (n <= FUSED_NMAX) {
    if (ph != 0) return CPD_OK;
    const SubspaceArgs a = subspace_args(q);
    cpd_status st;
    if ((st = put_args(&a, 1, q.desc, s))) return st;
    hipLaunchKernelGGL(subspace_kernel, dim3(1), dim3(FNT), 0, s, (const SubspaceArgs*)q.desc);
    CPD_LAUNCH_CHECK();
    q.done = true;
    return CPD_OK;
  }
  if (ph == 0) {
    hipLaunchKernelGGL(init_block_kernel, dim3((n * k + 255) / 256), dim3(256), 0, s, q.Y, n, k, q.seed);
    CPD_LAUNCH_CHECK();
    // a Gaussian-like start block is well conditioned: one Cholesky-QR pass
    return chol_qr(q.Y, n, k, q.Q, q.B, q.Ri, q.Dv, q.Qt, q.flags, false, q.seed + 1, s);
  }
  if (ph <= 4) {
    // plain power steps Q <- orth(G Q) before the first Rayleigh-Ritz check; the last one
    // re-orthogonalises (two passes) since G Q is ill-conditioned
    const int it = ph - 1;
    cpd_status st;
    if ((st = gemm_f64(n, k, n, 1.0, q.G, n, 0, false, q.Q, CPD_F64, k, 0, false, 0.0, q.Y, k, 0, 1, s))) return st;
    return chol_qr(q.Y, n, k, q.Q, q.B, q.Ri, q.Dv, q.Qt, q.flags, it == 3, q.seed + 100 + it, s);
  }
  return sp_rr(q, s);
}

cpd_status sp_start(SubProblem& q, hipStream_t s) {
  cpd_status st;
  for (int ph = 0; ph < START_PHASES; ++ph)
    if ((st = sp_start_phase(q, ph, s))) return st;
  return CPD_OK;
}

// After the stream has been synchronised: finish, or enqueue the next basis and Ritz step.
cpd_status sp_continue(SubProblem& q, hipStream_t s) {
  if (*q.r_host <= 1e-13 || q.it >= 199) {
    q.done = true;   // the outputs were written by the last Rayleigh-Ritz step
    return CPD_OK;
  }
  // next basis: orthonormalised G (Q Vb); its columns are nearly orthogonal (G times Ritz
  // vectors), but a second pass keeps the Rayleigh-Ritz basis orthonormal to rounding
  cpd_status st;
  if ((st = chol_qr(q.Y, q.n, q.k, q.Q, q.B, q.Ri, q.Dv, q.Qt, q.flags, true, q.seed + 2 + q.it, s))) return st;
  ++q.it;
  return sp_rr(q, s);
}

// Pinned host slots for the Ritz residual ratios of up to NSIDE problems, one set per host thread,
// kept until the process ends.  A copy into pageable memory returns only when the stream reaches
// it, which would serialise the problems' Rayleigh-Ritz steps behind the host.  Every use ends
// with a synchronisation of the problem's stream before the next call on the thread.
double* ratio_slots() {
  static thread_local double* buf = nullptr;
  static thread_local bool tried = false;
  if (!tried) {
    tried = true;
    if (hipHostMalloc((void**)&buf, NSIDE * sizeof(double), hipHostMallocPortable) != hipSuccess) {
      buf = nullptr;
      (void)hipGetLastError();
    }
  }
  return buf;
}

void sp_bind_ratio(SubProblem& q, int slot) {
  double* b = ratio_slots();
  q.r_host = b ? b + slot : &q.r_own;
}

// Streams (default priority) and events for running up to three problems side by side; created
// once per host thread.
struct SideStreams {
  hipStream_t st[NSIDE];
  hipEvent_t fork, join[NSIDE];
  bool ok;
};

SideStreams* side_streams() {
  static thread_local SideStreams ss = {};
  static thread_local bool tried = false;
  if (!tried) {
    tried = true;
    ss.ok = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < NSIDE && ss.ok; ++i)
      ss.ok = hipStreamCreateWithFlags(&ss.st[i], hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&ss.join[i], hipEventDisableTiming) == hipSuccess;
  }
  return ss.ok ? &ss : nullptr;
}

}  // namespace

cpd_status eig_top(const double* G, int n, int P, double* U, double* lam, void* ws,
                   size_t ws_bytes, hipStream_t s) {
  cpd_status st;
  if ((st = sp_check(n, P, G, U, lam))) return st;
  if (ws == nullptr || ws_bytes < eig_ws_bytes(n, P)) {
    set_error("eig_top: workspace too small");
    return CPD_E_WORKSPACE;
  }
  SubProblem q;
  sp_describe(q, G, n, P, U, lam);
  sp_bind_ratio(q, 0);
  Arena ar(ws, ws_bytes);
  q.desc = &carve_desc(ar)[0].s;
  sp_carve(ar, q);
  if ((st = sp_start(q, s))) return st;
  while (!q.done) {
    CPD_HIP_CHECK(hipStreamSynchronize(s));
    if ((st = sp_continue(q, s))) return st;
  }
  return CPD_OK;
}

size_t eig_ws_bytes(int n, int P) {
  SubProblem q;
  sp_describe(q, nullptr, n, P, nullptr, nullptr);
  Sizer z;
  carve_desc(z);
  sp_carve(z, q);
  return z.off;
}

// Up to three problems: each runs on its own stream (forked from and joined back to s), so their
// single-workgroup kernels execute concurrently; one host loop advances them all.
size_t eig_ws_bytes3(const int* n, const int* P, int nprob) {
  Sizer z;
  carve_desc(z);
  for (int i = 0; i < nprob; ++i) {
    SubProblem q;
    sp_describe(q, nullptr, n[i], P[i], nullptr, nullptr);
    sp_carve(z, q);
  }
  return z.off;
}

cpd_status eig_top3(const double* const* G, const int* n, const int* P, double* const* U, double* const* lam,
                    int nprob, void* ws, size_t ws_bytes, hipStream_t s) {
  if (nprob < 1 || nprob > NSIDE) {
    set_error("eig_top: 1..%d problems per call", NSIDE);
    return CPD_E_INVALID;
  }
  cpd_status st;
  for (int i = 0; i < nprob; ++i)
    if ((st = sp_check(n[i], P[i], G[i], U[i], lam[i]))) return st;
  if (ws == nullptr || ws_bytes < eig_ws_bytes3(n, P, nprob)) {
    set_error("eig_top: workspace too small");
    return CPD_E_WORKSPACE;
  }
  SubProblem q[NSIDE];
  Arena ar(ws, ws_bytes);
  EigDesc* desc = carve_desc(ar);
  for (int i = 0; i < nprob; ++i) {
    sp_describe(q[i], G[i], n[i], P[i], U[i], lam[i]);
    sp_bind_ratio(q[i], i);
    q[i].desc = &desc[i].s;
    sp_carve(ar, q[i]);
  }
  // every problem small enough for the direct solve, or every one on the one-workgroup subspace
  // solver: one launch, one workgroup per problem, on s itself
  bool all_fused = true, all_direct = true;
  for (int i = 0; i < nprob; ++i) {
    all_fused = all_fused && sp_fused(q[i]);
    all_direct = all_direct && q[i].direct;
  }
  if (all_direct) {
    // contiguous DirectArgs array at the start of the descriptor block
    DirectArgs a[NSIDE];
    for (int i = 0; i < nprob; ++i) a[i] = {q[i].G, q[i].n, q[i].P, q[i].V, q[i].lall, q[i].U, q[i].lam};
    DirectArgs* dev = reinterpret_cast<DirectArgs*>(desc);
    if ((st = put_args(a, nprob, dev, s))) return st;
    hipLaunchKernelGGL(direct_kernel, dim3(nprob), dim3(JNT), 0, s, (const DirectArgs*)dev);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
  }
  if (all_fused) {
    SubspaceArgs a[NSIDE];
    for (int i = 0; i < nprob; ++i) a[i] = subspace_args(q[i]);
    SubspaceArgs* dev = reinterpret_cast<SubspaceArgs*>(desc);
    if ((st = put_args(a, nprob, dev, s))) return st;
    hipLaunchKernelGGL(subspace_kernel, dim3(nprob), dim3(FNT), 0, s, (const SubspaceArgs*)dev);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
  }
  SideStreams* ss = side_streams();
  if (ss == nullptr) {
    set_error("eig_top: could not create side streams");
    return CPD_E_HIP;
  }
  CPD_HIP_CHECK(hipEventRecord(ss->fork, s));
  for (int i = 0; i < nprob; ++i) CPD_HIP_CHECK(hipStreamWaitEvent(ss->st[i], ss->fork, 0));
  for (int ph = 0; ph < START_PHASES; ++ph)
    for (int i = 0; i < nprob; ++i)
      if ((st = sp_start_phase(q[i], ph, ss->st[i]))) return st;
  for (;;) {
    bool all = true;
    for (int i = 0; i < nprob; ++i) {
      if (q[i].done) continue;
      CPD_HIP_CHECK(hipStreamSynchronize(ss->st[i]));
      if ((st = sp_continue(q[i], ss->st[i]))) return st;
      all = all && q[i].done;
    }
    if (all) break;
  }
  for (int i = 0; i < nprob; ++i) {
    CPD_HIP_CHECK(hipEventRecord(ss->join[i], ss->st[i]));
    CPD_HIP_CHECK(hipStreamWaitEvent(s, ss->join[i], 0));
  }
  return CPD_OK;
}

}  // namespace cpd
