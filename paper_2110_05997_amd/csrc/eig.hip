// Leading eigenpairs of the symmetric unfolding Gram G_l = T_(l) T_(l)^T.  Its eigenvectors are
// the mode-l left singular vectors and sigma = sqrt(lambda) (App. B lemma relating the SVD of M to
// the eigendecomposition of M M^T); only the P_l = min(I_l, R) leading ones are needed (ch.4
// Alg. Compression, truncated SVD).
//
//  n <= 64 : cyclic Jacobi with the round-robin parallel ordering, the whole matrix in LDS of one
//            workgroup (exact to rounding, no spectral-gap assumption).
//  n  > 64 : subspace iteration on k = min(n, max(P + 8, 2P), 64) vectors with Rayleigh-Ritz
//            (Jacobi on the k x k projection), stopped when every wanted Ritz pair has residual
//            ||G u - theta u|| <= 1e-13 theta_1 (at most 200 iterations).
// Eigenvectors are signed so that each one's largest-magnitude entry is positive (ties: lowest
// index), the convention the oracle applies to its singular vectors.
#include "common.h"

#include <vector>

namespace cpd {
namespace {

constexpr int JMAX = 64;
constexpr int JNT = 256;

// Jacobi eigendecomposition of an n x n symmetric matrix (row-major, leading dim lda).
// Outputs: lam[n] descending, V[n*n] row-major with eigenvector j in column j (ldv = n).
__global__ __launch_bounds__(JNT) void jacobi_kernel(const double* __restrict__ Ag, int n, int lda,
                                                     double* __restrict__ lam,
                                                     double* __restrict__ Vout) {
  __shared__ double A[JMAX][JMAX + 1];
  __shared__ double V[JMAX][JMAX + 1];
  __shared__ double cs[JMAX / 2], sn[JMAX / 2];
  __shared__ int pp[JMAX / 2], qq[JMAX / 2];
  __shared__ double red[2][JNT / 64];
  __shared__ int rank_of[JMAX];
  const int tid = threadIdx.x;
  const int np = (n + 1) & ~1;   // even number of slots (one padding slot when n is odd)
  for (int e = tid; e < JMAX * JMAX; e += JNT) {
    const int i = e / JMAX, j = e % JMAX;
    A[i][j] = (i < n && j < n) ? Ag[(long long)i * lda + j] : 0.0;
    V[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  double fro2 = 0.0;
  for (int e = tid; e < n * n; e += JNT) fro2 += A[e / n][e % n] * A[e / n][e % n];
  fro2 = block_sum(fro2, red[0]);
  const int half = np / 2;
  for (int sweep = 0; sweep < 60 && np >= 2; ++sweep) {
    double off = 0.0;
    for (int e = tid; e < n * n; e += JNT) {
      const int i = e / n, j = e % n;
      if (i != j) off += A[i][j] * A[i][j];
    }
    off = block_sum(off, red[(sweep + 1) & 1]);
    if (off <= 1e-30 * fro2 || off == 0.0) break;
    for (int round = 0; round < np - 1; ++round) {
      if (tid < half) {
        // round-robin: slot 0 fixed, the others rotate
        const int i = tid;
        const int a = (i == 0) ? 0 : 1 + ((i - 1 + round) % (np - 1));
        const int bslot = np - 1 - i;
        const int b = 1 + ((bslot - 1 + round) % (np - 1));
        const int p = min(a, b), q = max(a, b);
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p][q];
          if (apq != 0.0) {
            const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        cs[i] = c; sn[i] = s; pp[i] = p; qq[i] = q;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int e = tid; e < half * np; e += JNT) {
        const int i = e / np, j = e % np;
        const int p = pp[i], q = qq[i];
        const double c = cs[i], s = sn[i];
        const double ap = A[p][j], aq = A[q][j];
        A[p][j] = c * ap - s * aq;
        A[q][j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int e = tid; e < half * np; e += JNT) {
        const int i = e / np, j = e % np;
        const int p = pp[i], q = qq[i];
        const double c = cs[i], s = sn[i];
        const double ap = A[j][p], aq = A[j][q];
        A[j][p] = c * ap - s * aq;
        A[j][q] = s * ap + c * aq;
        const double vp = V[j][p], vq = V[j][q];
        V[j][p] = c * vp - s * vq;
        V[j][q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  // rank sort, descending eigenvalue, ties by index
  if (tid < n) {
    const double li = A[tid][tid];
    int r = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = A[j][j];
      if (lj > li || (lj == li && j < tid)) ++r;
    }
    rank_of[tid] = r;
  }
  __syncthreads();
  if (tid < n) lam[rank_of[tid]] = A[tid][tid];
  for (int e = tid; e < n * n; e += JNT) {
    const int i = e / n, j = e % n;   // component i of eigenvector j
    Vout[(long long)i * n + rank_of[j]] = V[i][j];
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
  int besti = 0x7fffffff;
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
__global__ __launch_bounds__(ONT) void orth_kernel(double* __restrict__ Z, int n, int k, uint64_t seed) {
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

// max_j ||ZV[:,j] - theta_j U[:,j]|| / |theta_0| over the P wanted pairs (one workgroup).
__global__ void ritz_residual_kernel(const double* __restrict__ ZV, const double* __restrict__ U,
                                     const double* __restrict__ theta, int n, int P,
                                     double* __restrict__ out) {
  __shared__ double red[2][256 / 64];
  double worst = 0.0;
  int flip = 0;
  for (int j = 0; j < P; ++j) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double r = ZV[(long long)i * P + j] - theta[j] * U[(long long)i * P + j];
      s += r * r;
    }
    s = block_sum(s, red[flip]); flip ^= 1;
    worst = fmax(worst, sqrt(s));
  }
  if (threadIdx.x == 0) {
    const double t0 = fabs(theta[0]);
    *out = (t0 > 0.0) ? worst / t0 : 0.0;
  }
}

int subspace_k(int n, int P) {
  int k = P + 8;
  if (2 * P > k) k = 2 * P;
  if (k > JMAX) k = JMAX;
  if (k > n) k = n;
  return k;
}

}  // namespace

size_t eig_ws_bytes(int n, int P) {
  if (n <= JMAX) {
    Sizer z;
    z.take<double>((size_t)n * n);
    z.take<double>(n);
    return z.off;
  }
  const int k = subspace_k(n, P);
  Sizer z;
  z.take<double>((size_t)n * k);   // Q
  z.take<double>((size_t)n * k);   // Z
  z.take<double>((size_t)k * k);   // B
  z.take<double>((size_t)k * k);   // Vb
  z.take<double>(k);               // theta
  z.take<double>((size_t)n * P);   // U work
  z.take<double>((size_t)n * P);   // ZV
  z.take<double>(1);               // residual ratio
  return z.off;
}

cpd_status eig_top(const double* G, int n, int P, double* U, double* lam, void* ws,
                   size_t ws_bytes, hipStream_t s) {
  if (n < 1 || P < 1 || P > n || G == nullptr || U == nullptr || lam == nullptr) {
    set_error("eig_top: bad arguments n=%d P=%d", n, P);
    return CPD_E_INVALID;
  }
  if (ws == nullptr || ws_bytes < eig_ws_bytes(n, P)) {
    set_error("eig_top: workspace too small");
    return CPD_E_WORKSPACE;
  }
  Arena ar(ws, ws_bytes);
  if (n <= JMAX) {
    double* V = ar.take<double>((size_t)n * n);
    double* lall = ar.take<double>(n);
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(JNT), 0, s, G, n, n, lall, V);
    CPD_LAUNCH_CHECK();
    CPD_HIP_CHECK(hipMemcpyAsync(lam, lall, sizeof(double) * P, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(sign_columns_kernel, dim3(P), dim3(256), 0, s, V, n, n, P, U);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
  }
  if (P > JMAX - 8) {
    set_error("eig_top: P=%d exceeds %d for n=%d > %d", P, JMAX - 8, n, JMAX);
    return CPD_E_UNSUPPORTED;
  }
  const int k = subspace_k(n, P);
  double* Q = ar.take<double>((size_t)n * k);
  double* Z = ar.take<double>((size_t)n * k);
  double* B = ar.take<double>((size_t)k * k);
  double* Vb = ar.take<double>((size_t)k * k);
  double* theta = ar.take<double>(k);
  double* Uw = ar.take<double>((size_t)n * P);
  double* ZV = ar.take<double>((size_t)n * P);
  double* ratio = ar.take<double>(1);
  const uint64_t seed = 0xC0FFEEull + (uint64_t)n * 131 + (uint64_t)P;
  hipLaunchKernelGGL(init_block_kernel, dim3((n * k + 255) / 256), dim3(256), 0, s, Q, n, k, seed);
  CPD_LAUNCH_CHECK();
  hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(ONT), 0, s, Q, n, k, seed + 1);
  CPD_LAUNCH_CHECK();
  cpd_status st;
  for (int it = 0; it < 200; ++it) {
    // Z = G Q ; B = Q^T Z ; Ritz pairs of B
    if ((st = gemm_f64(n, k, n, 1.0, G, n, 0, false, Q, CPD_F64, k, 0, false, 0.0, Z, k, 0, 1, s))) return st;
    if ((st = gemm_f64(k, k, n, 1.0, Q, k, 0, true, Z, CPD_F64, k, 0, false, 0.0, B, k, 0, 1, s))) return st;
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(JNT), 0, s, B, k, k, theta, Vb);
    CPD_LAUNCH_CHECK();
    // U = Q Vb[:, :P], ZV = Z Vb[:, :P]
    if ((st = gemm_f64(n, P, k, 1.0, Q, k, 0, false, Vb, CPD_F64, k, 0, false, 0.0, Uw, P, 0, 1, s))) return st;
    if ((st = gemm_f64(n, P, k, 1.0, Z, k, 0, false, Vb, CPD_F64, k, 0, false, 0.0, ZV, P, 0, 1, s))) return st;
    hipLaunchKernelGGL(ritz_residual_kernel, dim3(1), dim3(256), 0, s, ZV, Uw, theta, n, P, ratio);
    CPD_LAUNCH_CHECK();
    double r = 0.0;
    CPD_HIP_CHECK(hipMemcpyAsync(&r, ratio, sizeof(double), hipMemcpyDeviceToHost, s));
    CPD_HIP_CHECK(hipStreamSynchronize(s));
    if (r <= 1e-13) break;
    // next block: orthonormalised Z
    CPD_HIP_CHECK(hipMemcpyAsync(Q, Z, sizeof(double) * (size_t)n * k, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(ONT), 0, s, Q, n, k, seed + 2 + it);
    CPD_LAUNCH_CHECK();
  }
  CPD_HIP_CHECK(hipMemcpyAsync(lam, theta, sizeof(double) * P, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(sign_columns_kernel, dim3(P), dim3(256), 0, s, Uw, n, P, P, U);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

}  // namespace cpd
