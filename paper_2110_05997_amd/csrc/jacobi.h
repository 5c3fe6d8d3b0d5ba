// Cyclic Jacobi eigensolver for a symmetric matrix of order n <= 64 held in the LDS of one
// workgroup of JNT threads (shared by the single-problem eigensolver and the batched solver).
#pragma once
#include "common.h"

namespace cpd {
namespace {

constexpr int JMAX = 64;
constexpr int JNT = 256;

// Jacobi with the parallel round-robin ordering.  Each round: the first np/2 threads compute the
// rotations of the round's disjoint pairs from A (one per pair); after a barrier every thread
// applies J_i^T A_ij J_j to the 2x2 blocks it owns, in place (a block's new value depends only on
// its own old entries), and V <- V J.  A rotation of pair (p, q) is skipped when
// |a_pq| <= 1e-15 sqrt(|a_pp a_qq|); a sweep without rotations, or with off(A)^2 <= 1e-30 ||A||^2,
// ends the iteration.
__device__ __forceinline__ void pair_of(int i, int round, int np, int& p, int& q) {
  const int a = (i == 0) ? 0 : 1 + ((i - 1 + round) % (np - 1));
  const int b = 1 + ((np - 2 - i + round) % (np - 1));
  p = min(a, b);
  q = max(a, b);
}

// Eigendecomposition of the symmetric n x n matrix Ag (leading dim lda, n <= 64).
// Outputs lam[n] descending and Vout (n x n row-major, eigenvector j in column j).
__device__ void jacobi_block(const double* __restrict__ Ag, int n, int lda, double* __restrict__ lam,
                             double* __restrict__ Vout) {
  __shared__ double A[JMAX][JMAX + 1];
  __shared__ double V[JMAX][JMAX + 1];
  __shared__ double rc[JMAX / 2], rs[JMAX / 2];
  __shared__ int rp[JMAX / 2], rq[JMAX / 2];
  __shared__ double red[2][JNT / 64];
  __shared__ int rank_of[JMAX];
  __shared__ int rotated[2];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int NWV = JNT / 64;
  const int np = (n + 1) & ~1;   // even number of slots (one zero padding slot when n is odd)
  const int half = np / 2;
  for (int i = w; i < JMAX; i += NWV) {
    A[i][lane] = (i < n && lane < n) ? Ag[(long long)i * lda + lane] : 0.0;
    V[i][lane] = (i == lane) ? 1.0 : 0.0;
  }
  __syncthreads();
  double fro2 = 0.0;
  for (int i = w; i < n; i += NWV)
    if (lane < n) fro2 += A[i][lane] * A[i][lane];
  fro2 = block_sum(fro2, red[0]);
  const int jj = tid & 31, i0 = tid >> 5;   // block column owned, first block row
  constexpr int ISTEP = JNT / 32;
  for (int sweep = 0; sweep < 60 && np >= 2; ++sweep) {
    double off = 0.0;
    for (int i = w; i < n; i += NWV)
      if (lane < n && lane != i) off += A[i][lane] * A[i][lane];
    off = block_sum(off, red[(sweep + 1) & 1]);
    if (off <= 1e-30 * fro2 || off == 0.0) break;
    if (tid == 0) rotated[sweep & 1] = 0;
    for (int round = 0; round < np - 1; ++round) {
      if (tid < half) {
        int p, q;
        pair_of(tid, round, np, p, q);
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p][q], app = A[p][p], aqq = A[q][q];
          if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > 1e-300) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            rotated[sweep & 1] = 1;
          }
        }
        rp[tid] = p; rq[tid] = q; rc[tid] = c; rs[tid] = s;
      }
      __syncthreads();
      if (jj < half) {
        const int pj = rp[jj], qj = rq[jj];
        const double cj = rc[jj], sj = rs[jj];
        for (int i = i0; i < half; i += ISTEP) {
          const int pi = rp[i], qi = rq[i];
          const double ci = rc[i], si = rs[i];
          const double a_pp = A[pi][pj], a_pq = A[pi][qj], a_qp = A[qi][pj], a_qq = A[qi][qj];
          const double b_pp = ci * a_pp - si * a_qp, b_pq = ci * a_pq - si * a_qq;
          const double b_qp = si * a_pp + ci * a_qp, b_qq = si * a_pq + ci * a_qq;
          A[pi][pj] = cj * b_pp - sj * b_pq;
          A[pi][qj] = sj * b_pp + cj * b_pq;
          A[qi][pj] = cj * b_qp - sj * b_qq;
          A[qi][qj] = sj * b_qp + cj * b_qq;
        }
        for (int x = i0; x < n; x += ISTEP) {
          const double vp = V[x][pj], vq = V[x][qj];
          V[x][pj] = cj * vp - sj * vq;
          V[x][qj] = sj * vp + cj * vq;
        }
      }
      __syncthreads();
    }
    if (rotated[sweep & 1] == 0) break;
  }
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
  for (int i = w; i < n; i += NWV)
    if (lane < n) Vout[(long long)i * n + rank_of[lane]] = V[i][lane];
}

}  // namespace
}  // namespace cpd
