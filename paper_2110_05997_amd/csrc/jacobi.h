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
  // round-robin ordering: slot 0 fixed, the others rotate; (x mod (np - 1)) for 0 <= x < 2(np - 1)
  const int m = np - 1;
  int x = i - 1 + round;
  x = (x >= m) ? x - m : x;
  int y = np - 2 - i + round;
  y = (y >= m) ? y - m : y;
  const int a = (i == 0) ? 0 : 1 + x;
  const int b = 1 + y;
  p = min(a, b);
  q = max(a, b);
}

// Rotation annihilating a_pq: with d = a_qq - a_pp and h = 2 a_pq, t = tan(theta) is
// sign(d) h / (|d| + sqrt(d^2 + h^2)) (the smaller root of t^2 + 2 (d/h) t - 1 = 0), c = 1/sqrt(1+t^2),
// s = t c.
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, double& c, double& s) {
  const double d = aqq - app, h = 2.0 * apq;
  const double r = sqrt(d * d + h * h);
  const double t = (d >= 0.0 ? h : -h) / (fabs(d) + r);
  c = rsqrt(1.0 + t * t);
  s = t * c;
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
  // thread map of the update phase: block column jj (pair), block rows i0, i0 + ISTEP, ...
  const int jj = tid & 31, i0 = tid >> 5;
  constexpr int ISTEP = JNT / 32;
  constexpr int NBI = (JMAX / 2 + ISTEP - 1) / ISTEP;   // block rows per thread
  constexpr int NVX = (JMAX + ISTEP - 1) / ISTEP;       // rows of V per thread
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
            jacobi_rotation(app, aqq, apq, c, s);
            rotated[sweep & 1] = 1;
          }
        }
        rp[tid] = p; rq[tid] = q; rc[tid] = c; rs[tid] = s;
      }
      __syncthreads();
      if (jj < half) {
        // gather every entry this thread owns, then rotate, then scatter (one LDS round trip
        // each way; the 2x2 blocks and V entries of different threads are disjoint)
        const int pj = rp[jj], qj = rq[jj];
        const double cj = rc[jj], sj = rs[jj];
        int pi[NBI], qi[NBI];
        double ci[NBI], si[NBI], a_pp[NBI], a_pq[NBI], a_qp[NBI], a_qq[NBI];
#pragma unroll
        for (int u = 0; u < NBI; ++u) {
          if (i0 + u * ISTEP < half) {
            const int i = i0 + u * ISTEP;
            pi[u] = rp[i]; qi[u] = rq[i]; ci[u] = rc[i]; si[u] = rs[i];
          }
        }
#pragma unroll
        for (int u = 0; u < NBI; ++u) {
          if (i0 + u * ISTEP < half) {
            a_pp[u] = A[pi[u]][pj]; a_pq[u] = A[pi[u]][qj];
            a_qp[u] = A[qi[u]][pj]; a_qq[u] = A[qi[u]][qj];
          }
        }
        double vp[NVX], vq[NVX];
#pragma unroll
        for (int u = 0; u < NVX; ++u) {
          const int x = i0 + u * ISTEP;
          if (x < n) { vp[u] = V[x][pj]; vq[u] = V[x][qj]; }
        }
#pragma unroll
        for (int u = 0; u < NBI; ++u) {
          if (i0 + u * ISTEP < half) {
            const double b_pp = ci[u] * a_pp[u] - si[u] * a_qp[u], b_pq = ci[u] * a_pq[u] - si[u] * a_qq[u];
            const double b_qp = si[u] * a_pp[u] + ci[u] * a_qp[u], b_qq = si[u] * a_pq[u] + ci[u] * a_qq[u];
            A[pi[u]][pj] = cj * b_pp - sj * b_pq;
            A[pi[u]][qj] = sj * b_pp + cj * b_pq;
            A[qi[u]][pj] = cj * b_qp - sj * b_qq;
            A[qi[u]][qj] = sj * b_qp + cj * b_qq;
          }
        }
#pragma unroll
        for (int u = 0; u < NVX; ++u) {
          const int x = i0 + u * ISTEP;
          if (x < n) {
            V[x][pj] = cj * vp[u] - sj * vq[u];
            V[x][qj] = sj * vp[u] + cj * vq[u];
          }
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
