// Cyclic Jacobi eigensolver for a symmetric matrix of order n <= 64 held in the LDS of one
// workgroup (shared by the single-problem eigensolvers and the batched solver).
#pragma once
#include "common.h"

namespace cpd {
namespace {

constexpr int JMAX = 64;
constexpr int JNT = 1024;   // threads of the standalone Jacobi kernels

// LDS of one Jacobi solve.  A is updated in place; the rotation inputs of the next round
// (diagonal entries and the off-diagonal entry of each pair) are copied into a small side
// buffer by the threads that produce them, so one barrier per round suffices.
struct JacobiLds {
  double A[JMAX][JMAX + 1];
  double V[JMAX][JMAX + 1];
  double dg[2][JMAX];    // A[x][x] for the round that reads this buffer
  double od[2][JMAX];    // A[p][q] of the pair (p < q) that contains p, indexed by p
  double rc[JMAX / 2], rs[JMAX / 2];   // rotations of the round (shared-rotation mode)
  double red[2][32];
  int rank_of[JMAX];
  int rotated[2];
};

// Round-robin ordering on np (even) slots: element 0 is fixed, elements 1..np-1 rotate.  Slot i
// of round t holds (p, q), p < q; 0 <= t < np - 1.
__device__ __forceinline__ void pair_of(int i, int round, int np, int& p, int& q) {
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

// Partner of element e in round t of the same ordering (the two non-zero elements of a slot sum
// to np - 3 + 2t modulo np - 1 after subtracting one from each; the element that would pair with
// itself pairs with 0).
__device__ __forceinline__ int partner_of(int e, int round, int np) {
  const int m = np - 1;
  if (e == 0) {
    const int y = np - 2 + round;
    return 1 + ((y >= m) ? y - m : y);
  }
  int v = np - 2 + 2 * round - e + m;   // in [m - 1, 4m - 1]
  v = (v >= m) ? v - m : v;
  v = (v >= m) ? v - m : v;
  v = (v >= m) ? v - m : v;
  const int f = 1 + v;
  return (f == e) ? 0 : f;
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

// Rotation of pair (p, q) from the side buffers; identity when q is the padding slot or when a_pq
// is negligible (|a_pq| <= 1e-15 sqrt(|a_pp a_qq|)).
__device__ __forceinline__ bool pair_rotation(const double* dg, const double* od, int p, int q, int n,
                                              double& c, double& s) {
  c = 1.0;
  s = 0.0;
  if (q >= n) return false;
  const double apq = od[p], app = dg[p], aqq = dg[q];
  if (!(apq * apq > 1e-30 * fabs(app * aqq)) || !(fabs(apq) > 1e-300)) return false;
  jacobi_rotation(app, aqq, apq, c, s);
  return true;
}

// Eigendecomposition of the symmetric n x n matrix Ag (leading dim lda, n <= 64) by NTH threads.
// Outputs lam[n] descending and Vout (n x n row-major, eigenvector j in column j).
// Each round applies the rotations of its disjoint pairs as A <- J^T A J, V <- V J; the thread of
// block (bi, bj) updates its 2x2 block in place (a block's new value depends only on its own old
// entries); V's column pairs are split the same way.  Rotations: with SHARED, one thread per pair
// forms it into LDS and a barrier publishes it (two barriers per round, least arithmetic: for many
// workgroups per CU); otherwise every thread forms the two rotations it needs from the side
// buffers (one barrier per round, shortest round: for a single latency-bound solve).  A sweep
// without rotations, or with off(A)^2 <= 1e-30 ||A||^2, ends the iteration (at most 60 sweeps).
template <int NTH, bool SHARED>
__device__ __forceinline__ void jacobi_block(JacobiLds& L, const double* __restrict__ Ag, int n, int lda,
                                             double* __restrict__ lam, double* __restrict__ Vout) {
  static_assert(NTH % 64 == 0 && NTH >= 64 && NTH <= 1024, "thread count");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int NWV = NTH / 64;
  const int np = (n + 1) & ~1;   // even number of slots (one zero padding slot when n is odd)
  const int half = np / 2;
  for (int i = w; i < JMAX; i += NWV) {
    L.A[i][lane] = (i < n && lane < n) ? Ag[(long long)i * lda + lane] : 0.0;
    L.V[i][lane] = (i == lane) ? 1.0 : 0.0;
  }
  __syncthreads();
  double fro2 = 0.0;
  for (int i = w; i < n; i += NWV)
    if (lane < n) fro2 += L.A[i][lane] * L.A[i][lane];
  if (tid == 0) { L.rotated[0] = 0; L.rotated[1] = 0; }
  fro2 = block_sum(fro2, L.red[0]);
  // rotation inputs of round 0
  if (tid < np) L.dg[0][tid] = L.A[tid][tid];
  if (tid < half) {
    int p, q;
    pair_of(tid, 0, np, p, q);
    L.od[0][p] = L.A[p][q];
  }
  // thread map: block column bj = tid % 32, block rows bi0, bi0 + ISTEP, ...
  const int bj = tid & 31, bi0 = tid >> 5;
  constexpr int ISTEP = NTH / 32;
  constexpr int NBI = (JMAX / 2 + ISTEP - 1) / ISTEP;   // block rows per thread
  constexpr int NVX = (JMAX + ISTEP - 1) / ISTEP;       // rows of V per thread
  int par = 0;
  for (int sweep = 0; sweep < 60 && np >= 2; ++sweep) {
    double off = 0.0;
    for (int i = w; i < n; i += NWV)
      if (lane < n && lane != i) off += L.A[i][lane] * L.A[i][lane];
    off = block_sum(off, L.red[(sweep + 1) & 1]);   // its barrier also publishes round 0's inputs
    if (off <= 1e-30 * fro2 || off == 0.0) break;
    // the flag of the next sweep is cleared here: nothing reads or sets it before the barriers
    // of this sweep's rounds
    if (tid == 0) L.rotated[(sweep + 1) & 1] = 0;
    for (int round = 0; round < np - 1; ++round) {
      const int nround = (round + 1 == np - 1) ? 0 : round + 1;
      const double* dg = L.dg[par];
      const double* od = L.od[par];
      double* dgn = L.dg[par ^ 1];
      double* odn = L.od[par ^ 1];
      if (SHARED) {
        if (tid < half) {
          int p, q;
          pair_of(tid, round, np, p, q);
          double c = 1.0, sn = 0.0;
          if (q < n) {
            const double apq = L.A[p][q], app = L.A[p][p], aqq = L.A[q][q];
            if (apq * apq > 1e-30 * fabs(app * aqq) && fabs(apq) > 1e-300) {
              jacobi_rotation(app, aqq, apq, c, sn);
              L.rotated[sweep & 1] = 1;
            }
          }
          L.rc[tid] = c;
          L.rs[tid] = sn;
        }
        __syncthreads();
      }
      if (bj < half) {
        int pj, qj;
        pair_of(bj, round, np, pj, qj);
        double cj, sj;
        if (SHARED) {
          cj = L.rc[bj];
          sj = L.rs[bj];
        } else if (pair_rotation(dg, od, pj, qj, n, cj, sj)) {
          L.rotated[sweep & 1] = 1;
        }
#pragma unroll
        for (int u = 0; u < NBI; ++u) {
          const int bi = bi0 + u * ISTEP;
          if (bi < half) {
            int pi, qi;
            pair_of(bi, round, np, pi, qi);
            double ci, si;
            if (SHARED) {
              ci = L.rc[bi];
              si = L.rs[bi];
            } else {
              pair_rotation(dg, od, pi, qi, n, ci, si);
            }
            const double a_pp = L.A[pi][pj], a_pq = L.A[pi][qj], a_qp = L.A[qi][pj], a_qq = L.A[qi][qj];
            const double b_pp = ci * a_pp - si * a_qp, b_pq = ci * a_pq - si * a_qq;
            const double b_qp = si * a_pp + ci * a_qp, b_qq = si * a_pq + ci * a_qq;
            const double n_pp = cj * b_pp - sj * b_pq, n_pq = sj * b_pp + cj * b_pq;
            const double n_qp = cj * b_qp - sj * b_qq, n_qq = sj * b_qp + cj * b_qq;
            L.A[pi][pj] = n_pp;
            L.A[pi][qj] = n_pq;
            L.A[qi][pj] = n_qp;
            L.A[qi][qj] = n_qq;
            if (!SHARED) {
              // inputs of the next round produced by this block
              if (bi == bj) { dgn[pi] = n_pp; dgn[qi] = n_qq; }
              const int ppi = partner_of(pi, nround, np), pqi = partner_of(qi, nround, np);
              if (pi < pj && ppi == pj) odn[pi] = n_pp;
              if (pi < qj && ppi == qj) odn[pi] = n_pq;
              if (qi < pj && pqi == pj) odn[qi] = n_qp;
              if (qi < qj && pqi == qj) odn[qi] = n_qq;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < NVX; ++u) {
          const int x = bi0 + u * ISTEP;
          if (x < n) {
            const double vp = L.V[x][pj], vq = L.V[x][qj];
            L.V[x][pj] = cj * vp - sj * vq;
            L.V[x][qj] = sj * vp + cj * vq;
          }
        }
      }
      par ^= 1;
      __syncthreads();
    }
    if (L.rotated[sweep & 1] == 0) break;
  }
  if (tid < n) {
    const double li = L.A[tid][tid];
    int r = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = L.A[j][j];
      if (lj > li || (lj == li && j < tid)) ++r;
    }
    L.rank_of[tid] = r;
  }
  __syncthreads();
  if (tid < n) lam[L.rank_of[tid]] = L.A[tid][tid];
  for (int i = w; i < n; i += NWV)
    if (lane < n) Vout[(long long)i * n + L.rank_of[lane]] = L.V[i][lane];
}



}  // namespace
}  // namespace cpd
