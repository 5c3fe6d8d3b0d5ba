// Damped Gauss-Newton on the compressed core, one persistent workgroup per CPD.
//
// Restates ch.4 "dGN" of the thesis for L = 3: at iteration k
//   pi^(l) = W^(l)T W^(l); Pi^(1) = pi2*pi3, Pi^(2) = pi1*pi3, Pi^(3) = pi1*pi2 (Hadamard), and the
//     pair products Pi^(a,b) = pi^(c) for the third mode c (ch.3 "Dealing with the Hessian");
//   gradient dF/dW^(l) = W^(l) Pi^(l) - S_(l) (KR of the others)         (gradient theorem)
//   D from the gammas, M = diag(J^T J) + mu D                          (ch.4 regularization)
//   CG on M^{-1/2}(J^T J + mu D)M^{-1/2} x_hat = M^{-1/2}(-grad F) with the random cap, the
//     product J^T J v from ch.3 Thm Hv, x = M^{-1/2} x_hat
//   predicted ||f + J x||^2 = ||f||^2 + 2 grad.x + x.J^T J x; w <- w + x (always accepted);
//   norm balancing; fused residual ||S - [[W]]||^2 with the MTTKRP of the next gradient;
//   gain ratio, damping rule (g < 0.25: 3 mu; g > 0.75: mu / 3), stopping conditions 1-7.
//
// Layout: the parameter vector is three row-major blocks W^(l) (d_l x R) back to back.  Every
// vector of the iteration (W, MTTKRP, gradient, CG x, r, p, z) and the R x R Grams live in LDS;
// the core S is read from global memory (L2-resident).  The dense contractions (Grams, the two
// products of Thm Hv, the three MTTKRPs and the residual model W^(1) (W^(3) (.) W^(2))^T) run on
// the FP64 matrix cores in 16x16 tiles spread over the waves, Khatri-Rao rows formed on the fly.
// All arithmetic is FP64; reductions use a fixed order, so a run is bit-reproducible.
#include "common.h"
#include "dgn_state.h"
#include "mfma_f64.h"

#include <math.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <vector>

namespace cpd {
namespace {


struct Ctx {
  int d0, d1, d2, off1, off2, R, np;
  int sp1, sp2;            // strides of S[i][j][k] (padded when S is staged in LDS)
  double *W, *MK, *G, *X, *Rv, *P, *Z;
  double *pi, *Pown, *Qb;   // 3 R^2 each
  double *msq, *gam;       // 3 R each
  double *red;             // 2 x NW
  double *U, *Ci;          // block-Jacobi only: one more vector and the three C_l^{-1} (R x R)
  const double* S;
};

// mode sizes and block offsets by selects (a dynamically indexed local array would live in
// scratch memory)
__device__ __forceinline__ int dimof(const Ctx& c, int a) { return a == 0 ? c.d0 : (a == 1 ? c.d1 : c.d2); }
__device__ __forceinline__ int offof(const Ctx& c, int a) { return a == 0 ? 0 : (a == 1 ? c.off1 : c.off2); }

__device__ __forceinline__ void split_index(const Ctx& c, int e, int& l, int& i, int& r) {
  l = (e >= c.off2) ? 2 : (e >= c.off1 ? 1 : 0);
  const int loc = e - offof(c, l);
  i = loc / c.R;
  r = loc - i * c.R;
}

// q = floor(x / d) for 0 <= x < 2^26 through a double reciprocal (exact: the error of
// (x + 0.5) * inv is far below the distance 0.5 / d to an integer).
__device__ __forceinline__ int div_by(int x, double inv) { return (int)(((double)x + 0.5) * inv); }

__device__ __forceinline__ double sel(bool ok, double v) { return ok ? v : 0.0; }

__device__ void setup_ctx(Ctx& c, double* lds, const int d[3], int R, const double* S, double* MK, double* G) {
  c.d0 = d[0]; c.d1 = d[1]; c.d2 = d[2]; c.R = R;
  c.off1 = d[0] * R; c.off2 = (d[0] + d[1]) * R;
  c.np = (d[0] + d[1] + d[2]) * R;
  c.sp1 = d[1] * d[2];
  c.sp2 = d[2];
  double* p = lds;
  c.W = p; p += c.np;
  c.MK = MK;
  c.G = G;
  c.X = p; p += c.np;
  c.Rv = p; p += c.np;
  c.P = p; p += c.np;
  c.Z = p; p += c.np;
  c.pi = p; p += 3 * R * R;
  c.Pown = p; p += 3 * R * R;
  c.Qb = p; p += 3 * R * R;
  c.msq = p; p += 3 * R;
  c.gam = p; p += 3 * R;
  c.red = p; p += 2 * NW;
  c.U = nullptr;
  c.Ci = nullptr;
  c.S = S;
}

// pi^(l) = W^(l)T W^(l) on the matrix cores, then Pi^(l); ends with a barrier.
__device__ void grams(Ctx& c) {
  const int R = c.R, RR = R * R, tr = tiles16(R);
  const int lane = threadIdx.x & 63, w = wave_id(), r16 = lane & 15, kq = lane >> 4;
  for (int t = w; t < 3 * tr * tr; t += NW) {
    const int l = t / (tr * tr), tt = t - l * tr * tr, tm = tt / tr, tn = tt - tm * tr;
    const double* Wl = c.W + offof(c, l);
    const int dl = dimof(c, l);
    const dbl4 acc = mfma_tile(tm * 16, tn * 16, dl,
        [&](int r, int i) { return sel(r < R && i < dl, Wl[min(i, dl - 1) * R + min(r, R - 1)]); },
        [&](int i, int q) { return sel(q < R && i < dl, Wl[min(i, dl - 1) * R + min(q, R - 1)]); });
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = tm * 16 + 4 * v + kq, q = tn * 16 + r16;
      if (r < R && q < R) c.pi[l * RR + r * R + q] = acc[v];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < RR; e += NT) {
    const double a = c.pi[e], b = c.pi[RR + e], d = c.pi[2 * RR + e];
    c.Pown[e] = b * d;
    c.Pown[RR + e] = a * d;
    c.Pown[2 * RR + e] = a * b;
  }
  __syncthreads();
}

// gammas of D and msq = M^{-1/2}, M = Pi^(l)_rr + mu gamma_l[r]; ends with a barrier.
__device__ void precond(Ctx& c, double mu) {
  const int R = c.R, RR = R * R;
  if (threadIdx.x < R) {
    double m = 0.0;
    for (int r = 0; r < R; ++r) {
      const double n0 = sqrt(c.pi[r * R + r]), n1 = sqrt(c.pi[RR + r * R + r]),
                   n2 = sqrt(c.pi[2 * RR + r * R + r]);
      m = fmax(m, fmax(n1 * n2, fmax(n0 * n2, n0 * n1)));
    }
    const int r = threadIdx.x;
    const double n0 = sqrt(c.pi[r * R + r]), n1 = sqrt(c.pi[RR + r * R + r]),
                 n2 = sqrt(c.pi[2 * RR + r * R + r]);
    const double g0 = n1 * n2 * m, g1 = n0 * n2 * m, g2 = n0 * n1 * m;
    c.gam[r] = g0; c.gam[R + r] = g1; c.gam[2 * R + r] = g2;
    c.msq[r] = 1.0 / sqrt(c.Pown[r * R + r] + mu * g0);
    c.msq[R + r] = 1.0 / sqrt(c.Pown[RR + r * R + r] + mu * g1);
    c.msq[2 * R + r] = 1.0 / sqrt(c.Pown[2 * RR + r * R + r] + mu * g2);
  }
  __syncthreads();
}

// The structured product of Thm Hv (same contract as hv below) on the vector units, for ranks whose
// 16 x 16 matrix-core tiles would be mostly padding.  Phase 1: the thread of position (s, r) forms
// Q_b[s][r] = v_b[:, s] . W_b[:, r] of all three modes and stores Y_0, Y_1, Y_2 in their place in Qb
// (one barrier).  Phase 2: the thread of entry (a, i, r) forms
// v_a[i, :] Pi^(a)[:, r] + W_a[i, :] Y_a[:, r].
constexpr int HV_VALU_RMAX = 24;
__device__ double hv_valu(Ctx& c, const double* V, double* out, double mu, bool scale) {
  const int R = c.R, RR = R * R, tid = threadIdx.x;
  const int d0 = c.d0, d1 = c.d1, d2 = c.d2;
  const double* V0 = V;
  const double* V1 = V + c.off1;
  const double* V2 = V + c.off2;
  const double* W0 = c.W;
  const double* W1 = c.W + c.off1;
  const double* W2 = c.W + c.off2;
  // column dot products in four interleaved partial sums (their loads overlap)
  auto coldot = [&](const double* Vb, const double* Wb, int db, int s, int r) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = 0;
    for (; i + 3 < db; i += 4) {
      a0 = fma(Vb[i * R + s], Wb[i * R + r], a0);
      a1 = fma(Vb[(i + 1) * R + s], Wb[(i + 1) * R + r], a1);
      a2 = fma(Vb[(i + 2) * R + s], Wb[(i + 2) * R + r], a2);
      a3 = fma(Vb[(i + 3) * R + s], Wb[(i + 3) * R + r], a3);
    }
    for (; i < db; ++i) a0 = fma(Vb[i * R + s], Wb[i * R + r], a0);
    return (a0 + a1) + (a2 + a3);
  };
  for (int sr = tid; sr < RR; sr += NT) {
    const int s = sr / R, r = sr - s * R;
    double q0 = coldot(V0, W0, d0, s, r);
    double q1 = coldot(V1, W1, d1, s, r);
    double q2 = coldot(V2, W2, d2, s, r);
    if (scale) {
      q0 *= c.msq[s];
      q1 *= c.msq[R + s];
      q2 *= c.msq[2 * R + s];
    }
    const double p0 = c.pi[sr], p1 = c.pi[RR + sr], p2 = c.pi[2 * RR + sr];
    c.Qb[sr] = p2 * q1 + p1 * q2;
    c.Qb[RR + sr] = p2 * q0 + p0 * q2;
    c.Qb[2 * RR + sr] = p1 * q0 + p0 * q1;
  }
  __syncthreads();
  double dotp = 0.0;
  for (int e = tid; e < c.np; e += NT) {
    int a, i, r;
    split_index(c, e, a, i, r);
    const double* Va = V + offof(c, a) + i * R;
    const double* Wa = c.W + offof(c, a) + i * R;
    const double* Pa = c.Pown + a * RR + r;
    const double* Ya = c.Qb + a * RR + r;
    const double* ma = c.msq + a * R;
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
    int s2 = 0;
    for (; s2 + 1 < R; s2 += 2) {
      a0 = fma(scale ? ma[s2] * Va[s2] : Va[s2], Pa[s2 * R], a0);
      b0 = fma(Wa[s2], Ya[s2 * R], b0);
      a1 = fma(scale ? ma[s2 + 1] * Va[s2 + 1] : Va[s2 + 1], Pa[(s2 + 1) * R], a1);
      b1 = fma(Wa[s2 + 1], Ya[(s2 + 1) * R], b1);
    }
    if (s2 < R) {
      a0 = fma(scale ? ma[s2] * Va[s2] : Va[s2], Pa[s2 * R], a0);
      b0 = fma(Wa[s2], Ya[s2 * R], b0);
    }
    double tv = (a0 + a1) + (b0 + b1);
    if (scale) tv = ma[r] * (tv + mu * c.gam[a * R + r] * (ma[r] * V[e]));
    else if (mu != 0.0) tv += mu * c.gam[a * R + r] * V[e];
    out[e] = tv;
    dotp += V[e] * tv;
  }
  return dotp;
}

// Structured product of Thm Hv.  With scale = true the input is v = msq * V and the output is
// msq * (J^T J v + mu D v) (the preconditioned CG operator); with scale = false it is
// J^T J V + mu D V (mu = 0: the plain J^T J V, D not read).
// Phase 1: Q_b = v_b^T W_b (R x R) for the three modes.  Phase 2, block a:
//   out_a = [v_a | W_a] [Pi^(a) ; Y_a],  Y_a = pi^(b2) * Q_b1 + pi^(b1) * Q_b2 ({b1, b2} = other modes),
// with Y formed inside the B-fragment loads (no barrier between the phases beyond the one that
// publishes Q).  Returns this thread's partial of <V, out>; ends
// without a barrier after phase 2.
// HVM 0: the vector-unit product for R <= HV_VALU_RMAX, the matrix cores above; 1: the matrix
// cores at any R (the batched kernel: carrying both paths spills its registers).
template <int HVM = 0>
__device__ double hv(Ctx& c, const double* V, double* out, double mu, bool scale) {
  if (HVM == 0 && c.R <= HV_VALU_RMAX) return hv_valu(c, V, out, mu, scale);
  const int R = c.R, RR = R * R, tr = tiles16(R);
  const int lane = threadIdx.x & 63, w = wave_id(), r16 = lane & 15, kq = lane >> 4;
  for (int t = w; t < 3 * tr * tr; t += NW) {
    const int b = t / (tr * tr), tt = t - b * tr * tr, tm = tt / tr, tn = tt - tm * tr;
    const double* Vb = V + offof(c, b);
    const double* Wb = c.W + offof(c, b);
    const int db = dimof(c, b);
    const dbl4 acc = mfma_tile(tm * 16, tn * 16, db,
        [&](int sidx, int i) { return sel(sidx < R && i < db, Vb[min(i, db - 1) * R + min(sidx, R - 1)]); },
        [&](int i, int r) { return sel(r < R && i < db, Wb[min(i, db - 1) * R + min(r, R - 1)]); });
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int sidx = tm * 16 + 4 * v + kq, r = tn * 16 + r16;
      if (sidx < R && r < R) c.Qb[b * RR + sidx * R + r] = scale ? c.msq[b * R + sidx] * acc[v] : acc[v];
    }
  }
  __syncthreads();
  double dotp = 0.0;
  const int t0 = tiles16(c.d0) * tr, t1 = t0 + tiles16(c.d1) * tr, t2 = t1 + tiles16(c.d2) * tr;
  for (int t = w; t < t2; t += NW) {
    const int a = (t >= t1) ? 2 : (t >= t0 ? 1 : 0);
    const int tt = t - (a == 0 ? 0 : (a == 1 ? t0 : t1));
    const int tm = tt / tr, tn = tt - tm * tr;
    const int da = dimof(c, a);
    const double* Va = V + offof(c, a);
    const double* Wa = c.W + offof(c, a);
    const double* Pa = c.Pown + a * RR;
    const double* ma = c.msq + a * R;
    // Y_a = pi^(b2) * Q_b1 + pi^(b1) * Q_b2 over the other two modes b1 < b2, formed in the loads
    const int b1 = (a == 0) ? 1 : 0, b2 = (a == 2) ? 1 : 2;
    const double* pb1 = c.pi + b1 * RR;
    const double* pb2 = c.pi + b2 * RR;
    const double* qb1 = c.Qb + b1 * RR;
    const double* qb2 = c.Qb + b2 * RR;
    // v_a Pi^(a) then W_a Y_a, accumulated into one tile
    const dbl4 acc1 = mfma_tile(tm * 16, tn * 16, R,
        [&](int i, int k) {
          const int kk = min(k, R - 1);
          const double v = Va[min(i, da - 1) * R + kk];
          return sel(i < da && k < R, scale ? ma[kk] * v : v);
        },
        [&](int k, int r) { return sel(r < R && k < R, Pa[min(k, R - 1) * R + min(r, R - 1)]); });
    const dbl4 acc2 = mfma_tile(tm * 16, tn * 16, R,
        [&](int i, int k) { return sel(i < da && k < R, Wa[min(i, da - 1) * R + min(k, R - 1)]); },
        [&](int k, int r) {
          const int q = min(k, R - 1) * R + min(r, R - 1);
          return sel(r < R && k < R, pb2[q] * qb1[q] + pb1[q] * qb2[q]);
        });
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = tm * 16 + 4 * v + kq, r = tn * 16 + r16;
      if (i < da && r < R) {
        const int e = offof(c, a) + i * R + r;
        double tv = acc1[v] + acc2[v];
        if (scale) tv = ma[r] * (tv + mu * c.gam[a * R + r] * (ma[r] * V[e]));
        else if (mu != 0.0) tv += mu * c.gam[a * R + r] * V[e];
        out[e] = tv;
        dotp += V[e] * tv;
      }
    }
  }
  return dotp;
}

// The same product for a working set in global memory (cores too large for LDS): each mode's
// operands are staged in LDS first with coalesced loads (phase 1: W_b and V_b; phase 2: W_a, the
// scaled V_a, Pi^(a) and the Hadamard combination Y_a), so the MFMA operands come from LDS instead
// of one L2 round trip per k-group.  Same tile products in the same order as hv, bit-identical
// results.  sh holds 2 dmax R + 2 R^2 doubles (hv_stage_doubles).
__device__ double hv_staged(Ctx& c, const double* V, double* out, double mu, bool scale, double* sh) {
  const int R = c.R, RR = R * R, tr = tiles16(R);
  const int tid = threadIdx.x, lane = tid & 63, w = wave_id(), r16 = lane & 15, kq = lane >> 4;
  const int dmax = max(c.d0, max(c.d1, c.d2));
  double* sW = sh;
  double* sV = sh + dmax * R;
  double* sP = sV + dmax * R;
  double* sY = sP + RR;
  for (int b = 0; b < 3; ++b) {
    const int db = dimof(c, b), ob = offof(c, b);
    for (int e = tid; e < db * R; e += NT) {
      sW[e] = c.W[ob + e];
      sV[e] = V[ob + e];
    }
    __syncthreads();
    for (int t = w; t < tr * tr; t += NW) {
      const int tm = t / tr, tn = t - tm * tr;
      const dbl4 acc = mfma_tile(tm * 16, tn * 16, db,
          [&](int sidx, int i) { return sel(sidx < R && i < db, sV[min(i, db - 1) * R + min(sidx, R - 1)]); },
          [&](int i, int r) { return sel(r < R && i < db, sW[min(i, db - 1) * R + min(r, R - 1)]); });
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int sidx = tm * 16 + 4 * v + kq, r = tn * 16 + r16;
        if (sidx < R && r < R) c.Qb[b * RR + sidx * R + r] = scale ? c.msq[b * R + sidx] * acc[v] : acc[v];
      }
    }
    __syncthreads();
  }
  double dotp = 0.0;
  for (int a = 0; a < 3; ++a) {
    const int da = dimof(c, a), oa = offof(c, a);
    const int b1 = (a == 0) ? 1 : 0, b2 = (a == 2) ? 1 : 2;
    const double* ma = c.msq + a * R;
    for (int e = tid; e < da * R; e += NT) {
      sW[e] = c.W[oa + e];
      const double v = V[oa + e];
      sV[e] = scale ? ma[e % R] * v : v;
    }
    for (int e = tid; e < RR; e += NT) {
      sP[e] = c.Pown[a * RR + e];
      sY[e] = c.pi[b2 * RR + e] * c.Qb[b1 * RR + e] + c.pi[b1 * RR + e] * c.Qb[b2 * RR + e];
    }
    __syncthreads();
    for (int t = w; t < tiles16(da) * tr; t += NW) {
      const int tm = t / tr, tn = t - tm * tr;
      const dbl4 acc1 = mfma_tile(tm * 16, tn * 16, R,
          [&](int i, int k) { return sel(i < da && k < R, sV[min(i, da - 1) * R + min(k, R - 1)]); },
          [&](int k, int r) { return sel(r < R && k < R, sP[min(k, R - 1) * R + min(r, R - 1)]); });
      const dbl4 acc2 = mfma_tile(tm * 16, tn * 16, R,
          [&](int i, int k) { return sel(i < da && k < R, sW[min(i, da - 1) * R + min(k, R - 1)]); },
          [&](int k, int r) { return sel(r < R && k < R, sY[min(k, R - 1) * R + min(r, R - 1)]); });
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = tm * 16 + 4 * v + kq, r = tn * 16 + r16;
        if (i < da && r < R) {
          const int e = oa + i * R + r;
          double tv = acc1[v] + acc2[v];
          if (scale) tv = ma[r] * (tv + mu * c.gam[a * R + r] * (ma[r] * V[e]));
          else if (mu != 0.0) tv += mu * c.gam[a * R + r] * V[e];
          out[e] = tv;
          dotp += V[e] * tv;
        }
      }
    }
    __syncthreads();
  }
  return dotp;
}

// Block-Jacobi preconditioner: the diagonal blocks of J^T J + mu D act on block l as
// V^(l) -> V^(l) K_l with K_l = Pi^(l) + mu diag(gamma_l) (ch.3 block structure), split as
// K_l = C_l C_l^T (Cholesky, lower).  C_l goes to Qb (free until the CG products), C_l^{-1} to Ci.
// Column j of C: every thread of the column forms the pivot itself in the same order, so one
// barrier per column suffices.  Needs Pown and gam (precond); ends with a barrier.
__device__ void block_chol(Ctx& c, double mu) {
  const int R = c.R, RR = R * R;
  for (int j = 0; j < R; ++j) {
    for (int e = threadIdx.x; e < 3 * R; e += NT) {
      const int l = e / R, i = e - l * R;
      if (i < j) continue;
      const double* K = c.Pown + l * RR;
      double* C = c.Qb + l * RR;
      double sd = K[j * R + j] + mu * c.gam[l * R + j];
      for (int q = 0; q < j; ++q) sd -= C[j * R + q] * C[j * R + q];
      const double piv = sqrt(sd);
      if (i == j) {
        C[j * R + j] = piv;
      } else {
        double sv = K[i * R + j];
        for (int q = 0; q < j; ++q) sv -= C[i * R + q] * C[j * R + q];
        C[i * R + j] = sv / piv;
      }
    }
    __syncthreads();
  }
  // C^{-1} (lower): column j solves C y = e_j by forward substitution, one thread per (l, j)
  for (int e = threadIdx.x; e < 3 * R; e += NT) {
    const int l = e / R, j = e - l * R;
    const double* C = c.Qb + l * RR;
    double* Y = c.Ci + l * RR;
    for (int i = 0; i < j; ++i) Y[i * R + j] = 0.0;
    Y[j * R + j] = 1.0 / C[j * R + j];
    for (int i = j + 1; i < R; ++i) {
      double sv = 0.0;
      for (int q = j; q < i; ++q) sv += C[i * R + q] * Y[q * R + j];
      Y[i * R + j] = -sv / C[i * R + i];
    }
  }
  __syncthreads();
}

// out_a = sgn In_a C_a^{-1} (trans = false: L^{-T} in vec form) or sgn In_a C_a^{-T} (trans = true:
// L^{-1}), block by block on the matrix cores; out2 (nullable) receives a copy.  Returns this
// thread's partial of <out, out>; ends without a barrier.
__device__ double tri_apply(Ctx& c, const double* In, double* out, bool trans, double sgn, double* out2) {
  const int R = c.R, RR = R * R, tr = tiles16(R);
  const int lane = threadIdx.x & 63, w = wave_id(), r16 = lane & 15, kq = lane >> 4;
  const int t0 = tiles16(c.d0) * tr, t1 = t0 + tiles16(c.d1) * tr, t2 = t1 + tiles16(c.d2) * tr;
  double ss = 0.0;
  for (int t = w; t < t2; t += NW) {
    const int a = (t >= t1) ? 2 : (t >= t0 ? 1 : 0);
    const int tt = t - (a == 0 ? 0 : (a == 1 ? t0 : t1));
    const int tm = tt / tr, tn = tt - tm * tr;
    const int da = dimof(c, a), oa = offof(c, a);
    const double* Ia = In + oa;
    const double* Ca = c.Ci + a * RR;
    const dbl4 acc = mfma_tile(tm * 16, tn * 16, R,
        [&](int i, int k) { return sel(i < da && k < R, Ia[min(i, da - 1) * R + min(k, R - 1)]); },
        [&](int k, int r) {
          const int kk = min(k, R - 1), rr = min(r, R - 1);
          return sel(k < R && r < R, trans ? Ca[rr * R + kk] : Ca[kk * R + rr]);
        });
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = tm * 16 + 4 * v + kq, r = tn * 16 + r16;
      if (i < da && r < R) {
        const int e = oa + i * R + r;
        const double val = sgn * acc[v];
        out[e] = val;
        if (out2) out2[e] = val;
        ss += val * val;
      }
    }
  }
  return ss;
}

// Norm balancing (ch.4 "Updates"): every rank-one term gets equal column norms.  Uses msq as
// scratch for the column norms.  Ends with a barrier.
// fix0: the first factor is held fixed; the rank-one terms are balanced over modes 2 and 3 only,
// alpha_r = sqrt(n_r^(2) n_r^(3)).
__device__ void norm_balance(Ctx& c, bool fix0 = false) {
  const int R = c.R;
  double* cn = c.msq;   // 3R scratch
  for (int e = threadIdx.x; e < 3 * R; e += NT) {
    const int l = e / R, r = e - l * R;
    const double* Wl = c.W + offof(c, l);
    double acc = 0.0;
    for (int i = 0; i < dimof(c, l); ++i) acc += Wl[i * R + r] * Wl[i * R + r];
    cn[e] = sqrt(acc);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < c.np; e += NT) {
    int l, i, r;
    split_index(c, e, l, i, r);
    const double n0 = cn[r], n1 = cn[R + r], n2 = cn[2 * R + r];
    if (fix0) {
      if (l == 0 || fmin(n1, n2) == 0.0) continue;
      const double alpha = sqrt(n1 * n2);
      c.W[e] *= alpha / cn[l * R + r];
      continue;
    }
    if (fmin(n0, fmin(n1, n2)) == 0.0) continue;
    const double alpha = pow(n0 * n1 * n2, 1.0 / 3.0);
    c.W[e] *= alpha / cn[l * R + r];
  }
  __syncthreads();
}

// ||S - [[W]]||^2 and MK = S_(l) KR(others) at the current W (ch.4 "Computing the residual" and
// the MTTKRP of the gradient), on the matrix cores:
//   MK_0 = S_(0) KR(W2, W1) over (j, k);  MK_1 over (i, k);  MK_2 over (i, j);
//   model = W0 KR12^T (d0 x d1 d2), and f = S - model squared and summed in the tile epilogue.
// Returns the block-wide ||f||^2.
__device__ double residual_mttkrp(Ctx& c, double* slots) {
  const int R = c.R, d0 = c.d0, d1 = c.d1, d2 = c.d2, tr = tiles16(R);
  const int d12 = d1 * d2, d02 = d0 * d2, d01 = d0 * d1;
  const double inv1 = 1.0 / d1, inv2 = 1.0 / d2;
  const double* W0 = c.W;
  const double* W1 = c.W + c.off1;
  const double* W2 = c.W + c.off2;
  const double* S = c.S;
  const int sp1 = c.sp1, sp2 = c.sp2;
  const int lane = threadIdx.x & 63, w = wave_id(), r16 = lane & 15, kq = lane >> 4;
  const int n0 = tiles16(d0) * tr, n1 = n0 + tiles16(d1) * tr, n2 = n1 + tiles16(d2) * tr;
  const int nres = tiles16(d0) * tiles16(d12);
  const int R1 = R - 1;
  double f2 = 0.0;
  for (int t = w; t < n2 + nres; t += NW) {
    if (t < n2) {
      const int l = (t >= n1) ? 2 : (t >= n0 ? 1 : 0);
      const int tt = t - (l == 0 ? 0 : (l == 1 ? n0 : n1));
      const int tm = tt / tr, tn = tt - tm * tr;
      const int dl = dimof(c, l);
      dbl4 acc;
      if (l == 0) {
        acc = mfma_tile(tm * 16, tn * 16, d12,
            [&](int i, int jk) {
              const int x = min(jk, d12 - 1), j = div_by(x, inv2), k = x - j * d2;
              return sel(i < d0 && jk < d12, S[min(i, d0 - 1) * sp1 + j * sp2 + k]);
            },
            [&](int jk, int r) {
              const int x = min(jk, d12 - 1), j = div_by(x, inv2), k = x - j * d2, rr = min(r, R1);
              return sel(r < R && jk < d12, W2[k * R + rr] * W1[j * R + rr]);
            });
      } else if (l == 1) {
        acc = mfma_tile(tm * 16, tn * 16, d02,
            [&](int j, int ik) {
              const int x = min(ik, d02 - 1), i = div_by(x, inv2), k = x - i * d2;
              return sel(j < d1 && ik < d02, S[i * sp1 + min(j, d1 - 1) * sp2 + k]);
            },
            [&](int ik, int r) {
              const int x = min(ik, d02 - 1), i = div_by(x, inv2), k = x - i * d2, rr = min(r, R1);
              return sel(r < R && ik < d02, W2[k * R + rr] * W0[i * R + rr]);
            });
      } else {
        acc = mfma_tile(tm * 16, tn * 16, d01,
            [&](int k, int ij) {
              const int x = min(ij, d01 - 1), i = div_by(x, inv1), j = x - i * d1;
              return sel(k < d2 && ij < d01, S[i * sp1 + j * sp2 + min(k, d2 - 1)]);
            },
            [&](int ij, int r) {
              const int x = min(ij, d01 - 1), i = div_by(x, inv1), j = x - i * d1, rr = min(r, R1);
              return sel(r < R && ij < d01, W1[j * R + rr] * W0[i * R + rr]);
            });
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = tm * 16 + 4 * v + kq, r = tn * 16 + r16;
        if (m < dl && r < R) c.MK[offof(c, l) + m * R + r] = acc[v];
      }
    } else {
      const int tt = t - n2, tcols = tiles16(d12);
      const int tm = tt / tcols, tn = tt - tm * tcols;
      const dbl4 acc = mfma_tile(tm * 16, tn * 16, R,
          [&](int i, int r) { return sel(i < d0 && r < R, W0[min(i, d0 - 1) * R + min(r, R1)]); },
          [&](int r, int jk) {
            const int x = min(jk, d12 - 1), j = div_by(x, inv2), k = x - j * d2, rr = min(r, R1);
            return sel(r < R && jk < d12, W1[j * R + rr] * W2[k * R + rr]);
          });
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = tm * 16 + 4 * v + kq, jk = tn * 16 + r16;
        if (i < d0 && jk < d12) {
          const int j = div_by(jk, inv2), k = jk - j * d2;
          const double f = S[i * sp1 + j * sp2 + k] - acc[v];
          f2 += f * f;
        }
      }
    }
  }
  return block_sum(f2, slots);
}

__device__ int stop_test(const double* errs, int k, double step, double grad_inf, double tol,
                         int maxiter, double div_ref) {
  const double err = errs[k];
  if (err < tol) return CPD_STOP_REL_ERR;
  if (step < tol) return CPD_STOP_STEP;
  if (fabs(errs[k - 1] - err) < tol) return CPD_STOP_IMPROVEMENT;
  if (grad_inf < tol) return CPD_STOP_GRAD;
  const int cw = 1 + (maxiter + 9) / 10;
  if (k % cw == 0 && k > 2 * cw) {
    double so = 0.0, sn = 0.0, si = 0.0;
    for (int j = k - 2 * cw + 1; j <= k - cw; ++j) so += errs[j];
    for (int j = k - cw + 1; j <= k; ++j) sn += errs[j];
    const double avg_old = so / cw, avg_new = sn / cw;
    if (avg_old - avg_new < tol) return CPD_STOP_AVG_ERR;
    for (int j = k - cw + 1; j <= k; ++j) si += fabs(errs[j - 1] - errs[j]);
    if (si / cw < 1e-3 * avg_new) return CPD_STOP_AVG_IMPR;
  }
  if (err > div_ref / (1e-16 + tol)) return CPD_STOP_DIVERGED;
  if (k >= maxiter) return CPD_STOP_MAXITER;
  return CPD_STOP_NONE;
}

// mode 0: initialise the state from the W stored in it; mode 1: run up to max_steps iterations;
// mode 2: one iteration up to the balanced update, its residual and MTTKRP left to other
// launches (dgn_tail_kernel finishes the step).
// SL: the core S is copied into LDS after the working set (the caller sized the LDS for it).
// GW: working set in global memory with hv_staged's LDS buffer at `stage`.
// OPT (mode 1, working set in LDS): DGN_OPT_BLOCK, DGN_OPT_DRAWBACK; with DGN_OPT_BLOCK the caller
// sized the LDS for np + 3 R^2 more doubles (block_lds_doubles), placed before the staged core.
// SOLO: a state the host may have modified (cpd_state_factors): honours HDR_DIRTY.
template <bool SL, bool GW = false, int OPT = 0, bool SOLO = false>
__device__ __forceinline__ void dgn_body(char* __restrict__ state, const double* __restrict__ S, int mode, int max_steps,
                         double* lds, int& s_stop, double* stage = nullptr) {
  constexpr int HVM = SOLO ? 0 : 1;   // structured-product path (see hv)
  Hdr* h = (Hdr*)state;
  const int R = h->R;
  int d[3] = {h->d[0], h->d[1], h->d[2]};
  const int maxiter = h->maxiter;
  const int np = (d[0] + d[1] + d[2]) * R;
  const Layout Lo = layout_of(np, R, maxiter);
  double* gW = (double*)(state + Lo.W);
  double* gMK = (double*)(state + Lo.MK);
  Ctx c;
  constexpr bool BLK = (OPT & DGN_OPT_BLOCK) != 0 && !GW;
  constexpr bool DRAW = (OPT & DGN_OPT_DRAWBACK) != 0 && !GW;
  const size_t blk_lds = (BLK && mode == 1) ? block_lds_doubles(np, R) : 0;
  if (SL) {
    // rows of S padded to odd strides (in doubles): the sixteen rows a matrix-core fragment reads
    // then fall into distinct LDS banks
    double* Sl = lds + lds_doubles(np, R) + blk_lds;
    const int p2 = d[2] | 1, p1 = (d[1] * p2) | 1;
    const int n3 = d[0] * d[1] * d[2], d12 = d[1] * d[2];
    for (int e = threadIdx.x; e < n3; e += NT) {
      const int i = e / d12, jk = e - i * d12, j = jk / d[2], k = jk - j * d[2];
      Sl[i * p1 + j * p2 + k] = S[e];
    }
    setup_ctx(c, lds, d, R, Sl, gMK, (double*)(state + Lo.G));
    c.sp1 = p1;
    c.sp2 = p2;
  } else {
    setup_ctx(c, lds, d, R, S, gMK, (double*)(state + Lo.G));
  }
  if (blk_lds) {
    c.U = lds + lds_doubles(np, R);
    c.Ci = c.U + np;
  }
  double* errs = (double*)(state + Lo.errs);
  const int* caps = (const int*)(state + Lo.caps);
  cpd_step_info* logp = (cpd_step_info*)(state + Lo.log);
  const int tid = threadIdx.x;
  double* slotA = c.red;
  double* slotB = c.red + NW;

  for (int e = tid; e < c.np; e += NT) c.W[e] = gW[e];
  const bool fix0 = (h->flags & HDR_FIX0) != 0;
  const bool dirty = SOLO && mode == 1 && (h->flags & HDR_DIRTY) != 0;   // read before any write
  __syncthreads();

  if (mode == 0 || mode == 3) {   // mode 3: the residual and MTTKRP are left to other launches
    // non-finite initial point?
    int bad = 0;
    for (int e = tid; e < c.np; e += NT) bad |= !isfinite(c.W[e]);
    const double nb = block_sum((double)bad, slotA);
    norm_balance(c, fix0);
    // a preset header (refinement on the input tensor) already holds ||S||, mu and the divergence
    // reference: the tensor is not read here
    const bool preset = (h->flags & HDR_PRESET) != 0;
    const int n = d[0] * d[1] * d[2];
    double s2 = 0.0, sa = 0.0;
    if (!preset)
      for (int e = tid; e < n; e += NT) { s2 += S[e] * S[e]; sa += fabs(S[e]); }
    s2 = block_sum(s2, slotB);
    sa = block_sum(sa, slotA);
    const double f2 = (mode == 3) ? 0.0 : residual_mttkrp(c, slotB);
    for (int e = tid; e < c.np; e += NT) gW[e] = c.W[e];
    if (tid == 0) {
      const double s_norm = preset ? h->s_norm : sqrt(s2);
      h->s_norm = s_norm;
      if (!preset) h->mu = h->init_damp * (sa / (double)n);
      h->f2 = f2;
      if (!preset) h->div_ref = fmax(1.0, (h->div_ref > 0.0) ? h->div_ref : s2);
      h->err0 = (s_norm > 0.0) ? sqrt(f2) / s_norm : 0.0;
      errs[0] = h->err0;
      h->k = 0;
      h->tol_iter = -1;
      h->stop = (nb > 0.0) ? -1 : CPD_STOP_NONE;
      h->flags = ((nb > 0.0) ? 1 : 0) | (preset ? HDR_PRESET : 0) | (fix0 ? HDR_FIX0 : 0);
      h->t_init = wall_clock64();
    }
    return;
  }

  double mu = h->mu, f2 = h->f2;
  const double s_norm = h->s_norm, div_ref = h->div_ref, tol = h->tol, cg_tol = h->cg_tol;
  int k = h->k, stop = h->stop, tol_iter = h->tol_iter;
  double err_prev = (k == 0) ? h->err0 : errs[k];
  if (dirty) {
    // factors replaced from outside: residual and MTTKRP at them; mu and the history continue
    f2 = residual_mttkrp(c, slotB);
    if (tid == 0) {
      h->f2 = f2;
      h->flags &= ~HDR_DIRTY;
    }
  }
  const bool blk = BLK && !fix0;
  const bool drawback = DRAW && !fix0;
  __syncthreads();

  // sum over the CG iterations of alpha_j ||r_j||^2 (x^T J^T J x of the step follows from it)
  double aff = 0.0;
  // Gradient and preconditioned CG step at the current W: Grams, D and the preconditioner first;
  // leaves the gradient in G and the step x in X.
  auto direction = [&](int cap, int& its, double& rr, double& grad_inf) __attribute__((always_inline)) {
    its = 0;
    rr = 0.0;
    aff = 0.0;
    grams(c);
    precond(c, mu);
    if constexpr (BLK) {
      if (blk) block_chol(c, mu);
    }
    // gradient; CG start x = 0 and r = p = M^{-1/2}(-grad) (block-Jacobi: L^{-1}(-grad), below).
    // With the working set in global memory, W and the Pi^(l) are staged in LDS first (same
    // values, same order of operations)
    const double* gWs = c.W;
    const double* gPs = c.Pown;
    if constexpr (GW) {
      for (int e = tid; e < c.np; e += NT) stage[e] = c.W[e];
      for (int e = tid; e < 3 * R * R; e += NT) stage[c.np + e] = c.Pown[e];
      __syncthreads();
      gWs = stage;
      gPs = stage + c.np;
    }
    double gi = 0.0;
    for (int e = tid; e < c.np; e += NT) {
      int l, i, r;
      split_index(c, e, l, i, r);
      const double* Wi = gWs + offof(c, l) + i * R;
      const double* Pl = gPs + l * R * R;
      double acc = 0.0;
      for (int s = 0; s < R; ++s) acc += Wi[s] * Pl[s * R + r];
      const double g = (fix0 && l == 0) ? 0.0 : acc - c.MK[e];   // a fixed factor has no step
      c.G[e] = g;
      gi = fmax(gi, fabs(g));
      c.X[e] = 0.0;
      if (!(BLK && blk)) {
        const double r0 = c.msq[l * R + r] * (-g);
        c.Rv[e] = r0;
        c.P[e] = r0;
        rr += r0 * r0;
      }
    }
    if (BLK && blk) {
      __syncthreads();
      rr = tri_apply(c, c.G, c.Rv, true, -1.0, c.P);
    }
    rr = block_sum(rr, slotA);
    grad_inf = block_max(gi, slotB);
    while (its < cap) {
      if (rr == 0.0) break;
      double pz;
      if (BLK && blk) {
        // z = L^{-1} (J^T J + mu D) L^{-T} p through u = L^{-T} p; <p, z> = <u, (J^T J + mu D) u>
        tri_apply(c, c.P, c.U, false, 1.0, nullptr);
        __syncthreads();
        pz = block_sum(hv<HVM>(c, c.U, c.Z, mu, false), slotA);
        tri_apply(c, c.Z, c.U, true, 1.0, nullptr);
        __syncthreads();
      } else {
        pz = block_sum(GW ? hv_staged(c, c.P, c.Z, mu, true, stage) : hv<HVM>(c, c.P, c.Z, mu, true), slotA);
      }
      if (!(pz > 0.0)) break;
      const double alpha = rr / pz;
      aff += alpha * rr;
      const double* Zv = (BLK && blk) ? c.U : c.Z;
      double eps = 0.0;
      const int zfree = fix0 ? c.off1 : 0;   // rows of J^T J v of a fixed factor are dropped
      for (int e = tid; e < c.np; e += NT) {
        c.X[e] += alpha * c.P[e];
        const double rv = c.Rv[e] - alpha * ((e < zfree) ? 0.0 : Zv[e]);
        c.Rv[e] = rv;
        eps += rv * rv;
      }
      eps = block_sum(eps, slotB);
      const double beta = eps / rr;
      for (int e = tid; e < c.np; e += NT) c.P[e] = c.Rv[e] + beta * c.P[e];
      __syncthreads();
      rr = eps;
      ++its;
      if (eps < cg_tol) break;
    }
    if (BLK && blk) {
      // x = L^{-T} x_hat, into U; the two buffers swap roles
      tri_apply(c, c.X, c.U, false, 1.0, nullptr);
      double* t = c.X;
      c.X = c.U;
      c.U = t;
    } else {
      // x = M^{-1/2} x_hat
      for (int e = tid; e < c.np; e += NT) {
        int l, i, r;
        split_index(c, e, l, i, r);
        c.X[e] *= c.msq[l * R + r];
      }
    }
    __syncthreads();
  };

  // Predicted ||f + J x||^2 from the residual f2_base at the start point, then w <- w + x (always
  // accepted) and norm balancing.
  // Predicted residual of the linearisation, the update and the balancing.  For the CG's own step
  // (from_cg) x^T J^T J x comes from the CG coefficients: with A the preconditioned operator, b its
  // right-hand side and x_hat_0 = 0, x_hat^T A x_hat = 2 b^T x_hat - sum_j alpha_j ||r_j||^2 (a
  // relation that persists in finite precision), b^T x_hat = -grad.x and x_hat^T A x_hat =
  // x^T (J^T J + mu D) x; a step changed after the CG (the dogleg) takes the product.
  auto predict_update = [&](double f2_base, double& f2_pred, double& xx, bool from_cg) __attribute__((always_inline)) {
    double xjx = 0.0;
    if (!from_cg)
      xjx = block_sum(GW ? hv_staged(c, c.X, c.Z, 0.0, false, stage) : hv<HVM>(c, c.X, c.Z, 0.0, false), slotA);
    double gx = 0.0, xs = 0.0, xd = 0.0;
    for (int e = tid; e < c.np; e += NT) {
      gx += c.G[e] * c.X[e];
      xs += c.X[e] * c.X[e];
      if (from_cg) {
        int l, i, r;
        split_index(c, e, l, i, r);
        xd += c.gam[l * R + r] * c.X[e] * c.X[e];
      }
    }
    gx = block_sum(gx, slotB);
    xx = block_sum(xs, slotA);
    if (from_cg) xjx = -2.0 * gx - aff - mu * block_sum(xd, slotB);
    f2_pred = f2_base + 2.0 * gx + xjx;
    for (int e = tid; e < c.np; e += NT) c.W[e] += c.X[e];
    __syncthreads();
    norm_balance(c, fix0);
  };

  // Dogleg step inside the radius delta from the Gauss-Newton step in X and the gradient in G
  // (Madsen-Nielsen-Tingleff): X itself if it fits; the steepest-descent step cut at delta when
  // the Cauchy point a = -(|g|^2 / |J g|^2) g lies outside; else a + beta (X - a) on the radius.
  auto dogleg = [&](double delta) __attribute__((always_inline)) {
    const double jg2 =
        block_sum(GW ? hv_staged(c, c.G, c.Z, 0.0, false, stage) : hv<HVM>(c, c.G, c.Z, 0.0, false), slotA);
    double hh = 0.0, gg = 0.0;
    for (int e = tid; e < c.np; e += NT) {
      hh += c.X[e] * c.X[e];
      gg += c.G[e] * c.G[e];
    }
    hh = block_sum(hh, slotB);
    gg = block_sum(gg, slotA);
    if (sqrt(hh) <= delta) return;
    const double alpha = gg / jg2, na = alpha * sqrt(gg);
    if (na >= delta) {
      const double sc = -(delta / sqrt(gg));
      for (int e = tid; e < c.np; e += NT) c.X[e] = sc * c.G[e];
      __syncthreads();
      return;
    }
    double cd = 0.0, dd = 0.0;
    for (int e = tid; e < c.np; e += NT) {
      const double av = -alpha * c.G[e], dv = c.X[e] - av;
      cd += av * dv;
      dd += dv * dv;
    }
    cd = block_sum(cd, slotB);
    dd = block_sum(dd, slotA);
    const double beta = (-cd + sqrt(cd * cd + dd * (delta * delta - na * na))) / dd;
    for (int e = tid; e < c.np; e += NT) {
      const double av = -alpha * c.G[e];
      c.X[e] = av + beta * (c.X[e] - av);
    }
    __syncthreads();
  };

  for (int step_i = 0; step_i < max_steps && stop == CPD_STOP_NONE; ++step_i) {
    ++k;
    int its = 0;
    double rr = 0.0, grad_inf = 0.0, f2_pred = 0.0, xx = 0.0;
    const int cap = caps[k - 1];
    direction(cap, its, rr, grad_inf);
    // the batched kernel keeps the product (its registers are at the limit)
    predict_update(f2, f2_pred, xx, SOLO);
    if (mode == 2) {
      if (tid == 0) {
        h->f2_pred = f2_pred; h->stepn = sqrt(xx); h->grad_inf = grad_inf; h->cg_resid = rr;
        h->its = its; h->cap = cap; h->pending = 1;
      }
      break;
    }
    double f2_new = residual_mttkrp(c, slotB);
    double err = sqrt(f2_new) / s_norm;
    double f2_base = f2;
    int drew = 0;
    if (DRAW && drawback && err > 100.0 * err_prev) {
      // draw back to N(w_k + x) - x, a new step there cut to half the failed one's length
      drew = 1;
      const double delta = 0.5 * sqrt(xx);
      for (int e = tid; e < c.np; e += NT) c.W[e] -= c.X[e];
      __syncthreads();
      f2_base = residual_mttkrp(c, slotB);   // and the MTTKRP of the new gradient
      direction(cap, its, rr, grad_inf);
      dogleg(delta);
      predict_update(f2_base, f2_pred, xx, false);
      f2_new = residual_mttkrp(c, slotB);
      err = sqrt(f2_new) / s_norm;
    }
    const double den = f2_base - f2_pred;
    const double g = (den > 0.0) ? (f2_base - f2_new) / den : 0.0;
    const double mu_new = (g < 0.25) ? 3.0 * mu : ((g > 0.75) ? mu / 3.0 : mu);
    const double stepn = sqrt(xx);
    if (tid == 0) {
      errs[k] = err;
      const int st = stop_test(errs, k, stepn, grad_inf, tol, maxiter, div_ref);
      s_stop = st;
      const long long now = wall_clock64();
      cpd_step_info inf;
      inf.k = k; inf.cg_iters = its; inf.cg_cap = cap; inf.stop = st;
      inf.rel_err = err; inf.step_norm = stepn; inf.grad_inf = grad_inf; inf.gain = g;
      inf.mu = mu_new; inf.cg_resid = rr;
      inf.t_ns = now - h->t_init;   // ticks here; the host converts to ns
      inf.drew_back = drew; inf.reserved = 0;
      logp[k - 1] = inf;
      if (tol_iter < 0 && err < tol) h->t_tol = now;
    }
    __syncthreads();
    stop = s_stop;
    if (tol_iter < 0 && err < tol) tol_iter = k;
    mu = mu_new;
    f2 = f2_new;
    err_prev = err;
  }
  for (int e = tid; e < c.np; e += NT) gW[e] = c.W[e];
  if (tid == 0) {
    h->mu = mu; h->f2 = f2; h->k = k; h->stop = stop; h->tol_iter = tol_iter;
  }
}

// Initialisation (mode 0) and iterations (mode 1) are separate kernels, so that traces and
// counters attribute them separately.
template <bool SL>
__global__ __launch_bounds__(NT) void dgn_init_kernel(char* __restrict__ state, const double* __restrict__ S) {
  extern __shared__ double lds[];
  __shared__ int s_stop;
  dgn_body<SL>(state, S, 0, 0, lds, s_stop);
}

template <bool SL, int OPT>
__global__ __launch_bounds__(NT) void dgn_kernel(char* __restrict__ state, const double* __restrict__ S,
                                                 int max_steps) {
  extern __shared__ double lds[];
  __shared__ int s_stop;
  dgn_body<SL, false, OPT, true>(state, S, 1, max_steps, lds, s_stop);
}

// Same iteration for states too large for LDS: the working set lives in the state's own work
// region (global memory; one workgroup, so its accesses stay coherent through the CU's cache).
// MODE 2 is the first half of one iteration (see dgn_tail_kernel).
// STG: the gradient and J^T J v read their operands from dynamic LDS (hv_stage_doubles).
template <int MODE, bool STG>
__global__ __launch_bounds__(NT) void dgn_kernel_g(char* __restrict__ state, const double* __restrict__ S,
                                                   int max_steps) {
  extern __shared__ double g_stage[];
  __shared__ int s_stop;
  const Hdr* h = (const Hdr*)state;
  const Layout Lo = layout_of(h->np, h->R, h->maxiter);
  dgn_body<false, STG>(state, S, MODE, max_steps, (double*)(state + Lo.work), s_stop, g_stage);
}

// Second half of an iteration split over launches: from the residual ||S - [[W]]||^2 of the
// balanced update (f2_new, computed by the full-tensor kernels on the core, which also refreshed
// the MTTKRP in the state) the error, gain ratio, damping update, stopping tests and log entry.
__device__ void tail_step(char* __restrict__ state) {
  Hdr* h = (Hdr*)state;
  if (h->pending != 1) return;
  h->pending = 0;
  const Layout Lo = layout_of(h->np, h->R, h->maxiter);
  double* errs = (double*)(state + Lo.errs);
  cpd_step_info* logp = (cpd_step_info*)(state + Lo.log);
  const int k = h->k;
  const double f2 = h->f2, f2_new = h->f2_new, mu = h->mu;
  const double err = sqrt(f2_new) / h->s_norm;
  const double den = f2 - h->f2_pred;
  const double g = (den > 0.0) ? (f2 - f2_new) / den : 0.0;
  const double mu_new = (g < 0.25) ? 3.0 * mu : ((g > 0.75) ? mu / 3.0 : mu);
  errs[k] = err;
  const int st = stop_test(errs, k, h->stepn, h->grad_inf, h->tol, h->maxiter, h->div_ref);
  const long long now = wall_clock64();
  cpd_step_info inf;
  inf.k = k; inf.cg_iters = h->its; inf.cg_cap = h->cap; inf.stop = st;
  inf.rel_err = err; inf.step_norm = h->stepn; inf.grad_inf = h->grad_inf; inf.gain = g;
  inf.mu = mu_new; inf.cg_resid = h->cg_resid;
  inf.t_ns = now - h->t_init;   // ticks here; the host converts to ns
  inf.drew_back = 0; inf.reserved = 0;
  logp[k - 1] = inf;
  if (h->tol_iter < 0 && err < h->tol) {
    h->tol_iter = k;
    h->t_tol = now;
  }
  h->mu = mu_new;
  h->f2 = f2_new;
  h->stop = st;
}

__global__ void dgn_tail_kernel(char* __restrict__ state) {
  if (threadIdx.x == 0) tail_step(state);
}

// ---- cooperative CG for cores whose working set lives in global memory -------------------------
// The CG of one dGN iteration (ch.4 Alg. "Conjugate gradient - dGN" on M^{-1/2}(J^T J + mu D)
// M^{-1/2}, the products of Thm Hv) spread over CG_WG workgroups of one cooperative launch, then
// x = M^{-1/2} x_hat and x^T J^T J x (from the CG coefficients) for the epilogue.  Per CG
// iteration j:
//   A: the R x R tiles of Q_b = (M^{-1/2} p_j)_b^T W_b, one tile per wave;            grid barrier
//   B: the tiles of z_j = M^{-1/2}(J^T J + mu D) M^{-1/2} p_j and their <p_j, z_j>, <r_j, z_j>
//      and <z_j, z_j> partials (one set per workgroup);                               grid barrier
//   C: every workgroup adds the partials in workgroup order (same alpha everywhere) and forms
//      ||r_j - alpha z_j||^2 = ||r_j||^2 - 2 alpha <r_j, z_j> + alpha^2 <z_j, z_j> (same beta
//      everywhere), then updates its own slice of x, r_{j+1}, p_{j+1} (r and p double-buffered by
//      the parity of j).
// Phase A of iteration j+1 forms p_{j+1} = r_j - alpha z_j + beta p_j from the parity-j buffers, so
// no barrier is needed after C; B reads the stored p_{j+1}, which the barrier after A publishes.
// Every exit test is taken on values that are identical in all workgroups.
//
// Launch and barrier: an ordinary launch of CG_WG x COOP_STRIDE workgroups, of which every
// COOP_STRIDE-th one works (few enough to be resident together; a cooperative launch measured
// ~23 us of extra latency and slowed the kernels after it).  The barriers up to the one after
// step 2 count arrivals and flip a generation word in a slot of fine-grained device memory, with
// agent-scope fences around each arrival (device-scope atomics on ordinary, coarse-grained memory
// are performed in the L2 of the issuing XCD, which the other XCDs do not see).  Before the one
// after step 2 each workgroup records its hardware XCD; when all share one (the dispatch hands
// workgroups to the eight XCDs in turn), every later barrier is XCD-local: counter and generation
// in ordinary memory with agent-scope atomics, which that XCD's L2 performs; each wave's stores
// are acknowledged by the L2 before the arrival, and the device-scope invalidate after it drops
// the L1 and the L2's clean lines but keeps the dirty lines the workgroups just wrote, with no L2
// write-back (the agent-scope fence's write-back left every CG phase starting from memory).  The
// workgroup-scope invalidate is not enough: the L1 keeps stale lines (wrong CG sums).  Every wait
// is bounded: after BAR_SPINS polls a workgroup records HDR_BAR_TIMEOUT in the header and goes on,
// so every wave reaches the end of the kernel, and the host reports an error.
// workgroups: at R = 50 (48 tiles per phase, one per wave at 6) the 600^3 solve's dGN takes
// 7.27 ms with 6 and 7.35 ms with 8 (memory-coherent barriers throughout: 7.68 ms with 6, 7.79 ms
// with 8, 10.8 ms with 4)
constexpr int CG_WG = 6;
// Partial-sum slots of the multi-workgroup iteration (doubles, after the second r, p and z
// buffers): each group is written before a barrier and read after it, and no group is written
// again until every workgroup has passed a later barrier.
constexpr int SLOT_RR = 0;                          // ||r_0||^2 (CG_WG), then max|g| (CG_WG)
constexpr int SLOT_COL = 2 * CG_WG;                 // column-norm partials, CG_WG x 3R (R <= 64)
constexpr int SLOT_DP = SLOT_COL + CG_WG * 3 * 64;  // <p_j, z_j> by the parity of j (2 CG_WG)
constexpr int SLOT_RZ = SLOT_DP + 2 * CG_WG;        // <r_j, z_j> (CG_WG)
constexpr int SLOT_ZZ = SLOT_RZ + CG_WG;            // <z_j, z_j> (CG_WG)
constexpr int SLOT_XJX = SLOT_ZZ + CG_WG;           // x^T D x (CG_WG)
constexpr int SLOT_GX = SLOT_XJX + CG_WG;           // grad.x and x.x (2 CG_WG)
constexpr int SLOT_END = SLOT_GX + 2 * CG_WG;
constexpr long long BAR_SPINS = 1ll << 22;

struct BarSlot {
  unsigned count;
  unsigned pad0[31];   // count and generation in separate 128-byte lines
  unsigned gen;
  unsigned xcc[8];     // the hardware XCD of each workgroup of the current launch
  unsigned pad1[23];
};
static_assert(CG_WG <= 8, "one XCD id slot per workgroup");

// The iteration kernel runs on every COOP_STRIDE-th workgroup of its launch: workgroups go to the
// eight XCDs in turn, so these normally share one XCD, whose L2 is then their common coherence
// point.  The others leave at once.
constexpr int COOP_STRIDE = 8;
__device__ __forceinline__ int coop_g() { return blockIdx.x / COOP_STRIDE; }
__device__ __forceinline__ int coop_G() { return gridDim.x / COOP_STRIDE; }

// Grid barrier for workgroups on one XCD: counter and generation in ordinary device memory, whose
// agent-scope atomics are performed in that XCD's L2.  Release: every wave waits until its stores
// are acknowledged (the L1 writes through to the L2).  Acquire: a device-scope invalidate, which
// drops the compute unit's L1 and the L2's clean lines and keeps its dirty ones, the data the
// group exchanges; there is no L2 write-back.  Same bounded wait as grid_barrier.
__device__ __forceinline__ void xcd_barrier(BarSlot* b, unsigned nblocks, int* flags) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned g = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // read before this arrival is counted
    const unsigned arrived = __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // the reset lands before the release
      __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long long spins = 0;
      while (__hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > BAR_SPINS) {
          atomicOr(flags, HDR_BAR_TIMEOUT);
          break;
        }
      }
    }
    asm volatile("s_waitcnt vmcnt(0)\n\tbuffer_inv sc1" ::: "memory");
  }
  __syncthreads();
}

__device__ __forceinline__ void grid_barrier(BarSlot* b, unsigned nblocks, int* flags) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();   // this workgroup's writes, visible device-wide (release)
    const unsigned g = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const unsigned arrived = __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_SYSTEM);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    } else {
      long long spins = 0;
      while (__hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > BAR_SPINS) {
          atomicOr(flags, HDR_BAR_TIMEOUT);
          break;
        }
      }
    }
    __threadfence();   // the other workgroups' writes (acquire)
  }
  __syncthreads();
}

// p_{j+1} entry e from the parity-j buffers (alpha = 0, beta = 0 reads p_j itself)
__device__ __forceinline__ double p_next(const double* Rj, const double* Zj, const double* Pj, int e, double alpha,
                                         double beta, int zfree) {
  return (Rj[e] - alpha * ((e < zfree) ? 0.0 : Zj[e])) + beta * Pj[e];
}

// Phase A: the tiles of Q_b = V_b^T W_b (rows scaled by msq when scale) for V given by vf(e), written
// as the two contributions Y_a needs, C[2a + j] = pi^(c) * Q_b for the modes a != b (j = 0 when b is
// the lower of a's other modes, c the third mode), so that phase B reads Y_a = C[2a] + C[2a + 1]
// without pi.  The pi entries are loaded with the tile's operands: one memory round per tile.
template <class VF>
__device__ void coop_phase_a(Ctx& c, double* C, VF vf, bool scale) {
  const int R = c.R, RR = R * R, tr = tiles16(R);
  const int lane = threadIdx.x & 63, w = wave_id(), r16 = lane & 15, kq = lane >> 4;
  const int nA = 3 * tr * tr;
  for (int t = coop_g() * NW + w; t < nA; t += coop_G() * NW) {
    const int b = t / (tr * tr), tt = t - b * tr * tr, tm = tt / tr, tn = tt - tm * tr;
    const int ob = offof(c, b), db = dimof(c, b);
    const double* Wb = c.W + ob;
    // the two modes a != b, and for each the third mode whose pi weighs Q_b
    const int a0 = (b == 0) ? 1 : 0, a1 = (b == 2) ? 1 : 2;
    const int c0 = 3 - b - a0, c1 = 3 - b - a1;
    double pw0[4], pw1[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = min(tm * 16 + 4 * v + kq, R - 1) * R + min(tn * 16 + r16, R - 1);
      pw0[v] = c.pi[c0 * RR + q];
      pw1[v] = c.pi[c1 * RR + q];
    }
    const dbl4 acc = mfma_tile_wide(tm * 16, tn * 16, db,
        [&](int sidx, int i) { return sel(sidx < R && i < db, vf(ob + min(i, db - 1) * R + min(sidx, R - 1))); },
        [&](int i, int r) { return sel(r < R && i < db, Wb[min(i, db - 1) * R + min(r, R - 1)]); });
    // slot of Q_b in Y_{a0} and Y_{a1}: j = 0 when b is the lower other mode of a
    const int j0 = (b == ((a0 == 0) ? 1 : 0)) ? 0 : 1, j1 = (b == ((a1 == 0) ? 1 : 0)) ? 0 : 1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int sidx = tm * 16 + 4 * v + kq, r = tn * 16 + r16;
      if (sidx < R && r < R) {
        const double qv = scale ? c.msq[b * R + sidx] * acc[v] : acc[v];
        const int q = sidx * R + r;
        C[(2 * a0 + j0) * RR + q] = pw0[v] * qv;
        C[(2 * a1 + j1) * RR + q] = pw1[v] * qv;
      }
    }
  }
}

// Phase B: out = the scaled (or plain) structured product of V (stored), tile by tile; returns this
// thread's partial of <V, out>.  Every global operand of a tile (the V and W fragments, the two
// contributions of Y_a at the B-fragment positions, V at the outputs) is loaded before its first
// product, so a tile costs one memory round; Pi^(a), M^{-1/2} and D come from LDS.  R <= 64: the
// contraction over R is a single 64-deep slice.
// With Rv (the stored r_j) also this thread's partials of <r_j, z> and <z, z> over the entries past
// zfree, from which every workgroup forms ||r_j - alpha z||^2 = ||r_j||^2 - 2 alpha <r_j, z> +
// alpha^2 <z, z> without a pass over the whole vector.
__device__ double coop_phase_b(Ctx& c, const double* C, const double* V, double* out, double mu, bool scale,
                               const double* Rv = nullptr, double* rz = nullptr, double* zz = nullptr,
                               int zfree = 0) {
  const int R = c.R, RR = R * R, tr = tiles16(R);
  const int lane = threadIdx.x & 63, w = wave_id(), r16 = lane & 15, kq = lane >> 4;
  const int t0 = tiles16(c.d0) * tr, t1 = t0 + tiles16(c.d1) * tr, t2 = t1 + tiles16(c.d2) * tr;
  double dotp = 0.0;
  for (int t = coop_g() * NW + w; t < t2; t += coop_G() * NW) {
    const int a = (t >= t1) ? 2 : (t >= t0 ? 1 : 0);
    const int tt = t - (a == 0 ? 0 : (a == 1 ? t0 : t1));
    const int tm = tt / tr, tn = tt - tm * tr;
    const int da = dimof(c, a), oa = offof(c, a);
    const double* Va = V + oa;
    const double* Wa = c.W + oa;
    const double* Pa = c.Pown + a * RR;
    const double* ma = c.msq + a * R;
    const double* ya0 = C + (2 * a) * RR;
    const double* ya1 = C + (2 * a + 1) * RR;
    const int irow = tm * 16 + r16, ic = min(irow, da - 1);
    const int rcol = tn * 16 + r16, rc = min(rcol, R - 1);
    double va[16], wa[16], y0[16], y1[16], ve[4], re[4];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int kc = min(4 * u + kq, R - 1);
      va[u] = Va[ic * R + kc];
      wa[u] = Wa[ic * R + kc];
      y0[u] = ya0[kc * R + rc];
      y1[u] = ya1[kc * R + rc];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = min(tm * 16 + 4 * v + kq, da - 1) * R + rc;
      ve[v] = Va[q];
      re[v] = Rv ? Rv[oa + q] : 0.0;
    }
    dbl4 acc1 = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = 4 * u + kq, kc = min(k, R - 1);
      const bool okA = irow < da && k < R, okB = rcol < R && k < R;
      const double a1 = sel(okA, scale ? ma[kc] * va[u] : va[u]);
      const double b1 = sel(okB, Pa[kc * R + rc]);
      const double a2 = sel(okA, wa[u]);
      const double b2 = sel(okB, y0[u] + y1[u]);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc1, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, b2, acc2, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = tm * 16 + 4 * v + kq, r = rcol;
      if (i < da && r < R) {
        const int e = oa + i * R + r;
        double tv = acc1[v] + acc2[v];
        if (scale) tv = ma[r] * (tv + mu * c.gam[a * R + r] * (ma[r] * ve[v]));
        out[e] = tv;
        dotp += ve[v] * tv;
        if (Rv && e >= zfree) {
          *rz += re[v] * tv;
          *zz += tv * tv;
        }
      }
    }
  }
  return dotp;
}

// Column-norm scratch of the iteration kernel's step 5: the M^{-1/2} slots, no longer needed then.
__device__ __forceinline__ double* slots_cn(Ctx& c) { return c.msq; }

// Sum of the per-workgroup partials in workgroup order (the same value in every workgroup).
__device__ __forceinline__ double sum_parts(const double* part, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  return s;
}

// One dGN iteration (ch.4 "dGN") of a core whose working set lives in global memory, on CG_WG
// workgroups: everything but the core's residual and MTTKRPs (the full-tensor kernels compute them
// next from the updated factors) and the scalar tail.  The factors are read and updated in the
// state's W region; Pi, M^{-1/2} and D sit in each workgroup's LDS.
//   1. pi^(l) = W^(l)T W^(l) tiles (one per wave), unless the previous launch left them; barrier
//   2. every workgroup: Pi^(l), the gammas and M^{-1/2}; gradient W Pi - MTTKRP on its own slice of
//      the parameter vector, r_0 = p_0 = M^{-1/2}(-grad), x = 0; partials of ||r_0||^2, max|g|; barrier
//   3. the CG described above;
//   4. own slice: x = M^{-1/2} x_hat, grad.x, x.x and x^T D x partials, w <- w + x and that
//      slice's part of every column norm; barrier (x^T J^T J x then follows from the CG coefficients)
//   5. every workgroup: the column norms (partials added in workgroup order), norm balancing of its
//      slice; workgroup 0 writes the step's values to the header for the tail.
// Dynamic LDS: 3 R^2 + 6 R doubles.
__global__ __launch_bounds__(NT) void dgn_iter_coop_kernel(char* __restrict__ state, double* __restrict__ P1,
                                                           double* __restrict__ R1, double* __restrict__ part,
                                                           BarSlot* __restrict__ bar, BarSlot* __restrict__ xbar,
                                                           int grams_ready) {
  extern __shared__ double lds_c[];
  __shared__ double slots[2][NW];
  __shared__ int s_same_xcd;
  if (blockIdx.x % COOP_STRIDE) return;
  Hdr* h = (Hdr*)state;
  if (h->stop != CPD_STOP_NONE) return;   // the header is the same for every workgroup
  int* hflags = &h->flags;
  const unsigned nblk = coop_G();
  // the barriers up to the one after step 2 are the memory-coherent kind; each workgroup publishes
  // its XCD before that one, and when all share one XCD the later barriers are XCD-local (the same
  // decision in every workgroup)
  bool same_xcd = false;
  auto sync_all = [&]() {
    if (same_xcd)
      xcd_barrier(xbar, nblk, hflags);
    else
      grid_barrier(bar, nblk, hflags);
  };
  const int R = h->R, RR = R * R;
  const int d[3] = {h->d[0], h->d[1], h->d[2]};
  const int np = (d[0] + d[1] + d[2]) * R;
  const Layout Lo = layout_of(np, R, h->maxiter);
  Ctx c;
  setup_ctx(c, (double*)(state + Lo.work), d, R, nullptr, (double*)(state + Lo.MK), (double*)(state + Lo.G));
  c.W = (double*)(state + Lo.W);
  // the work region's Pi and Q areas (adjacent, 6 R^2) hold phase A's contributions to Y
  double* Cy = c.Pown;
  c.Pown = lds_c;
  c.msq = lds_c + 3 * RR;
  c.gam = c.msq + 3 * R;
  const int* caps = (const int*)(state + Lo.caps);
  const bool fix0 = (h->flags & HDR_FIX0) != 0;
  const int zfree = fix0 ? c.off1 : 0;
  const double mu = h->mu, cg_tol = h->cg_tol;
  const int k = h->k + 1;
  const int cap = caps[k - 1];
  const int G = coop_G(), g = coop_g(), tid = threadIdx.x;
  const int chunk = (np + G - 1) / G, e0 = g * chunk, e1 = min(np, e0 + chunk);
  const int tr = tiles16(R);
  const int lane = tid & 63, w = wave_id(), r16 = lane & 15, kq = lane >> 4;

  // 1. factor Grams (unless the previous launch, core_finish_kernel, left them in the state)
  if (!grams_ready) {
  for (int t = g * NW + w; t < 3 * tr * tr; t += G * NW) {
    const int l = t / (tr * tr), tt = t - l * tr * tr, tm = tt / tr, tn = tt - tm * tr;
    const double* Wl = c.W + offof(c, l);
    const int dl = dimof(c, l);
    const dbl4 acc = mfma_tile_wide(tm * 16, tn * 16, dl,
        [&](int r, int i) { return sel(r < R && i < dl, Wl[min(i, dl - 1) * R + min(r, R - 1)]); },
        [&](int i, int q) { return sel(q < R && i < dl, Wl[min(i, dl - 1) * R + min(q, R - 1)]); });
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = tm * 16 + 4 * v + kq, q = tn * 16 + r16;
      if (r < R && q < R) c.pi[l * RR + r * R + q] = acc[v];
    }
  }
  sync_all();
  }
  // 2. Pi, D, M^{-1/2} (each workgroup for itself, same values), gradient and CG start on the slice
  for (int e = tid; e < RR; e += NT) {
    const double a = c.pi[e], b = c.pi[RR + e], dd = c.pi[2 * RR + e];
    c.Pown[e] = b * dd;
    c.Pown[RR + e] = a * dd;
    c.Pown[2 * RR + e] = a * b;
  }
  __syncthreads();
  precond(c, mu);
  double rr = 0.0, gi = 0.0;
  for (int e = e0 + tid; e < e1; e += NT) {
    int l, i, r;
    split_index(c, e, l, i, r);
    const double* Wi = c.W + offof(c, l) + i * R;
    const double* Pl = c.Pown + l * RR;
    double acc = 0.0;
    for (int s2 = 0; s2 < R; ++s2) acc += Wi[s2] * Pl[s2 * R + r];
    const double gv = (fix0 && l == 0) ? 0.0 : acc - c.MK[e];   // a fixed factor has no step
    c.G[e] = gv;
    gi = fmax(gi, fabs(gv));
    const double r0 = c.msq[l * R + r] * (-gv);
    c.Rv[e] = r0;
    c.P[e] = r0;
    c.X[e] = 0.0;
    rr += r0 * r0;
  }
  rr = block_sum(rr, slots[0]);
  gi = block_max(gi, slots[1]);
  if (tid == 0) {
    part[g] = rr;
    part[G + g] = gi;
    unsigned x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    __hip_atomic_store(&bar->xcc[g], x & 0xfu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  grid_barrier(bar, nblk, hflags);
  if (tid == 0) {
    const unsigned x0 = __hip_atomic_load(&bar->xcc[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    int same = 1;
    for (unsigned i = 1; i < nblk; ++i)
      same &= __hip_atomic_load(&bar->xcc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) == x0;
    s_same_xcd = same;
  }
  __syncthreads();
  same_xcd = __builtin_amdgcn_readfirstlane(s_same_xcd) != 0;
  rr = sum_parts(part, G);
  double grad_inf = 0.0;
  for (int q = 0; q < G; ++q) grad_inf = fmax(grad_inf, part[G + q]);

  // 3. CG
  double* Pb[2] = {c.P, P1};
  double* Rb[2] = {c.Rv, R1};
  int its = 0, par = 0;
  double alpha = 0.0, beta = 0.0;   // of the previous CG iteration (p_0 is stored)
  double aff = 0.0;                 // sum over the CG iterations of alpha_j ||r_j||^2
  bool first = true;
  while (its < cap) {
    if (rr == 0.0) break;
    const double* Rj = Rb[par];
    const double* Pj = Pb[par];
    // A: Q from p_j (p_0 stored; later p_j formed from the previous parity's buffers)
    {
      const double* Rq = Rb[par ^ 1];
      const double* Pq = Pb[par ^ 1];
      const double* Zq = c.Z;
      const double al = alpha, be = beta;
      if (first)
        coop_phase_a(c, Cy, [&](int e) { return Pj[e]; }, true);
      else
        coop_phase_a(c, Cy, [&](int e) { return p_next(Rq, Zq, Pq, e, al, be, zfree); }, true);
    }
    sync_all();
    // B: z_j, and the partials of <p_j, z_j>, <r_j, z_j> and <z_j, z_j>
    double rzp = 0.0, zzp = 0.0;
    const double dp = block_sum(coop_phase_b(c, Cy, Pj, c.Z, mu, true, Rj, &rzp, &zzp, zfree), slots[0]);
    rzp = block_sum(rzp, slots[1]);
    zzp = block_sum(zzp, slots[0]);
    if (tid == 0) {
      part[SLOT_DP + g] = dp;
      part[SLOT_RZ + g] = rzp;
      part[SLOT_ZZ + g] = zzp;
    }
    sync_all();
    const double pz = sum_parts(part + SLOT_DP, G);
    if (!(pz > 0.0)) break;
    alpha = rr / pz;
    aff += alpha * rr;
    // C: ||r_j - alpha z_j||^2 from the partials (the same in every workgroup; rounding can only
    // make a vanishing value slightly negative, read as 0), own slice update
    const double rzs = sum_parts(part + SLOT_RZ, G), zzs = sum_parts(part + SLOT_ZZ, G);
    const double eps = fmax(rr - 2.0 * alpha * rzs + alpha * alpha * zzs, 0.0);
    beta = eps / rr;
    double* Rn = Rb[par ^ 1];
    double* Pn = Pb[par ^ 1];
#pragma unroll 2
    for (int e = e0 + tid; e < e1; e += NT) {
      c.X[e] += alpha * Pj[e];
      const double rv = Rj[e] - alpha * ((e < zfree) ? 0.0 : c.Z[e]);
      Rn[e] = rv;
      Pn[e] = rv + beta * Pj[e];
    }
    rr = eps;
    ++its;
    par ^= 1;
    first = false;
    if (eps < cg_tol) break;
  }
  // 4. own slice (no barrier before it: after the last barrier of the CG every workgroup reads and
  // writes only its own slice): x = M^{-1/2} x_hat, grad.x, x.x, x^T D x, the update, and the
  // slice's share of every column norm.  x^T J^T J x needs no product of its own: with A the CG
  // operator, b = -M^{-1/2} grad its right-hand side and x_hat_0 = 0, the CG iterates satisfy
  // x_hat^T A x_hat = 2 b^T x_hat - sum_j alpha_j ||r_j||^2 (a relation that persists in finite
  // precision), b^T x_hat = -grad.x, and x_hat^T A x_hat = x^T (J^T J + mu D) x.
  double gx = 0.0, xx = 0.0, xdx = 0.0;
  for (int e = e0 + tid; e < e1; e += NT) {
    int l, i, r;
    split_index(c, e, l, i, r);
    const double xv = c.X[e] * c.msq[l * R + r];
    c.X[e] = xv;
    gx += c.G[e] * xv;
    xx += xv * xv;
    xdx += c.gam[l * R + r] * xv * xv;
    c.W[e] += xv;
  }
  gx = block_sum(gx, slots[0]);
  xx = block_sum(xx, slots[1]);
  xdx = block_sum(xdx, slots[0]);
  double* colp = part + SLOT_COL;   // CG_WG rows of 3R column partials
  for (int q = tid; q < 3 * R; q += NT) {
    const int l = q / R, r = q - l * R;
    const int ol = offof(c, l), dl = dimof(c, l);
    // rows i of mode l whose entry ol + i R + r lies in [e0, e1)
    int ib = (e0 - ol - r + R - 1) / R;
    if (e0 <= ol + r) ib = 0;
    double acc = 0.0;
    for (int i = ib; i < dl; ++i) {
      const int e = ol + i * R + r;
      if (e >= e1) break;
      acc += c.W[e] * c.W[e];
    }
    colp[g * 3 * R + q] = acc;
  }
  if (tid == 0) {
    part[SLOT_GX + g] = gx;
    part[SLOT_GX + G + g] = xx;
    part[SLOT_XJX + g] = xdx;
  }
  sync_all();
  // 5. column norms, balancing of the own slice, header
  gx = sum_parts(part + SLOT_GX, G);
  xx = sum_parts(part + SLOT_GX + G, G);
  xdx = sum_parts(part + SLOT_XJX, G);
  const double xjx = -2.0 * gx - aff - mu * xdx;
  double* cn = slots_cn(c);   // 3R doubles of LDS (reuses msq: no longer needed)
  for (int q = tid; q < 3 * R; q += NT) {
    double s2 = 0.0;
    for (int q2 = 0; q2 < G; ++q2) s2 += colp[q2 * 3 * R + q];
    cn[q] = sqrt(s2);
  }
  __syncthreads();
  for (int e = e0 + tid; e < e1; e += NT) {
    int l, i, r;
    split_index(c, e, l, i, r);
    const double n0 = cn[r], n1 = cn[R + r], n2 = cn[2 * R + r];
    if (fix0) {
      if (l == 0 || fmin(n1, n2) == 0.0) continue;
      c.W[e] *= sqrt(n1 * n2) / cn[l * R + r];
      continue;
    }
    if (fmin(n0, fmin(n1, n2)) == 0.0) continue;
    c.W[e] *= pow(n0 * n1 * n2, 1.0 / 3.0) / cn[l * R + r];
  }
  if (g == 0 && tid == 0) {
    h->f2_pred = h->f2 + 2.0 * gx + xjx;
    h->stepn = sqrt(xx);
    h->grad_inf = grad_inf;
    h->cg_resid = rr;
    h->its = its;
    h->cap = cap;
    h->pending = 1;
    h->k = k;
  }
}

// Finishes an initialisation whose residual ||S - [[W]]||^2 (into f2_new) and MTTKRP (into the
// state's MK) were computed by the full-tensor kernels on the core.
__device__ void tail_init(char* __restrict__ state) {
  Hdr* h = (Hdr*)state;
  const Layout Lo = layout_of(h->np, h->R, h->maxiter);
  double* errs = (double*)(state + Lo.errs);
  h->f2 = h->f2_new;
  h->err0 = (h->s_norm > 0.0) ? sqrt(h->f2_new) / h->s_norm : 0.0;
  errs[0] = h->err0;
  h->t_init = wall_clock64();
}

__global__ void dgn_init_tail_kernel(char* __restrict__ state) {
  if (threadIdx.x == 0) tail_init(state);
}

// ---- residual and MTTKRPs of a large core in two launches ----------------------------------------
// For an FP64 core whose dGN working set exceeds LDS, the MTTKRPs MK_l = S_(l) KR(other factors)
// of the next gradient (ch.4 gradient theorem) and ||S - [[W]]||^2 (ch.4 residual) come from one
// launch of independent wave items on the FP64 matrix cores:
//   MTTKRP items: a 16x16 tile of MK_l over a chunk of CR_KC contraction indices (Khatri-Rao rows
//     formed in the loads), written as a partial tile;
//   residual items: a 16x16 tile of the model W^(1) (W^(2) kr W^(3))^T (contraction over R, one
//     64-deep slice), whose squared differences with S are summed per wave.
// core_finish_kernel adds the partials in a fixed order into MK and f2_new and runs the step's
// tail (or the initialisation's), so a dGN iteration of a large core is three launches.
constexpr int CR_KC = 256;

struct CoreGeom {
  int d0, d1, d2, R, tr;
  int ns[3];        // contraction chunks per mode
  int base[3];      // first partial tile of each mode
  int nm;           // MTTKRP items (= partial tiles)
  int nres;         // residual items
  double inv1, inv2;
};

__host__ __device__ inline CoreGeom core_geom(const int d[3], int R) {
  CoreGeom g;
  g.d0 = d[0]; g.d1 = d[1]; g.d2 = d[2]; g.R = R; g.tr = (R + 15) / 16;
  const long long K[3] = {(long long)d[1] * d[2], (long long)d[0] * d[2], (long long)d[0] * d[1]};
  int b = 0;
  for (int l = 0; l < 3; ++l) {
    g.ns[l] = (int)((K[l] + CR_KC - 1) / CR_KC);
    g.base[l] = b;
    b += ((d[l] + 15) / 16) * g.tr * g.ns[l];
  }
  g.nm = b;
  g.nres = ((d[0] + 15) / 16) * (int)(((long long)d[1] * d[2] + 15) / 16);
  g.inv1 = 1.0 / d[1];
  g.inv2 = 1.0 / d[2];
  return g;
}

__global__ __launch_bounds__(NT) void core_refresh_kernel(const double* __restrict__ S, const double* __restrict__ W,
                                                          CoreGeom g, double* __restrict__ mpart,
                                                          double* __restrict__ rpart, const Hdr* __restrict__ h) {
  // a stopped solve's W is unchanged: nothing to recompute (iterations enqueued past the stop)
  if (h->stop != CPD_STOP_NONE) return;
  const int item = blockIdx.x * NW + wave_id();
  if (item >= g.nm + g.nres) return;
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  const int R = g.R, R1 = R - 1, d0 = g.d0, d1 = g.d1, d2 = g.d2, d12 = d1 * d2;
  const double* W0 = W;
  const double* W1 = W + d0 * R;
  const double* W2 = W + (d0 + d1) * R;
  if (item < g.nm) {
    const int l = item >= g.base[2] ? 2 : (item >= g.base[1] ? 1 : 0);
    const int loc = item - g.base[l];
    const int ns = g.ns[l];
    const int tile = loc / ns, sp = loc - tile * ns;
    const int tm = tile / g.tr, tn = tile - tm * g.tr;
    const int dl = l == 0 ? d0 : (l == 1 ? d1 : d2);
    const int K = l == 0 ? d12 : (l == 1 ? d0 * d2 : d0 * d1);
    const int kb = sp * CR_KC, kn = min(CR_KC, K - kb);
    dbl4 acc;
    if (l == 0) {
      acc = mfma_tile_wide(tm * 16, tn * 16, kn,
          [&](int i, int x) {
            const int xx = kb + min(x, kn - 1);
            return sel(i < d0 && x < kn, S[(long long)min(i, d0 - 1) * d12 + xx]);
          },
          [&](int x, int r) {
            const int xx = kb + min(x, kn - 1), j = div_by(xx, g.inv2), k = xx - j * d2, rr = min(r, R1);
            return sel(r < R && x < kn, W1[j * R + rr] * W2[k * R + rr]);
          });
    } else if (l == 1) {
      acc = mfma_tile_wide(tm * 16, tn * 16, kn,
          [&](int j, int x) {
            const int xx = kb + min(x, kn - 1), i = div_by(xx, g.inv2), k = xx - i * d2;
            return sel(j < d1 && x < kn, S[(long long)i * d12 + min(j, d1 - 1) * d2 + k]);
          },
          [&](int x, int r) {
            const int xx = kb + min(x, kn - 1), i = div_by(xx, g.inv2), k = xx - i * d2, rr = min(r, R1);
            return sel(r < R && x < kn, W0[i * R + rr] * W2[k * R + rr]);
          });
    } else {
      acc = mfma_tile_wide(tm * 16, tn * 16, kn,
          [&](int k, int x) {
            const int xx = kb + min(x, kn - 1);
            return sel(k < d2 && x < kn, S[(long long)xx * d2 + min(k, d2 - 1)]);
          },
          [&](int x, int r) {
            const int xx = kb + min(x, kn - 1), i = div_by(xx, g.inv1), j = xx - i * d1, rr = min(r, R1);
            return sel(r < R && x < kn, W0[i * R + rr] * W1[j * R + rr]);
          });
    }
    double* out = mpart + (long long)item * 256;
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(4 * v + kq) * 16 + r16] = acc[v];
    (void)dl;
    return;
  }
  // residual item: rows tm of mode 1 times columns tn of the (j, k) index
  const int it = item - g.nm;
  const int tcols = (d12 + 15) / 16;
  const int tm = it / tcols, tn = it - tm * tcols;
  double sv[4];
  const int x = tn * 16 + r16, xc = min(x, d12 - 1);
#pragma unroll
  for (int v = 0; v < 4; ++v) sv[v] = S[(long long)min(tm * 16 + 4 * v + kq, d0 - 1) * d12 + xc];
  const dbl4 acc = mfma_tile_wide(tm * 16, tn * 16, R,
      [&](int i, int r) { return sel(i < d0 && r < R, W0[min(i, d0 - 1) * R + min(r, R1)]); },
      [&](int r, int xx) {
        const int xcl = min(xx, d12 - 1), j = div_by(xcl, g.inv2), k = xcl - j * d2, rr = min(r, R1);
        return sel(r < R && xx < d12, W1[j * R + rr] * W2[k * R + rr]);
      });
  double f2 = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = tm * 16 + 4 * v + kq;
    if (i < d0 && x < d12) {
      const double f = sv[v] - acc[v];
      f2 += f * f;
    }
  }
  f2 = wave_sum(f2);
  if (lane == 0) rpart[it] = f2;
}

// MK from the partial tiles and f2_new from the residual partials (fixed orders), then the tail of
// the step (init = 0) or of the initialisation (init = 1): workgroup 0 adds the residual partials
// and runs the tail (which reads no MK), the others one entry of MK per thread.
__global__ __launch_bounds__(NT) void core_finish_kernel(char* __restrict__ state, CoreGeom g,
                                                         const double* __restrict__ mpart,
                                                         const double* __restrict__ rpart, int init) {
  __shared__ double slots[NW];
  Hdr* h = (Hdr*)state;
  const int R = g.R;
  // (a stopped state has an unchanged W: its MK is recomputed unchanged, and tail_step returns on
  // pending == 0; workgroup 0 alone reads and clears pending)
  if (blockIdx.x == 0) {
    double f2 = 0.0;
    for (int it = threadIdx.x; it < g.nres; it += NT) f2 += rpart[it];
    f2 = block_sum(f2, slots);
    if (threadIdx.x == 0) {
      h->f2_new = f2;
      if (init) tail_init(state); else tail_step(state);
    }
    return;
  }
  const Layout Lo = layout_of(h->np, R, h->maxiter);
  const int np = (g.d0 + g.d1 + g.d2) * R;
  const int nmk = (np + NT - 1) / NT;   // workgroups 1..nmk: MTTKRP entries; then the Grams
  if ((int)blockIdx.x > nmk) {
    // pi^(l) = W^(l)T W^(l) of the factors this step's residual was taken at, for the next
    // iteration launch (one 16x16 tile per wave)
    const int d[3] = {g.d0, g.d1, g.d2};
    Ctx c;
    setup_ctx(c, (double*)(state + Lo.work), d, R, nullptr, nullptr, nullptr);
    const double* W = (const double*)(state + Lo.W);
    const int tr = g.tr, lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
    const int t = ((int)blockIdx.x - 1 - nmk) * NW + wave_id();
    if (t >= 3 * tr * tr) return;
    const int l = t / (tr * tr), tt = t - l * tr * tr, tm = tt / tr, tn = tt - tm * tr;
    const double* Wl = W + offof(c, l);
    const int dl = dimof(c, l);
    const dbl4 acc = mfma_tile_wide(tm * 16, tn * 16, dl,
        [&](int r, int i) { return sel(r < R && i < dl, Wl[min(i, dl - 1) * R + min(r, R - 1)]); },
        [&](int i, int q) { return sel(q < R && i < dl, Wl[min(i, dl - 1) * R + min(q, R - 1)]); });
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = tm * 16 + 4 * v + kq, q = tn * 16 + r16;
      if (r < R && q < R) c.pi[l * R * R + r * R + q] = acc[v];
    }
    return;
  }
  double* MK = (double*)(state + Lo.MK);
  int e = (blockIdx.x - 1) * NT + threadIdx.x;
  if (e >= np) return;
  const int n0 = g.d0 * R, n1 = g.d1 * R;
  const int l = e >= n0 + n1 ? 2 : (e >= n0 ? 1 : 0);
  const int el = e - (l == 0 ? 0 : (l == 1 ? n0 : n0 + n1));
  const int i = el / R, r = el - i * R, ns = g.ns[l];
  const int tile = (i >> 4) * g.tr + (r >> 4);
  const double* p = mpart + ((long long)g.base[l] + (long long)tile * ns) * 256 + (i & 15) * 16 + (r & 15);
  double acc = 0.0;
  for (int sp = 0; sp < ns; ++sp) acc += p[(long long)sp * 256];
  MK[e] = acc;
}

// The fused launches serve tensors up to CR_MAXN entries (compressed cores; larger tensors, met by a
// refinement on the input, take the full-tensor kernels).
constexpr long long CR_MAXN = 1ll << 22;

bool core_fused(const int d[3], int sdtype) {
  return sdtype == CPD_F64 && (long long)d[0] * d[1] * d[2] <= CR_MAXN;
}

size_t core_refresh_bytes(const int d[3], int R) {
  if ((long long)d[0] * d[1] * d[2] > CR_MAXN) return 0;
  const CoreGeom g = core_geom(d, R);
  return align_up(((size_t)g.nm * 256 + (size_t)g.nres) * sizeof(double), 256);
}

// Batched: workgroup b initialises state b (header, caps and W already written) and iterates it
// to a stopping rule.  Dynamic LDS must cover the largest member.
__global__ __launch_bounds__(NT) void dgn_batch_kernel(char* const* __restrict__ states,
                                                       const double* const* __restrict__ S, int n) {
  extern __shared__ double lds[];
  __shared__ int s_stop;
  const int b = blockIdx.x;
  if (b >= n) return;
  char* st = states[b];
  if (((const Hdr*)st)->flags & 2) return;   // member rejected (zero or non-finite tensor)
  dgn_body<false>(st, S[b], 0, 0, lds, s_stop);
  __syncthreads();
  const int maxiter = ((const Hdr*)st)->maxiter;
  dgn_body<false>(st, S[b], 1, maxiter, lds, s_stop);
}

// MLSVD-energy initial point (ch.4 "Initialization"): the R entries of largest |s| (ties: smallest
// C-order index) placed on canonical vectors; W^(1) carries the value.  Extra columns (R larger
// than the core) come from `extra` (packed like W) when given.
__global__ __launch_bounds__(256) void smart_init_kernel(const double* __restrict__ S, int d0, int d1,
                                                         int d2, int R, const double* __restrict__ extra,
                                                         double* __restrict__ W) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  __shared__ int chosen[64];
  const int tid = threadIdx.x;
  const int n = d0 * d1 * d2, np = (d0 + d1 + d2) * R;
  for (int e = tid; e < np; e += 256) W[e] = extra ? extra[e] : 0.0;
  __syncthreads();
  const int take = min(R, n);
  for (int t = 0; t < take; ++t) {
    double best = -1.0;
    int besti = 0;   // stays a valid index if every entry is NaN
    for (int e = tid; e < n; e += 256) {
      bool used = false;
      for (int u = 0; u < t; ++u) used |= (chosen[u] == e);
      if (used) continue;
      const double a = fabs(S[e]);
      if (a > best || (a == best && e < besti)) { best = a; besti = e; }
    }
    bv[tid] = best; bi[tid] = besti;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) {
        const double a = bv[tid + s];
        const int ia = bi[tid + s];
        if (a > bv[tid] || (a == bv[tid] && ia < bi[tid])) { bv[tid] = a; bi[tid] = ia; }
      }
      __syncthreads();
    }
    if (tid == 0) chosen[t] = bi[0];
    __syncthreads();
  }
  if (tid < take) {
    const int r = tid, e = chosen[r];
    const int i = e / (d1 * d2), j = (e / d2) % d1, k = e % d2;
    for (int x = 0; x < d0; ++x) W[x * R + r] = 0.0;
    for (int x = 0; x < d1; ++x) W[d0 * R + x * R + r] = 0.0;
    for (int x = 0; x < d2; ++x) W[(d0 + d1) * R + x * R + r] = 0.0;
    W[i * R + r] = S[e];
    W[d0 * R + j * R + r] = 1.0;
    W[(d0 + d1) * R + k * R + r] = 1.0;
  }
}

// N(0,1) entries by Box-Muller on SplitMix64 counters.
// A new state's header and CG caps, built on the host and passed by value, are written by one
// kernel together with a given start: setting up a state needs no host copy and no
// synchronisation.  Up to SETUP_CAPS dGN iterations; longer runs copy the caps from the host.
constexpr int SETUP_CAPS = 512;
struct SetupArgs {
  Hdr h;
  int32_t caps[SETUP_CAPS];
};
static_assert(sizeof(SetupArgs) <= 3072, "setup arguments must fit the kernel argument segment");
static_assert(sizeof(Hdr) % 4 == 0, "header copied in 4-byte words");

__global__ __launch_bounds__(256) void state_setup_kernel(const SetupArgs a, int ncaps, char* __restrict__ st,
                                                          size_t caps_off, const double* __restrict__ W0,
                                                          double* __restrict__ gW, int nw) {
  if (blockIdx.x == 0) {
    const int32_t* hw = reinterpret_cast<const int32_t*>(&a.h);
    int32_t* dh = reinterpret_cast<int32_t*>(st);
    for (int i = threadIdx.x; i < (int)(sizeof(Hdr) / 4); i += 256) dh[i] = hw[i];
    int32_t* dc = reinterpret_cast<int32_t*>(st + caps_off);
    for (int i = threadIdx.x; i < ncaps; i += 256) dc[i] = a.caps[i];
  }
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nw; i += gridDim.x * 256) gW[i] = W0[i];
}

__global__ void randn_kernel(double* W, int n, uint64_t seed) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const uint64_t a = splitmix64(seed * 0x9E3779B97F4A7C15ull + 2 * (uint64_t)e);
  const uint64_t b = splitmix64(seed * 0x9E3779B97F4A7C15ull + 2 * (uint64_t)e + 1);
  const double u1 = 1.0 - u01_from_bits(a), u2 = u01_from_bits(b);
  W[e] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Standalone J^T J v (ch.3 Thm Hv) for parity tests; one workgroup.
__global__ __launch_bounds__(NT) void jtjv_kernel(const double* W0, const double* W1, const double* W2,
                                                  const double* V0, const double* V1, const double* V2,
                                                  int d0, int d1, int d2, int R, double* O0, double* O1,
                                                  double* O2) {
  extern __shared__ double lds[];
  Ctx c;
  int d[3] = {d0, d1, d2};
  setup_ctx(c, lds, d, R, nullptr, nullptr, nullptr);
  const double* Ws[3] = {W0, W1, W2};
  const double* Vs[3] = {V0, V1, V2};
  double* Os[3] = {O0, O1, O2};
  for (int e = threadIdx.x; e < c.np; e += NT) {
    int l, i, r;
    split_index(c, e, l, i, r);
    c.W[e] = Ws[l][i * R + r];
    c.X[e] = Vs[l][i * R + r];
  }
  __syncthreads();
  grams(c);
  hv(c, c.X, c.Z, 0.0, false);
  __syncthreads();
  for (int e = threadIdx.x; e < c.np; e += NT) {
    int l, i, r;
    split_index(c, e, l, i, r);
    Os[l][i * R + r] = c.Z[e];
  }
}

constexpr size_t LDS_LIMIT = 160 * 1024 - 1024;   // dynamic LDS available next to the static slots

bool lds_fits(int np, int R, size_t* bytes) {
  const size_t b = lds_doubles(np, R) * sizeof(double);
  if (bytes) *bytes = b;
  return b <= LDS_LIMIT;
}

}  // namespace

int cg_cap_for(int k, double u) {
  // exact ceilings: smallest m with m^5 >= k^2 and smallest m with m^10 >= k^9
  auto ceil_pow = [](long long kk, int p, int q) {
    unsigned __int128 target = 1;
    for (int i = 0; i < p; ++i) target *= (unsigned __int128)kk;
    long long m = (long long)floor(pow((double)kk, (double)p / q));
    m = m > 2 ? m - 2 : 0;
    for (;; ++m) {
      unsigned __int128 v = 1;
      for (int i = 0; i < q; ++i) v *= (unsigned __int128)m;
      if (v >= target) return m;
    }
  };
  const long long lo = 1 + ceil_pow(k, 2, 5);
  const long long hi = 2 + ceil_pow(k, 9, 10);
  const long long n = hi - lo + 1;
  long long off = (long long)floor(u * (double)n);
  if (off > n - 1) off = n - 1;
  if (off < 0) off = 0;
  return (int)(lo + off);
}

size_t full_aux_bytes(const int d[3], int R);
size_t full_kernels_aux_bytes(const int d[3], int R);
size_t coop_cg_bytes(int np);

namespace {
// Barrier slots of the multi-workgroup CG: per device one pool of fine-grained device memory (the
// memory-coherent barrier) and one of ordinary device memory (the XCD-local one), allocated and
// zeroed on first use and held until the process ends (both barriers leave a slot's count at zero,
// so it needs no reset between launches).  A host thread keeps its own slot: calls on one thread
// are ordered (every solve synchronises), and different threads never share one.
constexpr int BAR_POOL = 256;
constexpr int BAR_MAX_DEVICES = 64;
BarSlot* g_bar_pool[BAR_MAX_DEVICES];
BarSlot* g_xbar_pool[BAR_MAX_DEVICES];
std::mutex g_bar_mu;
std::atomic<int> g_bar_next{0};

cpd_status barrier_slot(BarSlot** out, BarSlot** xout) {
  int dev = 0;
  CPD_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= BAR_MAX_DEVICES) {
    set_error("dgn: device %d beyond %d", dev, BAR_MAX_DEVICES);
    return CPD_E_UNSUPPORTED;
  }
  static thread_local int slot = -1;
  if (slot < 0) slot = g_bar_next.fetch_add(1) % BAR_POOL;
  std::lock_guard<std::mutex> lk(g_bar_mu);
  if (g_bar_pool[dev] == nullptr) {
    void* p = nullptr;
    hipError_t e = hipExtMallocWithFlags(&p, sizeof(BarSlot) * BAR_POOL, hipDeviceMallocFinegrained);
    if (e == hipSuccess) e = hipMemset(p, 0, sizeof(BarSlot) * BAR_POOL);
    if (e != hipSuccess) {
      set_error("dgn: barrier pool allocation failed: %s", hipGetErrorString(e));
      return CPD_E_HIP;
    }
    g_bar_pool[dev] = (BarSlot*)p;
  }
  if (g_xbar_pool[dev] == nullptr) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(BarSlot) * BAR_POOL);
    if (e == hipSuccess) e = hipMemset(p, 0, sizeof(BarSlot) * BAR_POOL);
    if (e != hipSuccess) {
      set_error("dgn: barrier pool allocation failed: %s", hipGetErrorString(e));
      return CPD_E_HIP;
    }
    g_xbar_pool[dev] = (BarSlot*)p;
  }
  *out = g_bar_pool[dev] + slot;
  *xout = g_xbar_pool[dev] + slot;
  return CPD_OK;
}
}  // namespace

namespace {
// Two pinned header slots and two events per host thread for the pipelined stop test of the
// multi-workgroup dGN, created on first use on the thread's current device and held until the
// process ends; nullptr (the synchronous test) when they cannot be had or the thread has moved to
// another device.  Calls on one thread are ordered, so one pair per thread suffices.
struct HeaderSlots {
  Hdr* h[2];
  hipEvent_t ev[2];
  int dev;
};
HeaderSlots* header_slots() {
  static thread_local HeaderSlots hs = {};
  static thread_local int state = 0;   // 0 untried, 1 ready, -1 unavailable
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  if (state == 0) {
    state = -1;
    void* p = nullptr;
    if (hipHostMalloc(&p, 2 * sizeof(Hdr), hipHostMallocPortable) == hipSuccess) {
      hs.h[0] = (Hdr*)p;
      hs.h[1] = hs.h[0] + 1;
      if (hipEventCreateWithFlags(&hs.ev[0], hipEventDisableTiming) == hipSuccess &&
          hipEventCreateWithFlags(&hs.ev[1], hipEventDisableTiming) == hipSuccess) {
        hs.dev = dev;
        state = 1;
      }
    }
    if (state < 0) (void)hipGetLastError();
  }
  return state == 1 && hs.dev == dev ? &hs : nullptr;
}
}  // namespace

namespace {
// LDS of the staged large-core kernel: hv_staged's operands, or W and the three Pi^(l) for the
// gradient, whichever is larger
size_t hv_stage_doubles(const int d[3], int R) {
  const int dmax = d[0] > d[1] ? (d[0] > d[2] ? d[0] : d[2]) : (d[1] > d[2] ? d[1] : d[2]);
  const size_t hvs = 2 * (size_t)dmax * R + 2 * (size_t)R * R;
  const size_t grs = (size_t)(d[0] + d[1] + d[2]) * R + 3 * (size_t)R * R;
  return hvs > grs ? hvs : grs;
}

// The persistent dGN kernel with its working set in LDS when it fits, else in the state's work
// region.
// sdtype: element type of S (FP64 for a core; the input tensor's type for a refinement, which also
// forces the global-memory path since the LDS paths read S as FP64).
// The iteration kernel instantiated for the options (the plain one carries no code of the others).
template <bool SL>
auto dgn_kernel_for(int opts) -> void (*)(char*, const double*, int) {
  switch (opts & (DGN_OPT_BLOCK | DGN_OPT_DRAWBACK)) {
    case DGN_OPT_BLOCK: return dgn_kernel<SL, DGN_OPT_BLOCK>;
    case DGN_OPT_DRAWBACK: return dgn_kernel<SL, DGN_OPT_DRAWBACK>;
    case DGN_OPT_BLOCK | DGN_OPT_DRAWBACK: return dgn_kernel<SL, DGN_OPT_BLOCK | DGN_OPT_DRAWBACK>;
    default: return dgn_kernel<SL, 0>;
  }
}

// known_maxiter >= 0: the header was just written by state_init with that maxiter and no factors
// replaced since, so the large-core path takes both from the caller instead of a blocking read.
cpd_status launch_dgn(char* state, const void* Sv, int mode, int max_steps, int np, int R, const int d[3],
                      hipStream_t s, int sdtype = CPD_F64, int opts = 0, int known_maxiter = -1) {
  const double* S = (const double*)Sv;
  const bool lds_ok = sdtype == CPD_F64;
  const int p2 = d[2] | 1, p1 = (d[1] * p2) | 1;
  const size_t s_lds = (size_t)(d[0] - 1) * p1 + (size_t)(d[1] - 1) * p2 + d[2];   // padded core in LDS
  if (mode == 0) opts = 0;
  // the block-Jacobi factors and one more vector sit between the working set and the staged core
  const size_t extra = (opts & DGN_OPT_BLOCK) ? block_lds_doubles(np, R) * sizeof(double) : 0;
  size_t lb;
  const bool fits = lds_ok && lds_fits(np, R, &lb);
  if (fits && lb + extra + (size_t)s_lds * sizeof(double) <= LDS_LIMIT) {
    lb += extra + (size_t)s_lds * sizeof(double);
    if (mode == 0) {
      CPD_HIP_CHECK(hipFuncSetAttribute((const void*)dgn_init_kernel<true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lb));
      hipLaunchKernelGGL(dgn_init_kernel<true>, dim3(1), dim3(NT), lb, s, state, S);
    } else {
      const auto kern = dgn_kernel_for<true>(opts);
      CPD_HIP_CHECK(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lb));
      hipLaunchKernelGGL(kern, dim3(1), dim3(NT), lb, s, state, S, max_steps);
    }
  } else if (fits && lb + extra <= LDS_LIMIT) {
    lb += extra;
    if (mode == 0) {
      CPD_HIP_CHECK(hipFuncSetAttribute((const void*)dgn_init_kernel<false>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lb));
      hipLaunchKernelGGL(dgn_init_kernel<false>, dim3(1), dim3(NT), lb, s, state, S);
    } else {
      const auto kern = dgn_kernel_for<false>(opts);
      CPD_HIP_CHECK(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lb));
      hipLaunchKernelGGL(kern, dim3(1), dim3(NT), lb, s, state, S, max_steps);
    }
  } else if (fits || (mode != 0 && opts != 0)) {
    set_error("dgn: the block-Jacobi preconditioner and the draw-back run on cores whose working set fits "
              "in one workgroup's LDS (np = %d, R = %d)", np, R);
    return CPD_E_UNSUPPORTED;
  } else {
    // Large core: the MTTKRPs and the residual run over the chip, on the fused core launches
    // (core_refresh_kernel + core_finish_kernel, which also runs the tail) or, for tensors too large
    // for them or not FP64 (a refinement on the input), on the full-tensor kernels and a one-thread
    // tail.  Initialisation: the single-workgroup part (balancing, norms, header), then those.  Each
    // iteration: the multi-workgroup half (Grams, gradient, CG, update), then those; the host checks
    // the stop flag after every few iterations.
    const int64_t dims[3] = {d[0], d[1], d[2]};
    Hdr hh{};
    if (known_maxiter >= 0) {
      hh.maxiter = known_maxiter;   // flags: no HDR_DIRTY
    } else {
      CPD_HIP_CHECK(hipMemcpyAsync(&hh, state, sizeof(Hdr), hipMemcpyDeviceToHost, s));
      CPD_HIP_CHECK(hipStreamSynchronize(s));
    }
    const Layout Lo = layout_of(np, R, hh.maxiter);
    const double* Wp[3] = {(const double*)(state + Lo.W), (const double*)(state + Lo.W) + d[0] * R,
                           (const double*)(state + Lo.W) + (d[0] + d[1]) * R};
    double* MK = (double*)(state + Lo.MK);
    double* MKp[3] = {MK, MK + d[0] * R, MK + (d[0] + d[1]) * R};
    char* aux = state + align_up(Lo.total, 256);
    const size_t aux_bytes = full_kernels_aux_bytes(d, R);   // the cooperative CG's buffers follow
    double* f2_new = (double*)(state + offsetof(Hdr, f2_new));
    // the fused core launches' partials follow the cooperative CG's buffers
    const bool fused = core_fused(d, sdtype);
    const CoreGeom cg = core_geom(d, R);
    double* mpart = (double*)(aux + aux_bytes + coop_cg_bytes(np));
    double* rpart = mpart + (size_t)cg.nm * 256;
    const int cr_blocks = (cg.nm + cg.nres + NW - 1) / NW;
    // residual and MTTKRPs at the current W, then the step's (or the initialisation's) tail
    auto refresh = [&](int init) -> cpd_status {
      if (fused) {
        hipLaunchKernelGGL(core_refresh_kernel, dim3(cr_blocks), dim3(NT), 0, s, S, (const double*)(state + Lo.W),
                           cg, mpart, rpart, (const Hdr*)state);
        CPD_LAUNCH_CHECK();
        const int fin_blocks = 1 + (np + NT - 1) / NT + (3 * cg.tr * cg.tr + NW - 1) / NW;
        hipLaunchKernelGGL(core_finish_kernel, dim3(fin_blocks), dim3(NT), 0, s, state, cg, (const double*)mpart,
                           (const double*)rpart, init);
        CPD_LAUNCH_CHECK();
        return CPD_OK;
      }
      cpd_status st;
      for (int l = 0; l < 3; ++l)
        if ((st = mttkrp_full(Sv, sdtype, dims, Wp, R, l, CPD_F64, MKp[l], aux, aux_bytes, s))) return st;
      if ((st = residual_full(Sv, sdtype, dims, Wp, R, f2_new, aux, aux_bytes, s))) return st;
      if (init)
        hipLaunchKernelGGL(dgn_init_tail_kernel, dim3(1), dim3(64), 0, s, state);
      else
        hipLaunchKernelGGL(dgn_tail_kernel, dim3(1), dim3(64), 0, s, state);
      CPD_LAUNCH_CHECK();
      return CPD_OK;
    };
    if (mode == 0) {
      hipLaunchKernelGGL((dgn_kernel_g<3, false>), dim3(1), dim3(NT), 0, s, state, S, max_steps);
      CPD_LAUNCH_CHECK();
      return refresh(1);
    }
    // the fused refresh leaves the Grams of the current factors in the state; the first launch after
    // replaced factors (or after the full-tensor kernels) forms them itself
    int grams_ready = (fused && !(hh.flags & HDR_DIRTY)) ? 1 : 0;
    if (hh.flags & HDR_DIRTY) {
      // factors replaced from outside: MTTKRP and residual at them, then clear the flag
      cpd_status st;
      for (int l = 0; l < 3; ++l)
        if ((st = mttkrp_full(Sv, sdtype, dims, Wp, R, l, CPD_F64, MKp[l], aux, aux_bytes, s))) return st;
      if ((st = residual_full(Sv, sdtype, dims, Wp, R, (double*)(state + offsetof(Hdr, f2)), aux, aux_bytes, s)))
        return st;
      const int32_t fl = hh.flags & ~HDR_DIRTY;
      CPD_HIP_CHECK(hipMemcpyAsync(state + offsetof(Hdr, flags), &fl, sizeof(fl), hipMemcpyHostToDevice, s));
      CPD_HIP_CHECK(hipStreamSynchronize(s));
    }
    // Pi, M^{-1/2} and D of the iteration kernel in LDS
    const size_t it_lds = ((size_t)3 * R * R + 6 * (size_t)R) * sizeof(double);
    if (it_lds > 64 * 1024)
      CPD_HIP_CHECK(hipFuncSetAttribute((const void*)dgn_iter_coop_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)it_lds));
    // buffers of the multi-workgroup iteration behind the full-tensor kernels' workspace
    double* cbuf = (double*)(aux + aux_bytes);
    double* cP1 = cbuf;
    double* cR1 = cbuf + np;
    double* cpart = cbuf + 2 * (size_t)np;
    BarSlot *bar = nullptr, *xbar = nullptr;
    cpd_status bst = barrier_slot(&bar, &xbar);
    if (bst) return bst;
    // Chunks of CHUNK iterations; the stop test reads the header after each chunk.  With the
    // pinned slots the copy of chunk c's header is waited for only once chunk c + 1 is enqueued,
    // so the device never idles on the host (a chunk enqueued past the stop returns at once).
    constexpr int CHUNK = 4;
    HeaderSlots* hs = header_slots();
    int pending = -1;   // chunk whose header copy is in flight
    for (int done = 0, c = 0; done < max_steps; done += CHUNK, ++c) {
      const int n = (max_steps - done < CHUNK) ? max_steps - done : CHUNK;
      for (int j = 0; j < n; ++j) {
        // Grams, gradient, CG, x^T J^T J x and the balanced update on CG_WG workgroups
        hipLaunchKernelGGL(dgn_iter_coop_kernel, dim3(CG_WG * COOP_STRIDE), dim3(NT), it_lds, s, state, cP1, cR1,
                           cpart, bar, xbar, grams_ready);
        CPD_LAUNCH_CHECK();
        grams_ready = fused ? 1 : 0;
        cpd_status st;
        if ((st = refresh(0))) return st;
      }
      if (done + n >= max_steps) break;
      if (hs == nullptr) {
        CPD_HIP_CHECK(hipMemcpyAsync(&hh, state, sizeof(Hdr), hipMemcpyDeviceToHost, s));
        CPD_HIP_CHECK(hipStreamSynchronize(s));
        if (hh.stop != CPD_STOP_NONE) break;
        continue;
      }
      CPD_HIP_CHECK(hipMemcpyAsync(hs->h[c & 1], state, sizeof(Hdr), hipMemcpyDeviceToHost, s));
      CPD_HIP_CHECK(hipEventRecord(hs->ev[c & 1], s));
      if (pending >= 0) {
        CPD_HIP_CHECK(hipEventSynchronize(hs->ev[pending & 1]));
        if (hs->h[pending & 1]->stop != CPD_STOP_NONE) break;
      }
      pending = c;
    }
    return CPD_OK;
  }
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}
}  // namespace

// Workspace of the full-tensor kernels that take over the core's residual and MTTKRPs when the
// working set does not fit in LDS (0 otherwise); it follows the state's own regions.
size_t dgn_aux_bytes(const int d[3], int R) {
  const int np = (d[0] + d[1] + d[2]) * R;
  if (lds_fits(np, R, nullptr)) return 0;
  return full_aux_bytes(d, R);
}

size_t full_aux_bytes(const int d[3], int R) {
  return full_kernels_aux_bytes(d, R) + coop_cg_bytes((d[0] + d[1] + d[2]) * R) + core_refresh_bytes(d, R);
}

// The multi-workgroup iteration's second r and p buffers and its per-workgroup partials.
size_t coop_cg_bytes(int np) {
  return align_up(((size_t)2 * np + SLOT_END) * sizeof(double), 256);
}

size_t full_kernels_aux_bytes(const int d[3], int R) {
  const int64_t dims[3] = {d[0], d[1], d[2]};
  size_t b = residual_ws_bytes(dims);
  for (int l = 0; l < 3; ++l) {
    const size_t m = mttkrp_ws_bytes(dims, R, l);
    if (m > b) b = m;
  }
  return align_up(b, 256);
}

size_t state_bytes(const int32_t core[3], int R, int maxiter) {
  const int np = (core[0] + core[1] + core[2]) * R;
  const int d[3] = {core[0], core[1], core[2]};
  return align_up(layout_of(np, R, maxiter).total, 256) + dgn_aux_bytes(d, R);
}

cpd_status state_init(void* state, const double* S, const int32_t core[3], int R,
                      const double* W0, double t_norm2, const cpd_params* p, hipStream_t s, bool check_flags,
                      int32_t hdr_flags) {
  if (state == nullptr || S == nullptr || p == nullptr || R < 1 || R > 64 || p->maxiter < 1) {
    set_error("state_init: bad arguments (R=%d)", R);
    return CPD_E_INVALID;
  }
  for (int l = 0; l < 3; ++l)
    if (core[l] < 1 || core[l] > 4096) {
      set_error("state_init: bad core dim %d", core[l]);
      return CPD_E_INVALID;
    }
  const int np = (core[0] + core[1] + core[2]) * R;
  const Layout Lo = layout_of(np, R, p->maxiter);
  char* st = (char*)state;
  double* gW = (double*)(st + Lo.W);
  // header and caps on the host
  const bool inline_args = p->maxiter <= SETUP_CAPS;
  std::vector<int32_t> caps_long(inline_args ? 0 : p->maxiter);
  SetupArgs a;
  memset(&a, 0, sizeof(a));
  Hdr& h = a.h;
  h.d[0] = core[0]; h.d[1] = core[1]; h.d[2] = core[2]; h.R = R;
  h.maxiter = p->maxiter; h.np = np; h.tol_iter = -1;
  h.tol = p->tol; h.cg_tol = (p->cg_tol > 0.0) ? p->cg_tol : p->tol;
  h.init_damp = p->init_damp; h.div_ref = t_norm2;
  h.flags = hdr_flags;
  int32_t* caps = inline_args ? a.caps : caps_long.data();
  for (int k = 1; k <= p->maxiter; ++k) {
    if (p->cg_fixed > 0) {
      caps[k - 1] = p->cg_fixed;
    } else {
      const double u = p->cg_uniforms ? p->cg_uniforms[k - 1]
                                      : u01_from_bits(splitmix64(p->seed * 0xD1B54A32D192ED03ull + (uint64_t)k));
      caps[k - 1] = cg_cap_for(k, u);
    }
  }
  // a given start is copied by the same kernel
  const bool given = p->init != CPD_INIT_MLSVD && W0 != nullptr;
  const int nw = given ? np : 0;
  int nb = (nw + 255) / 256;
  nb = nb < 1 ? 1 : (nb > 256 ? 256 : nb);
  if (inline_args) {
    hipLaunchKernelGGL(state_setup_kernel, dim3(nb), dim3(256), 0, s, a, p->maxiter, st, Lo.caps, W0, gW, nw);
    CPD_LAUNCH_CHECK();
  } else {
    // long runs: the caps from host memory; the synchronisation keeps the host buffers alive
    // until the copies have read them
    hipError_t ce = hipMemcpyAsync(st, &h, sizeof(h), hipMemcpyHostToDevice, s);
    if (ce == hipSuccess)
      ce = hipMemcpyAsync(st + Lo.caps, caps, sizeof(int32_t) * p->maxiter, hipMemcpyHostToDevice, s);
    if (ce == hipSuccess) ce = hipStreamSynchronize(s);
    if (ce != hipSuccess) {
      set_error("state_init: copy failed: %s", hipGetErrorString(ce));
      return CPD_E_HIP;
    }
    if (given) {
      hipLaunchKernelGGL(state_setup_kernel, dim3(nb), dim3(256), 0, s, a, 0, st, Lo.caps, W0, gW, nw);
      CPD_LAUNCH_CHECK();
    }
  }
  if (p->init == CPD_INIT_MLSVD) {
    hipLaunchKernelGGL(smart_init_kernel, dim3(1), dim3(256), 0, s, S, core[0], core[1], core[2],
                       R, W0, gW);
    CPD_LAUNCH_CHECK();
    if (W0 == nullptr && R > core[0] * core[1] * core[2]) {
      set_error("state_init: MLSVD init with R > prod(core) needs W0 for the extra columns");
      return CPD_E_INVALID;
    }
  } else if (W0 != nullptr) {
    // copied above
  } else if (p->init == CPD_INIT_RANDOM) {
    hipLaunchKernelGGL(randn_kernel, dim3((np + 255) / 256), dim3(256), 0, s, gW, np, p->seed);
    CPD_LAUNCH_CHECK();
  } else {
    set_error("state_init: CPD_INIT_GIVEN needs W0");
    return CPD_E_INVALID;
  }
  cpd_status lst;
  const int dc[3] = {core[0], core[1], core[2]};
  if ((lst = launch_dgn(st, S, 0, 0, np, R, dc, s, CPD_F64, 0, p->maxiter))) return lst;
  if (!check_flags) return CPD_OK;
  int flags = 0;
  CPD_HIP_CHECK(hipMemcpyAsync(&flags, st + offsetof(Hdr, flags), sizeof(int), hipMemcpyDeviceToHost, s));
  CPD_HIP_CHECK(hipStreamSynchronize(s));
  if (flags & 1) {
    set_error("state_init: non-finite initial factors");
    return CPD_E_NONFINITE;
  }
  return CPD_OK;
}

// ---- refinement on the input tensor -----------------------------------------------------------
// A state over the input tensor's dimensions that always takes the global-memory path (the
// full-tensor MTTKRP and residual read the tensor in its own dtype).
size_t refine_state_bytes(const int64_t dims[3], int R, int n_iters) {
  const int d[3] = {(int)dims[0], (int)dims[1], (int)dims[2]};
  const int np = (d[0] + d[1] + d[2]) * R;
  return align_up(layout_of(np, R, n_iters).total, 256) + full_aux_bytes(d, R);
}

size_t refine_w_offset(const int64_t dims[3], int R, int n_iters) {
  const int np = (int)(dims[0] + dims[1] + dims[2]) * R;
  return layout_of(np, R, n_iters).W;
}

// Header and CG caps of a refinement: n_iters further iterations continuing the compressed run
// (its damping parameter mu and iteration count k0: iteration j uses the cap of iteration k0 + j),
// errors relative to ||T|| = sqrt(t_norm2).  The caller then writes the start W~ into the state
// (refine_w_offset) and calls refine_run.
cpd_status refine_setup(void* state, const int64_t dims[3], int R, int n_iters, double t_norm2, double mu, int k0,
                        const cpd_params* p, hipStream_t s) {
  if (n_iters < 1 || n_iters > SETUP_CAPS || R < 1 || R > 64 || !(t_norm2 > 0.0)) {
    set_error("refine: bad arguments (iterations %d, R %d)", n_iters, R);
    return CPD_E_INVALID;
  }
  const int np = (int)(dims[0] + dims[1] + dims[2]) * R;
  const Layout Lo = layout_of(np, R, n_iters);
  SetupArgs a;
  memset(&a, 0, sizeof(a));
  Hdr& h = a.h;
  h.d[0] = (int)dims[0]; h.d[1] = (int)dims[1]; h.d[2] = (int)dims[2]; h.R = R;
  h.maxiter = n_iters; h.np = np; h.tol_iter = -1;
  h.tol = p->tol; h.cg_tol = (p->cg_tol > 0.0) ? p->cg_tol : p->tol;
  h.init_damp = p->init_damp;
  h.div_ref = fmax(1.0, t_norm2);
  h.s_norm = sqrt(t_norm2);
  h.mu = mu;
  h.flags = HDR_PRESET;
  for (int j = 1; j <= n_iters; ++j) {
    const int k = k0 + j;
    if (p->cg_fixed > 0) {
      a.caps[j - 1] = p->cg_fixed;
    } else {
      const int ku = (p->cg_uniforms && k > p->maxiter) ? p->maxiter : k;
      const double u = p->cg_uniforms ? p->cg_uniforms[ku - 1]
                                      : u01_from_bits(splitmix64(p->seed * 0xD1B54A32D192ED03ull + (uint64_t)k));
      a.caps[j - 1] = cg_cap_for(k, u);
    }
  }
  hipLaunchKernelGGL(state_setup_kernel, dim3(1), dim3(256), 0, s, a, n_iters, (char*)state, Lo.caps,
                     (const double*)nullptr, (double*)nullptr, 0);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

// Initialisation (balancing, residual and MTTKRP on T) and up to n_iters iterations.
cpd_status refine_run(void* state, const void* T, int dtype, const int64_t dims[3], int R, int n_iters,
                      hipStream_t s) {
  const int d[3] = {(int)dims[0], (int)dims[1], (int)dims[2]};
  const int np = (d[0] + d[1] + d[2]) * R;
  cpd_status st;
  if ((st = launch_dgn((char*)state, T, 0, 0, np, R, d, s, dtype))) return st;
  prof_begin(CPD_PK_DGN, s);
  st = launch_dgn((char*)state, T, 1, n_iters, np, R, d, s, dtype);
  prof_end(CPD_PK_DGN, s);
  return st;
}

size_t dgn_lds_bytes(int np, int R) { return lds_doubles(np, R) * sizeof(double); }

cpd_status fill_randn(double* W, int n, uint64_t seed, hipStream_t s) {
  if (n <= 0) return CPD_OK;
  hipLaunchKernelGGL(randn_kernel, dim3((n + 255) / 256), dim3(256), 0, s, W, n, seed);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

cpd_status dgn_batch_prepare(size_t lds_bytes) {
  if (lds_bytes > LDS_LIMIT) {
    set_error("dgn batch: a member needs %zu bytes of LDS", lds_bytes);
    return CPD_E_UNSUPPORTED;
  }
  CPD_HIP_CHECK(hipFuncSetAttribute((const void*)dgn_batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds_bytes));
  return CPD_OK;
}

cpd_status dgn_batch_launch(char* const* states, const double* const* S, int n, size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL(dgn_batch_kernel, dim3(n), dim3(NT), lds_bytes, s, states, S, n);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

cpd_status dgn_iterate(void* state, const double* S, int max_steps, hipStream_t s, int opts) {
  Hdr h;
  CPD_HIP_CHECK(hipMemcpyAsync(&h, state, sizeof(h), hipMemcpyDeviceToHost, s));
  CPD_HIP_CHECK(hipStreamSynchronize(s));
  if (h.R < 1 || h.np != (h.d[0] + h.d[1] + h.d[2]) * h.R) {
    set_error("dgn_iterate: state not initialised");
    return CPD_E_INVALID;
  }
  prof_begin(CPD_PK_DGN, s);
  const int dc[3] = {h.d[0], h.d[1], h.d[2]};
  const cpd_status st = launch_dgn((char*)state, S, 1, max_steps, h.np, h.R, dc, s, CPD_F64, opts);
  prof_end(CPD_PK_DGN, s);
  return st;
}

cpd_status dgn_iterate_known(void* state, const double* S, const int32_t core[3], int R, int max_steps,
                             hipStream_t s, int opts) {
  const int np = (core[0] + core[1] + core[2]) * R;
  const int dc[3] = {core[0], core[1], core[2]};
  prof_begin(CPD_PK_DGN, s);
  const cpd_status st = launch_dgn((char*)state, S, 1, max_steps, np, R, dc, s, CPD_F64, opts, max_steps);
  prof_end(CPD_PK_DGN, s);
  return st;
}

cpd_status state_read(void* state, int* k, int* stop, int* tol_iter, double* err, hipStream_t s) {
  Hdr h;
  CPD_HIP_CHECK(hipMemcpyAsync(&h, state, sizeof(h), hipMemcpyDeviceToHost, s));
  CPD_HIP_CHECK(hipStreamSynchronize(s));
  if (h.flags & HDR_BAR_TIMEOUT) {
    set_error("dgn: a grid barrier of the multi-workgroup CG timed out");
    return CPD_E_HIP;
  }
  if (k) *k = h.k;
  if (stop) *stop = h.stop;
  if (tol_iter) *tol_iter = h.tol_iter;
  if (err) {
    const Layout Lo = layout_of(h.np, h.R, h.maxiter);
    CPD_HIP_CHECK(hipMemcpyAsync(err, (char*)state + Lo.errs + sizeof(double) * h.k, sizeof(double),
                                 hipMemcpyDeviceToHost, s));
    CPD_HIP_CHECK(hipStreamSynchronize(s));
  }
  return CPD_OK;
}

cpd_status state_log(void* state, int first, int count, cpd_step_info* out, hipStream_t s) {
  Hdr h;
  CPD_HIP_CHECK(hipMemcpyAsync(&h, state, sizeof(h), hipMemcpyDeviceToHost, s));
  CPD_HIP_CHECK(hipStreamSynchronize(s));
  if (first < 0 || count < 0 || first + count > h.maxiter) {
    set_error("state_log: range out of bounds");
    return CPD_E_INVALID;
  }
  const Layout Lo = layout_of(h.np, h.R, h.maxiter);
  if (count > 0) {
    CPD_HIP_CHECK(hipMemcpyAsync(out, (char*)state + Lo.log + sizeof(cpd_step_info) * first,
                                 sizeof(cpd_step_info) * count, hipMemcpyDeviceToHost, s));
    CPD_HIP_CHECK(hipStreamSynchronize(s));
    const double f = wall_ns_per_tick();
    for (int i = 0; i < count; ++i) out[i].t_ns = (int64_t)llround((double)out[i].t_ns * f);
  }
  return CPD_OK;
}

cpd_status state_factors(void* state, double* W, int set, hipStream_t s) {
  Hdr h;
  CPD_HIP_CHECK(hipMemcpyAsync(&h, state, sizeof(h), hipMemcpyDeviceToHost, s));
  CPD_HIP_CHECK(hipStreamSynchronize(s));
  const Layout Lo = layout_of(h.np, h.R, h.maxiter);
  char* gW = (char*)state + Lo.W;
  if (set) {
    CPD_HIP_CHECK(hipMemcpyAsync(gW, W, sizeof(double) * h.np, hipMemcpyDeviceToDevice, s));
    // the next iteration recomputes the residual and the MTTKRP at the new factors
    const int32_t fl = h.flags | HDR_DIRTY;
    CPD_HIP_CHECK(hipMemcpyAsync((char*)state + offsetof(Hdr, flags), &fl, sizeof(fl), hipMemcpyHostToDevice, s));
    CPD_HIP_CHECK(hipStreamSynchronize(s));
  } else
    CPD_HIP_CHECK(hipMemcpyAsync(W, gW, sizeof(double) * h.np, hipMemcpyDeviceToDevice, s));
  return CPD_OK;
}

cpd_status jtj_v(const double* const W[3], const double* const V[3], const int32_t dims[3], int R,
                 double* const out[3], hipStream_t s) {
  if (R < 1 || R > 64) {
    set_error("jtj_v: R=%d out of range", R);
    return CPD_E_INVALID;
  }
  for (int l = 0; l < 3; ++l)
    if (dims[l] < 1 || dims[l] > 4096 || !W[l] || !V[l] || !out[l]) {
      set_error("jtj_v: bad mode %d", l);
      return CPD_E_INVALID;
    }
  const int np = (dims[0] + dims[1] + dims[2]) * R;
  size_t lb;
  if (!lds_fits(np, R, &lb)) {
    set_error("jtj_v: problem too large for LDS");
    return CPD_E_UNSUPPORTED;
  }
  CPD_HIP_CHECK(hipFuncSetAttribute((const void*)jtjv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lb));
  hipLaunchKernelGGL(jtjv_kernel, dim3(1), dim3(NT), lb, s, W[0], W[1], W[2], V[0], V[1], V[2],
                     dims[0], dims[1], dims[2], R, out[0], out[1], out[2]);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

}  // namespace cpd
