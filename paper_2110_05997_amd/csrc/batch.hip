// Batched solve of many small independent CPDs (modes <= 64): the whole hot path of ch.4
// (MLSVD compression -> dGN with PCG on the core -> uncompression) for every member, one
// workgroup per member and stage, five launches in total with no host round trip between them:
//   1. Gram G_l = T_(l) T_(l)^T of every mode on FP64 MFMA (one workgroup per member and mode),
//   2. cyclic Jacobi eigendecomposition of every G_l, canonical signs of the leading P_l vectors,
//   3. truncation rule, core projection S = T x1 U1^T x2 U2^T x3 U3^T, ||T||^2, dGN header,
//      CG caps and initial point,
//   4. the persistent dGN kernel (initialisation and iterations to a stopping rule),
//   5. uncompression W~ = U W, full-tensor residual and output normalisation.
// A plan captures the five launches in a hipGraph once; the Gram tile variant is chosen by timing
// the candidates on the plan's own batch.
#include "common.h"
#include "dgn_state.h"
#include "jacobi.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

namespace cpd {
namespace {

constexpr int BMAX_DIM = 64;
constexpr int PROJ_NT = 512;
constexpr int FIN_NT = 256;

struct BItem {
  const void* T;
  int d[3];
  int R;
  int P[3];
  int pad;
  const double* W0[3];
  double* Wout[3];
  double* lam;
  double* G[3];
  double* V[3];
  double* ev[3];
  double* U[3];
  double* Wt[3];
  double* Y1;
  double* Y2;
  double* S;
  char* state;
  cpd_solve_info* info;
};

typedef double dbl4 __attribute__((ext_vector_type(4)));

template <class TT>
__device__ __forceinline__ double ld_elem(const TT* p) { return (double)*p; }

// Element (row, c) of the mode-`mode` unfolding of a C-ordered I1 x I2 x I3 tensor, with the
// column index c running over the other two modes in C order.
template <class TT>
__device__ __forceinline__ double unf(const TT* T, int mode, int row, int c, int I2, int I3, int K,
                                      double inv3) {
  if (mode == 0) return ld_elem(T + (long long)row * K + c);
  if (mode == 2) return ld_elem(T + (long long)c * I3 + row);
  const int i = (int)(((double)c + 0.5) * inv3);
  const int kk = c - i * I3;
  return ld_elem(T + ((long long)i * I2 + row) * I3 + kk);
}

// ---- 1. Grams ---------------------------------------------------------------------------------
// Upper-triangle 16x16 tiles of G = A A^T (A = T_(mode), I x K) on v_mfma_f64_16x16x4f64; the
// waves of the workgroup take tiles round robin; each tile's result is written to both halves.
// NWAVE and UNR (MFMAs per k-chunk) are the tuned parameters.
template <class TT, int NWAVE, int UNR>
__global__ __launch_bounds__(NWAVE * 64) void batch_gram_kernel(const BItem* __restrict__ items, int n) {
  const int b = blockIdx.x / 3, mode = blockIdx.x - 3 * (blockIdx.x / 3);
  if (b >= n) return;
  const BItem& it = items[b];
  const TT* T = (const TT*)it.T;
  const int I2 = it.d[1], I3 = it.d[2];
  const int I = it.d[mode];
  const int K = (int)(((long long)it.d[0] * I2 * I3) / I);
  double* G = it.G[mode];
  const double inv3 = 1.0 / (double)I3;
  const int nt = (I + 15) >> 4, nup = nt * (nt + 1) / 2;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r16 = lane & 15, kq = lane >> 4;
  for (int t = w; t < nup; t += NWAVE) {
    int ti = 0, rem = t;
    while (rem >= nt - ti) { rem -= nt - ti; ++ti; }
    const int tj = ti + rem;
    const int m0 = ti * 16, n0 = tj * 16;
    const int ra = min(m0 + r16, I - 1), rb = min(n0 + r16, I - 1);
    const bool oka = (m0 + r16) < I, okb = (n0 + r16) < I;
    dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 4 * UNR) {
      double a[UNR], bb[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int c = k0 + 4 * u + kq;
        const bool okc = c < K;
        const int cc = okc ? c : K - 1;
        const double va = unf(T, mode, ra, cc, I2, I3, K, inv3);
        const double vb = unf(T, mode, rb, cc, I2, I3, K, inv3);
        a[u] = (oka && okc) ? va : 0.0;
        bb[u] = (okb && okc) ? vb : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        if (u & 1) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bb[u], acc1, 0, 0, 0);
        else acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bb[u], acc0, 0, 0, 0);
      }
    }
    const dbl4 D = acc0 + acc1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = m0 + 4 * v + kq, col = n0 + r16;
      if (row < I && col < I && (ti != tj || row <= col)) {
        G[row * I + col] = D[v];
        G[col * I + row] = D[v];
      }
    }
  }
}

// ---- 2. eigenpairs ------------------------------------------------------------------------------
// 256 threads per member: many members share each CU, so throughput (fewer redundant rotation
// evaluations per round) matters more than the latency of one member.
constexpr int BJNT = 256;
__global__ __launch_bounds__(BJNT) void batch_eig_kernel(const BItem* __restrict__ items, int n) {
  const int b = blockIdx.x / 3, mode = blockIdx.x - 3 * (blockIdx.x / 3);
  if (b >= n) return;
  const BItem& it = items[b];
  const int I = it.d[mode], P = it.P[mode];
  double* V = it.V[mode];
  __shared__ JacobiLds L;
  jacobi_block<BJNT, true>(L, it.G[mode], I, I, it.ev[mode], V);
  __syncthreads();
  // first P eigenvectors, each signed so that its largest-|.| entry is positive (ties: lowest
  // index); one wave per column
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double* U = it.U[mode];
  for (int j = w; j < P; j += BJNT / 64) {
    double best = -1.0;
    int bi = 0;
    for (int i = lane; i < I; i += 64) {
      const double a = fabs(V[i * I + j]);
      if (a > best || (a == best && i < bi)) { best = a; bi = i; }
    }
    for (int off = 32; off >= 1; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const double sgn = (V[bi * I + j] < 0.0) ? -1.0 : 1.0;
    for (int i = lane; i < I; i += 64) U[i * P + j] = sgn * V[i * I + j];
  }
}

// ---- 3. truncation, projection, dGN set-up ------------------------------------------------------
struct SetupArgs {
  const int* caps;   // maxiter entries
  int maxiter, fixed, random_init, pad;
  double tol, cg_tol, init_damp, mlsvd_tol;
  uint64_t seed;
};

// Truncation rule of Alg. Compression on the leading P eigenvalues (sigma^2, clamped at 0).
__device__ int trunc_rank(const double* lam, int P, double mlsvd_tol) {
  double total = 0.0;
  for (int r = 0; r < P; ++r) total += fmax(lam[r], 0.0);
  if (total == 0.0) return P;
  for (int i = 1; i <= P; ++i) {
    double tail = 0.0;
    for (int r = i; r < P; ++r) tail += fmax(lam[r], 0.0);
    if (tail / total < mlsvd_tol / 3.0) return i;
  }
  return P;
}

template <class TT>
__global__ __launch_bounds__(PROJ_NT) void batch_project_kernel(const BItem* __restrict__ items, int n,
                                                                SetupArgs a) {
  __shared__ int core[3];
  __shared__ double red[2][PROJ_NT / 64];
  __shared__ double U1s[BMAX_DIM * BMAX_DIM];
  const int b = blockIdx.x;
  if (b >= n) return;
  const BItem& it = items[b];
  const TT* T = (const TT*)it.T;
  const int tid = threadIdx.x;
  const int I1 = it.d[0], I2 = it.d[1], I3 = it.d[2], R = it.R;
  const int P1 = it.P[0], P2 = it.P[1], P3 = it.P[2];
  const int K1 = I2 * I3;
  const long long N = (long long)I1 * K1;
  if (tid == 0)
    for (int l = 0; l < 3; ++l) core[l] = a.fixed ? it.P[l] : trunc_rank(it.ev[l], it.P[l], a.mlsvd_tol);
  double s2 = 0.0, bad = 0.0;
  for (long long e = tid; e < N; e += PROJ_NT) {
    const double v = ld_elem(T + e);
    s2 += v * v;
    bad += isfinite(v) ? 0.0 : 1.0;
  }
  s2 = block_sum(s2, red[0]);
  bad = block_sum(bad, red[1]);
  const int c1 = core[0], c2 = core[1], c3 = core[2];
  // Y1[a][j k] = sum_i U1[i][a] T[i][j][k]: U1 staged in LDS, up to 16 outputs per thread from one
  // read of T[:, j, k] (each output accumulated over i in increasing order)
  for (int e = tid; e < I1 * P1; e += PROJ_NT) U1s[e] = it.U[0][e];
  __syncthreads();
  for (int a0 = 0; a0 < c1; a0 += 16) {
    const int na = min(16, c1 - a0);
    for (int jk = tid; jk < K1; jk += PROJ_NT) {
      double acc[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = 0.0;
      for (int i = 0; i < I1; ++i) {
        const double t = ld_elem(T + (long long)i * K1 + jk);
        const double* u = U1s + i * P1 + a0;
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (q < na) acc[q] = fma(u[q], t, acc[q]);
      }
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (q < na) it.Y1[(long long)(a0 + q) * K1 + jk] = acc[q];
    }
  }
  __syncthreads();
  // Y2[a][b][k] = sum_j U2[j][b] Y1[a][j][k]
  for (int e = tid; e < c1 * c2 * I3; e += PROJ_NT) {
    const int ab = e / I3, k = e - ab * I3;
    const int aa = ab / c2, bb = ab - aa * c2;
    double acc = 0.0;
    for (int j = 0; j < I2; ++j) acc = fma(it.U[1][j * P2 + bb], it.Y1[(long long)aa * K1 + j * I3 + k], acc);
    it.Y2[e] = acc;
  }
  __syncthreads();
  // S[a][b][c] = sum_k U3[k][c] Y2[a][b][k]
  for (int e = tid; e < c1 * c2 * c3; e += PROJ_NT) {
    const int ab = e / c3, cc = e - ab * c3;
    double acc = 0.0;
    for (int k = 0; k < I3; ++k) acc = fma(it.U[2][k * P3 + cc], it.Y2[ab * I3 + k], acc);
    it.S[e] = acc;
  }
  // dGN state: header, caps, initial point (first c_l rows of W0, or N(0,1))
  const int np = (c1 + c2 + c3) * R;
  const Layout Lo = layout_of(np, R, a.maxiter);
  char* st = it.state;
  int* caps = (int*)(st + Lo.caps);
  for (int k = tid; k < a.maxiter; k += PROJ_NT) caps[k] = a.caps[k];
  double* W = (double*)(st + Lo.W);
  const int cs[3] = {c1, c2, c3};
  int off = 0;
  for (int l = 0; l < 3; ++l) {
    for (int e = tid; e < cs[l] * R; e += PROJ_NT) {
      double v;
      if (!a.random_init) {
        v = it.W0[l][e];   // row i < c_l of the P_l x R block, same index
      } else {
        const uint64_t base = a.seed * 0x9E3779B97F4A7C15ull + (uint64_t)b * 0xD1B54A32D192ED03ull;
        const uint64_t ctr = (uint64_t)(off + e);
        const double u1 = u01_from_bits(splitmix64(base + 2 * ctr));
        const double u2 = u01_from_bits(splitmix64(base + 2 * ctr + 1));
        v = sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586 * u2);
      }
      W[off + e] = v;
    }
    off += cs[l] * R;
  }
  if (tid == 0) {
    Hdr* h = (Hdr*)st;
    memset(h, 0, sizeof(Hdr));
    h->d[0] = c1; h->d[1] = c2; h->d[2] = c3; h->R = R;
    h->maxiter = a.maxiter; h->np = np; h->tol_iter = -1; h->k = 0; h->stop = CPD_STOP_NONE;
    h->tol = a.tol; h->cg_tol = a.cg_tol; h->init_damp = a.init_damp; h->div_ref = s2;
    h->flags = (bad > 0.0 || !(s2 > 0.0)) ? 2 : 0;
    cpd_solve_info* inf = it.info;
    inf->t_norm = sqrt(s2);
    inf->core_dims[0] = c1; inf->core_dims[1] = c2; inf->core_dims[2] = c3;
  }
}

// ---- 5. uncompression, residual, normalisation --------------------------------------------------
template <class TT>
__global__ __launch_bounds__(FIN_NT) void batch_finish_kernel(const BItem* __restrict__ items, int n,
                                                              int maxiter, double ns_per_tick) {
  __shared__ double red[2][FIN_NT / 64];
  __shared__ double nrm[3][64];
  __shared__ double sgn[2][64];
  __shared__ double lamv[64];
  __shared__ double scale[3][64];
  __shared__ int dest[64];
  __shared__ double W1s[BMAX_DIM * 64], W2s[BMAX_DIM * 64];   // modes <= 64, R <= 64
  const int b = blockIdx.x;
  if (b >= n) return;
  const BItem& it = items[b];
  const TT* T = (const TT*)it.T;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const Hdr* h = (const Hdr*)it.state;
  const int R = it.R;
  const int cs[3] = {h->d[0], h->d[1], h->d[2]};
  const int np = (cs[0] + cs[1] + cs[2]) * R;
  const Layout Lo = layout_of(np, R, maxiter);
  const double* Wc = (const double*)(it.state + Lo.W);
  const double* errs = (const double*)(it.state + Lo.errs);
  const bool skipped = (h->flags & 2) != 0;
  // W~_l = U_l[:, :c_l] W_l
  int off = 0;
  for (int l = 0; l < 3; ++l) {
    const int I = it.d[l], P = it.P[l];
    for (int e = tid; e < I * R; e += FIN_NT) {
      const int i = e / R, r = e - (e / R) * R;
      double acc = 0.0;
      for (int q = 0; q < cs[l]; ++q) acc = fma(it.U[l][i * P + q], Wc[off + q * R + r], acc);
      it.Wt[l][e] = acc;
    }
    off += cs[l] * R;
  }
  __syncthreads();
  // ||T - [[W~]]||^2, with the mode-2 and mode-3 factors staged in LDS
  const int I1 = it.d[0], I2 = it.d[1], I3 = it.d[2], K1 = I2 * I3;
  for (int e = tid; e < I2 * R; e += FIN_NT) W1s[e] = it.Wt[1][e];
  for (int e = tid; e < I3 * R; e += FIN_NT) W2s[e] = it.Wt[2][e];
  __syncthreads();
  const double inv3 = 1.0 / (double)I3;
  double res = 0.0;
  for (int i = 0; i < I1; ++i) {
    const double* A = it.Wt[0] + i * R;
    for (int jk = tid; jk < K1; jk += FIN_NT) {
      const int j = (int)(((double)jk + 0.5) * inv3), k = jk - j * I3;
      const double* B = W1s + j * R;
      const double* C = W2s + k * R;
      double m = 0.0;
      for (int r = 0; r < R; ++r) m = fma(A[r] * B[r], C[r], m);
      const double d = ld_elem(T + (long long)i * K1 + jk) - m;
      res += d * d;
    }
  }
  res = block_sum(res, red[0]);
  // column norms, signs of modes 1 and 2, lambda and the order by decreasing lambda
  for (int c = w; c < 3 * R; c += FIN_NT / 64) {
    const int l = c / R, r = c - (c / R) * R;
    double s = 0.0;
    for (int i = lane; i < it.d[l]; i += 64) s += it.Wt[l][i * R + r] * it.Wt[l][i * R + r];
    s = wave_sum(s);
    if (lane == 0) nrm[l][r] = sqrt(s);
  }
  for (int c = w; c < 2 * R; c += FIN_NT / 64) {
    const int l = c / R, r = c - (c / R) * R;
    double best = -1.0;
    int bi = 0;
    for (int i = lane; i < it.d[l]; i += 64) {
      const double a = fabs(it.Wt[l][i * R + r]);
      if (a > best || (a == best && i < bi)) { best = a; bi = i; }
    }
    for (int o = 32; o >= 1; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) sgn[l][r] = (it.Wt[l][bi * R + r] < 0.0) ? -1.0 : 1.0;
  }
  __syncthreads();
  if (tid < R) lamv[tid] = (nrm[0][tid] * nrm[1][tid]) * nrm[2][tid];
  __syncthreads();
  if (tid < R) {
    const int r = tid;
    int rank = 0;
    for (int q = 0; q < R; ++q)
      if (lamv[q] > lamv[r] || (lamv[q] == lamv[r] && q < r)) ++rank;
    dest[r] = rank;
    it.lam[rank] = lamv[r];
    for (int l = 0; l < 3; ++l) {
      double sc = (nrm[l][r] > 0.0) ? 1.0 / nrm[l][r] : 1.0;
      sc *= (l < 2) ? sgn[l][r] : sgn[0][r] * sgn[1][r];
      scale[l][r] = sc;
    }
  }
  __syncthreads();
  for (int l = 0; l < 3; ++l)
    for (int e = tid; e < it.d[l] * R; e += FIN_NT) {
      const int i = e / R, r = e - (e / R) * R;
      it.Wout[l][i * R + dest[r]] = it.Wt[l][e] * scale[l][r];
    }
  if (tid == 0) {
    cpd_solve_info* inf = it.info;
    inf->iters = h->k;
    inf->stop_reason = skipped ? -1 : h->stop;
    inf->tol_iter = h->tol_iter;
    // per member: from its dGN start to its first iteration below tol (members run side by side)
    inf->time_to_tol_ns = (!skipped && h->tol_iter > 0) ? llround((double)(h->t_tol - h->t_init) * ns_per_tick) : -1;
    inf->refine_iters = 0;   // batched solves do not refine
    inf->refine_stop = 0;
    inf->rel_err_core = skipped ? NAN : errs[h->k];
    const double tn = inf->t_norm;
    inf->rel_err_full = (tn > 0.0) ? sqrt(fmax(res, 0.0)) / tn : 0.0;
  }
}

// ---- host side ----------------------------------------------------------------------------------
bool item_ok(const cpd_batch_item& x) {
  if (!x.T || !x.W[0] || !x.W[1] || !x.W[2] || !x.lambda || x.R < 1 || x.R > 64) return false;
  for (int l = 0; l < 3; ++l)
    if (x.dims[l] < 1 || x.dims[l] > BMAX_DIM) return false;
  const bool any = x.W0[0] || x.W0[1] || x.W0[2];
  const bool all = x.W0[0] && x.W0[1] && x.W0[2];
  return !any || all;
}

void item_P(const cpd_batch_item& x, const cpd_params* p, int P[3]) {
  const bool fixed = p->core_dims[0] > 0 && p->core_dims[1] > 0 && p->core_dims[2] > 0;
  for (int l = 0; l < 3; ++l) {
    const int I = (int)x.dims[l];
    const int want = fixed ? p->core_dims[l] : x.R;
    P[l] = want < I ? want : I;
  }
}

// Carves the batch workspace (Sizer and Arena share this sequence).
template <class Carver>
void carve_batch(Carver& z, const cpd_batch_item* items, int n, const cpd_params* p, BItem** d_items,
                 char*** d_states, const double*** d_S, int** d_caps, cpd_solve_info** d_info,
                 std::vector<BItem>* host) {
  *d_items = z.template take<BItem>(n);
  *d_states = z.template take<char*>(n);
  *d_S = z.template take<const double*>(n);
  *d_caps = z.template take<int>(p->maxiter);
  *d_info = z.template take<cpd_solve_info>(n);
  for (int b = 0; b < n; ++b) {
    const cpd_batch_item& x = items[b];
    BItem it;
    memset(&it, 0, sizeof(it));
    it.T = x.T;
    it.R = x.R;
    int P[3];
    item_P(x, p, P);
    for (int l = 0; l < 3; ++l) {
      it.d[l] = (int)x.dims[l];
      it.P[l] = P[l];
      it.W0[l] = x.W0[l];
      it.Wout[l] = x.W[l];
    }
    it.lam = x.lambda;
    for (int l = 0; l < 3; ++l) {
      const size_t I = (size_t)x.dims[l];
      it.G[l] = z.template take<double>(I * I);
      it.V[l] = z.template take<double>(I * I);
      it.ev[l] = z.template take<double>(I);
      it.U[l] = z.template take<double>(I * P[l]);
      it.Wt[l] = z.template take<double>(I * x.R);
    }
    it.Y1 = z.template take<double>((size_t)P[0] * x.dims[1] * x.dims[2]);
    it.Y2 = z.template take<double>((size_t)P[0] * P[1] * x.dims[2]);
    it.S = z.template take<double>((size_t)P[0] * P[1] * P[2]);
    const int32_t pc[3] = {P[0], P[1], P[2]};
    it.state = z.template take<char>(state_bytes(pc, x.R, p->maxiter));
    it.info = (*d_info) ? (*d_info) + b : nullptr;
    if (host) host->push_back(it);
  }
}

cpd_status check_batch(const cpd_batch_item* items, int n, int dtype, const cpd_params* p, size_t* lds) {
  if (!items || n < 1 || !p || p->maxiter < 1 || (dtype != CPD_F64 && dtype != CPD_F32)) {
    set_error("batch: bad arguments (n=%d dtype=%d)", n, dtype);
    return CPD_E_INVALID;
  }
  if (dgn_opts(p)) {
    set_error("batch: the batched solver runs the plain dGN (precond 0, no draw-back)");
    return CPD_E_UNSUPPORTED;
  }
  size_t mx = 0;
  for (int b = 0; b < n; ++b) {
    if (!item_ok(items[b])) {
      set_error("batch: member %d invalid (modes 1..%d, R 1..64, W0 all or none)", b, BMAX_DIM);
      return CPD_E_INVALID;
    }
    int P[3];
    item_P(items[b], p, P);
    const int np = (P[0] + P[1] + P[2]) * items[b].R;
    const size_t lb = dgn_lds_bytes(np, items[b].R);
    mx = lb > mx ? lb : mx;
  }
  if (mx > 160 * 1024 - 1024) {
    set_error("batch: a member's dGN state needs %zu bytes of LDS", mx);
    return CPD_E_UNSUPPORTED;
  }
  *lds = mx;
  return CPD_OK;
}

void host_caps(const cpd_params* p, std::vector<int>& caps) {
  caps.resize(p->maxiter);
  for (int k = 1; k <= p->maxiter; ++k) {
    if (p->cg_fixed > 0) {
      caps[k - 1] = p->cg_fixed;
    } else {
      const double u = p->cg_uniforms ? p->cg_uniforms[k - 1]
                                      : u01_from_bits(splitmix64(p->seed * 0xD1B54A32D192ED03ull + (uint64_t)k));
      caps[k - 1] = cg_cap_for(k, u);
    }
  }
}

typedef void (*gram_fn)(const BItem*, int);

template <class TT>
gram_fn gram_variant(int v) {
  switch (v) {
    case 0: return batch_gram_kernel<TT, 4, 4>;
    case 1: return batch_gram_kernel<TT, 4, 8>;
    case 2: return batch_gram_kernel<TT, 8, 4>;
    default: return batch_gram_kernel<TT, 8, 8>;
  }
}
constexpr int N_GRAM_VARIANTS = 4;
int variant_threads(int v) { return (v >= 2) ? 512 : 256; }

struct Launch {
  const BItem* items;
  char* const* states;
  const double* const* S;
  int n, dtype, variant, maxiter;
  size_t lds;
  SetupArgs setup;
  double ns_per_tick;
};

cpd_status launch_gram(const Launch& L, hipStream_t s) {
  gram_fn f = (L.dtype == CPD_F64) ? gram_variant<double>(L.variant) : gram_variant<float>(L.variant);
  hipLaunchKernelGGL(f, dim3(3 * L.n), dim3(variant_threads(L.variant)), 0, s, L.items, L.n);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

cpd_status launch_all(const Launch& L, hipStream_t s) {
  cpd_status st;
  if ((st = launch_gram(L, s))) return st;
  hipLaunchKernelGGL(batch_eig_kernel, dim3(3 * L.n), dim3(BJNT), 0, s, L.items, L.n);
  CPD_LAUNCH_CHECK();
  if (L.dtype == CPD_F64)
    hipLaunchKernelGGL(batch_project_kernel<double>, dim3(L.n), dim3(PROJ_NT), 0, s, L.items, L.n, L.setup);
  else
    hipLaunchKernelGGL(batch_project_kernel<float>, dim3(L.n), dim3(PROJ_NT), 0, s, L.items, L.n, L.setup);
  CPD_LAUNCH_CHECK();
  if ((st = dgn_batch_launch(L.states, L.S, L.n, L.lds, s))) return st;
  if (L.dtype == CPD_F64)
    hipLaunchKernelGGL(batch_finish_kernel<double>, dim3(L.n), dim3(FIN_NT), 0, s, L.items, L.n, L.maxiter, L.ns_per_tick);
  else
    hipLaunchKernelGGL(batch_finish_kernel<float>, dim3(L.n), dim3(FIN_NT), 0, s, L.items, L.n, L.maxiter, L.ns_per_tick);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

// Uploads descriptors and caps (synchronises the stream) and fills the launch record.
cpd_status prepare(const cpd_batch_item* items, int n, int dtype, const cpd_params* p, void* ws, size_t ws_bytes,
                   hipStream_t s, Launch& L, cpd_solve_info** d_info) {
  size_t lds = 0;
  cpd_status st;
  if ((st = check_batch(items, n, dtype, p, &lds))) return st;
  Sizer z;
  BItem* di = nullptr;
  char** dst = nullptr;
  const double** dS = nullptr;
  int* dc = nullptr;
  cpd_solve_info* dinf = nullptr;
  carve_batch(z, items, n, p, &di, &dst, &dS, &dc, &dinf, nullptr);
  if (!ws || ws_bytes < z.off) {
    set_error("batch: workspace %zu < %zu", ws_bytes, z.off);
    return CPD_E_WORKSPACE;
  }
  if ((st = dgn_batch_prepare(lds))) return st;
  Arena ar(ws, ws_bytes);
  std::vector<BItem> host;
  host.reserve(n);
  carve_batch(ar, items, n, p, &di, &dst, &dS, &dc, &dinf, &host);
  std::vector<char*> hst(n);
  std::vector<const double*> hS(n);
  for (int b = 0; b < n; ++b) {
    host[b].info = dinf + b;
    hst[b] = host[b].state;
    hS[b] = host[b].S;
  }
  std::vector<int> caps;
  host_caps(p, caps);
  CPD_HIP_CHECK(hipMemcpyAsync(di, host.data(), sizeof(BItem) * n, hipMemcpyHostToDevice, s));
  CPD_HIP_CHECK(hipMemcpyAsync(dst, hst.data(), sizeof(char*) * n, hipMemcpyHostToDevice, s));
  CPD_HIP_CHECK(hipMemcpyAsync(dS, hS.data(), sizeof(double*) * n, hipMemcpyHostToDevice, s));
  CPD_HIP_CHECK(hipMemcpyAsync(dc, caps.data(), sizeof(int) * p->maxiter, hipMemcpyHostToDevice, s));
  CPD_HIP_CHECK(hipStreamSynchronize(s));
  L.items = di;
  L.states = dst;
  L.S = dS;
  L.n = n;
  L.dtype = dtype;
  L.variant = 0;
  L.maxiter = p->maxiter;
  L.ns_per_tick = wall_ns_per_tick();
  L.lds = lds;
  L.setup.caps = dc;
  L.setup.maxiter = p->maxiter;
  L.setup.fixed = (p->core_dims[0] > 0 && p->core_dims[1] > 0 && p->core_dims[2] > 0) ? 1 : 0;
  L.setup.random_init = items[0].W0[0] ? 0 : 1;
  for (int b = 1; b < n; ++b)
    if ((items[b].W0[0] != nullptr) != (items[0].W0[0] != nullptr)) {
      set_error("batch: W0 must be given for every member or for none");
      return CPD_E_INVALID;
    }
  L.setup.tol = p->tol;
  L.setup.cg_tol = (p->cg_tol > 0.0) ? p->cg_tol : p->tol;
  L.setup.init_damp = p->init_damp;
  L.setup.mlsvd_tol = p->mlsvd_tol;
  L.setup.seed = p->seed;
  *d_info = dinf;
  return CPD_OK;
}

cpd_status read_info(cpd_solve_info* d_info, int n, cpd_solve_info* info, hipStream_t s) {
  if (info) CPD_HIP_CHECK(hipMemcpyAsync(info, d_info, sizeof(cpd_solve_info) * n, hipMemcpyDeviceToHost, s));
  CPD_HIP_CHECK(hipStreamSynchronize(s));
  return CPD_OK;
}

}  // namespace
}  // namespace cpd

using namespace cpd;

struct cpd_batch_plan {
  Launch L;
  cpd_solve_info* d_info;
  hipGraph_t graph;
  hipGraphExec_t exec;
  float variant_ms[N_GRAM_VARIANTS];
};

extern "C" {

size_t cpd_batch_workspace_bytes(const cpd_batch_item* items, int32_t n, const cpd_params* p) {
  cpd_params def;
  if (!p) { cpd_default_params(&def); p = &def; }
  size_t lds;
  if (check_batch(items, n, CPD_F64, p, &lds)) return 0;
  Sizer z;
  BItem* di = nullptr;
  char** dst = nullptr;
  const double** dS = nullptr;
  int* dc = nullptr;
  cpd_solve_info* dinf = nullptr;
  carve_batch(z, items, n, p, &di, &dst, &dS, &dc, &dinf, nullptr);
  return z.off;
}

cpd_status cpd_solve_batched(const cpd_batch_item* items, int32_t n, int32_t dtype, const cpd_params* p,
                             cpd_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  cpd_params def;
  if (!p) { cpd_default_params(&def); p = &def; }
  hipStream_t s = (hipStream_t)stream;
  Launch L;
  cpd_solve_info* d_info = nullptr;
  cpd_status st;
  if ((st = prepare(items, n, dtype, p, ws, ws_bytes, s, L, &d_info))) return st;
  if ((st = launch_all(L, s))) return st;
  return read_info(d_info, n, info, s);
}

cpd_status cpd_batch_plan_create(const cpd_batch_item* items, int32_t n, int32_t dtype, const cpd_params* p,
                                 void* ws, size_t ws_bytes, void* stream, cpd_batch_plan** out) {
  CPD_REQUIRE(out != nullptr, "cpd_batch_plan_create: null out");
  *out = nullptr;
  cpd_params def;
  if (!p) { cpd_default_params(&def); p = &def; }
  hipStream_t s = (hipStream_t)stream;
  cpd_batch_plan* plan = (cpd_batch_plan*)calloc(1, sizeof(cpd_batch_plan));
  if (!plan) {
    set_error("cpd_batch_plan_create: host allocation failed");
    return CPD_E_INVALID;
  }
  cpd_status st = prepare(items, n, dtype, p, ws, ws_bytes, s, plan->L, &plan->d_info);
  if (st) { free(plan); return st; }
  // autotune the Gram tile variant on this batch: each candidate once to warm up, then timed
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("cpd_batch_plan_create: event creation failed");
    free(plan);
    return CPD_E_HIP;
  }
  int best = 0;
  float best_ms = 1e30f;
  for (int v = 0; v < N_GRAM_VARIANTS && !st; ++v) {
    Launch Lv = plan->L;
    Lv.variant = v;
    st = launch_gram(Lv, s);
    if (!st && hipEventRecord(e0, s) != hipSuccess) st = CPD_E_HIP;
    if (!st) st = launch_gram(Lv, s);
    if (!st && hipEventRecord(e1, s) != hipSuccess) st = CPD_E_HIP;
    float ms = 0.0f;
    if (!st && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = CPD_E_HIP;
    plan->variant_ms[v] = ms;
    if (!st && ms < best_ms) { best_ms = ms; best = v; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    set_error("cpd_batch_plan_create: autotuning failed");
    free(plan);
    return st;
  }
  plan->L.variant = best;
  // capture the five launches on a private stream (default priority)
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    set_error("cpd_batch_plan_create: stream creation failed");
    free(plan);
    return CPD_E_HIP;
  }
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = launch_all(plan->L, cs);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (!st && e2 == hipSuccess) {
      plan->graph = g;
      if (hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0) != hipSuccess) st = CPD_E_HIP;
    } else if (!st) {
      st = CPD_E_HIP;
    }
  } else {
    st = CPD_E_HIP;
  }
  (void)hipStreamDestroy(cs);
  if (st) {
    set_error("cpd_batch_plan_create: graph capture failed");
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    free(plan);
    return st;
  }
  *out = plan;
  return CPD_OK;
}

cpd_status cpd_batch_plan_run(cpd_batch_plan* plan, cpd_solve_info* info, void* stream) {
  CPD_REQUIRE(plan != nullptr && plan->exec != nullptr, "cpd_batch_plan_run: no plan");
  hipStream_t s = (hipStream_t)stream;
  CPD_HIP_CHECK(hipGraphLaunch(plan->exec, s));
  if (!info) return CPD_OK;
  return read_info(plan->d_info, plan->L.n, info, s);
}

int32_t cpd_batch_plan_variant(const cpd_batch_plan* plan, float* variant_ms) {
  if (!plan) return -1;
  if (variant_ms)
    for (int v = 0; v < N_GRAM_VARIANTS; ++v) variant_ms[v] = plan->variant_ms[v];
  return plan->L.variant;
}

void cpd_batch_plan_destroy(cpd_batch_plan* plan) {
  if (!plan) return;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  free(plan);
}

}  // extern "C"
