// The tensor-train route to the CPD of a tensor of order L >= 4 (ch.4 "Tensor train and the CPD"):
// Alg. TT-SVD with every TT-rank equal to R, a rank-R CPD of the second core, a Bi-CPD (first factor
// fixed) of each further core, and the outer factors from the first and last cores (Alg. CPD-TTD).
//
// TT-SVD step l works on M, the (r_{l-1} I_l) x n_l row-major reshape of the current tensor
// (C order: no data movement): its left singular vectors are the eigenvectors of the Gram M M^T
// (the App. B lemma; the same Gram and eigensolver kernels as the MLSVD, the Gram taken as mode 1
// of an m x 1 x n tensor), core l is their (r_{l-1}, I_l, R) reshape, and M <- U^T M (= Sigma V^T)
// on the generic GEMM.  The inner CPDs are the third-order path (compression, dGN with CG,
// uncompression); a Bi-CPD is the dGN with its first factor's block of the step held at zero.
// Every factor is returned with unit columns, lambda_r >= 0, modes 1..L-1 signed so each column's
// largest-|.| entry is positive (the sign goes to mode L), and terms by decreasing lambda.
#include "common.h"
#include "dgn_state.h"

#include <math.h>
#include <string.h>

#include <vector>

namespace cpd {
namespace {

constexpr int TT_MAXL = 16;
constexpr int TT_NT = 256;
constexpr int TT_RB = 1024;   // residual partial sums (fixed grid: bit-reproducible)

// out = (A^{-1})^T for an R x R matrix (R <= 64), Gauss-Jordan with partial pivoting in LDS (one
// workgroup): pivot rows are chosen by the largest |.| in the column (ties: lowest row).  A zero
// pivot sets *singular (never cleared here).
__global__ __launch_bounds__(TT_NT) void inverse_transpose_kernel(const double* __restrict__ A, int R,
                                                                  double* __restrict__ out, int* __restrict__ singular) {
  __shared__ double M[64][128];   // [A | I]
  __shared__ int piv;
  const int tid = threadIdx.x;
  for (int e = tid; e < R * 2 * R; e += TT_NT) {
    const int i = e / (2 * R), j = e - i * 2 * R;
    M[i][j] = (j < R) ? A[i * R + j] : (j - R == i ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int c = 0; c < R; ++c) {
    if (tid == 0) {
      int best = c;
      double bv = fabs(M[c][c]);
      for (int i = c + 1; i < R; ++i)
        if (fabs(M[i][c]) > bv) { bv = fabs(M[i][c]); best = i; }
      piv = best;
      if (!(bv > 0.0)) *singular = 1;
    }
    __syncthreads();
    const int pr = piv;
    if (pr != c)
      for (int j = tid; j < 2 * R; j += TT_NT) {
        const double t = M[c][j];
        M[c][j] = M[pr][j];
        M[pr][j] = t;
      }
    __syncthreads();
    const double d = M[c][c];
    __syncthreads();
    for (int j = tid; j < 2 * R; j += TT_NT) M[c][j] = M[c][j] / d;
    __syncthreads();
    for (int e = tid; e < R * 2 * R; e += TT_NT) {
      const int i = e / (2 * R), j = e - i * 2 * R;
      if (i != c) {
        const double f = M[i][c];
        if (j != c) M[i][j] -= f * M[c][j];
      }
    }
    __syncthreads();
    for (int i = tid; i < R; i += TT_NT)
      if (i != c) M[i][c] = 0.0;
    __syncthreads();
  }
  // A^{-1} sits in the right half; write its transpose
  for (int e = tid; e < R * R; e += TT_NT) {
    const int i = e / R, j = e - i * R;
    out[i * R + j] = M[j][R + i];
  }
}

// Shapes of the L factors in one device array: dims[l], row offsets (in rows of R) off[l].
struct TtShape {
  int L, R;
  int dims[TT_MAXL];
  long long off[TT_MAXL];
};

// ||T - sum_r w_r^(1) o ... o w_r^(L)||^2 partials: entry e of T (C order) is split into its L
// indices, the model is sum_r prod_l W_l[i_l][r] (W packed per mode, row-major).  One partial per
// block, summed later in a fixed order.
template <class TT>
__global__ __launch_bounds__(TT_NT) void tt_residual_kernel(const TT* __restrict__ X, long long n,
                                                            const TtShape* __restrict__ sh,
                                                            const double* __restrict__ W,
                                                            double* __restrict__ part) {
  __shared__ double slots[TT_NT / 64];
  __shared__ TtShape s;
  if (threadIdx.x == 0) s = *sh;
  __syncthreads();
  const int L = s.L, R = s.R;
  double acc = 0.0;
  for (long long e = (long long)blockIdx.x * TT_NT + threadIdx.x; e < n; e += (long long)gridDim.x * TT_NT) {
    double prod[64];
    for (int r = 0; r < R; ++r) prod[r] = 1.0;
    long long rem = e;
    for (int l = L - 1; l >= 0; --l) {
      const int d = s.dims[l];
      const long long i = rem % d;
      rem /= d;
      const double* Wl = W + (s.off[l] + i) * R;
      for (int r = 0; r < R; ++r) prod[r] *= Wl[r];
    }
    double model = 0.0;
    for (int r = 0; r < R; ++r) model += prod[r];
    const double f = (double)X[e] - model;
    acc += f * f;
  }
  const double b = block_sum(acc, slots);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

__global__ void tt_final_sum_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double slots[TT_NT / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += TT_NT) acc += part[i];
  const double s = block_sum(acc, slots);
  if (threadIdx.x == 0) *out = s;
}

// Output normalisation for L modes (one workgroup, R <= 64): column norms, lambda = their product,
// signs of modes 1..L-1 from the largest-|.| entry (ties: lowest row) with the sign moved into mode
// L, terms ordered by decreasing lambda (ties: lower index).  scale[l * 64 + r] and dest[r] drive
// tt_normalize_apply_kernel.
__global__ __launch_bounds__(TT_NT) void tt_normalize_plan_kernel(const TtShape* __restrict__ sh,
                                                                  const double* __restrict__ W,
                                                                  double* __restrict__ scale, int* __restrict__ dest,
                                                                  double* __restrict__ lambda) {
  __shared__ TtShape s;
  __shared__ double nrm[TT_MAXL][64];
  __shared__ double sgn[TT_MAXL][64];
  __shared__ double lam[64];
  if (threadIdx.x == 0) s = *sh;
  __syncthreads();
  const int L = s.L, R = s.R;
  for (int e = threadIdx.x; e < L * R; e += TT_NT) {
    const int l = e / R, r = e - l * R;
    const double* Wl = W + s.off[l] * R;
    double acc = 0.0, best = -1.0;
    int bi = 0;
    for (int i = 0; i < s.dims[l]; ++i) {
      const double v = Wl[(long long)i * R + r];
      acc += v * v;
      if (fabs(v) > best) { best = fabs(v); bi = i; }
    }
    nrm[l][r] = sqrt(acc);
    sgn[l][r] = (Wl[(long long)bi * R + r] < 0.0) ? -1.0 : 1.0;
  }
  __syncthreads();
  if (threadIdx.x < R) {
    const int r = threadIdx.x;
    double p = 1.0;
    for (int l = 0; l < L; ++l) p *= nrm[l][r];
    lam[r] = p;
  }
  __syncthreads();
  if (threadIdx.x < R) {
    const int r = threadIdx.x;
    int rank = 0;
    for (int q = 0; q < R; ++q)
      if (lam[q] > lam[r] || (lam[q] == lam[r] && q < r)) ++rank;
    dest[r] = rank;
    lambda[rank] = lam[r];
    double last = 1.0;
    for (int l = 0; l < L - 1; ++l) {
      scale[l * 64 + r] = ((nrm[l][r] > 0.0) ? 1.0 / nrm[l][r] : 1.0) * sgn[l][r];
      last *= sgn[l][r];
    }
    scale[(L - 1) * 64 + r] = ((nrm[L - 1][r] > 0.0) ? 1.0 / nrm[L - 1][r] : 1.0) * last;
  }
}

__global__ void tt_normalize_apply_kernel(const double* __restrict__ Wl, long long rows, int R,
                                          const double* __restrict__ scale, const int* __restrict__ dest,
                                          double* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * R) return;
  const long long i = e / R;
  const int r = (int)(e - i * R);
  out[i * R + dest[r]] = Wl[e] * scale[r];
}

struct TtPlan {
  int L, R;
  int64_t dims[TT_MAXL];
  int64_t N;
  int m[TT_MAXL];          // rows of M at step l (r_{l-1} I_l)
  int64_t n[TT_MAXL];      // columns of M at step l
  size_t gram_b, eig_b, inner_b;
  int64_t mbuf;            // doubles of each ping-pong buffer
  int Gmax;                // largest Gram order
  int64_t wrows;           // total factor rows
};

bool tt_plan(int L, const int64_t* dims, int R, const cpd_params* p, TtPlan& q) {
  if (L < 4 || L > TT_MAXL || R < 1 || R > 64 || dims == nullptr) return false;
  q.L = L;
  q.R = R;
  q.N = 1;
  q.wrows = 0;
  for (int l = 0; l < L; ++l) {
    if (dims[l] < 1 || dims[l] > 4096) return false;
    q.dims[l] = dims[l];
    q.N *= dims[l];
    q.wrows += dims[l];
  }
  if (R > dims[0] || R > dims[L - 1]) return false;   // every TT-rank must reach R
  q.gram_b = q.eig_b = q.inner_b = 0;
  q.Gmax = 0;
  q.mbuf = 0;
  int64_t rem = q.N;
  for (int l = 0; l < L - 1; ++l) {
    const int64_t m = (l == 0 ? 1 : R) * dims[l];
    rem /= dims[l];
    if (m > 4096 || (m > 64 && R > 56) || rem < R || rem > 0x7fffffffLL) return false;
    q.m[l] = (int)m;
    q.n[l] = rem;
    const int64_t gd[3] = {m, 1, rem};
    const size_t gb = gram_ws_bytes(gd, 0);
    q.gram_b = q.gram_b > gb ? q.gram_b : gb;
    const size_t eb = eig_ws_bytes((int)m, R);
    q.eig_b = q.eig_b > eb ? q.eig_b : eb;
    q.Gmax = q.Gmax > (int)m ? q.Gmax : (int)m;
    const int64_t out = (int64_t)R * rem;
    q.mbuf = q.mbuf > out ? q.mbuf : out;
  }
  // the CPD of the second core and the Bi-CPD states
  const int64_t d2[3] = {R, dims[1], R};
  q.inner_b = solve_ws_bytes(d2, R, p);
  for (int l = 2; l < L - 1; ++l) {
    const int32_t cd[3] = {R, (int32_t)dims[l], R};
    const size_t sb = state_bytes(cd, R, p->maxiter);
    q.inner_b = q.inner_b > sb ? q.inner_b : sb;
  }
  return true;
}

// Workspace carving, in this order (the size query mirrors it).
template <class Carver>
struct TtWs {
  double *chk, *Ma, *Mb, *G, *lam, *U[TT_MAXL], *W2raw, *Minv, *Mprev, *Wall, *W0pack, *part, *res, *scale;
  int *dest, *flag;
  TtShape* shape;
  char *sws, *gws, *ews, *inner;
  void carve(Carver& ar, const TtPlan& q) {
    const int R = q.R;
    chk = ar.template take<double>(2);
    sws = ar.template take<char>(sumsq_ws_bytes());
    Ma = ar.template take<double>(q.mbuf);
    Mb = ar.template take<double>(q.mbuf);
    G = ar.template take<double>((size_t)q.Gmax * q.Gmax);
    lam = ar.template take<double>(R);
    for (int l = 0; l < q.L - 1; ++l) U[l] = ar.template take<double>((size_t)q.m[l] * R);
    W2raw = ar.template take<double>((size_t)(2 * R + q.dims[1]) * R);
    Minv = ar.template take<double>((size_t)R * R);
    Mprev = ar.template take<double>((size_t)R * R);
    Wall = ar.template take<double>((size_t)q.wrows * R);
    int64_t dmax = 0;
    for (int l = 0; l < q.L; ++l) dmax = dmax > q.dims[l] ? dmax : q.dims[l];
    W0pack = ar.template take<double>((size_t)(2 * R + dmax) * R);
    part = ar.template take<double>(TT_RB);
    res = ar.template take<double>(1);
    scale = ar.template take<double>((size_t)TT_MAXL * 64);
    dest = ar.template take<int>(64);
    flag = ar.template take<int>(1);
    shape = ar.template take<TtShape>(1);
    gws = ar.template take<char>(q.gram_b);
    ews = ar.template take<char>(q.eig_b);
    inner = ar.template take<char>(q.inner_b);
  }
};

// Offsets (doubles) of the start factors of inner CPD c in the packed W0 (the order of the
// seeded generator): core 2: R x R, min(I_2, R) x R, R x R; cores l >= 3: I_l x R, R x R.
int64_t w0_offset(const TtPlan& q, int core) {
  const int R = q.R;
  int64_t o = (int64_t)(2 * R + (q.dims[1] < R ? q.dims[1] : R)) * R;
  if (core == 1) return 0;
  for (int l = 2; l < core; ++l) o += (q.dims[l] + R) * R;
  return o;
}

}  // namespace

size_t tt_ws_bytes(int L, const int64_t* dims, int R, const cpd_params* p) {
  TtPlan q;
  if (!tt_plan(L, dims, R, p, q)) return 0;
  Sizer z;
  TtWs<Sizer> w;
  w.carve(z, q);
  return z.off;
}

cpd_status solve_tt(const void* T, int dtype, int L, const int64_t* dims, int R, const cpd_params* p0,
                    const double* W0, double* const* W_out, double* lambda_out, cpd_solve_info* info, void* ws,
                    size_t ws_bytes, hipStream_t s) {
  TtPlan q;
  if (!tt_plan(L, dims, R, p0, q)) {
    set_error("cpd_solve_tt: needs 4 <= L <= %d, every dim in 1..4096, R <= min(I_1, I_L), R <= 64 (56 when "
              "R I_l > 64), R I_l <= 4096 and R <= the product of the trailing dims", TT_MAXL);
    return CPD_E_INVALID;
  }
  if (dgn_opts(p0)) {
    set_error("cpd_solve_tt: the tensor-train route runs the plain dGN (precond 0, no draw-back)");
    return CPD_E_UNSUPPORTED;
  }
  if (!ws || ws_bytes < tt_ws_bytes(L, dims, R, p0)) {
    set_error("cpd_solve_tt: workspace too small");
    return CPD_E_WORKSPACE;
  }
  // the inner CPDs: classic compression, FP64, the caller's dGN parameters; starts given or random
  cpd_params p = *p0;
  p.st_mlsvd = 0;
  p.refine_iters = 0;
  p.compute_dtype = CPD_F64;
  p.core_dims[0] = p.core_dims[1] = p.core_dims[2] = 0;
  p.init = CPD_INIT_RANDOM;
  Arena ar(ws, ws_bytes);
  TtWs<Arena> w;
  w.carve(ar, q);
  if (!w.inner) {
    set_error("cpd_solve_tt: workspace too small");
    return CPD_E_WORKSPACE;
  }
  cpd_status st;
  // shapes of the factors for the output kernels (one synchronised copy)
  TtShape hs;
  memset(&hs, 0, sizeof(hs));
  hs.L = L;
  hs.R = R;
  long long off = 0;
  for (int l = 0; l < L; ++l) {
    hs.dims[l] = (int)dims[l];
    hs.off[l] = off;
    off += dims[l];
  }
  CPD_HIP_CHECK(hipMemcpyAsync(w.shape, &hs, sizeof(hs), hipMemcpyHostToDevice, s));
  // ||T||^2 and the non-finite check
  if ((st = sumsq_full(T, dtype, q.N, w.chk, (int*)(w.chk + 1), w.sws, sumsq_ws_bytes(), s))) return st;
  double hchk[2];
  CPD_HIP_CHECK(hipMemcpyAsync(hchk, w.chk, sizeof(hchk), hipMemcpyDeviceToHost, s));
  CPD_HIP_CHECK(hipStreamSynchronize(s));
  int bad = 0;
  memcpy(&bad, &hchk[1], sizeof(int));
  if (bad) { set_error("cpd_solve_tt: non-finite entries in T"); return CPD_E_NONFINITE; }
  if (!(hchk[0] > 0.0)) { set_error("cpd_solve_tt: ||T|| = 0"); return CPD_E_ZERO_TENSOR; }

  // TT-SVD: M (m x n) = the current tensor; U = leading R eigenvectors of M M^T; M <- U^T M
  const void* M = T;
  int mdt = dtype;
  double* bufs[2] = {w.Ma, w.Mb};
  for (int l = 0; l < L - 1; ++l) {
    const int m = q.m[l];
    const int64_t n = q.n[l];
    const int64_t gd[3] = {m, 1, n};
    if ((st = gram(M, mdt, gd, 0, CPD_F64, w.G, w.gws, q.gram_b, s))) return st;
    if ((st = eig_top(w.G, m, R, w.U[l], w.lam, w.ews, q.eig_b, s))) return st;
    double* out = bufs[l & 1];
    if ((st = gemm_f64(R, (int)n, m, 1.0, w.U[l], R, 0, true, M, mdt, n, 0, false, 0.0, out, n, 0, 1, s))) return st;
    M = out;
    mdt = CPD_F64;
  }
  const double* GL = (const double*)M;   // R x I_L

  // CPD of the second core (R x I_2 x R): (M1, W2, M2)
  const int64_t d2[3] = {R, dims[1], R};
  int it2 = 0, stop2 = 0;
  double err2 = 0.0;
  if ((st = solve3_raw(w.U[1], d2, R, &p, W0 ? W0 + w0_offset(q, 1) : nullptr, w.W2raw, &it2, &stop2, &err2, w.inner,
                       q.inner_b, s)))
    return st;
  const double* M1 = w.W2raw;
  double* Wall = w.Wall;
  // W2 into the packed output rows of mode 2
  CPD_HIP_CHECK(hipMemcpyAsync(Wall + hs.off[1] * R, w.W2raw + (size_t)R * R, sizeof(double) * dims[1] * R,
                               hipMemcpyDeviceToDevice, s));
  CPD_HIP_CHECK(hipMemcpyAsync(w.Mprev, w.W2raw + (size_t)(R + dims[1]) * R, sizeof(double) * R * R,
                               hipMemcpyDeviceToDevice, s));
  int iters_total = it2, last_stop = stop2;
  double worst_err = err2;
  CPD_HIP_CHECK(hipMemsetAsync(w.flag, 0, sizeof(int), s));   // set by a singular third factor
  // Bi-CPDs of cores 3..L-1 with the first factor fixed to M_prev^{-T}
  for (int l = 2; l < L - 1; ++l) {
    hipLaunchKernelGGL(inverse_transpose_kernel, dim3(1), dim3(TT_NT), 0, s, w.Mprev, R, w.Minv, w.flag);
    CPD_LAUNCH_CHECK();
    const int Il = (int)dims[l];
    // start: [F; W_l; M_l], packed rows
    CPD_HIP_CHECK(hipMemcpyAsync(w.W0pack, w.Minv, sizeof(double) * R * R, hipMemcpyDeviceToDevice, s));
    if (W0) {
      CPD_HIP_CHECK(hipMemcpyAsync(w.W0pack + (size_t)R * R, W0 + w0_offset(q, l), sizeof(double) * (Il + R) * R,
                                   hipMemcpyDeviceToDevice, s));
    } else {
      if ((st = fill_randn(w.W0pack + (size_t)R * R, (Il + R) * R, p.seed * 131 + l, s))) return st;
    }
    const int32_t cd[3] = {R, Il, R};
    char* state = w.inner;
    cpd_params pg = p;
    pg.init = CPD_INIT_GIVEN;
    if ((st = state_init(state, w.U[l], cd, R, w.W0pack, 0.0, &pg, s, true, HDR_FIX0))) return st;
    if ((st = dgn_iterate_known(state, w.U[l], cd, R, pg.maxiter, s))) return st;
    const int np = (R + Il + R) * R;
    const double* Wst = (const double*)(state + layout_of(np, R, pg.maxiter).W);
    CPD_HIP_CHECK(hipMemcpyAsync(Wall + hs.off[l] * R, Wst + (size_t)R * R, sizeof(double) * Il * R,
                                 hipMemcpyDeviceToDevice, s));
    CPD_HIP_CHECK(hipMemcpyAsync(w.Mprev, Wst + (size_t)(R + Il) * R, sizeof(double) * R * R,
                                 hipMemcpyDeviceToDevice, s));
    int k = 0, sr = 0;
    double e = 0.0;
    if ((st = state_read(state, &k, &sr, nullptr, &e, s))) return st;
    iters_total += k;
    last_stop = sr;
    worst_err = worst_err > e ? worst_err : e;
  }
  // outer factors: W1 = G1 M1 (I_1 x R), W_L = G_L^T M_{L-1} (I_L x R)
  if ((st = gemm_f64((int)dims[0], R, R, 1.0, w.U[0], R, 0, false, M1, CPD_F64, R, 0, false, 0.0, Wall, R, 0, 1, s)))
    return st;
  if ((st = gemm_f64((int)dims[L - 1], R, R, 1.0, GL, (int)dims[L - 1], 0, true, w.Mprev, CPD_F64, R, 0, false, 0.0,
                     Wall + hs.off[L - 1] * R, R, 0, 1, s)))
    return st;
  // full error on the input tensor, then the normalised output
  switch (dtype) {
    case CPD_F64:
      hipLaunchKernelGGL(tt_residual_kernel<double>, dim3(TT_RB), dim3(TT_NT), 0, s, (const double*)T, (long long)q.N,
                         w.shape, Wall, w.part);
      break;
    case CPD_F32:
      hipLaunchKernelGGL(tt_residual_kernel<float>, dim3(TT_RB), dim3(TT_NT), 0, s, (const float*)T, (long long)q.N,
                         w.shape, Wall, w.part);
      break;
    default:
      set_error("cpd_solve_tt: dtype must be CPD_F64 or CPD_F32");
      return CPD_E_INVALID;
  }
  CPD_LAUNCH_CHECK();
  hipLaunchKernelGGL(tt_final_sum_kernel, dim3(1), dim3(TT_NT), 0, s, w.part, TT_RB, w.res);
  CPD_LAUNCH_CHECK();
  hipLaunchKernelGGL(tt_normalize_plan_kernel, dim3(1), dim3(TT_NT), 0, s, w.shape, Wall, w.scale, w.dest, lambda_out);
  CPD_LAUNCH_CHECK();
  for (int l = 0; l < L; ++l) {
    const long long rows = dims[l];
    hipLaunchKernelGGL(tt_normalize_apply_kernel, dim3((unsigned)((rows * R + 255) / 256)), dim3(256), 0, s,
                       Wall + hs.off[l] * R, rows, R, w.scale + l * 64, w.dest, W_out[l]);
    CPD_LAUNCH_CHECK();
  }
  double h_res = 0.0;
  int h_sing = 0;
  CPD_HIP_CHECK(hipMemcpyAsync(&h_res, w.res, sizeof(double), hipMemcpyDeviceToHost, s));
  CPD_HIP_CHECK(hipMemcpyAsync(&h_sing, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  CPD_HIP_CHECK(hipStreamSynchronize(s));
  memset(info, 0, sizeof(*info));
  info->iters = iters_total;
  info->stop_reason = last_stop;
  info->core_dims[0] = info->core_dims[1] = info->core_dims[2] = R;
  info->tol_iter = -1;
  info->rel_err_core = worst_err;
  info->t_norm = sqrt(hchk[0]);
  info->rel_err_full = sqrt(h_res > 0.0 ? h_res : 0.0) / info->t_norm;
  info->time_to_tol_ns = -1;
  if (h_sing) {
    set_error("cpd_solve_tt: a core's third factor is singular");
    return CPD_E_NONFINITE;
  }
  return CPD_OK;
}

}  // namespace cpd
