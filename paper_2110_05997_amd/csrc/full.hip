// Kernels on the full (uncompressed) tensor and the output stage.
//  * residual_full: ||T - sum_r w_r^(1) o w_r^(2) o w_r^(3)||^2 fused with its reduction (the
//    residual of ch.4 "Computing the residual" evaluated on T instead of the core);
//  * sumsq_full: ||T||^2 with detection of NaN/Inf;
//  * normalize_output: unit columns and lambda (ch.4 flow chart output).
// Reductions go through per-block partials summed in a fixed order (bit-reproducible).
#include "common.h"

#include <mutex>

namespace cpd {
namespace {

constexpr int RB = 1024;   // number of partial sums (fixed grid for determinism)
constexpr int RNT = 256;

template <class T>
__device__ __forceinline__ double ldv(const T* p, long long i) { return (double)p[i]; }
template <class T>
__device__ __forceinline__ double to_f64(T v) { return (double)v; }
template <>
__device__ __forceinline__ double to_f64<uint16_t>(uint16_t v) { return bf16_bits_to_f64(v); }
template <>
__device__ __forceinline__ double ldv<uint16_t>(const uint16_t* p, long long i) { return bf16_bits_to_f64(p[i]); }

// Tiles of RJB fibres (i, j0..j0+RJB-1) with threads over k: the R values W2[k][.] of a thread's k
// stay in registers (R <= 8 RC), a_jr = W0[i][r] W1[j][r] of the tile is staged in LDS and read
// by broadcast, and the RJB model values of a thread are independent FMA chains.  Each model
// value is sum_r a_jr W2[k][r] in increasing r.  Fixed grid, fixed order: bit-reproducible.
constexpr int RJB = 8;

template <class T, int RC>
__global__ __launch_bounds__(RNT) void residual_kernel(const T* __restrict__ X, int I1, int I2, int I3,
                                                       const double* __restrict__ W0,
                                                       const double* __restrict__ W1,
                                                       const double* __restrict__ W2, int R,
                                                       double* __restrict__ part) {
  constexpr int RM = 8 * RC;
  __shared__ double a[RJB][RM];
  __shared__ double slots[RNT / 64];
  const int njb = (I2 + RJB - 1) / RJB;
  const int ntiles = I1 * njb;
  const int R1 = R - 1;
  double acc = 0.0;
  for (int k0 = 0; k0 < I3; k0 += RNT) {
    const int k = k0 + (int)threadIdx.x;
    const bool kin = k < I3;
    const int kc = kin ? k : I3 - 1;
    double w[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) w[r] = (r < R) ? W2[(size_t)kc * R + min(r, R1)] : 0.0;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
      const int i = t / njb, j0 = (t - i * njb) * RJB;
      __syncthreads();
      for (int e = threadIdx.x; e < RJB * RM; e += RNT) {
        const int jj = e / RM, r = e - jj * RM;
        const int j = j0 + jj;
        a[jj][r] = (j < I2 && r < R) ? W0[(size_t)i * R + min(r, R1)] * W1[(size_t)min(j, I2 - 1) * R + min(r, R1)] : 0.0;
      }
      __syncthreads();
      const int nj = min(RJB, I2 - j0);
      const T* x = X + ((size_t)i * I2 + j0) * I3 + kc;
#pragma unroll
      for (int jj = 0; jj < RJB; ++jj) {
        double model = 0.0;
#pragma unroll
        for (int r = 0; r < RM; ++r) model += a[jj][r] * w[r];
        const double d = ldv(x, (long long)min(jj, nj - 1) * I3) - model;
        acc += (kin && jj < nj) ? d * d : 0.0;
      }
    }
  }
  const double s = block_sum(acc, slots);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Residual on the FP64 matrix cores (R <= 64), work in tasks (row i of mode 1, RM_KW columns k of
// mode 3): the task's B[r][kk] = W0[i][r] W2[k0 + kk][r] is staged in LDS once, and the model of
// 16 rows (i, j0..j0+15) by RM_KW columns is the product of the W1 rows j (the A fragments, one
// load each) with B, a 16 x 64 MFMA tile over the R <= 4 NU contraction.  Each wave takes every
// fourth block of rows j, and for up to 13 contraction steps (NU, fixed at compile time) loads the
// tensor values and A fragments of its next block while it multiplies the current one.  The grid is fixed (RB workgroups, each a contiguous run
// of tasks) and every sum runs in a fixed order: bit-reproducible.
constexpr int RM_KW = 64;
typedef double rdbl4 __attribute__((ext_vector_type(4)));

// two waves per SIMD where the register sets fit in 256 registers (FP32/BF16 input, or up to 8
// contraction steps), else one
template <class T, int NU>
constexpr int res_waves() { return sizeof(T) <= 4 || NU <= 8 ? 2 : 1; }

// EXACT: the contraction takes all NU steps ((R + 3) / 4 == NU), so no step needs its test
template <class T, int NU, bool EXACT>
__global__ __launch_bounds__(RNT, (res_waves<T, NU>())) void residual_mfma_kernel(const T* __restrict__ X, int I1, int I2, int I3,
                                                            const double* __restrict__ W0,
                                                            const double* __restrict__ W1,
                                                            const double* __restrict__ W2, int R,
                                                            double* __restrict__ part) {
  __shared__ double slots[RNT / 64];
  // row pitch 80 doubles: the four rows kq of a fragment read fall 32 banks apart, so the 64 lanes'
  // 8-byte reads are free of bank conflicts
  __shared__ double Bs[64][RM_KW + 16];
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4, w = threadIdx.x >> 6;
  constexpr int NWV = RNT / 64;
  const int nkr = (I3 + RM_KW - 1) / RM_KW;
  const long long ntask = (long long)I1 * nkr;
  const int njb = (I2 + 15) / 16;
  const int nu = (R + 3) / 4;   // contraction steps of four (at most NU)
  double acc = 0.0;
  // one block: tensor values tv[v][n] at row j0 + 4 v + kq, column k0 + 16 n + r16, and the A
  // fragments av[u] = W1[j0 + r16][4 u + kq] (zero outside the matrices; addresses clamped)
  auto load = [&](int i, int k0, int jb, T (&tv)[4][4], double (&av)[NU]) {
    const int j = jb * 16 + r16;
    const bool jok = j < I2;
    const double* w1 = W1 + (long long)(jok ? j : I2 - 1) * R;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int r = 4 * u + kq;
      const double x = w1[r < R ? r : R - 1];
      av[u] = (jok && r < R) ? x : 0.0;
    }
    // raw tensor values (converted at the products): in the input's own width, so the prefetched
    // set costs half the registers for FP32 input
    const T* xr = X + ((long long)i * I2 + (long long)jb * 16) * I3 + k0;
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const int jr = jb * 16 + 4 * v + kq, k = k0 + 16 * n + r16;
        const bool ok = jr < I2 && k < I3;
        tv[v][n] = xr[ok ? (long long)(4 * v + kq) * I3 + 16 * n + r16 : 0ll];
      }
  };
  auto compute = [&](int jb, int k0, const T (&tv)[4][4], const double (&av)[NU]) {
    // B is reread from LDS for every block (kept in registers it would leave room for one wave per
    // SIMD only); the next step's fragments are read while the current step's MFMAs run
    asm volatile("" ::: "memory");
    rdbl4 am[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) am[n] = rdbl4{0.0, 0.0, 0.0, 0.0};
    double bf[4], bn[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) bf[n] = Bs[kq][16 * n + r16];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      if (EXACT || u < nu) {
        const int un = u + 1 < NU ? u + 1 : u;
#pragma unroll
        for (int n = 0; n < 4; ++n) bn[n] = Bs[4 * un + kq][16 * n + r16];
#pragma unroll
        for (int n = 0; n < 4; ++n) am[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bf[n], am[n], 0, 0, 0);
#pragma unroll
        for (int n = 0; n < 4; ++n) bf[n] = bn[n];
      }
      __builtin_amdgcn_sched_barrier(0);   // two steps' B fragments in registers at a time
    }
    // am[n][v] is the model at row 4 v + kq of the block, column 16 n + r16 (zero where tv is)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const int jr = jb * 16 + 4 * v + kq, k = k0 + 16 * n + r16;
        const double d = (jr < I2 && k < I3) ? to_f64(tv[v][n]) - am[n][v] : 0.0;
        acc += d * d;
      }
  };
  T tA[4][4], tB[4][4];
  double aA[NU], aB[NU];
  // a contiguous run of tasks per workgroup: neighbouring column ranges of one row i follow each
  // other on the same compute unit, so the cache lines they share (rows are not line-aligned) are
  // read from memory once
  const long long tb = ntask * blockIdx.x / gridDim.x, te = ntask * (blockIdx.x + 1) / gridDim.x;
  for (long long t = tb; t < te; ++t) {
    const int i = (int)(t / nkr), kr = (int)(t - (long long)i * nkr), k0 = kr * RM_KW;
    __syncthreads();   // the previous task's products no longer read Bs
    const double* w0 = W0 + (long long)i * R;
    for (int e = threadIdx.x; e < 64 * RM_KW; e += RNT) {
      const int r = e / RM_KW, kk = e - r * RM_KW, k = k0 + kk;   // lanes along a row of B
      const bool ok = r < R && k < I3;
      const double x = W2[(long long)(ok ? k : 0) * R + (ok ? r : 0)] * w0[ok ? r : 0];
      Bs[r][kk] = ok ? x : 0.0;
    }
    __syncthreads();
    if constexpr (NU > 13) {
      // one register set (two would not fit two waves per SIMD)
      for (int jb = w; jb < njb; jb += NWV) {
        load(i, k0, jb, tA, aA);
        compute(jb, k0, tA, aA);
      }
      continue;
    }
    // two register sets in turn; the loads of a block past the last are clamped and unused
    if (w < njb) load(i, k0, w, tA, aA);
    for (int jb = w; jb < njb; jb += 2 * NWV) {
      load(i, k0, min(jb + NWV, njb - 1), tB, aB);
      __builtin_amdgcn_sched_barrier(0);
      compute(jb, k0, tA, aA);
      __builtin_amdgcn_sched_barrier(0);
      if (jb + NWV >= njb) break;
      load(i, k0, min(jb + 2 * NWV, njb - 1), tA, aA);
      __builtin_amdgcn_sched_barrier(0);
      compute(jb + NWV, k0, tB, aB);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  const double sres = block_sum(acc, slots);
  if (threadIdx.x == 0) part[blockIdx.x] = sres;
}

template <class T>
void launch_residual(const T* X, int I1, int I2, int I3, const double* const W[3], int R, double* part,
                     hipStream_t s) {
  if (R <= 64 && (long long)I1 * I2 < (1ll << 31) - 16) {
    const int nu = (R + 3) / 4;
    auto k = nu == 13 ? residual_mfma_kernel<T, 13, true> : nu == 16 ? residual_mfma_kernel<T, 16, true>
           : R <= 16 ? residual_mfma_kernel<T, 4, false> : R <= 32 ? residual_mfma_kernel<T, 8, false>
           : R <= 52 ? residual_mfma_kernel<T, 13, false> : residual_mfma_kernel<T, 16, false>;
    hipLaunchKernelGGL(k, dim3(RB), dim3(RNT), 0, s, X, I1, I2, I3, W[0], W[1], W[2], R, part);
    return;
  }
  switch ((R + 7) / 8) {
#define CPD_RES_CASE(rc)                                                                               \
  case rc:                                                                                             \
    hipLaunchKernelGGL((residual_kernel<T, rc>), dim3(RB), dim3(RNT), 0, s, X, I1, I2, I3, W[0], W[1], \
                       W[2], R, part);                                                                 \
    break;
    CPD_RES_CASE(1) CPD_RES_CASE(2) CPD_RES_CASE(3) CPD_RES_CASE(4)
    CPD_RES_CASE(5) CPD_RES_CASE(6) CPD_RES_CASE(7) CPD_RES_CASE(8)
#undef CPD_RES_CASE
    default: break;
  }
}

// Squares of the 16 / sizeof(T) entries packed in one 16-byte word, added in order; a
// non-finite entry sets nf.
template <class T>
__device__ __forceinline__ void sumsq_word(const uint4& q, double& acc, double& nf) {
  const uint32_t w[4] = {q.x, q.y, q.z, q.w};
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double v = __builtin_bit_cast(double, ((uint64_t)w[2 * i + 1] << 32) | w[2 * i]);
      if (!isfinite(v)) nf = 1.0;
      acc += v * v;
    }
  } else if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double v = (double)__builtin_bit_cast(float, w[i]);
      if (!isfinite(v)) nf = 1.0;
      acc += v * v;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double lo = (double)__builtin_bit_cast(float, w[i] << 16);
      const double hi = (double)__builtin_bit_cast(float, w[i] & 0xffff0000u);
      if (!isfinite(lo) || !isfinite(hi)) nf = 1.0;
      acc += lo * lo;
      acc += hi * hi;
    }
  }
}

// ||X||^2 partials, one per block: the 16-byte words of the aligned body are strided over the
// grid with SQ_U loads in flight per thread; the unaligned head and the tail (fewer than one
// word per thread of the grid) go entry by entry.  Fixed grid, fixed order: bit-reproducible.
constexpr int SQ_U = 4;

template <class T>
__global__ __launch_bounds__(RNT) void sumsq_kernel(const T* __restrict__ X, long long n,
                                                    double* __restrict__ part, double* __restrict__ badp,
                                                    long long* __restrict__ stamp) {
  __shared__ double slots[2][RNT / 64];
  // the first kernel of a solve: its start is the solve's device entry time
  if (stamp != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *stamp = wall_clock64();
  constexpr int EPW = 16 / (int)sizeof(T);   // entries per word
  const long long head = (long long)((16 - ((uintptr_t)X & 15)) & 15) / (long long)sizeof(T);
  const bool aligned = ((uintptr_t)X % sizeof(T)) == 0;
  const long long h = aligned ? (head < n ? head : n) : n;
  const long long nw = (n - h) / EPW;        // whole words of the body
  const uint4* Xw = reinterpret_cast<const uint4*>(X + h);
  const long long gid = (long long)blockIdx.x * RNT + threadIdx.x;
  const long long stride = (long long)gridDim.x * RNT;
  double acc = 0.0, nf = 0.0;
  long long v = gid;
  for (; v + (SQ_U - 1) * stride < nw; v += SQ_U * stride) {
    uint4 q[SQ_U];
#pragma unroll
    for (int u = 0; u < SQ_U; ++u) q[u] = Xw[v + u * stride];
#pragma unroll
    for (int u = 0; u < SQ_U; ++u) sumsq_word<T>(q[u], acc, nf);
  }
  for (; v < nw; v += stride) sumsq_word<T>(Xw[v], acc, nf);
  // head entries, then the tail entries after the last whole word
  for (long long e = gid; e < h; e += stride) {
    const double x = ldv(X, e);
    if (!isfinite(x)) nf = 1.0;
    acc += x * x;
  }
  for (long long e = h + nw * EPW + gid; e < n; e += stride) {
    const double x = ldv(X, e);
    if (!isfinite(x)) nf = 1.0;
    acc += x * x;
  }
  const double s = block_sum(acc, slots[0]);
  const double b = block_sum(nf, slots[1]);
  if (threadIdx.x == 0) { part[blockIdx.x] = s; badp[blockIdx.x] = b; }
}

// The sum of the per-block partials and, when `out_flag` is given, whether any block saw a
// non-finite entry: one launch for both.
__global__ void final_sum_flag_kernel(const double* __restrict__ part, const double* __restrict__ badp, int n,
                                      double* __restrict__ out, int* __restrict__ out_flag) {
  __shared__ double slots[2][RNT / 64];
  double acc = 0.0, nb = 0.0;
  for (int i = threadIdx.x; i < n; i += RNT) {
    acc += part[i];
    if (out_flag) nb += badp[i];
  }
  const double s = block_sum(acc, slots[0]);
  const double b = block_sum(nb, slots[1]);
  if (threadIdx.x == 0) {
    *out = s;
    if (out_flag) *out_flag = (b > 0.0) ? 1 : 0;
  }
}

__global__ void final_sum_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double slots[RNT / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += RNT) acc += part[i];
  const double s = block_sum(acc, slots);
  if (threadIdx.x == 0) *out = s;
}

// Column norms, lambda, signs and order of the uncompressed factors (one workgroup).  Lane =
// column (loads along a row are coalesced), 16 row groups of 1024 threads, partial results
// combined in a fixed order; the sign comes from the largest-|.| entry of modes 1 and 2 (ties:
// lowest index).
constexpr int NP_NT = 1024;
constexpr int NP_G = NP_NT / 64;

__global__ __launch_bounds__(NP_NT) void normalize_plan_kernel(const double* __restrict__ W0, const double* __restrict__ W1,
                                                              const double* __restrict__ W2, int I1, int I2, int I3, int R,
                                                              double* __restrict__ scale, int* __restrict__ dest,
                                                              double* __restrict__ lambda, const int* __restrict__ skip) {
  __shared__ double ps[NP_G][64];
  __shared__ double pb[NP_G][64];
  __shared__ int px[NP_G][64];
  __shared__ double nrm[3][64];
  __shared__ double lam[64];
  __shared__ double sgn[2][64];
  const int tid = threadIdx.x, r = tid & 63, q = tid >> 6;
  for (int l = 0; l < 3; ++l) {
    const double* W = (l == 0) ? W0 : (l == 1 ? W1 : W2);
    const int I = (l == 0) ? I1 : (l == 1 ? I2 : I3);
    double s = 0.0, best = -1.0;
    int bi = 0;   // stays a valid index if every entry is NaN
    if (r < R) {
      for (int i = q; i < I; i += NP_G) {
        const double v = W[(long long)i * R + r];
        s += v * v;
        const double a = fabs(v);
        if (a > best) { best = a; bi = i; }   // rows ascend: the first maximum is kept
      }
    }
    ps[q][r] = s;
    pb[q][r] = best;
    px[q][r] = bi;
    __syncthreads();
    if (q == 0 && r < R) {
      double t = 0.0;
      for (int g = 0; g < NP_G; ++g) t += ps[g][r];
      nrm[l][r] = sqrt(t);
      if (l < 2) {
        double b = pb[0][r];
        int ix = px[0][r];
        for (int g = 1; g < NP_G; ++g)
          if (pb[g][r] > b || (pb[g][r] == b && px[g][r] < ix)) { b = pb[g][r]; ix = px[g][r]; }
        sgn[l][r] = (W[(long long)ix * R + r] < 0.0) ? -1.0 : 1.0;
      }
    }
    __syncthreads();
  }
  if (tid < R) lam[tid] = (nrm[0][tid] * nrm[1][tid]) * nrm[2][tid];
  __syncthreads();
  if (tid < R) {
    const int rr = tid;
    int rank = 0;
    for (int s2 = 0; s2 < R; ++s2)
      if (lam[s2] > lam[rr] || (lam[s2] == lam[rr] && s2 < rr)) ++rank;
    dest[rr] = rank;
    if (!(skip && (*skip & 1))) lambda[rank] = lam[rr];
    for (int l = 0; l < 3; ++l) {
      double sc = (nrm[l][rr] > 0.0) ? 1.0 / nrm[l][rr] : 1.0;
      if (l < 2) sc *= sgn[l][rr];
      else sc *= sgn[0][rr] * sgn[1][rr];
      scale[l * 64 + rr] = sc;
    }
  }
}

__global__ void normalize_apply_kernel(const double* __restrict__ Wt, int I, int R,
                                       const double* __restrict__ scale, const int* __restrict__ dest,
                                       double* __restrict__ Wout, const int* __restrict__ skip) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)I * R || (skip && (*skip & 1))) return;
  const int r = (int)(e % R);
  const long long i = e / R;
  Wout[i * R + dest[r]] = Wt[e] * scale[r];
}

}  // namespace

size_t residual_ws_bytes(const int64_t dims[3]) {
  (void)dims;
  return align_up(RB * sizeof(double), 256);
}

size_t sumsq_ws_bytes() { return 2 * align_up(RB * sizeof(double), 256); }

namespace {
// The two launches of the fused residual: per-block partials in `part` (RB doubles), then their sum
// in a fixed order into *out.  Arguments already checked.
cpd_status residual_launch(const void* T, int dtype, const int64_t dims[3], const double* const W[3], int R,
                           double* out, double* part, hipStream_t s, bool timed) {
  const int I1 = (int)dims[0], I2 = (int)dims[1], I3 = (int)dims[2];
  if (timed) prof_begin(CPD_PK_RESIDUAL, s);
  switch (dtype) {
    case CPD_F64:
      launch_residual((const double*)T, I1, I2, I3, W, R, part, s);
      break;
    case CPD_F32:
      launch_residual((const float*)T, I1, I2, I3, W, R, part, s);
      break;
    case CPD_BF16:
      launch_residual((const uint16_t*)T, I1, I2, I3, W, R, part, s);
      break;
    default:
      set_error("residual_full: bad dtype");
      return CPD_E_INVALID;
  }
  if (timed) prof_end(CPD_PK_RESIDUAL, s);
  CPD_LAUNCH_CHECK();
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(RNT), 0, s, part, RB, out);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

bool residual_args_ok(const void* T, int dtype, const double* const W[3], int R, const double* out) {
  if (R < 1 || R > 64 || !T || !out || !W[0] || !W[1] || !W[2]) {
    set_error("residual_full: bad arguments");
    return false;
  }
  if (dtype != CPD_F64 && dtype != CPD_F32 && dtype != CPD_BF16) {
    set_error("residual_full: bad dtype");
    return false;
  }
  return true;
}

// Scratch of the allocation-free residual (cpd_residual_norm2_noalloc): the per-block partial sums.
// One copy per GPU, held until the process ends; every call on a GPU shares it.
constexpr size_t NOALLOC_SCRATCH_BYTES = 64 * 1024;
__device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on each GPU, looked up once per device with that device current (in
// host code the array's name is only a stand-in for the symbol).
constexpr int NOALLOC_MAX_DEVICES = 64;
char* g_scratch_ptr[NOALLOC_MAX_DEVICES];
std::mutex g_scratch_mu;

cpd_status scratch_address(char** out) {
  int dev = 0;
  CPD_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    set_error("residual_norm2_noalloc: device %d beyond %d", dev, NOALLOC_MAX_DEVICES);
    return CPD_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error("residual_norm2_noalloc: hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
      return CPD_E_HIP;
    }
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return CPD_OK;
}
}  // namespace

cpd_status residual_full(const void* T, int dtype, const int64_t dims[3], const double* const W[3],
                         int R, double* out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!residual_args_ok(T, dtype, W, R, out)) return CPD_E_INVALID;
  if (!ws || ws_bytes < residual_ws_bytes(dims)) {
    set_error("residual_full: workspace too small");
    return CPD_E_WORKSPACE;
  }
  return residual_launch(T, dtype, dims, W, R, out, (double*)ws, s, true);
}

cpd_status residual_full_noalloc(const void* T, int dtype, const int64_t dims[3], const double* const W[3],
                                 int R, double* out, hipStream_t s) {
  if (!residual_args_ok(T, dtype, W, R, out)) return CPD_E_INVALID;
  const size_t need = residual_ws_bytes(dims);
  if (need > NOALLOC_SCRATCH_BYTES) {
    set_error("residual_norm2_noalloc: needs %zu scratch bytes, the static buffer holds %zu", need,
              NOALLOC_SCRATCH_BYTES);
    return CPD_E_UNSUPPORTED;
  }
  char* sp = nullptr;
  cpd_status st = scratch_address(&sp);
  if (st) return st;
  // every partial is written by the first launch before the second reads it: nothing to clear
  return residual_launch(T, dtype, dims, W, R, out, (double*)sp, s, false);
}

cpd_status sumsq_full(const void* T, int dtype, int64_t n, double* out, int* nonfinite, void* ws,
                      size_t ws_bytes, hipStream_t s, long long* stamp) {
  if (!ws || ws_bytes < sumsq_ws_bytes()) {
    set_error("sumsq_full: workspace too small");
    return CPD_E_WORKSPACE;
  }
  double* part = (double*)ws;
  double* bad = (double*)((char*)ws + align_up(RB * sizeof(double), 256));
  switch (dtype) {
    case CPD_F64:
      hipLaunchKernelGGL(sumsq_kernel<double>, dim3(RB), dim3(RNT), 0, s, (const double*)T, (long long)n, part, bad, stamp);
      break;
    case CPD_F32:
      hipLaunchKernelGGL(sumsq_kernel<float>, dim3(RB), dim3(RNT), 0, s, (const float*)T, (long long)n, part, bad, stamp);
      break;
    case CPD_BF16:
      hipLaunchKernelGGL(sumsq_kernel<uint16_t>, dim3(RB), dim3(RNT), 0, s, (const uint16_t*)T, (long long)n, part, bad, stamp);
      break;
    default:
      set_error("sumsq_full: bad dtype");
      return CPD_E_INVALID;
  }
  CPD_LAUNCH_CHECK();
  hipLaunchKernelGGL(final_sum_flag_kernel, dim3(1), dim3(RNT), 0, s, part, bad, RB, out, nonfinite);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

// ||T||^2 and the non-finite flag from the mode-1 Gram when it was formed from T in FP64: its
// trace is the sum of the squared entries (each product exact, FP64 accumulation), and a NaN or
// infinite entry leaves a non-finite diagonal entry.  Saves a pass over T; the sum runs in a
// fixed order (bit-reproducible).
__global__ void gram_trace_flag_kernel(const double* __restrict__ G, int n, double* __restrict__ out,
                                       int* __restrict__ out_flag) {
  __shared__ double slots[2][RNT / 64];
  double acc = 0.0, nb = 0.0;
  for (int i = threadIdx.x; i < n; i += RNT) {
    const double d = G[(long long)i * n + i];
    acc += d;
    nb += isfinite(d) ? 0.0 : 1.0;
  }
  const double sum = block_sum(acc, slots[0]);
  const double b = block_sum(nb, slots[1]);
  if (threadIdx.x == 0) {
    *out = sum;
    *out_flag = (b > 0.0 || !isfinite(sum)) ? 1 : 0;
  }
}

// The device wall clock at the start of a solve (its entry stamp).
__global__ void stamp_kernel(long long* __restrict__ t) { *t = wall_clock64(); }

cpd_status gram_trace_check(const double* G, int n, double* out, int* nonfinite, hipStream_t s) {
  hipLaunchKernelGGL(gram_trace_flag_kernel, dim3(1), dim3(RNT), 0, s, G, n, out, nonfinite);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

cpd_status device_stamp(long long* t, hipStream_t s) {
  hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(1), 0, s, t);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

size_t normalize_ws_bytes(int R) {
  (void)R;
  return align_up(3 * 64 * sizeof(double), 256) + align_up(64 * sizeof(int), 256);
}

cpd_status normalize_output(const double* const Wt[3], const int64_t dims[3], int R,
                            double* const Wout[3], double* lambda, void* ws, size_t ws_bytes,
                            hipStream_t s, const int* skip) {
  if (R < 1 || R > 64) {
    set_error("normalize_output: R out of range");
    return CPD_E_INVALID;
  }
  if (!ws || ws_bytes < normalize_ws_bytes(R)) {
    set_error("normalize_output: workspace too small");
    return CPD_E_WORKSPACE;
  }
  double* scale = (double*)ws;
  int* dest = (int*)((char*)ws + align_up(3 * 64 * sizeof(double), 256));
  hipLaunchKernelGGL(normalize_plan_kernel, dim3(1), dim3(NP_NT), 0, s, Wt[0], Wt[1], Wt[2], (int)dims[0],
                     (int)dims[1], (int)dims[2], R, scale, dest, lambda, skip);
  CPD_LAUNCH_CHECK();
  for (int l = 0; l < 3; ++l) {
    const long long n = dims[l] * (long long)R;
    hipLaunchKernelGGL(normalize_apply_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Wt[l],
                       (int)dims[l], R, scale + l * 64, dest, Wout[l], skip);
    CPD_LAUNCH_CHECK();
  }
  return CPD_OK;
}

}  // namespace cpd
