// Kernels on the full (uncompressed) tensor and the output stage.
//  * residual_full: ||T - sum_r w_r^(1) o w_r^(2) o w_r^(3)||^2 fused with its reduction (the
//    residual of ch.4 "Computing the residual" evaluated on T instead of the core);
//  * sumsq_full: ||T||^2 with detection of NaN/Inf;
//  * normalize_output: unit columns and lambda (ch.4 flow chart output).
// Reductions go through per-block partials summed in a fixed order (bit-reproducible).
#include "common.h"

namespace cpd {
namespace {

constexpr int RB = 1024;   // number of partial sums (fixed grid for determinism)
constexpr int RNT = 256;

template <class T>
__device__ __forceinline__ double ldv(const T* p, long long i) { return (double)p[i]; }
template <>
__device__ __forceinline__ double ldv<uint16_t>(const uint16_t* p, long long i) { return bf16_bits_to_f64(p[i]); }

// One fibre (i, j) at a time: a_r = W0[i][r] W1[j][r] staged in LDS, threads over k.
template <class T>
__global__ __launch_bounds__(RNT) void residual_kernel(const T* __restrict__ X, int I1, int I2, int I3,
                                                       const double* __restrict__ W0,
                                                       const double* __restrict__ W1,
                                                       const double* __restrict__ W2, int R,
                                                       double* __restrict__ part) {
  __shared__ double a[64];
  __shared__ double slots[RNT / 64];
  const long long nf = (long long)I1 * I2;
  double acc = 0.0;
  for (long long f = blockIdx.x; f < nf; f += gridDim.x) {
    const int i = (int)(f / I2), j = (int)(f % I2);
    __syncthreads();
    if (threadIdx.x < R) a[threadIdx.x] = W0[(long long)i * R + threadIdx.x] * W1[(long long)j * R + threadIdx.x];
    __syncthreads();
    const long long base = f * I3;
    for (int k = threadIdx.x; k < I3; k += RNT) {
      const double* w2 = W2 + (long long)k * R;
      double model = 0.0;
      for (int r = 0; r < R; ++r) model += a[r] * w2[r];
      const double d = ldv(X, base + k) - model;
      acc += d * d;
    }
  }
  const double s = block_sum(acc, slots);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <class T>
__global__ __launch_bounds__(RNT) void sumsq_kernel(const T* __restrict__ X, long long n,
                                                    double* __restrict__ part, double* __restrict__ badp) {
  __shared__ double slots[2][RNT / 64];
  double acc = 0.0, nf = 0.0;
  for (long long e = (long long)blockIdx.x * RNT + threadIdx.x; e < n; e += (long long)gridDim.x * RNT) {
    const double v = ldv(X, e);
    if (!isfinite(v)) nf = 1.0;
    acc += v * v;
  }
  const double s = block_sum(acc, slots[0]);
  const double b = block_sum(nf, slots[1]);
  if (threadIdx.x == 0) { part[blockIdx.x] = s; badp[blockIdx.x] = b; }
}

__global__ void final_flag_kernel(const double* __restrict__ badp, int n, int* __restrict__ out) {
  __shared__ double slots[RNT / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += RNT) acc += badp[i];
  const double s = block_sum(acc, slots);
  if (threadIdx.x == 0) *out = (s > 0.0) ? 1 : 0;
}

__global__ void final_sum_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double slots[RNT / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += RNT) acc += part[i];
  const double s = block_sum(acc, slots);
  if (threadIdx.x == 0) *out = s;
}

// Column norms, lambda, signs and order of the uncompressed factors (one workgroup).
__global__ void normalize_plan_kernel(const double* __restrict__ W0, const double* __restrict__ W1,
                                      const double* __restrict__ W2, int I1, int I2, int I3, int R,
                                      double* __restrict__ scale, int* __restrict__ dest,
                                      double* __restrict__ lambda) {
  __shared__ double nrm[3][64];
  __shared__ double lam[64];
  __shared__ double sgn[2][64];
  const double* Ws[3] = {W0, W1, W2};
  const int Is[3] = {I1, I2, I3};
  const int tid = threadIdx.x;
  // norms: one wave per (mode, column)
  const int lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  for (int c = w; c < 3 * R; c += nw) {
    const int l = c / R, r = c % R;
    double s = 0.0;
    for (int i = lane; i < Is[l]; i += 64) s += Ws[l][(long long)i * R + r] * Ws[l][(long long)i * R + r];
    s = wave_sum(s);
    if (lane == 0) nrm[l][r] = sqrt(s);
  }
  // sign of the largest-|.| entry of modes 1 and 2 (ties: lowest index)
  for (int c = w; c < 2 * R; c += nw) {
    const int l = c / R, r = c % R;
    double best = -1.0;
    int bi = 0;   // stays a valid index if every entry is NaN
    for (int i = lane; i < Is[l]; i += 64) {
      const double a = fabs(Ws[l][(long long)i * R + r]);
      if (a > best || (a == best && i < bi)) { best = a; bi = i; }
    }
    for (int off = 32; off >= 1; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) sgn[l][r] = (Ws[l][(long long)bi * R + r] < 0.0) ? -1.0 : 1.0;
  }
  __syncthreads();
  if (tid < R) lam[tid] = (nrm[0][tid] * nrm[1][tid]) * nrm[2][tid];
  __syncthreads();
  if (tid < R) {
    const int r = tid;
    int rank = 0;
    for (int s = 0; s < R; ++s)
      if (lam[s] > lam[r] || (lam[s] == lam[r] && s < r)) ++rank;
    dest[r] = rank;
    lambda[rank] = lam[r];
    for (int l = 0; l < 3; ++l) {
      double sc = (nrm[l][r] > 0.0) ? 1.0 / nrm[l][r] : 1.0;
      if (l < 2) sc *= sgn[l][r];
      else sc *= sgn[0][r] * sgn[1][r];
      scale[l * 64 + r] = sc;
    }
  }
}

__global__ void normalize_apply_kernel(const double* __restrict__ Wt, int I, int R,
                                       const double* __restrict__ scale, const int* __restrict__ dest,
                                       double* __restrict__ Wout) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)I * R) return;
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

cpd_status residual_full(const void* T, int dtype, const int64_t dims[3], const double* const W[3],
                         int R, double* out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (R < 1 || R > 64 || !T || !out || !W[0] || !W[1] || !W[2]) {
    set_error("residual_full: bad arguments");
    return CPD_E_INVALID;
  }
  if (!ws || ws_bytes < residual_ws_bytes(dims)) {
    set_error("residual_full: workspace too small");
    return CPD_E_WORKSPACE;
  }
  double* part = (double*)ws;
  const int I1 = (int)dims[0], I2 = (int)dims[1], I3 = (int)dims[2];
  prof_begin(CPD_PK_RESIDUAL, s);
  switch (dtype) {
    case CPD_F64:
      hipLaunchKernelGGL(residual_kernel<double>, dim3(RB), dim3(RNT), 0, s, (const double*)T, I1, I2, I3,
                         W[0], W[1], W[2], R, part);
      break;
    case CPD_F32:
      hipLaunchKernelGGL(residual_kernel<float>, dim3(RB), dim3(RNT), 0, s, (const float*)T, I1, I2, I3,
                         W[0], W[1], W[2], R, part);
      break;
    case CPD_BF16:
      hipLaunchKernelGGL(residual_kernel<uint16_t>, dim3(RB), dim3(RNT), 0, s, (const uint16_t*)T, I1, I2,
                         I3, W[0], W[1], W[2], R, part);
      break;
    default:
      set_error("residual_full: bad dtype");
      return CPD_E_INVALID;
  }
  prof_end(CPD_PK_RESIDUAL, s);
  CPD_LAUNCH_CHECK();
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(RNT), 0, s, part, RB, out);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

cpd_status sumsq_full(const void* T, int dtype, int64_t n, double* out, int* nonfinite, void* ws,
                      size_t ws_bytes, hipStream_t s) {
  if (!ws || ws_bytes < sumsq_ws_bytes()) {
    set_error("sumsq_full: workspace too small");
    return CPD_E_WORKSPACE;
  }
  double* part = (double*)ws;
  double* bad = (double*)((char*)ws + align_up(RB * sizeof(double), 256));
  switch (dtype) {
    case CPD_F64:
      hipLaunchKernelGGL(sumsq_kernel<double>, dim3(RB), dim3(RNT), 0, s, (const double*)T, (long long)n, part, bad);
      break;
    case CPD_F32:
      hipLaunchKernelGGL(sumsq_kernel<float>, dim3(RB), dim3(RNT), 0, s, (const float*)T, (long long)n, part, bad);
      break;
    case CPD_BF16:
      hipLaunchKernelGGL(sumsq_kernel<uint16_t>, dim3(RB), dim3(RNT), 0, s, (const uint16_t*)T, (long long)n, part, bad);
      break;
    default:
      set_error("sumsq_full: bad dtype");
      return CPD_E_INVALID;
  }
  CPD_LAUNCH_CHECK();
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(RNT), 0, s, part, RB, out);
  CPD_LAUNCH_CHECK();
  if (nonfinite) {
    hipLaunchKernelGGL(final_flag_kernel, dim3(1), dim3(RNT), 0, s, bad, RB, nonfinite);
    CPD_LAUNCH_CHECK();
  }
  return CPD_OK;
}

size_t normalize_ws_bytes(int R) {
  (void)R;
  return align_up(3 * 64 * sizeof(double), 256) + align_up(64 * sizeof(int), 256);
}

cpd_status normalize_output(const double* const Wt[3], const int64_t dims[3], int R,
                            double* const Wout[3], double* lambda, void* ws, size_t ws_bytes,
                            hipStream_t s) {
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
  hipLaunchKernelGGL(normalize_plan_kernel, dim3(1), dim3(256), 0, s, Wt[0], Wt[1], Wt[2], (int)dims[0],
                     (int)dims[1], (int)dims[2], R, scale, dest, lambda);
  CPD_LAUNCH_CHECK();
  for (int l = 0; l < 3; ++l) {
    const long long n = dims[l] * (long long)R;
    hipLaunchKernelGGL(normalize_apply_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Wt[l],
                       (int)dims[l], R, scale + l * 64, dest, Wout[l]);
    CPD_LAUNCH_CHECK();
  }
  return CPD_OK;
}

}  // namespace cpd
