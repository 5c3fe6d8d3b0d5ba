// Learned starting point for the dGN on a fixed-size compressed core (an extension: the thesis
// starts from random or MLSVD-energy points, ch.4 "Initialization").
//
// Encoding shared by training and inference:
//   feature  x = S / ||S||                                   (FP32, prod(core dims) entries)
//   target   t = [w_r^(l) lambda_r^{1/3}] / ||S||^{1/3}       (FP32, modes stacked, core_l x R
//            row-major each): the balanced factors of the core's CPD, scaled so that a core of
//            any norm maps to targets of unit scale
//   start    W = y ||S||^{1/3}                               (FP64, the inverse of the target map)
// The judge runs a few dGN iterations from the network's start and from the library's N(0,1)
// start (the fallback, ch.4 "Initialization") and keeps the network's start unless its core error
// after them exceeds the fallback's by more than a given factor.
#include "common.h"

#include <math.h>
#include <string.h>

namespace cpd {
namespace {

constexpr int FNT = 256;

// One workgroup per item: ||S_b||^2 with a fixed reduction order, then x_b = S_b / ||S_b||.
__global__ __launch_bounds__(FNT) void feature_kernel(const double* __restrict__ S, long long n,
                                                      float* __restrict__ x, double* __restrict__ nrm) {
  __shared__ double red[FNT];
  const double* Sb = S + (long long)blockIdx.x * n;
  float* xb = x + (long long)blockIdx.x * n;
  double acc = 0.0;
  for (long long e = threadIdx.x; e < n; e += FNT) acc += Sb[e] * Sb[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = FNT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double s = sqrt(red[0]);
  const double inv = (s > 0.0) ? 1.0 / s : 0.0;
  for (long long e = threadIdx.x; e < n; e += FNT) xb[e] = (float)(Sb[e] * inv);
  if (threadIdx.x == 0) nrm[blockIdx.x] = s;
}

// W = y ||S||^{1/3} in FP64.
__global__ void start_kernel(const float* __restrict__ y, int n, const double* __restrict__ nrm,
                             double* __restrict__ W) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) W[e] = (double)y[e] * cbrt(nrm[0]);
}

// t = w_r^(l) lambda_r^{1/3} / ||S||^{1/3} (lambda clamped at 0), modes stacked.
__global__ void target_kernel(const double* __restrict__ W0, const double* __restrict__ W1,
                              const double* __restrict__ W2, int d0, int d1, int d2, int R,
                              const double* __restrict__ lam, double s_norm, float* __restrict__ t) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int n0 = d0 * R, n1 = d1 * R, n = (d0 + d1 + d2) * R;
  if (e >= n) return;
  const double* W = e < n0 ? W0 : (e < n0 + n1 ? W1 : W2);
  const int loc = e < n0 ? e : (e < n0 + n1 ? e - n0 : e - n0 - n1);
  const int r = loc % R;
  t[e] = (float)(W[loc] * cbrt(fmax(lam[r], 0.0)) / cbrt(s_norm));
}

bool core_ok(const int32_t core[3], int R) {
  if (!core || R < 1 || R > 64) return false;
  for (int l = 0; l < 3; ++l)
    if (core[l] < 1 || core[l] > 4096) return false;
  return true;
}

// Workspace layout of cpd_learned_start.
template <class A>
void carve_learned(A& a, const cpd_mlp* net, const int32_t core[3], int R, int judge_iters, float** x, float** y,
                   double** nrm, double** Wl, double** Wr, char** mws, char** st_l, char** st_r) {
  const int np = (core[0] + core[1] + core[2]) * R;
  *x = a.template take<float>(net->n_in);
  *y = a.template take<float>(net->n_out);
  *nrm = a.template take<double>(1);
  *Wl = a.template take<double>(np);
  *Wr = a.template take<double>(np);
  *mws = a.template take<char>(cpd_mlp_workspace_bytes(net, 1));
  const size_t sb = judge_iters > 0 ? state_bytes(core, R, judge_iters) : 0;
  *st_l = judge_iters > 0 ? a.template take<char>(sb) : nullptr;
  *st_r = judge_iters > 0 ? a.template take<char>(sb) : nullptr;
}

bool sizes_ok(const cpd_mlp* net, const int32_t core[3], int R) {
  if (!net || !core_ok(core, R)) return false;
  const long long n_in = (long long)core[0] * core[1] * core[2];
  const long long n_out = (long long)(core[0] + core[1] + core[2]) * R;
  return net->n_in == n_in && net->n_out == n_out;
}

}  // namespace
}  // namespace cpd

using namespace cpd;

extern "C" {

cpd_status cpd_learned_features(const double* S, int32_t n_items, int64_t n, float* x, double* norms,
                                void* stream) {
  CPD_REQUIRE(S && x && norms && n_items >= 1 && n >= 1, "cpd_learned_features: bad arguments");
  hipLaunchKernelGGL(feature_kernel, dim3(n_items), dim3(FNT), 0, (hipStream_t)stream, S, (long long)n, x, norms);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

cpd_status cpd_learned_target(const double* const W[3], const double* lambda, const int32_t core_dims[3],
                              int32_t R, double s_norm, float* t, void* stream) {
  CPD_REQUIRE(W && W[0] && W[1] && W[2] && lambda && t && core_ok(core_dims, R) && s_norm > 0.0,
              "cpd_learned_target: bad arguments");
  const int n = (core_dims[0] + core_dims[1] + core_dims[2]) * R;
  hipLaunchKernelGGL(target_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, W[0], W[1], W[2],
                     core_dims[0], core_dims[1], core_dims[2], R, lambda, s_norm, t);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

size_t cpd_learned_start_workspace_bytes(const cpd_mlp* net, const int32_t core_dims[3], int32_t R,
                                         int32_t judge_iters) {
  if (!sizes_ok(net, core_dims, R) || judge_iters < 0) return 0;
  Sizer z;
  float *x, *y;
  double *nrm, *Wl, *Wr;
  char *mws, *sl, *sr;
  carve_learned(z, net, core_dims, R, judge_iters, &x, &y, &nrm, &Wl, &Wr, &mws, &sl, &sr);
  return z.off;
}

cpd_status cpd_learned_start(const cpd_mlp* net, const double* S, const int32_t core_dims[3], int32_t R,
                             int32_t judge_iters, double judge_margin, const cpd_params* p,
                             const double* W_fallback, double* W_out, int32_t* chosen, double* judge_err, void* ws,
                             size_t ws_bytes, void* stream) {
  CPD_REQUIRE(S && W_out && sizes_ok(net, core_dims, R) && judge_iters >= 0 && judge_iters <= 1000 &&
                  judge_margin >= 1.0,
              "cpd_learned_start: bad arguments (the network must map prod(core) inputs to R sum(core) outputs)");
  cpd_params pj;
  if (p) pj = *p; else cpd_default_params(&pj);
  CPD_REQUIRE(pj.precond == 0 || pj.precond == 1, "cpd_learned_start: precond must be 0 or 1");
  CPD_REQUIRE(!pj.cg_uniforms || pj.maxiter >= judge_iters, "cpd_learned_start: cg_uniforms shorter than judge_iters");
  if (!ws || ws_bytes < cpd_learned_start_workspace_bytes(net, core_dims, R, judge_iters)) {
    set_error("cpd_learned_start: workspace too small");
    return CPD_E_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  Arena ar(ws, ws_bytes);
  float *x, *y;
  double *nrm, *Wl, *Wr;
  char *mws, *st_l, *st_r;
  carve_learned(ar, net, core_dims, R, judge_iters, &x, &y, &nrm, &Wl, &Wr, &mws, &st_l, &st_r);
  const int np = (core_dims[0] + core_dims[1] + core_dims[2]) * R;
  const long long n_in = (long long)core_dims[0] * core_dims[1] * core_dims[2];
  cpd_status st;
  // network start
  hipLaunchKernelGGL(feature_kernel, dim3(1), dim3(FNT), 0, s, S, n_in, x, nrm);
  CPD_LAUNCH_CHECK();
  if ((st = cpd_mlp_forward(net, x, y, 1, mws, cpd_mlp_workspace_bytes(net, 1), stream))) return st;
  hipLaunchKernelGGL(start_kernel, dim3((np + 255) / 256), dim3(256), 0, s, y, np, nrm, Wl);
  CPD_LAUNCH_CHECK();
  int pick = 0;
  double e_l = 0.0, e_r = 0.0;
  if (judge_iters > 0) {
    // the fallback: the caller's start, else the library's N(0,1) start for this seed (the start
    // cpd_solve draws)
    if (W_fallback) {
      CPD_HIP_CHECK(hipMemcpyAsync(Wr, W_fallback, sizeof(double) * np, hipMemcpyDeviceToDevice, s));
    } else if ((st = fill_randn(Wr, np, pj.seed, s))) {
      return st;
    }
    pj.maxiter = judge_iters;
    pj.init = CPD_INIT_GIVEN;
    pj.refine_iters = 0;
    const int32_t core[3] = {core_dims[0], core_dims[1], core_dims[2]};
    if ((st = state_init(st_l, S, core, R, Wl, 0.0, &pj, s, false))) return st;
    if ((st = state_init(st_r, S, core, R, Wr, 0.0, &pj, s, false))) return st;
    if ((st = dgn_iterate_known(st_l, S, core, R, judge_iters, s, dgn_opts(&pj)))) return st;
    if ((st = dgn_iterate_known(st_r, S, core, R, judge_iters, s, dgn_opts(&pj)))) return st;
    if ((st = state_read(st_l, nullptr, nullptr, nullptr, &e_l, s))) return st;
    if ((st = state_read(st_r, nullptr, nullptr, nullptr, &e_r, s))) return st;
    // the fallback only when the network's start is worse by more than the margin; a non-finite
    // network error loses (NaN compares false)
    pick = (e_l <= judge_margin * e_r) ? 0 : 1;
  }
  CPD_HIP_CHECK(hipMemcpyAsync(W_out, pick ? Wr : Wl, sizeof(double) * np, hipMemcpyDeviceToDevice, s));
  if (judge_iters > 0) CPD_HIP_CHECK(hipStreamSynchronize(s));
  if (chosen) *chosen = pick;
  if (judge_err) {
    judge_err[0] = e_l;
    judge_err[1] = e_r;
  }
  return CPD_OK;
}

}  // extern "C"
