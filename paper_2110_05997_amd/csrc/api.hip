// C ABI of libcpd: argument checking, workspace carving and the host-side sequencing of the
// Tensor Fox pipeline (ch.4 flow chart: Compress -> Initialize -> dGN -> Uncompress).
#include "common.h"
#include "dgn_state.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <vector>

namespace cpd {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

namespace {

bool dims_ok(const int64_t dims[3]) {
  if (!dims) return false;
  for (int l = 0; l < 3; ++l)
    if (dims[l] < 1 || dims[l] > 4096) return false;
  return true;
}

bool dtype_ok(int dt) { return dt == CPD_F64 || dt == CPD_F32 || dt == CPD_BF16; }

void pdims(const int64_t dims[3], int R, const cpd_params* p, int P[3]) {
  const bool fixed = p && p->core_dims[0] > 0 && p->core_dims[1] > 0 && p->core_dims[2] > 0;
  for (int l = 0; l < 3; ++l) {
    if (fixed) P[l] = p->core_dims[l];
    else P[l] = (int)(dims[l] < R ? dims[l] : R);
  }
}

// Truncation rule of Alg. Compression: smallest i with sum_{r >= i} lam_r / sum_r lam_r < tol / 3.
int truncation_rank(const double* lam, int P, double mlsvd_tol) {
  double total = 0.0;
  for (int r = 0; r < P; ++r) total += (lam[r] > 0.0 ? lam[r] : 0.0);
  if (total == 0.0) return P;
  for (int i = 1; i <= P; ++i) {
    double tail = 0.0;
    for (int r = i; r < P; ++r) tail += (lam[r] > 0.0 ? lam[r] : 0.0);
    if (tail / total < mlsvd_tol / 3.0) return i;
  }
  return P;
}

struct CompressWs {
  size_t G, gram, eig, Uf, lam, Y1, Y2;
};

void compress_sizes(const int64_t dims[3], const int P[3], Sizer& z) {
  size_t gram = 0;
  const int64_t d2[3] = {P[0], dims[1], dims[2]}, d3[3] = {P[0], P[1], dims[2]};
  for (int l = 0; l < 3; ++l) {
    z.take<double>((size_t)(dims[l] * dims[l]));         // G_l
    size_t g = gram_ws_bytes(dims, l);
    gram = gram > g ? gram : g;
  }
  // the sequentially truncated variant's Grams of the projected tensors
  const size_t g2 = gram_ws_bytes(d2, 1), g3 = gram_ws_bytes(d3, 2);
  gram = gram > g2 ? gram : g2;
  gram = gram > g3 ? gram : g3;
  const int n[3] = {(int)dims[0], (int)dims[1], (int)dims[2]};
  z.take<char>(gram);                                    // gram partials
  z.take<char>(eig_ws_bytes3(n, P, 3));                  // eigensolver
  for (int l = 0; l < 3; ++l) z.take<double>((size_t)dims[l] * P[l]);   // U full
  z.take<double>(P[0] + P[1] + P[2]);                    // eigenvalues
  z.take<double>((size_t)P[0] * dims[1] * dims[2]);      // Y1
  z.take<double>((size_t)P[0] * P[1] * dims[2]);         // Y2
}

// Host memory for a solve's read-backs: a 4 KB pinned buffer per host thread, so the copies write
// host memory directly instead of going through a staging copy.  Every use ends with a
// synchronisation before the next one starts, so one buffer per thread suffices; it lives until
// the process ends.  Falls back to `spill` (pageable) when the buffer cannot be had or is too small.
constexpr size_t READBACK_BYTES = 4096;
char* readback_host(size_t bytes, std::vector<char>& spill) {
  static thread_local char* buf = nullptr;
  static thread_local bool tried = false;
  if (!tried) {
    tried = true;
    if (hipHostMalloc((void**)&buf, READBACK_BYTES, hipHostMallocPortable) != hipSuccess) {
      buf = nullptr;
      (void)hipGetLastError();
    }
  }
  if (buf && bytes <= READBACK_BYTES) return buf;
  spill.resize(bytes);
  return spill.data();
}

// An event per host thread for waiting on one read-back while later work stays enqueued, created
// on first use on the thread's current device and held until the process ends; nullptr (wait for
// the stream instead) when it cannot be had or the thread has moved to another device.
hipEvent_t readback_event() {
  static thread_local hipEvent_t ev = nullptr;
  static thread_local int dev_of = -1;
  static thread_local bool tried = false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  if (!tried) {
    tried = true;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
      dev_of = dev;
    } else {
      ev = nullptr;
      (void)hipGetLastError();
    }
  }
  return ev != nullptr && dev_of == dev ? ev : nullptr;
}

// The three mode products of the core projection S = T x1 U1^T x2 U2^T x3 U3^T.
// Y1[a][i2 i3] = sum_i1 U1[i1][a] T[i1][i2 i3] (T in its own dtype)
cpd_status project_mode1(const void* T, int dtype, int I1, int I2, int I3, const double* U1, int r1, double* Y1,
                         hipStream_t s) {
  cpd_status st;
  prof_begin(CPD_PK_PROJECT, s);
  if (r1 <= 64)
    st = project_mfma(T, dtype, I1, (long long)I2 * I3, 1, 0, U1, r1, Y1, 0, s);
  else if (mode_product_mid_fits(I1, r1))
    st = mode_product_mid(T, dtype, 1, I1, (long long)I2 * I3, U1, r1, Y1, s);
  else
    st = gemm_f64(r1, I2 * I3, I1, 1.0, U1, r1, 0, true, T, dtype, (long long)I2 * I3, 0, false, 0.0, Y1,
                  (long long)I2 * I3, 0, 1, s);
  prof_end(CPD_PK_PROJECT, s);
  return st;
}
// Y2[a][b][i3] = sum_i2 U2[i2][b] Y1[a][i2][i3]
cpd_status project_mode2(const double* Y1, int r1, int I2, int I3, const double* U2, int r2, double* Y2,
                         hipStream_t s) {
  if (r2 <= 64 && r1 <= 65535)
    return project_mfma(Y1, CPD_F64, I2, I3, r1, (long long)I2 * I3, U2, r2, Y2, (long long)r2 * I3, s);
  if (mode_product_mid_fits(I2, r2)) return mode_product_mid(Y1, CPD_F64, r1, I2, I3, U2, r2, Y2, s);
  return gemm_f64(r2, I3, I2, 1.0, U2, r2, 0, true, Y1, CPD_F64, I3, (long long)I2 * I3, false, 0.0, Y2, I3,
                  (long long)r2 * I3, r1, s);
}
// S[ab][c] = sum_i3 Y2[ab][i3] U3[i3][c]
cpd_status project_mode3(const double* Y2, int r12, int I3, const double* U3, int r3, double* S, hipStream_t s) {
  return gemm_f64(r12, r3, I3, 1.0, Y2, I3, 0, false, U3, CPD_F64, r3, 0, false, 0.0, S, r3, 0, 1, s);
}

// Runs compression with carved workspace; outputs U (compact I_l x R~_l), sigma, S.
// T_gram / gram_dtype / gram_compute: the tensor copy and precision the Grams are formed from
// (normally T itself); the projection always reads T.
// U_out[l] holds dims[l] x P_l doubles: the eigensolver writes the full basis there and only a
// truncated mode is compacted (through workspace) afterwards.
// chk (optional, device, 2 + P_1 + P_2 + P_3 doubles): the input tensor's ||T||^2 in chk[0] and
// the non-finite flag (an int) in chk[1] from sumsq_full; the eigenvalues are written behind them,
// so one copy brings all three back (one host round trip) and the checks are made before any host
// decision; h_tn2 receives ||T||^2.  A zero or non-finite tensor only runs the Gram and eigen
// kernels on workspace (their loops are bounded) before the error is returned.
cpd_status run_compress(const void* T, int dtype, const void* T_gram, int gram_dtype, int gram_compute,
                        const int64_t dims[3], int R, const cpd_params* p,
                        double* const U_out[3], double* const sigma_out[3], double* S_out,
                        int core_out[3], Arena& ar, hipStream_t s, double* chk = nullptr,
                        double* h_tn2 = nullptr, bool chk_from_gram = false) {
  int P[3];
  pdims(dims, R, p, P);
  size_t gram_b = 0;
  for (int l = 0; l < 3; ++l) {
    if (P[l] < 1 || P[l] > dims[l]) {
      set_error("compress: core dim %d invalid for mode %d of size %lld", P[l], l, (long long)dims[l]);
      return CPD_E_INVALID;
    }
    if (dims[l] > 64 && P[l] > 56) {
      set_error("compress: P=%d > 56 for mode size %lld > 64 is not supported", P[l], (long long)dims[l]);
      return CPD_E_UNSUPPORTED;
    }
    size_t g = gram_ws_bytes(dims, l);
    gram_b = gram_b > g ? gram_b : g;
  }
  const int n[3] = {(int)dims[0], (int)dims[1], (int)dims[2]};
  const size_t eig_b = eig_ws_bytes3(n, P, 3);
  double* G[3];
  for (int l = 0; l < 3; ++l) G[l] = ar.take<double>((size_t)(dims[l] * dims[l]));
  char* gws = ar.take<char>(gram_b);
  char* ews = ar.take<char>(eig_b);
  double* Uf[3];
  for (int l = 0; l < 3; ++l) Uf[l] = ar.take<double>((size_t)dims[l] * P[l]);
  double* lam = ar.take<double>(P[0] + P[1] + P[2]);
  if (chk) lam = chk + 2;
  double* Y1 = ar.take<double>((size_t)P[0] * dims[1] * dims[2]);
  double* Y2 = ar.take<double>((size_t)P[0] * P[1] * dims[2]);
  if (!Y2) {
    set_error("compress: workspace too small (%zu bytes)", ar.cap);
    return CPD_E_WORKSPACE;
  }
  double* laml[3] = {lam, lam + P[0], lam + P[0] + P[1]};
  cpd_status st;
  for (int l = 0; l < 3; ++l) {
    if ((st = gram(T_gram, gram_dtype, dims, l, gram_compute, G[l], gws, gram_b, s))) return st;
    if (l == 0 && chk && chk_from_gram && (st = gram_trace_check(G[0], n[0], chk, (int*)(chk + 1), s))) return st;
  }
  // the three eigenproblems run side by side
  prof_begin(CPD_PK_EIG, s);
  st = eig_top3(G, n, P, U_out, laml, 3, ews, eig_b, s);
  prof_end(CPD_PK_EIG, s);
  if (st) return st;
  const int ptot = P[0] + P[1] + P[2];
  std::vector<char> spill;
  double* hbuf = (double*)readback_host(sizeof(double) * (ptot + 2), spill);
  const int h0 = chk ? 0 : 2;   // host index of the first copied double
  CPD_HIP_CHECK(hipMemcpyAsync(hbuf + h0, chk ? chk : lam, sizeof(double) * (ptot + 2 - h0),
                               hipMemcpyDeviceToHost, s));
  // the core projection at the full ranks P goes in behind the copy, so that the device works
  // while the host waits for the eigenvalues (only the copy is waited for); a truncation below P
  // repeats it at the truncated ranks
  const int I1 = (int)dims[0], I2 = (int)dims[1], I3 = (int)dims[2];
  hipEvent_t ev = readback_event();
  bool speculated = false;
  if (ev != nullptr) {
    CPD_HIP_CHECK(hipEventRecord(ev, s));
    if ((st = project_mode1(T, dtype, I1, I2, I3, U_out[0], P[0], Y1, s))) return st;
    if ((st = project_mode2(Y1, P[0], I2, I3, U_out[1], P[1], Y2, s))) return st;
    if ((st = project_mode3(Y2, P[0] * P[1], I3, U_out[2], P[2], S_out, s))) return st;
    speculated = true;
    CPD_HIP_CHECK(hipEventSynchronize(ev));
  } else {
    CPD_HIP_CHECK(hipStreamSynchronize(s));
  }
  const std::vector<double> hlv(hbuf + 2, hbuf + 2 + ptot);   // the buffer is reused at the end
  const double* hlam = hlv.data();
  if (chk) {
    const double c_tn2 = hbuf[0];
    int c_bad = 0;
    memcpy(&c_bad, &hbuf[1], sizeof(int));
    if (c_bad) { set_error("cpd_solve: non-finite entries in T"); return CPD_E_NONFINITE; }
    if (!(c_tn2 > 0.0)) { set_error("cpd_solve: ||T|| = 0"); return CPD_E_ZERO_TENSOR; }
    if (h_tn2) *h_tn2 = c_tn2;
  }
  const bool fixed = p && p->core_dims[0] > 0 && p->core_dims[1] > 0 && p->core_dims[2] > 0;
  int rk[3];
  int o = 0;
  for (int l = 0; l < 3; ++l) {
    rk[l] = fixed ? P[l] : truncation_rank(hlam + o, P[l], p ? p->mlsvd_tol : 1e-6);
    o += P[l];
  }
  // sigma = sqrt(max(lambda, 0))
  if (sigma_out) {
    o = 0;
    for (int l = 0; l < 3; ++l) {
      if (sigma_out[l]) {
        std::vector<double> tmpv(P[l]);
        double* tmp = tmpv.data();
        for (int r = 0; r < P[l]; ++r) tmp[r] = sqrt(hlam[o + r] > 0.0 ? hlam[o + r] : 0.0);
        CPD_HIP_CHECK(hipMemcpyAsync(sigma_out[l], tmp, sizeof(double) * P[l], hipMemcpyHostToDevice, s));
        CPD_HIP_CHECK(hipStreamSynchronize(s));
      }
      o += P[l];
    }
  }
  // compact a truncated U (rows of P_l doubles to rows of R~_l) through the workspace
  for (int l = 0; l < 3; ++l) {
    if (rk[l] == P[l]) continue;
    CPD_HIP_CHECK(hipMemcpy2DAsync(Uf[l], sizeof(double) * rk[l], U_out[l], sizeof(double) * P[l],
                                   sizeof(double) * rk[l], dims[l], hipMemcpyDeviceToDevice, s));
    CPD_HIP_CHECK(hipMemcpyAsync(U_out[l], Uf[l], sizeof(double) * rk[l] * dims[l], hipMemcpyDeviceToDevice, s));
  }
  // S = T x1 U1^T x2 U2^T x3 U3^T (already enqueued when no mode was truncated)
  if (!(speculated && rk[0] == P[0] && rk[1] == P[1] && rk[2] == P[2])) {
    if ((st = project_mode1(T, dtype, I1, I2, I3, U_out[0], rk[0], Y1, s))) return st;
    if ((st = project_mode2(Y1, rk[0], I2, I3, U_out[1], rk[1], Y2, s))) return st;
    if ((st = project_mode3(Y2, rk[0] * rk[1], I3, U_out[2], rk[2], S_out, s))) return st;
  }
  for (int l = 0; l < 3; ++l) core_out[l] = rk[l];
  return CPD_OK;
}

// Sequentially truncated compression (ch.2 Alg. ST-MLSVD): mode l's Gram, eigenvectors and
// truncation are taken on the tensor already projected in the modes before it, Y1 = T x1 U1^T and
// Y2 = Y1 x2 U2^T, so the second and third Grams read R~1 I2 I3 and R~1 R~2 I3 entries instead of
// I1 I2 I3.  Same outputs, workspace and read-back conventions as run_compress (the eigenvalues of
// mode 1 come back with the input checks; modes 2 and 3 take one read-back each).
cpd_status run_compress_st(const void* T, int dtype, const void* T_gram, int gram_dtype, int gram_compute,
                           const int64_t dims[3], int R, const cpd_params* p,
                           double* const U_out[3], double* const sigma_out[3], double* S_out,
                           int core_out[3], Arena& ar, hipStream_t s, double* chk = nullptr,
                           double* h_tn2 = nullptr, bool chk_from_gram = false) {
  int P[3];
  pdims(dims, R, p, P);
  for (int l = 0; l < 3; ++l) {
    if (P[l] < 1 || P[l] > dims[l]) {
      set_error("compress: core dim %d invalid for mode %d of size %lld", P[l], l, (long long)dims[l]);
      return CPD_E_INVALID;
    }
    if (dims[l] > 64 && P[l] > 56) {
      set_error("compress: P=%d > 56 for mode size %lld > 64 is not supported", P[l], (long long)dims[l]);
      return CPD_E_UNSUPPORTED;
    }
  }
  const int I1 = (int)dims[0], I2 = (int)dims[1], I3 = (int)dims[2];
  const int64_t d1[3] = {dims[0], dims[1], dims[2]};
  const int64_t d2[3] = {P[0], dims[1], dims[2]};           // Y1 (at most P1 rows)
  const int64_t d3[3] = {P[0], P[1], dims[2]};              // Y2
  size_t gram_b = gram_ws_bytes(d1, 0);
  const size_t g2 = gram_ws_bytes(d2, 1), g3 = gram_ws_bytes(d3, 2);
  gram_b = gram_b > g2 ? gram_b : g2;
  gram_b = gram_b > g3 ? gram_b : g3;
  const int n[3] = {I1, I2, I3};
  const size_t eig_b = eig_ws_bytes3(n, P, 3);
  double* G[3];
  for (int l = 0; l < 3; ++l) G[l] = ar.take<double>((size_t)(dims[l] * dims[l]));
  char* gws = ar.take<char>(gram_b);
  char* ews = ar.take<char>(eig_b);
  double* Uf[3];
  for (int l = 0; l < 3; ++l) Uf[l] = ar.take<double>((size_t)dims[l] * P[l]);
  double* lam = ar.take<double>(P[0] + P[1] + P[2]);
  if (chk) lam = chk + 2;
  double* Y1 = ar.take<double>((size_t)P[0] * dims[1] * dims[2]);
  double* Y2 = ar.take<double>((size_t)P[0] * P[1] * dims[2]);
  if (!Y2) {
    set_error("compress: workspace too small (%zu bytes)", ar.cap);
    return CPD_E_WORKSPACE;
  }
  const bool fixed = p && p->core_dims[0] > 0 && p->core_dims[1] > 0 && p->core_dims[2] > 0;
  const double mtol = p ? p->mlsvd_tol : 1e-6;
  std::vector<char> spill;
  double* hbuf = (double*)readback_host(sizeof(double) * (P[0] + P[1] + P[2] + 2), spill);
  double* laml[3] = {lam, lam + P[0], lam + P[0] + P[1]};
  int rk[3];
  cpd_status st;
  for (int l = 0; l < 3; ++l) {
    // the tensor this mode's Gram reads: T, then Y1 (rk[0] x I2 x I3), then Y2 (rk[0] x rk[1] x I3)
    if (l == 0) {
      if ((st = gram(T_gram, gram_dtype, dims, 0, gram_compute, G[0], gws, gram_b, s))) return st;
      if (chk && chk_from_gram && (st = gram_trace_check(G[0], (int)dims[0], chk, (int*)(chk + 1), s))) return st;
    } else if (l == 1) {
      const int64_t dy[3] = {rk[0], dims[1], dims[2]};
      if ((st = gram(Y1, CPD_F64, dy, 1, CPD_F64, G[1], gws, gram_b, s))) return st;
    } else {
      const int64_t dy[3] = {rk[0], rk[1], dims[2]};
      if ((st = gram(Y2, CPD_F64, dy, 2, CPD_F64, G[2], gws, gram_b, s))) return st;
    }
    prof_begin(CPD_PK_EIG, s);
    st = eig_top(G[l], n[l], P[l], U_out[l], laml[l], ews, eig_b, s);
    prof_end(CPD_PK_EIG, s);
    if (st) return st;
    // eigenvalues of this mode (and, for mode 1 of a solve, the input checks in front of them)
    const int h0 = (l == 0 && chk) ? 0 : 2;
    const double* src = (l == 0 && chk) ? chk : laml[l];
    CPD_HIP_CHECK(hipMemcpyAsync(hbuf + h0, src, sizeof(double) * (P[l] + 2 - h0), hipMemcpyDeviceToHost, s));
    CPD_HIP_CHECK(hipStreamSynchronize(s));
    if (l == 0 && chk) {
      const double c_tn2 = hbuf[0];
      int c_bad = 0;
      memcpy(&c_bad, &hbuf[1], sizeof(int));
      if (c_bad) { set_error("cpd_solve: non-finite entries in T"); return CPD_E_NONFINITE; }
      if (!(c_tn2 > 0.0)) { set_error("cpd_solve: ||T|| = 0"); return CPD_E_ZERO_TENSOR; }
      if (h_tn2) *h_tn2 = c_tn2;
    }
    rk[l] = fixed ? P[l] : truncation_rank(hbuf + 2, P[l], mtol);
    if (sigma_out && sigma_out[l]) {
      std::vector<double> tmpv(P[l]);
      for (int r = 0; r < P[l]; ++r) tmpv[r] = sqrt(hbuf[2 + r] > 0.0 ? hbuf[2 + r] : 0.0);
      CPD_HIP_CHECK(hipMemcpyAsync(sigma_out[l], tmpv.data(), sizeof(double) * P[l], hipMemcpyHostToDevice, s));
      CPD_HIP_CHECK(hipStreamSynchronize(s));
    }
    if (rk[l] != P[l]) {
      CPD_HIP_CHECK(hipMemcpy2DAsync(Uf[l], sizeof(double) * rk[l], U_out[l], sizeof(double) * P[l],
                                     sizeof(double) * rk[l], dims[l], hipMemcpyDeviceToDevice, s));
      CPD_HIP_CHECK(hipMemcpyAsync(U_out[l], Uf[l], sizeof(double) * rk[l] * dims[l], hipMemcpyDeviceToDevice, s));
    }
    if (l == 0) st = project_mode1(T, dtype, I1, I2, I3, U_out[0], rk[0], Y1, s);
    else if (l == 1) st = project_mode2(Y1, rk[0], I2, I3, U_out[1], rk[1], Y2, s);
    else st = project_mode3(Y2, rk[0] * rk[1], I3, U_out[2], rk[2], S_out, s);
    if (st) return st;
  }
  for (int l = 0; l < 3; ++l) core_out[l] = rk[l];
  return CPD_OK;
}

size_t solve_ws(const int64_t dims[3], int R, const cpd_params* p) {
  int P[3];
  pdims(dims, R, p, P);
  // the carving order of solve_impl
  Sizer z;
  z.take<double>(2 + P[0] + P[1] + P[2]);  // ||T||^2, non-finite flag, eigenvalues
  z.take<char>(sumsq_ws_bytes());
  for (int l = 0; l < 3; ++l) z.take<double>((size_t)dims[l] * P[l]);   // U
  z.take<double>((size_t)P[0] * P[1] * P[2]);                            // S
  const int32_t pc[3] = {P[0], P[1], P[2]};
  z.take<double>(1);                                                     // final residual
  z.take<char>(state_bytes(pc, R, p ? p->maxiter : 200));
  z.take<double>((size_t)(P[0] + P[1] + P[2]) * R);                      // core factors
  for (int l = 0; l < 3; ++l) z.take<double>((size_t)dims[l] * R);       // uncompressed
  z.take<char>(normalize_ws_bytes(R));
  z.take<char>(residual_ws_bytes(dims));
  if (p && p->refine_iters > 0) z.take<char>(refine_state_bytes(dims, R, p->refine_iters));
  Sizer zc;
  compress_sizes(dims, P, zc);
  z.take<char>(zc.off);
  return z.off;
}

}  // namespace

size_t solve_ws_bytes(const int64_t dims[3], int R, const cpd_params* p) { return solve_ws(dims, R, p); }

cpd_status solve3_raw(const double* T, const int64_t dims[3], int R, const cpd_params* p, const double* W0,
                      double* Wt, int* iters, int* stop, double* rel_err, void* ws, size_t ws_bytes, hipStream_t s) {
  const size_t need = solve_ws(dims, R, p);
  if (!ws || ws_bytes < need) {
    set_error("solve3_raw: workspace %zu < %zu", ws_bytes, need);
    return CPD_E_WORKSPACE;
  }
  int P[3];
  pdims(dims, R, p, P);
  Arena ar(ws, ws_bytes);
  double* chk = ar.take<double>(2 + P[0] + P[1] + P[2]);
  char* sws = ar.take<char>(sumsq_ws_bytes());
  double* U[3];
  for (int l = 0; l < 3; ++l) U[l] = ar.take<double>((size_t)dims[l] * P[l]);
  double* S = ar.take<double>((size_t)P[0] * P[1] * P[2]);
  const int32_t pc[3] = {P[0], P[1], P[2]};
  char* state = ar.take<char>(state_bytes(pc, R, p->maxiter));
  if (!state) {
    set_error("solve3_raw: workspace too small");
    return CPD_E_WORKSPACE;
  }
  cpd_status st;
  if ((st = sumsq_full(T, CPD_F64, dims[0] * dims[1] * dims[2], chk, (int*)(chk + 1), sws, sumsq_ws_bytes(), s)))
    return st;
  double h_tn2 = 0.0;
  int core[3];
  if ((st = run_compress(T, CPD_F64, T, CPD_F64, CPD_F64, dims, R, p, U, nullptr, S, core, ar, s, chk, &h_tn2)))
    return st;
  if ((st = state_init(state, S, core, R, W0, h_tn2, p, s, true))) return st;
  if ((st = dgn_iterate_known(state, S, core, R, p->maxiter, s, dgn_opts(p)))) return st;
  const int npc = (core[0] + core[1] + core[2]) * R;
  const double* Wst = (const double*)(state + layout_of(npc, R, p->maxiter).W);
  size_t o = 0, ot = 0;
  for (int l = 0; l < 3; ++l) {
    if ((st = gemm_f64((int)dims[l], R, core[l], 1.0, U[l], core[l], 0, false, Wst + o, CPD_F64, R, 0, false, 0.0,
                       Wt + ot, R, 0, 1, s)))
      return st;
    o += (size_t)core[l] * R;
    ot += (size_t)dims[l] * R;
  }
  Hdr h;
  CPD_HIP_CHECK(hipMemcpyAsync(&h, state, sizeof(Hdr), hipMemcpyDeviceToHost, s));
  CPD_HIP_CHECK(hipStreamSynchronize(s));
  if (iters) *iters = h.k;
  if (stop) *stop = h.stop;
  if (rel_err) *rel_err = (h.s_norm > 0.0) ? sqrt(h.f2) / h.s_norm : 0.0;
  return CPD_OK;
}
}  // namespace cpd

using namespace cpd;

extern "C" {

const char* cpd_last_error(void) { return g_err; }

const char* cpd_version(void) { return "libcpd 0.1 (gfx950)"; }

void cpd_default_params(cpd_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->maxiter = 200;
  p->tol = 1e-6;
  p->mlsvd_tol = 1e-6;
  p->init_damp = 1.0;
  p->cg_tol = 0.0;
  p->cg_fixed = 0;
  p->cg_uniforms = nullptr;
  p->seed = 0;
  p->init = CPD_INIT_RANDOM;
  p->compute_dtype = CPD_F64;
}

size_t cpd_workspace_bytes(const int64_t dims[3], int32_t R, const cpd_params* p) {
  if (!dims_ok(dims) || R < 1) return 0;
  return solve_ws(dims, R, p);
}

cpd_status cpd_compress(const void* T, int32_t dtype, const int64_t dims[3], int32_t R,
                        const cpd_params* p, double* U_out[3], double* sigma_out[3], double* S_out,
                        int32_t core_dims_out[3], void* ws, size_t ws_bytes, void* stream) {
  CPD_REQUIRE(T && U_out && U_out[0] && U_out[1] && U_out[2] && S_out && core_dims_out, "cpd_compress: null argument");
  CPD_REQUIRE(dims_ok(dims) && dtype_ok(dtype) && R >= 1 && R <= 64, "cpd_compress: bad dims/dtype/R");
  cpd_params def;
  if (!p) { cpd_default_params(&def); p = &def; }
  Arena ar(ws, ws_bytes);
  int core[3];
  cpd_status st = p->st_mlsvd
                      ? run_compress_st(T, dtype, T, dtype, p->compute_dtype, dims, R, p, U_out, sigma_out, S_out,
                                        core, ar, (hipStream_t)stream)
                      : run_compress(T, dtype, T, dtype, p->compute_dtype, dims, R, p, U_out, sigma_out, S_out, core,
                                     ar, (hipStream_t)stream);
  if (st) return st;
  CPD_HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
  for (int l = 0; l < 3; ++l) core_dims_out[l] = core[l];
  return CPD_OK;
}

size_t cpd_state_bytes(const int32_t core_dims[3], int32_t R, const cpd_params* p) {
  if (!core_dims || R < 1) return 0;
  return state_bytes(core_dims, R, p ? p->maxiter : 200);
}

cpd_status cpd_state_init(void* state, const double* S, const int32_t core_dims[3], int32_t R,
                          const double* W0, double t_norm2, const cpd_params* p, void* stream) {
  CPD_REQUIRE(state && S && core_dims, "cpd_state_init: null argument");
  cpd_params def;
  if (!p) { cpd_default_params(&def); p = &def; }
  return state_init(state, S, core_dims, R, W0, t_norm2, p, (hipStream_t)stream);
}

cpd_status cpd_dgn_step(void* state, const double* S, const cpd_params* p, cpd_step_info* info,
                        void* stream) {
  CPD_REQUIRE(state && S && info, "cpd_dgn_step: null argument");
  CPD_REQUIRE(!p || p->precond == 0 || p->precond == 1, "cpd_dgn_step: precond must be 0 or 1");
  hipStream_t s = (hipStream_t)stream;
  cpd_status st = dgn_iterate(state, S, 1, s, dgn_opts(p));
  if (st) return st;
  int k = 0, stop = 0, ti = 0;
  if ((st = state_read(state, &k, &stop, &ti, nullptr, s))) return st;
  memset(info, 0, sizeof(*info));
  if (k > 0) {
    if ((st = state_log(state, k - 1, 1, info, s))) return st;
  }
  info->stop = stop;
  return CPD_OK;
}

cpd_status cpd_dgn_run(void* state, const double* S, const cpd_params* p, int32_t* iters,
                       int32_t* stop, cpd_step_info* log, int32_t log_cap, void* stream) {
  CPD_REQUIRE(state && S, "cpd_dgn_run: null argument");
  CPD_REQUIRE(!p || p->precond == 0 || p->precond == 1, "cpd_dgn_run: precond must be 0 or 1");
  hipStream_t s = (hipStream_t)stream;
  const int maxiter = p ? p->maxiter : 200;
  cpd_status st = dgn_iterate(state, S, maxiter, s, dgn_opts(p));
  if (st) return st;
  int k = 0, sr = 0, ti = 0;
  if ((st = state_read(state, &k, &sr, &ti, nullptr, s))) return st;
  if (iters) *iters = k;
  if (stop) *stop = sr;
  if (log && log_cap > 0 && k > 0) {
    const int n = k < log_cap ? k : log_cap;
    if ((st = state_log(state, 0, n, log, s))) return st;
  }
  return CPD_OK;
}

cpd_status cpd_state_factors(void* state, double* W, int32_t set, void* stream) {
  CPD_REQUIRE(state && W, "cpd_state_factors: null argument");
  return state_factors(state, W, set, (hipStream_t)stream);
}

namespace {
cpd_status solve_impl(const void* T_gram, int32_t gram_dtype, int gram_compute, const void* T, int32_t dtype,
                      const int64_t dims[3], int32_t R, const cpd_params* p, const double* W0, double* W_out[3],
                      double* lambda_out, cpd_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  CPD_REQUIRE(T && W_out && W_out[0] && W_out[1] && W_out[2] && lambda_out && info, "cpd_solve: null argument");
  CPD_REQUIRE(dims_ok(dims) && dtype_ok(dtype) && R >= 1 && R <= 64, "cpd_solve: bad dims/dtype/R");
  CPD_REQUIRE(p->maxiter >= 1 && p->tol >= 0.0, "cpd_solve: bad parameters");
  CPD_REQUIRE(p->precond == 0 || p->precond == 1, "cpd_solve: precond must be 0 or 1");
  if (p->refine_iters > 0 && dgn_opts(p)) {
    set_error("cpd_solve: the refinement runs the plain dGN (no block-Jacobi preconditioner or draw-back)");
    return CPD_E_UNSUPPORTED;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t need = solve_ws(dims, R, p);
  if (!ws || ws_bytes < need) {
    set_error("cpd_solve: workspace %zu < %zu", ws_bytes, need);
    return CPD_E_WORKSPACE;
  }
  int P[3];
  pdims(dims, R, p, P);
  Arena ar(ws, ws_bytes);
  // ||T||^2, the non-finite flag and the eigenvalues, adjacent so that one copy reads them back
  double* chk = ar.take<double>(2 + P[0] + P[1] + P[2]);
  char* sws = ar.take<char>(sumsq_ws_bytes());
  double* U[3];
  for (int l = 0; l < 3; ++l) U[l] = ar.take<double>((size_t)dims[l] * P[l]);
  double* S = ar.take<double>((size_t)P[0] * P[1] * P[2]);
  const int32_t pc[3] = {P[0], P[1], P[2]};
  // the final residual one 256-byte slot before the state: one copy reads it with the header
  double* res = ar.take<double>(1);
  char* state = ar.take<char>(state_bytes(pc, R, p->maxiter));
  if (state != (char*)res + 256) {
    set_error("cpd_solve: workspace too small");
    return CPD_E_WORKSPACE;
  }
  double* Wc = ar.take<double>((size_t)(P[0] + P[1] + P[2]) * R);
  double* Wt[3];
  for (int l = 0; l < 3; ++l) Wt[l] = ar.take<double>((size_t)dims[l] * R);
  char* nws = ar.take<char>(normalize_ws_bytes(R));
  char* rws = ar.take<char>(residual_ws_bytes(dims));
  const int n_ref = p->refine_iters > 0 ? p->refine_iters : 0;
  char* rstate = n_ref ? ar.take<char>(refine_state_bytes(dims, R, n_ref)) : nullptr;
  if (!rws || (n_ref && !rstate)) {
    set_error("cpd_solve: workspace too small");
    return CPD_E_WORKSPACE;
  }
  cpd_status st;
  const int64_t n = dims[0] * dims[1] * dims[2];
  // the solve's device entry stamp goes next to the final residual (read back with it)
  long long* t_entry = (long long*)(res + 1);
  // ||T||^2 and the non-finite check: from the mode-1 Gram's trace when that Gram is the FP64 one
  // of T itself, else a pass over T (which also takes the entry stamp)
  const bool chk_from_gram = T_gram == T && gram_dtype == dtype && gram_compute != CPD_BF16;
  if (chk_from_gram) {
    if ((st = device_stamp(t_entry, s))) return st;
  } else if ((st = sumsq_full(T, dtype, n, chk, (int*)(chk + 1), sws, sumsq_ws_bytes(), s, t_entry))) {
    return st;
  }
  // ||T||^2 and the non-finite flag come back with the eigenvalues (one host round trip)
  double h_tn2 = 0.0;
  int core[3];
  st = p->st_mlsvd ? run_compress_st(T, dtype, T_gram, gram_dtype, gram_compute, dims, R, p, U, nullptr, S, core, ar,
                                     s, chk, &h_tn2, chk_from_gram)
                   : run_compress(T, dtype, T_gram, gram_dtype, gram_compute, dims, R, p, U, nullptr, S, core, ar, s,
                                  chk, &h_tn2, chk_from_gram);
  if (st) return st;
  // the header and CG caps go to the device as kernel arguments: no host synchronisation here
  if ((st = state_init(state, S, core, R, W0, h_tn2, p, s, false))) return st;
  if ((st = dgn_iterate_known(state, S, core, R, p->maxiter, s, dgn_opts(p)))) return st;
  // no read-back here: the header is read with the final residual; the output writes check its
  // non-finite flag on the device, so a rejected initial point leaves the outputs untouched
  (void)Wc;
  const int npc = (core[0] + core[1] + core[2]) * R;
  const double* Wst = (const double*)(state + layout_of(npc, R, p->maxiter).W);
  const int* flags_dev = (const int*)(state + offsetof(Hdr, flags));
  // refinement: the compressed run's iteration count and damping parameter continue on T (one
  // read-back of the core header)
  int ref_k0 = 0;
  double ref_mu = 0.0;
  bool refining = false;
  if (n_ref) {
    Hdr hc;
    CPD_HIP_CHECK(hipMemcpyAsync(&hc, state, sizeof(Hdr), hipMemcpyDeviceToHost, s));
    CPD_HIP_CHECK(hipStreamSynchronize(s));
    refining = !(hc.flags & 1);
    ref_k0 = hc.k;
    ref_mu = hc.mu;
    if (refining) {
      // the uncompressed start is written straight into the refinement state's factors
      double* Wr = (double*)(rstate + refine_w_offset(dims, R, n_ref));
      Wt[0] = Wr;
      Wt[1] = Wr + dims[0] * R;
      Wt[2] = Wr + (dims[0] + dims[1]) * R;
      if ((st = refine_setup(rstate, dims, R, n_ref, h_tn2, ref_mu, ref_k0, p, s))) return st;
    }
  }
  // uncompress W~ = U W
  size_t o = 0;
  for (int l = 0; l < 3; ++l) {
    if ((st = gemm_f64((int)dims[l], R, core[l], 1.0, U[l], core[l], 0, false, Wst + o, CPD_F64, R, 0, false,
                       0.0, Wt[l], R, 0, 1, s)))
      return st;
    o += (size_t)core[l] * R;
  }
  if (refining && (st = refine_run(rstate, T, dtype, dims, R, n_ref, s))) return st;
  const double* Wtc[3] = {Wt[0], Wt[1], Wt[2]};
  if ((st = residual_full(T, dtype, dims, Wtc, R, res, rws, residual_ws_bytes(dims), s))) return st;
  if ((st = normalize_output(Wtc, dims, R, W_out, lambda_out, nws, normalize_ws_bytes(R), s, flags_dev))) return st;
  std::vector<char> spill;
  const size_t hbytes = 256 + sizeof(Hdr);
  char* hb = readback_host(hbytes, spill);
  CPD_HIP_CHECK(hipMemcpyAsync(hb, res, hbytes, hipMemcpyDeviceToHost, s));
  CPD_HIP_CHECK(hipStreamSynchronize(s));
  double h_res;
  long long h_entry;
  Hdr h;
  memcpy(&h_res, hb, sizeof(double));
  memcpy(&h_entry, hb + sizeof(double), sizeof(long long));
  memcpy(&h, hb + 256, sizeof(Hdr));
  if (h.flags & 1) {
    set_error("state_init: non-finite initial factors");
    return CPD_E_NONFINITE;
  }
  if (h.flags & HDR_BAR_TIMEOUT) {
    set_error("dgn: a grid barrier of the multi-workgroup CG timed out");
    return CPD_E_HIP;
  }
  const int k = h.k, stop = h.stop, ti = h.tol_iter;
  const double err = (h.s_norm > 0.0) ? sqrt(h.f2) / h.s_norm : 0.0;   // = the logged error of step k
  info->iters = k;
  info->stop_reason = stop;
  for (int l = 0; l < 3; ++l) info->core_dims[l] = core[l];
  info->tol_iter = ti;
  info->rel_err_core = err;
  info->t_norm = sqrt(h_tn2);
  info->rel_err_full = sqrt(h_res > 0.0 ? h_res : 0.0) / sqrt(h_tn2);
  info->time_to_tol_ns = (ti > 0) ? (int64_t)llround((double)(h.t_tol - h_entry) * wall_ns_per_tick()) : -1;
  info->refine_iters = 0;
  info->refine_stop = 0;
  if (refining) {
    Hdr hr;
    CPD_HIP_CHECK(hipMemcpyAsync(&hr, rstate, sizeof(Hdr), hipMemcpyDeviceToHost, s));
    CPD_HIP_CHECK(hipStreamSynchronize(s));
    info->refine_iters = hr.k;
    info->refine_stop = hr.stop;
    if (hr.flags & HDR_BAR_TIMEOUT) {
      set_error("refinement: a grid barrier of the multi-workgroup CG timed out");
      return CPD_E_HIP;
    }
  }
  return CPD_OK;
}
}  // namespace

cpd_status cpd_solve(const void* T, int32_t dtype, const int64_t dims[3], int32_t R,
                     const cpd_params* p, const double* W0, double* W_out[3], double* lambda_out,
                     cpd_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  cpd_params def;
  if (!p) { cpd_default_params(&def); p = &def; }
  return solve_impl(T, dtype, p->compute_dtype, T, dtype, dims, R, p, W0, W_out, lambda_out, info, ws, ws_bytes,
                    stream);
}

cpd_status cpd_solve_mixed(const void* T_lo, int32_t lo_dtype, const void* T, int32_t dtype, const int64_t dims[3],
                           int32_t R, const cpd_params* p, const double* W0, double* W_out[3], double* lambda_out,
                           cpd_solve_info* info, void* ws, size_t ws_bytes, void* stream) {
  CPD_REQUIRE(T_lo && lo_dtype == CPD_BF16, "cpd_solve_mixed: T_lo must be a BF16 tensor");
  cpd_params def;
  if (!p) { cpd_default_params(&def); p = &def; }
  return solve_impl(T_lo, lo_dtype, CPD_BF16, T, dtype, dims, R, p, W0, W_out, lambda_out, info, ws, ws_bytes, stream);
}

size_t cpd_gram_workspace_bytes(const int64_t dims[3], int32_t mode) {
  if (!dims_ok(dims) || mode < 0 || mode > 2) return 0;
  return gram_ws_bytes(dims, mode);
}

cpd_status cpd_gram(const void* T, int32_t dtype, const int64_t dims[3], int32_t mode,
                    int32_t compute_dtype, double* G, void* ws, size_t ws_bytes, void* stream) {
  CPD_REQUIRE(T && G && dims_ok(dims) && dtype_ok(dtype) && mode >= 0 && mode <= 2, "cpd_gram: bad arguments");
  return gram(T, dtype, dims, mode, compute_dtype, G, ws, ws_bytes, (hipStream_t)stream);
}

size_t cpd_eig_workspace_bytes(int32_t n, int32_t P) {
  if (n < 1 || P < 1 || P > n) return 0;
  return eig_ws_bytes(n, P);
}

cpd_status cpd_eig_top(const double* G, int32_t n, int32_t P, double* U, double* lam, void* ws,
                       size_t ws_bytes, void* stream) {
  CPD_REQUIRE(G && U && lam && n >= 1 && n <= 4096 && P >= 1 && P <= n, "cpd_eig_top: bad arguments");
  return eig_top(G, n, P, U, lam, ws, ws_bytes, (hipStream_t)stream);
}

size_t cpd_mttkrp_workspace_bytes(const int64_t dims[3], int32_t R, int32_t mode) {
  if (!dims_ok(dims) || R < 1 || mode < 0 || mode > 2) return 0;
  return mttkrp_ws_bytes(dims, R, mode);
}

cpd_status cpd_mttkrp(const void* T, int32_t dtype, const int64_t dims[3], const double* const W[3],
                      int32_t R, int32_t mode, int32_t compute_dtype, double* M, void* ws, size_t ws_bytes,
                      void* stream) {
  CPD_REQUIRE(T && W && W[0] && W[1] && W[2] && M && dims_ok(dims) && dtype_ok(dtype) && dtype_ok(compute_dtype) &&
                  R >= 1 && R <= 64,
              "cpd_mttkrp: bad arguments");
  return mttkrp_full(T, dtype, dims, W, R, mode, compute_dtype, M, ws, ws_bytes, (hipStream_t)stream);
}

size_t cpd_residual_workspace_bytes(const int64_t dims[3]) {
  if (!dims_ok(dims)) return 0;
  return residual_ws_bytes(dims);
}

cpd_status cpd_residual_norm2(const void* T, int32_t dtype, const int64_t dims[3],
                              const double* const W[3], int32_t R, double* out, void* ws,
                              size_t ws_bytes, void* stream) {
  CPD_REQUIRE(T && W && out && dims_ok(dims) && dtype_ok(dtype), "cpd_residual_norm2: bad arguments");
  return residual_full(T, dtype, dims, W, R, out, ws, ws_bytes, (hipStream_t)stream);
}

size_t cpd_tt_workspace_bytes(int32_t L, const int64_t* dims, int32_t R, const cpd_params* p) {
  cpd_params def;
  if (!p) { cpd_default_params(&def); p = &def; }
  return tt_ws_bytes(L, dims, R, p);
}

cpd_status cpd_solve_tt(const void* T, int32_t dtype, int32_t L, const int64_t* dims, int32_t R, const cpd_params* p,
                        const double* W0, double* const* W_out, double* lambda_out, cpd_solve_info* info, void* ws,
                        size_t ws_bytes, void* stream) {
  CPD_REQUIRE(T && dims && W_out && lambda_out && info && (dtype == CPD_F64 || dtype == CPD_F32),
              "cpd_solve_tt: bad arguments");
  CPD_REQUIRE(L >= 4 && L <= 16, "cpd_solve_tt: order L must be 4..16");
  for (int l = 0; l < L; ++l) CPD_REQUIRE(W_out[l] != nullptr, "cpd_solve_tt: null output factor");
  cpd_params def;
  if (!p) { cpd_default_params(&def); p = &def; }
  CPD_REQUIRE(p->maxiter >= 1 && p->tol >= 0.0, "cpd_solve_tt: bad parameters");
  return solve_tt(T, dtype, L, dims, R, p, W0, W_out, lambda_out, info, ws, ws_bytes, (hipStream_t)stream);
}

cpd_status cpd_residual_norm2_noalloc(const void* T, int32_t dtype, const int64_t dims[3],
                                      const double* const W[3], int32_t R, double* out, void* stream) {
  CPD_REQUIRE(T && W && out && dims_ok(dims) && dtype_ok(dtype), "cpd_residual_norm2_noalloc: bad arguments");
  return residual_full_noalloc(T, dtype, dims, W, R, out, (hipStream_t)stream);
}

cpd_status cpd_jtj_v(const double* const W[3], const double* const V[3], const int32_t dims[3],
                     int32_t R, double* const out[3], void* stream) {
  CPD_REQUIRE(W && V && dims && out, "cpd_jtj_v: null argument");
  return jtj_v(W, V, dims, R, out, (hipStream_t)stream);
}

}  // extern "C"
