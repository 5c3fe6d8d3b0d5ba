// Learned initialisation: a multilayer perceptron x -> relu(x W1 + b1) -> relu(. W2 + b2) ->
// . W3 + b3 that maps a normalised compressed core to initial core factors, trained with the
// squared error and Adam (Kingma & Ba 2015, Algorithm 1).  Not part of the thesis's method: an
// extension that feeds the dGN of ch.4 a starting point.
//
// Every product is one tiled FP32 GEMM on the matrix cores (v_mfma_f32_16x16x4f32, FP32
// accumulation) with the bias / ReLU / ReLU-derivative applied in its epilogue:
//   forward   H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2), Y = H2 W3 + b3
//   backward  dW3 = H2^T G3, G2 = (G3 W3^T) * [H2 > 0], dW2 = H1^T G2, G1 = (G2 W2^T) * [H1 > 0],
//             dW1 = X^T G1, db_l = column sums of G_l.
// Result layout of v_mfma_f32_16x16x4f32 (checked on the device): A[i][k] from lane i + 16 k,
// B[k][j] from lane j + 16 k, acc[v] of lane l is D[4 (l / 16) + v][l % 16].
#include "common.h"

#include <math.h>

namespace cpd {
namespace {

typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;    // output tile edge
constexpr int GK = 16;    // k-tile
constexpr int GNT = 256;  // 4 waves, each a 32 x 32 quarter

enum { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_RELU = 2, EPI_RELU_MASK = 3 };

// C (M x N, ldc) = op(A) op(B), then the epilogue:
//   op(A)(m, k) = TA ? A[k lda + m] : A[m lda + k];  op(B)(k, n) = TB ? B[n ldb + k] : B[k ldb + n]
//   EPI_BIAS: + bias[n];  EPI_BIAS_RELU: max(. + bias[n], 0);  EPI_RELU_MASK: . * [H[m ldh + n] > 0]
template <bool TA, bool TB>
__global__ __launch_bounds__(GNT) void mlp_gemm_kernel(int M, int N, int K, const float* __restrict__ A, int lda,
                                                       const float* __restrict__ B, int ldb, float* __restrict__ C,
                                                       int ldc, const float* __restrict__ bias,
                                                       const float* __restrict__ H, int ldh, int epi) {
  __shared__ float As[GT][GK + 1];
  __shared__ float Bs[GK][GT + 1];
  const int n0 = blockIdx.x * GT, m0 = blockIdx.y * GT;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  constexpr int PER = GT * GK / GNT;   // 4 elements of each operand per thread and tile
  // staging slots: threads run along the operand's contiguous index
  int am[PER], ak[PER], bk[PER], bn[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + u * GNT;
    if (TA) { ak[u] = e / GT; am[u] = e % GT; } else { am[u] = e / GK; ak[u] = e % GK; }
    if (TB) { bn[u] = e / GK; bk[u] = e % GK; } else { bk[u] = e / GT; bn[u] = e % GT; }
  }
  float ra[PER], rb[PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int m = m0 + am[u], k = k0 + ak[u];
      const bool ok = m < M && k < K;
      const int mc = ok ? m : 0, kc = ok ? k : 0;
      const float v = TA ? A[(long long)kc * lda + mc] : A[(long long)mc * lda + kc];
      ra[u] = ok ? v : 0.f;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int n = n0 + bn[u], k = k0 + bk[u];
      const bool ok = n < N && k < K;
      const int nc = ok ? n : 0, kc = ok ? k : 0;
      const float v = TB ? B[(long long)nc * ldb + kc] : B[(long long)kc * ldb + nc];
      rb[u] = ok ? v : 0.f;
    }
  };
  flt4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
  if (K > 0) fetch(0);
  for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      As[am[u]][ak[u]] = ra[u];
      Bs[bk[u]][bn[u]] = rb[u];
    }
    __syncthreads();
    if (k0 + GK < K) fetch(k0 + GK);
#pragma unroll
    for (int s = 0; s < GK / 4; ++s) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[wm + 16 * i + (lane & 15)][4 * s + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[4 * s + (lane >> 4)][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + v;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m < M && n < N) {
          float c = acc[i][j][v];
          if (epi == EPI_BIAS || epi == EPI_BIAS_RELU) c += bias[n];
          if (epi == EPI_BIAS_RELU) c = fmaxf(c, 0.f);
          if (epi == EPI_RELU_MASK) c = (H[(long long)m * ldh + n] > 0.f) ? c : 0.f;
          C[(long long)m * ldc + n] = c;
        }
      }
}

// db[n] = sum_m G[m][n]: one thread per column, rows in a fixed order.
__global__ void colsum_kernel(const float* __restrict__ G, int M, int N, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  int m = 0;
  for (; m + 3 < M; m += 4) {
    s0 += G[(long long)m * N + n];
    s1 += G[(long long)(m + 1) * N + n];
    s2 += G[(long long)(m + 2) * N + n];
    s3 += G[(long long)(m + 3) * N + n];
  }
  for (; m < M; ++m) s0 += G[(long long)m * N + n];
  db[n] = (s0 + s1) + (s2 + s3);
}

// dy = 2 (y - t) / n and per-block partial sums of (y - t)^2
constexpr int LNT = 256;
__global__ __launch_bounds__(LNT) void mse_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                  long long n, float* __restrict__ dy, double* __restrict__ part) {
  __shared__ double slots[LNT / 64];
  double s = 0.0;
  const float scale = 2.f / (float)n;
  for (long long e = (long long)blockIdx.x * LNT + threadIdx.x; e < n; e += (long long)gridDim.x * LNT) {
    const float d = y[e] - t[e];
    dy[e] = scale * d;
    s += (double)d * (double)d;
  }
  s = block_sum(s, slots);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void mse_final_kernel(const double* __restrict__ part, int nb, long long n, float* __restrict__ loss) {
  __shared__ double slots[256 / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
  s = block_sum(s, slots);
  if (threadIdx.x == 0) *loss = (float)(s / (double)n);
}

// One Adam update of n parameters (bias-corrected moments).
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

cpd_status gemm32(bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C,
                  int ldc, const float* bias, const float* H, int ldh, int epi, hipStream_t s) {
  if (M < 1 || N < 1 || K < 1) return CPD_OK;
  const dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  if (!ta && !tb)
    hipLaunchKernelGGL((mlp_gemm_kernel<false, false>), grid, dim3(GNT), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, H, ldh, epi);
  else if (!ta && tb)
    hipLaunchKernelGGL((mlp_gemm_kernel<false, true>), grid, dim3(GNT), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, H, ldh, epi);
  else if (ta && !tb)
    hipLaunchKernelGGL((mlp_gemm_kernel<true, false>), grid, dim3(GNT), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, H, ldh, epi);
  else
    hipLaunchKernelGGL((mlp_gemm_kernel<true, true>), grid, dim3(GNT), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, H, ldh, epi);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

// Small batches (B <= VB, inference on one or a few cores): each layer as a split-K matrix-vector
// product streaming the weights once with coalesced loads (the tiled GEMM would run a handful of
// workgroups over the whole K), then a fixed-order reduction of the partial sums with the bias and
// ReLU.  part[ks][b][n] = sum over rows k of chunk ks of x[b][k] W[k][n].
constexpr int VB = 8;
constexpr int VNT = 256;
constexpr int VROWS = 256;                  // rows of x staged in LDS at a time
constexpr size_t VPART = (size_t)1024 * VNT;   // bound on KS * N (KS <= 1024 / column blocks)

__global__ __launch_bounds__(VNT) void gemv_part_kernel(int B, int N, int K, int chunk, const float* __restrict__ x,
                                                        int ldx, const float* __restrict__ W,
                                                        float* __restrict__ part) {
  __shared__ float xs[VB][VROWS];
  const int n = blockIdx.x * VNT + threadIdx.x;
  const int k0 = blockIdx.y * chunk;
  const int k1 = min(K, k0 + chunk);
  float acc[VB];
#pragma unroll
  for (int b = 0; b < VB; ++b) acc[b] = 0.f;
  for (int kb = k0; kb < k1; kb += VROWS) {
    const int kn = min(VROWS, k1 - kb);
    __syncthreads();
    for (int e = threadIdx.x; e < B * kn; e += VNT) {
      const int b = e / kn, kk = e - b * kn;
      xs[b][kk] = x[(long long)b * ldx + kb + kk];
    }
    __syncthreads();
    if (n < N) {
      for (int kk = 0; kk < kn; ++kk) {
        const float w = W[(long long)(kb + kk) * N + n];
#pragma unroll
        for (int b = 0; b < VB; ++b)
          if (b < B) acc[b] += xs[b][kk] * w;
      }
    }
  }
  if (n < N)
    for (int b = 0; b < B; ++b) part[((long long)blockIdx.y * B + b) * N + n] = acc[b];
}

__global__ void gemv_reduce_kernel(int B, int N, int KS, const float* __restrict__ part,
                                   const float* __restrict__ bias, int relu, float* __restrict__ y, int ldy) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * N) return;
  const int b = e / N, n = e - b * N;
  float s = 0.f;
  for (int ks = 0; ks < KS; ++ks) s += part[((long long)ks * B + b) * N + n];
  s += bias[n];
  y[(long long)b * ldy + n] = relu ? fmaxf(s, 0.f) : s;
}

// y (B x N) = epi(x (B x K) W (K x N) + bias) for B <= VB; part holds VPART * B floats.
cpd_status gemv32(int B, int N, int K, const float* x, const float* W, const float* bias, bool relu, float* y,
                  float* part, hipStream_t s) {
  const int cols = (N + VNT - 1) / VNT;
  int ks = 1024 / cols;
  const int kmax = (K + 7) / 8;   // at least eight rows per chunk
  ks = ks < 1 ? 1 : (ks > kmax ? kmax : ks);
  const int chunk = (K + ks - 1) / ks;
  ks = (K + chunk - 1) / chunk;
  hipLaunchKernelGGL(gemv_part_kernel, dim3(cols, ks), dim3(VNT), 0, s, B, N, K, chunk, x, K, W, part);
  CPD_LAUNCH_CHECK();
  hipLaunchKernelGGL(gemv_reduce_kernel, dim3((B * N + 255) / 256), dim3(256), 0, s, B, N, ks, part, bias,
                     relu ? 1 : 0, y, N);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

bool net_ok(const cpd_mlp* net) {
  if (!net) return false;
  const int d[4] = {net->n_in, net->n_h1, net->n_h2, net->n_out};
  for (int i = 0; i < 4; ++i)
    if (d[i] < 1 || d[i] > (1 << 20)) return false;
  for (int l = 0; l < 3; ++l)
    if (!net->W[l] || !net->b[l]) return false;
  return true;
}

// Workspace: H1 (B x h1), H2 (B x h2), G2 (B x h2), G1 (B x h1); for B <= VB also the partial sums
// of the small-batch forward (VPART * B).
template <class Carver>
void carve_mlp(Carver& z, const cpd_mlp* net, int B, float** H1, float** H2, float** G2, float** G1,
               float** part) {
  *H1 = z.template take<float>((size_t)B * net->n_h1);
  *H2 = z.template take<float>((size_t)B * net->n_h2);
  *G2 = z.template take<float>((size_t)B * net->n_h2);
  *G1 = z.template take<float>((size_t)B * net->n_h1);
  *part = B <= VB ? z.template take<float>(VPART * B) : nullptr;
}

}  // namespace
}  // namespace cpd

using namespace cpd;

extern "C" {

size_t cpd_mlp_workspace_bytes(const cpd_mlp* net, int32_t B) {
  if (!net_ok(net) || B < 1) return 0;
  Sizer z;
  float *a, *b, *c, *d, *e;
  carve_mlp(z, net, B, &a, &b, &c, &d, &e);
  return z.off;
}

cpd_status cpd_mlp_forward(const cpd_mlp* net, const float* x, float* y, int32_t B, void* ws, size_t ws_bytes,
                           void* stream) {
  CPD_REQUIRE(net_ok(net) && x && y && B >= 1, "cpd_mlp_forward: bad arguments");
  if (!ws || ws_bytes < cpd_mlp_workspace_bytes(net, B)) {
    set_error("cpd_mlp_forward: workspace too small");
    return CPD_E_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  Arena ar(ws, ws_bytes);
  float *H1, *H2, *G2, *G1, *part;
  carve_mlp(ar, net, B, &H1, &H2, &G2, &G1, &part);
  cpd_status st;
  if (B <= VB) {
    if ((st = gemv32(B, net->n_h1, net->n_in, x, net->W[0], net->b[0], true, H1, part, s))) return st;
    if ((st = gemv32(B, net->n_h2, net->n_h1, H1, net->W[1], net->b[1], true, H2, part, s))) return st;
    return gemv32(B, net->n_out, net->n_h2, H2, net->W[2], net->b[2], false, y, part, s);
  }
  if ((st = gemm32(false, false, B, net->n_h1, net->n_in, x, net->n_in, net->W[0], net->n_h1, H1, net->n_h1,
                   net->b[0], nullptr, 0, EPI_BIAS_RELU, s)))
    return st;
  if ((st = gemm32(false, false, B, net->n_h2, net->n_h1, H1, net->n_h1, net->W[1], net->n_h2, H2, net->n_h2,
                   net->b[1], nullptr, 0, EPI_BIAS_RELU, s)))
    return st;
  return gemm32(false, false, B, net->n_out, net->n_h2, H2, net->n_h2, net->W[2], net->n_out, y, net->n_out,
                net->b[2], nullptr, 0, EPI_BIAS, s);
}

cpd_status cpd_mlp_mse(const float* y, const float* t, int64_t n, float* dy, float* loss, void* ws, size_t ws_bytes,
                       void* stream) {
  CPD_REQUIRE(y && t && dy && loss && n >= 1, "cpd_mlp_mse: bad arguments");
  int nb = (int)((n + LNT - 1) / LNT);
  if (nb > 1024) nb = 1024;
  if (!ws || ws_bytes < (size_t)nb * sizeof(double)) {
    set_error("cpd_mlp_mse: workspace too small (needs 8 KiB)");
    return CPD_E_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(LNT), 0, s, y, t, (long long)n, dy, (double*)ws);
  hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(256), 0, s, (const double*)ws, nb, (long long)n, loss);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

cpd_status cpd_mlp_backward(const cpd_mlp* net, const float* x, const float* dy, cpd_mlp_grads* g, int32_t B,
                            void* ws, size_t ws_bytes, void* stream) {
  CPD_REQUIRE(net_ok(net) && x && dy && g && B >= 1, "cpd_mlp_backward: bad arguments");
  for (int l = 0; l < 3; ++l) CPD_REQUIRE(g->dW[l] && g->db[l], "cpd_mlp_backward: null gradient buffer");
  if (!ws || ws_bytes < cpd_mlp_workspace_bytes(net, B)) {
    set_error("cpd_mlp_backward: workspace too small");
    return CPD_E_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  Arena ar(ws, ws_bytes);
  float *H1, *H2, *G2, *G1;
  float* part;
  carve_mlp(ar, net, B, &H1, &H2, &G2, &G1, &part);
  const int h1 = net->n_h1, h2 = net->n_h2, no = net->n_out, ni = net->n_in;
  cpd_status st;
  // layer 3
  if ((st = gemm32(true, false, h2, no, B, H2, h2, dy, no, g->dW[2], no, nullptr, nullptr, 0, EPI_NONE, s))) return st;
  hipLaunchKernelGGL(colsum_kernel, dim3((no + 255) / 256), dim3(256), 0, s, dy, B, no, g->db[2]);
  if ((st = gemm32(false, true, B, h2, no, dy, no, net->W[2], no, G2, h2, nullptr, H2, h2, EPI_RELU_MASK, s))) return st;
  // layer 2
  if ((st = gemm32(true, false, h1, h2, B, H1, h1, G2, h2, g->dW[1], h2, nullptr, nullptr, 0, EPI_NONE, s))) return st;
  hipLaunchKernelGGL(colsum_kernel, dim3((h2 + 255) / 256), dim3(256), 0, s, G2, B, h2, g->db[1]);
  if ((st = gemm32(false, true, B, h1, h2, G2, h2, net->W[1], h2, G1, h1, nullptr, H1, h1, EPI_RELU_MASK, s))) return st;
  // layer 1
  if ((st = gemm32(true, false, ni, h1, B, x, ni, G1, h1, g->dW[0], h1, nullptr, nullptr, 0, EPI_NONE, s))) return st;
  hipLaunchKernelGGL(colsum_kernel, dim3((h1 + 255) / 256), dim3(256), 0, s, G1, B, h1, g->db[0]);
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

cpd_status cpd_mlp_adam_step(cpd_mlp* net, const cpd_mlp_grads* g, cpd_adam* a, void* stream) {
  CPD_REQUIRE(net_ok(net) && g && a && a->lr > 0.f && a->beta1 >= 0.f && a->beta1 < 1.f && a->beta2 >= 0.f &&
                  a->beta2 < 1.f,
              "cpd_mlp_adam_step: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  a->step += 1;
  const float c1 = 1.f - powf(a->beta1, (float)a->step), c2 = 1.f - powf(a->beta2, (float)a->step);
  const int d[4] = {net->n_in, net->n_h1, net->n_h2, net->n_out};
  for (int l = 0; l < 3; ++l) {
    CPD_REQUIRE(a->mW[l] && a->vW[l] && a->mb[l] && a->vb[l] && g->dW[l] && g->db[l], "cpd_mlp_adam_step: null state");
    const long long nw = (long long)d[l] * d[l + 1], nbias = d[l + 1];
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, net->W[l], g->dW[l], a->mW[l],
                       a->vW[l], nw, a->lr, a->beta1, a->beta2, a->eps, c1, c2);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((nbias + 255) / 256)), dim3(256), 0, s, net->b[l], g->db[l],
                       a->mb[l], a->vb[l], nbias, a->lr, a->beta1, a->beta2, a->eps, c1, c2);
  }
  CPD_LAUNCH_CHECK();
  return CPD_OK;
}

}  // extern "C"
