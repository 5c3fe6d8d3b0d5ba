// Internal helpers shared by the libcpd translation units (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/cpd.h"

namespace cpd {

// ---- error reporting -------------------------------------------------------------------------
void set_error(const char* fmt, ...);

#define CPD_HIP_CHECK(expr)                                                         \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess) {                                                         \
      ::cpd::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e),       \
                       __FILE__, __LINE__);                                         \
      return CPD_E_HIP;                                                             \
    }                                                                               \
  } while (0)

#define CPD_LAUNCH_CHECK() CPD_HIP_CHECK(hipGetLastError())

#define CPD_REQUIRE(cond, ...)                                                      \
  do {                                                                              \
    if (!(cond)) {                                                                  \
      ::cpd::set_error(__VA_ARGS__);                                                \
      return CPD_E_INVALID;                                                         \
    }                                                                               \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over the caller's workspace.
struct Arena {
  char* base;
  size_t cap;
  size_t off;
  Arena(void* b, size_t c) : base((char*)b), cap(c), off(0) {}
  template <class T>
  T* take(size_t n) {
    size_t o = align_up(off, 256);
    size_t bytes = align_up(n * sizeof(T), 256);
    if (base == nullptr || o + bytes > cap) return nullptr;
    off = o + bytes;
    return (T*)(base + o);
  }
};

// Byte-size accumulator mirroring Arena::take, for the workspace queries.
struct Sizer {
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = align_up(off, 256) + align_up(n * sizeof(T), 256);
    return nullptr;
  }
};

// ---- device helpers --------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ double to_f64(T v) { return (double)v; }

__device__ __forceinline__ double bf16_bits_to_f64(uint16_t b) {
  uint32_t u = ((uint32_t)b) << 16;
  return (double)__uint_as_float(u);
}

// Sum over a 64-wide wavefront; every lane gets the result.  Fixed butterfly order keeps the
// result identical run to run.
// Index of the calling wave within its workgroup, as a wave-uniform (scalar) value, so that
// tile indices derived from it stay in scalar registers and branches on them are uniform.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Block-wide sum: `slots` is LDS with room for blockDim.x/64 doubles.  Contains one barrier;
// callers alternate between two slot arrays so back-to-back reductions need no second barrier.
__device__ __forceinline__ double block_sum(double v, double* slots) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) slots[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += slots[i];
  return s;
}

__device__ __forceinline__ double block_max(double v, double* slots) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) slots[w] = v;
  __syncthreads();
  double s = slots[0];
  for (int i = 1; i < nw; ++i) s = fmax(s, slots[i]);
  return s;
}

// SplitMix64 (Steele, Lea, Flood 2014): counter-based 64-bit generator.
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__host__ __device__ __forceinline__ double u01_from_bits(uint64_t x) {
  return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

// ---- host launchers implemented in the .hip files ---------------------------------------------
// Batched FP64 GEMM: C[b] = alpha * op(A[b]) op(B[b]) + beta * C[b].
//   op(A)(m,k) = ta ? A[k*lda + m] : A[m*lda + k];  op(B)(k,n) = tb ? B[n*ldb + k] : B[k*ldb + n]
//   C(m,n) = tc ? C[n*ldc + m] : C[m*ldc + n]
//   bdtype: element type of B (CPD_F64, CPD_F32 or CPD_BF16); A and C are FP64.
// Y[a][b][k] = sum_j U[j][b] X[a][j][k] (U is J x nb row-major, X and Y dense, k contiguous).
cpd_status mode_product_mid(const void* X, int xdtype, int A, int J, long long K, const double* U, int nb,
                            double* Y, hipStream_t s);
bool mode_product_mid_fits(int J, int nb);   // whether mode_product_mid supports J rows of U
// Y[b] (r x N) = U^T X[b] for U (K x r, r <= 64) and row-major X[b] (K x N), b < batch, on the FP64
// matrix cores (the first two mode products of the core projection).
cpd_status project_mfma(const void* X, int xdtype, int K, long long N, int batch, long long sX, const double* U,
                        int r, double* Y, long long sY, hipStream_t s);
cpd_status gemm_f64(int M, int N, int K, double alpha, const double* A, int lda, long long sA,
                    bool ta, const void* B, int bdtype, long long ldb, long long sB, bool tb,
                    double beta, double* C, long long ldc, long long sC, int batch,
                    hipStream_t s, bool tc = false);

// Gram G = T_(mode) T_(mode)^T (I_mode x I_mode, FP64).
size_t gram_ws_bytes(const int64_t dims[3], int mode);
cpd_status gram(const void* T, int dtype, const int64_t dims[3], int mode, int compute_dtype,
                double* G, void* ws, size_t ws_bytes, hipStream_t s);

// Eigen solvers.
size_t eig_ws_bytes(int n, int P);
size_t eig_ws_bytes3(const int* n, const int* P, int nprob);
// Several independent problems in one call.
cpd_status eig_top3(const double* const* G, const int* n, const int* P, double* const* U,
                    double* const* lam, int nprob, void* ws, size_t ws_bytes, hipStream_t s);
cpd_status eig_top(const double* G, int n, int P, double* U, double* lam, void* ws,
                   size_t ws_bytes, hipStream_t s);

// Full-tensor kernels.
cpd_status mttkrp_full(const void* T, int dtype, const int64_t dims[3], const double* const W[3],
                       int R, int mode, int compute_dtype, double* M, void* ws, size_t ws_bytes, hipStream_t s);
size_t residual_ws_bytes(const int64_t dims[3]);
size_t sumsq_ws_bytes();
cpd_status residual_full(const void* T, int dtype, const int64_t dims[3],
                         const double* const W[3], int R, double* out, void* ws, size_t ws_bytes,
                         hipStream_t s);
// The same with its partial sums in the library's static device scratch (no workspace, no
// allocation; calls that overlap on one GPU race on that scratch).
cpd_status residual_full_noalloc(const void* T, int dtype, const int64_t dims[3], const double* const W[3],
                                 int R, double* out, hipStream_t s);
// stamp (device, nullable): receives the device wall clock when the kernel starts.
cpd_status sumsq_full(const void* T, int dtype, int64_t n, double* out, int* nonfinite, void* ws,
                      size_t ws_bytes, hipStream_t s, long long* stamp = nullptr);
// ||T||^2 and the non-finite flag from the trace of an FP64 Gram of T's mode-1 unfolding.
cpd_status gram_trace_check(const double* G, int n, double* out, int* nonfinite, hipStream_t s);
// writes the device wall clock to t
cpd_status device_stamp(long long* t, hipStream_t s);
// Nanoseconds per tick of the device wall clock (wall_clock64) of the current device.
double wall_ns_per_tick();

// dGN.
size_t state_bytes(const int32_t core[3], int R, int maxiter);
size_t dgn_aux_bytes(const int d[3], int R);
// check_flags = false leaves the non-finite-start flag in the header for the caller to read.
// hdr_flags: initial header flags (HDR_FIX0 for a fixed first factor).
cpd_status state_init(void* state, const double* S, const int32_t core[3], int R,
                      const double* W0, double t_norm2, const cpd_params* p, hipStream_t s,
                      bool check_flags = true, int32_t hdr_flags = 0);
// A third-order CPD of a device FP64 tensor (compression, dGN, uncompression) whose factors are
// returned unnormalised: uncompressed and balanced, in the dGN's column order, packed
// (d0 + d1 + d2) x R in Wt.  Workspace: solve_ws_bytes(dims, R, p).  Synchronises the stream.
size_t solve_ws_bytes(const int64_t dims[3], int R, const cpd_params* p);
cpd_status solve3_raw(const double* T, const int64_t dims[3], int R, const cpd_params* p, const double* W0,
                      double* Wt, int* iters, int* stop, double* rel_err, void* ws, size_t ws_bytes, hipStream_t s);
// Options of the iteration launches, from cpd_params.precond / drawback (kernel arguments; the
// state does not record them)
constexpr int DGN_OPT_BLOCK = 1;      // block-Jacobi preconditioner
constexpr int DGN_OPT_DRAWBACK = 2;   // draw-back with a dogleg step on a hundredfold error jump
inline int dgn_opts(const cpd_params* p) {
  return p ? ((p->precond == 1 ? DGN_OPT_BLOCK : 0) | (p->drawback ? DGN_OPT_DRAWBACK : 0)) : 0;
}
// dgn_iterate for a state just set up by state_init with maxiter = max_steps and no factors
// replaced since: the caller knows its sizes, so there is no header read-back.
cpd_status dgn_iterate_known(void* state, const double* S, const int32_t core[3], int R, int max_steps,
                             hipStream_t s, int opts = 0);
size_t dgn_lds_bytes(int np, int R);
// N(0,1) entries (Box-Muller on SplitMix64 counters), the library's own random start.
cpd_status fill_randn(double* W, int n, uint64_t seed, hipStream_t s);
// The tensor-train route for order L >= 4 (cpd_solve_tt).
size_t tt_ws_bytes(int L, const int64_t* dims, int R, const cpd_params* p);
cpd_status solve_tt(const void* T, int dtype, int L, const int64_t* dims, int R, const cpd_params* p,
                    const double* W0, double* const* W_out, double* lambda_out, cpd_solve_info* info, void* ws,
                    size_t ws_bytes, hipStream_t s);
// Refinement in the original space: a dGN state over the input tensor (global-memory path).
size_t refine_state_bytes(const int64_t dims[3], int R, int n_iters);
size_t refine_w_offset(const int64_t dims[3], int R, int n_iters);
cpd_status refine_setup(void* state, const int64_t dims[3], int R, int n_iters, double t_norm2, double mu, int k0,
                        const cpd_params* p, hipStream_t s);
cpd_status refine_run(void* state, const void* T, int dtype, const int64_t dims[3], int R, int n_iters,
                      hipStream_t s);
// Batched persistent dGN: one workgroup per state (header, caps and W written beforehand).
// dgn_batch_prepare sets the kernel's dynamic-LDS limit (call outside graph capture).
cpd_status dgn_batch_prepare(size_t lds_bytes);
cpd_status dgn_batch_launch(char* const* states, const double* const* S, int n, size_t lds_bytes,
                            hipStream_t s);
cpd_status dgn_iterate(void* state, const double* S, int max_steps, hipStream_t s, int opts = 0);
cpd_status state_read(void* state, int* k, int* stop, int* tol_iter, double* err,
                      hipStream_t s);
cpd_status state_log(void* state, int first, int count, cpd_step_info* out, hipStream_t s);
cpd_status state_factors(void* state, double* W, int set, hipStream_t s);
cpd_status jtj_v(const double* const W[3], const double* const V[3], const int32_t dims[3],
                 int R, double* const out[3], hipStream_t s);

// Output stage: unit columns, lambda >= 0, signs and ordering of the uncompressed factors.
size_t normalize_ws_bytes(int R);
cpd_status normalize_output(const double* const Wt[3], const int64_t dims[3], int R,
                            double* const Wout[3], double* lambda, void* ws, size_t ws_bytes,
                            hipStream_t s,
                            const int* skip = nullptr);   // device flag: bit 0 set -> write nothing
size_t mttkrp_ws_bytes(const int64_t dims[3], int R, int mode);

// Kernel timing (see cpd_profile_* in cpd.h).  No-ops unless enabled.
void prof_begin(int which, hipStream_t s);
void prof_end(int which, hipStream_t s);

// Host-side CG cap schedule (exact integer ceilings).
int cg_cap_for(int k, double u);

}  // namespace cpd
