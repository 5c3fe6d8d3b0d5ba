// Device-resident state of the persistent dGN kernel (shared by the single solve and the batched
// solver, which writes headers on the device).
#pragma once
#include "common.h"

namespace cpd {

constexpr int DGN_NT = 512;   // threads of the persistent dGN workgroup

namespace {
constexpr int NT = DGN_NT;
constexpr int NW = NT / 64;
}  // namespace

// Hdr::flags bits: 1 non-finite start (set by the initialisation), 2 rejected batch member,
// HDR_PRESET the header arrives with ||S||, mu and the divergence reference already set (refinement)
constexpr int32_t HDR_PRESET = 4;
// HDR_FIX0: the first factor is fixed (the Bi-CPD of the tensor-train route): its block of the step,
// gradient and CG vectors stays zero and only modes 2 and 3 are balanced
constexpr int32_t HDR_FIX0 = 8;
// HDR_BAR_TIMEOUT: a grid barrier of the multi-workgroup CG stopped waiting (the results are invalid)
constexpr int32_t HDR_BAR_TIMEOUT = 16;
// HDR_DIRTY: the factors were replaced from outside (cpd_state_factors); the next iteration launch
// first recomputes the residual and the MTTKRP at them
constexpr int32_t HDR_DIRTY = 32;

struct Hdr {
  int32_t d[3];
  int32_t R;
  int32_t k, stop, maxiter, tol_iter;
  int32_t np, flags, pad0, pad1;
  double mu, f2, s_norm, div_ref, tol, cg_tol, init_damp, err0;
  // one iteration split over launches (large cores): values of the step awaiting its residual
  double f2_pred, stepn, grad_inf, cg_resid, f2_new;
  int32_t its, cap, pending, pad2;
  // device wall-clock ticks (constant-rate counter): end of initialisation, and the end of the
  // first iteration whose error fell below tol (valid when tol_iter > 0)
  int64_t t_init, t_tol;
};
static_assert(sizeof(Hdr) <= 256, "header must fit its slot");

struct Layout {
  size_t W, MK, G, errs, caps, log, work, total;
};

__host__ __device__ inline size_t lds_doubles(int np, int R);

// Regions of a state (the work region holds the working set when it does not fit in LDS)
__host__ __device__ inline Layout layout_of(int np, int R, int maxiter) {
  Layout L;
  size_t off = 256;
  L.W = off; off += (size_t)np * 8;
  L.MK = off; off += (size_t)np * 8;
  L.G = off; off += (size_t)np * 8;
  L.errs = off; off += (size_t)(maxiter + 1) * 8;
  L.caps = off; off += ((size_t)maxiter * 4 + 7) / 8 * 8;
  L.log = off; off += (size_t)maxiter * sizeof(cpd_step_info);
  off = (off + 255) / 256 * 256;
  L.work = off; off += lds_doubles(np, R) * 8;
  L.total = (off + 255) / 256 * 256;
  return L;
}

// LDS footprint in doubles of the working set (W and the CG vectors X, r, p, z; the R x R
// Grams and products; preconditioner and regularisation scalars; reduction slots).  The MTTKRP and
// the gradient stay in the state (each is written and read once per iteration); the core S is
// staged after the working set when it fits.
__host__ __device__ inline size_t lds_doubles(int np, int R) {
  return (size_t)5 * np + (size_t)9 * R * R + (size_t)6 * R + 2 * NW + 16;
}

// Extra LDS of the block-Jacobi preconditioner: one more vector and the three R x R inverse factors
__host__ __device__ inline size_t block_lds_doubles(int np, int R) { return (size_t)np + (size_t)3 * R * R; }

}  // namespace cpd
