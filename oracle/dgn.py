"""Damped Gauss-Newton with Jacobi-preconditioned CG on the compressed core (oracle; test
infrastructure only).

Restates, for third-order tensors (L = 3):
* ch.3 Thm "JfT_Jf" and the Pi matrices built from factor Grams, and
  Thm "Hv" (structured J^T J v product);
* ch.4 "dGN": residual, gradient theorem (W Pi - T_(l) KR), Alg. "Conjugate
  gradient - dGN" with the random iteration cap, updates (step always taken,
  norm balancing), gain ratio, the Tensor Fox damping rule (g < 0.25: mu*3;
  g > 0.75: mu/3) and the seven stopping conditions in their stated order;
* ch.4 "Regularization and preconditioning": the gammas of D and the Jacobi
  preconditioner M = diag(J^T J) + mu D;
* App. A: preconditioned CG on M^{-1/2} A M^{-1/2}.

Vectors in the parameter space are kept in block form, a list of L matrices
V^(l) of shape R~_l x R (vec(V^(l)) stacks columns, ch.3 definition of w).

Readings (listed in the design doc): gradient sign grad F = J^T f = W Pi - MTTKRP;
CG product uses mu*D; the CG output is mapped back x = M^{-1/2} x_hat;
the gain ratio uses squared norms in both terms with the undamped linear
model; the step-size test uses ||x||; the windowed tests run when
k % c == 0 and k > 2c on non-overlapping windows of c errors; the CG cap
bounds use exact integer ceilings; CG and the gain ratio have breakdown
guards (see ``pcg`` and ``gain_ratio``).
"""
from dataclasses import dataclass, field
import math

import numpy as np

from .multilinear import unfold, khatri_rao_except, cpd_full

STOP_NONE = 0
STOP_REL_ERR = 1
STOP_STEP = 2
STOP_IMPROVEMENT = 3
STOP_GRAD = 4
STOP_AVG_ERR = 5
STOP_AVG_IMPR = 6
STOP_DIVERGED = 7
STOP_MAXITER = 8


# ---------------------------------------------------------------------------
# Grams and Pi matrices (ch.3, "Dealing with the Hessian")
# ---------------------------------------------------------------------------
def grams(Ws):
    """pi^(l) = W^(l)T W^(l), R x R."""
    return [W.T @ W for W in Ws]


def pi_pair(pis, a, b):
    """Pi^(a,b): Hadamard product of pi^(l) over l not in {a, b}."""
    out = np.ones_like(pis[0])
    for l, p in enumerate(pis):
        if l != a and l != b:
            out = out * p
    return out


def pi_own(pis, a):
    """Pi^(a): Hadamard product of pi^(l) over l != a."""
    out = np.ones_like(pis[0])
    for l, p in enumerate(pis):
        if l != a:
            out = out * p
    return out


# ---------------------------------------------------------------------------
# Residual, MTTKRP and gradient (ch.4 "Computing the residual / gradient")
# ---------------------------------------------------------------------------
def residual(S, Ws):
    """f = S - sum_r w_r^(1) (x) w_r^(2) (x) w_r^(3)."""
    return np.asarray(S, dtype=np.float64) - cpd_full(Ws)


def mttkrp(S, Ws, l):
    """S_(l) (W^(L) (.) ... (.) W^(l+1) (.) W^(l-1) (.) ... (.) W^(1)), R~_l x R."""
    return unfold(S, l) @ khatri_rao_except(Ws, l)


def gradient(S, Ws, pis=None):
    """dF/dW^(l) = W^(l) Pi^(l) - S_(l) KR^(l) (gradient theorem of ch.4); grad F = J^T f."""
    if pis is None:
        pis = grams(Ws)
    return [Ws[l] @ pi_own(pis, l) - mttkrp(S, Ws, l) for l in range(len(Ws))]


# ---------------------------------------------------------------------------
# Regularisation D and preconditioner M (ch.4 "Diagonal regularization")
# ---------------------------------------------------------------------------
def column_norms(Ws):
    return [np.sqrt(np.sum(W * W, axis=0)) for W in Ws]


def regularization(Ws):
    """gamma_X^(r) = ||Y_r|| ||Z_r|| m, gamma_Y^(r) = ||X_r|| ||Z_r|| m, gamma_Z^(r) = ||X_r|| ||Y_r|| m,
    m = max(max_r ||Y_r|| ||Z_r||, max_r ||X_r|| ||Z_r||, max_r ||X_r|| ||Y_r||).

    D is diagonal and constant over the rows of each column block, so it is
    returned as L vectors of length R.
    """
    assert len(Ws) == 3, "the thesis defines D for third-order tensors"
    nX, nY, nZ = column_norms(Ws)
    m = max(np.max(nY * nZ), np.max(nX * nZ), np.max(nX * nY))
    return [nY * nZ * m, nX * nZ * m, nX * nY * m]


def preconditioner(pis, gammas, mu):
    """M = diag(J^T J) + mu D; diag(J^T J) in block (l, r) is Pi^(l)_rr = prod_{l' != l} ||w_r^(l')||^2."""
    return [np.diag(pi_own(pis, l)).copy() + mu * gammas[l] for l in range(len(pis))]


# ---------------------------------------------------------------------------
# Structured J^T J v (ch.3 Thm "Hv")
# ---------------------------------------------------------------------------
def jtj_v(Ws, pis, Vs):
    """Block l' of J^T J v = V^(l') Pi^(l') + sum_{l'' != l'} W^(l') (Pi^(l',l'') * (V^(l'')T W^(l'')))."""
    L = len(Ws)
    out = []
    for a in range(L):
        blk = Vs[a] @ pi_own(pis, a)
        for b in range(L):
            if b != a:
                blk = blk + Ws[a] @ (pi_pair(pis, a, b) * (Vs[b].T @ Ws[b]))
        out.append(blk)
    return out


def dot(As, Bs):
    return float(sum(np.sum(A * B) for A, B in zip(As, Bs)))


def pcg(Ws, pis, gammas, mu, rhs, M, cap, cg_tol):
    """Alg. "Conjugate gradient - dGN" on B = M^{-1/2}(J^T J + mu D)M^{-1/2}, right-hand side
    M^{-1/2} rhs, with rhs = A^T b = -grad F.

    The product B p is formed in three steps (scale, J^T J + mu D, scale).
    Returns (x, iterations, final ||r||^2) with x = M^{-1/2} x_hat mapped back
    to the unpreconditioned variables.  Breakdown guard: the loop ends early
    when ||r||^2 = 0 or <p, Bp> <= 0.
    """
    msq = [1.0 / np.sqrt(m) for m in M]          # per (l, r) scalars
    x = [np.zeros_like(W) for W in Ws]
    r = [b * s for b, s in zip(rhs, msq)]
    p = [v.copy() for v in r]
    rr = dot(r, r)
    its = 0
    for _ in range(cap):
        if rr == 0.0:
            break
        z = [v * s for v, s in zip(p, msq)]
        jz = jtj_v(Ws, pis, z)
        z = [(j + mu * g * v) * s for j, g, v, s in zip(jz, gammas, z, msq)]
        pz = dot(p, z)
        if not pz > 0.0:
            break
        alpha = rr / pz
        x = [xv + alpha * pv for xv, pv in zip(x, p)]
        r = [rv - alpha * zv for rv, zv in zip(r, z)]
        eps = dot(r, r)
        beta = eps / rr
        p = [rv + beta * pv for rv, pv in zip(r, p)]
        rr = eps
        its += 1
        if eps < cg_tol:
            break
    return [xv * s for xv, s in zip(x, msq)], its, rr


def block_factors(pis, gammas, mu):
    """Block-Jacobi preconditioner (the block-diagonal preconditioner of ch.4 "Tensor Fox vs. other
    implementations" and the Conclusions): the diagonal blocks of J^T J + mu D.  Block l acts on
    V^(l) as V^(l) K_l with K_l = Pi^(l) + mu diag(gamma_l) (ch.3 block structure of J^T J), so it is
    K_l (x) I in vec form.  Returns the inverses C_l^{-1} of the Cholesky factors K_l = C_l C_l^T."""
    out = []
    for l in range(len(pis)):
        K = pi_own(pis, l) + mu * np.diag(gammas[l])
        C = np.linalg.cholesky(K)
        out.append(np.linalg.inv(C))
    return out


def pcg_block(Ws, pis, gammas, mu, rhs, Cinv, cap, cg_tol):
    """The CG of ``pcg`` with the block-Jacobi split L = C (x) I: CG on
    L^{-1} (J^T J + mu D) L^{-T} x_hat = L^{-1} rhs, x = L^{-T} x_hat.  In block form
    L^{-1} V = V C^{-T} and L^{-T} V = V C^{-1}; same loop, same breakdown guards."""
    lt = lambda Vs: [V @ Ci for V, Ci in zip(Vs, Cinv)]           # L^{-T}
    li = lambda Vs: [V @ Ci.T for V, Ci in zip(Vs, Cinv)]         # L^{-1}
    x = [np.zeros_like(W) for W in Ws]
    r = li(rhs)
    p = [v.copy() for v in r]
    rr = dot(r, r)
    its = 0
    for _ in range(cap):
        if rr == 0.0:
            break
        u = lt(p)
        ju = jtj_v(Ws, pis, u)
        z = li([j + mu * g * v for j, g, v in zip(ju, gammas, u)])
        pz = dot(p, z)
        if not pz > 0.0:
            break
        alpha = rr / pz
        x = [xv + alpha * pv for xv, pv in zip(x, p)]
        r = [rv - alpha * zv for rv, zv in zip(r, z)]
        eps = dot(r, r)
        beta = eps / rr
        p = [rv + beta * pv for rv, pv in zip(r, p)]
        rr = eps
        its += 1
        if eps < cg_tol:
            break
    return lt(x), its, rr


def dogleg(h_gn, g, jg2, delta):
    """Dogleg step inside the trust radius delta (Madsen, Nielsen & Tingleff, the method ch.4
    "Conditioning" applies after a draw-back): the Gauss-Newton step h_gn if it fits; else the
    steepest-descent step -g cut at delta when the Cauchy point a = -(|g|^2/|Jg|^2) g lies outside;
    else a + beta (h_gn - a) with beta >= 0 putting the step on the radius."""
    ngn = math.sqrt(dot(h_gn, h_gn))
    if ngn <= delta:
        return h_gn
    gg = dot(g, g)
    alpha = gg / jg2
    a = [-alpha * gv for gv in g]
    na = alpha * math.sqrt(gg)
    if na >= delta:
        return [-(delta / math.sqrt(gg)) * gv for gv in g]
    d = [hv - av for hv, av in zip(h_gn, a)]
    c = dot(a, d)
    dd = dot(d, d)
    beta = (-c + math.sqrt(c * c + dd * (delta * delta - na * na))) / dd
    return [av + beta * dv for av, dv in zip(a, d)]


# ---------------------------------------------------------------------------
# Updates (ch.4 "Updates")
# ---------------------------------------------------------------------------
def norm_balance(Ws):
    """Rescale each rank-one term so ||w_r^(1)|| = ... = ||w_r^(L)|| without changing the tensor:
    w_r^(l) <- (alpha_r / n_r^(l)) w_r^(l), alpha_r = (prod_l n_r^(l))^{1/L}.  Terms with a
    zero column are left unchanged."""
    Ws = [np.array(W, dtype=np.float64, copy=True) for W in Ws]
    L = len(Ws)
    norms = column_norms(Ws)
    for r in range(Ws[0].shape[1]):
        n = [norms[l][r] for l in range(L)]
        if min(n) == 0.0:
            continue
        alpha = float(np.prod(n)) ** (1.0 / L)
        for l in range(L):
            Ws[l][:, r] *= alpha / n[l]
    return Ws


def gain_ratio(f2_old, f2_new, f2_pred):
    """g = (||f_k||^2 - ||f_{k+1}||^2) / (||f_k||^2 - ||f_k + J x||^2).  Guard: a non-positive
    predicted reduction gives g = 0."""
    den = f2_old - f2_pred
    if not den > 0.0:
        return 0.0
    return (f2_old - f2_new) / den


def damping_update(mu, g):
    """Tensor Fox rule: g < 0.25 -> 3 mu; g > 0.75 -> mu / 3."""
    if g < 0.25:
        return 3.0 * mu
    if g > 0.75:
        return mu / 3.0
    return mu


# ---------------------------------------------------------------------------
# CG cap schedule (ch.4 "Conjugate gradient")
# ---------------------------------------------------------------------------
def ceil_rational_power(k, p, q):
    """Exact ceil(k^(p/q)) for integers k >= 0: the smallest m >= 0 with m^q >= k^p."""
    target = k ** p
    m = int(math.floor(float(k) ** (p / q)))
    m = max(m - 2, 0)
    while m ** q < target:
        m += 1
    return m


def cg_cap_bounds(k):
    """Inclusive interval [1 + ceil(k^0.4), 2 + ceil(k^0.9)] for dGN iteration k (1-based)."""
    return 1 + ceil_rational_power(k, 2, 5), 2 + ceil_rational_power(k, 9, 10)


def cg_cap(k, u):
    """Uniform integer in the cap interval from one uniform draw u in [0, 1)."""
    lo, hi = cg_cap_bounds(k)
    n = hi - lo + 1
    return lo + min(int(math.floor(u * n)), n - 1)


# ---------------------------------------------------------------------------
# One dGN iteration and the stopping conditions
# ---------------------------------------------------------------------------
@dataclass
class Params:
    maxiter: int = 200
    tol: float = 1e-6
    mlsvd_tol: float = 1e-6
    init_damp: float = 1.0
    cg_tol: float = None     # None -> tol
    cg_fixed: int = 0        # > 0: fixed CG cap instead of the random schedule
    block_precond: bool = False   # block-Jacobi preconditioner instead of the diagonal one
    drawback: bool = False   # draw back and take a dogleg step when the error jumps 100-fold

    def cg_tol_value(self):
        return self.tol if self.cg_tol is None else self.cg_tol


def window_c(maxiter):
    """c = 1 + ceil(maxiter / 10) of stopping conditions 5 and 6."""
    return 1 + (maxiter + 9) // 10


@dataclass
class State:
    Ws: list
    mu: float
    k: int                      # iterations done
    f2: float                   # ||S - [[W]]||^2 at the current W
    s_norm: float               # ||S||
    div_ref: float              # max(1, ||T||^2) for the divergence test
    errs: list = field(default_factory=list)   # errs[j] = relative error after iteration j (errs[0]: initial)
    stop: int = STOP_NONE


def init_state(S, Ws0, params, tnorm2=None):
    """Norm-balance the initial point, take mu0 = tau * mean|S| (ch.4 "Main parameters")."""
    S = np.asarray(S, dtype=np.float64)
    Ws = norm_balance(Ws0)
    f = residual(S, Ws)
    f2 = float(np.sum(f * f))
    s_norm = float(np.sqrt(np.sum(S * S)))
    if tnorm2 is None:
        tnorm2 = s_norm ** 2
    mu = params.init_damp * float(np.mean(np.abs(S)))
    return State(Ws=Ws, mu=mu, k=0, f2=f2, s_norm=s_norm, div_ref=max(1.0, tnorm2),
                 errs=[math.sqrt(f2) / s_norm])


def step_direction(S, Ws, mu, params, cap):
    """Gradient, Grams and the preconditioned CG step at Ws (the diagonal or block-Jacobi
    preconditioner): returns (grad, pis, x, CG iterations, final ||r||^2)."""
    pis = grams(Ws)
    grad = gradient(S, Ws, pis)
    gammas = regularization(Ws)
    rhs = [-g for g in grad]
    if params.block_precond:
        x, its, cg_res = pcg_block(Ws, pis, gammas, mu, rhs, block_factors(pis, gammas, mu), cap,
                                   params.cg_tol_value())
    else:
        M = preconditioner(pis, gammas, mu)
        x, its, cg_res = pcg(Ws, pis, gammas, mu, rhs, M, cap, params.cg_tol_value())
    return grad, pis, x, its, cg_res


def dgn_step(S, st, params, cap):
    """One iteration of the Tensor Fox dGN; returns (new_state, info dict).

    With params.drawback, an iteration whose error exceeds 100 times the previous one (the
    divergence test of ch.4 "Conditioning") is redone from the drawn-back point N(w_k) - x (the
    balanced bad point shifted back by the step): a new CG step there, cut by the dogleg method to
    the trust radius |x| / 2 (reading: half the failed step), then the usual update."""
    S = np.asarray(S, dtype=np.float64)
    Ws = st.Ws
    k = st.k + 1
    grad, pis, x, its, cg_res = step_direction(S, Ws, st.mu, params, cap)
    jx = jtj_v(Ws, pis, x)
    f2_pred = st.f2 + 2.0 * dot(grad, x) + dot(x, jx)
    Wn = norm_balance([W + dx for W, dx in zip(Ws, x)])
    fn = residual(S, Wn)
    f2_new = float(np.sum(fn * fn))
    err = math.sqrt(f2_new) / st.s_norm
    f2_base = st.f2
    drew_back = False
    if params.drawback and err > 100.0 * st.errs[-1]:
        drew_back = True
        Wd = [W - dx for W, dx in zip(Wn, x)]
        fd = residual(S, Wd)
        f2_base = float(np.sum(fd * fd))
        delta = 0.5 * math.sqrt(dot(x, x))
        grad, pis, h_gn, its, cg_res = step_direction(S, Wd, st.mu, params, cap)
        jg2 = dot(grad, jtj_v(Wd, pis, grad))
        x = dogleg(h_gn, grad, jg2, delta)
        jx = jtj_v(Wd, pis, x)
        f2_pred = f2_base + 2.0 * dot(grad, x) + dot(x, jx)
        Wn = norm_balance([W + dx for W, dx in zip(Wd, x)])
        fn = residual(S, Wn)
        f2_new = float(np.sum(fn * fn))
        err = math.sqrt(f2_new) / st.s_norm
    g = gain_ratio(f2_base, f2_new, f2_pred)
    mu = damping_update(st.mu, g)
    step = math.sqrt(dot(x, x))
    grad_inf = max(float(np.max(np.abs(gv))) for gv in grad)
    errs = st.errs + [err]
    stop = stop_test(errs, k, step, grad_inf, params, st.div_ref)
    new = State(Ws=Wn, mu=mu, k=k, f2=f2_new, s_norm=st.s_norm, div_ref=st.div_ref,
                errs=errs, stop=stop)
    info = dict(k=k, cg_iters=its, cg_resid=cg_res, rel_err=err, step_norm=step,
                grad_inf=grad_inf, gain=g, mu=mu, stop=stop, f2_pred=f2_pred, drew_back=drew_back)
    return new, info


def stop_test(errs, k, step, grad_inf, params, div_ref):
    """Stopping conditions 1-7 in the thesis's order, then maxiter."""
    tol = params.tol
    err = errs[k]
    if err < tol:
        return STOP_REL_ERR
    if step < tol:
        return STOP_STEP
    if abs(errs[k - 1] - err) < tol:
        return STOP_IMPROVEMENT
    if grad_inf < tol:
        return STOP_GRAD
    c = window_c(params.maxiter)
    if k % c == 0 and k > 2 * c:
        old = errs[k - 2 * c + 1: k - c + 1]
        new = errs[k - c + 1: k + 1]
        avg_old = sum(old) / c
        avg_new = sum(new) / c
        if avg_old - avg_new < tol:
            return STOP_AVG_ERR
        impr = sum(abs(errs[j - 1] - errs[j]) for j in range(k - c + 1, k + 1)) / c
        if impr < 1e-3 * avg_new:
            return STOP_AVG_IMPR
    if err > div_ref / (1e-16 + tol):
        return STOP_DIVERGED
    if k >= params.maxiter:
        return STOP_MAXITER
    return STOP_NONE


def run_dgn(S, Ws0, params, cg_uniforms=None, tnorm2=None, log=None):
    """dGN loop from an initial point until a stopping condition fires."""
    st = init_state(S, Ws0, params, tnorm2)
    infos = []
    while st.stop == STOP_NONE:
        k = st.k + 1
        if params.cg_fixed > 0:
            cap = params.cg_fixed
        else:
            cap = cg_cap(k, cg_uniforms[k - 1])
        st, info = dgn_step(S, st, params, cap)
        infos.append(info)
        if log is not None:
            log(info)
    return st, infos
