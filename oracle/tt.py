"""Tensor-train route to the CPD of tensors of order L > 3 (oracle; test infrastructure only).

Restates ch.4 "Tensor train and the CPD": Alg. TT-SVD (successive SVDs of reshaped unfoldings,
here with every TT-rank truncated to R), Thm CPD_to_TT (a rank-R CPD gives a TT whose inner cores
are (I, W^(l), I) . I) and Alg. CPD-TTD: a rank-R CPD of the second core, then for l = 3..L-1 a
"Bi-CPD" of core l whose first factor is fixed to the inverse transpose of the previous core's
third factor, and the outer factors from the first and last cores.

Readings (listed in the design doc):
* reshapes are C-order (row-major), consistent with the C-order unfoldings used here: core l is
  the r_{l-1} x I_l x r_l tensor whose (a, i) rows are the left singular vectors;
* singular-vector signs as in the MLSVD (largest-|.| entry positive);
* with the TT link index as the row index of M^(l), W^(1) = G^(1) M^(1) and
  W^(L) = G^(L)T M^(L-1) (the thesis writes the transposes for its own index order);
* Bi-CPD: the damped Gauss-Newton of oracle.dgn with the first factor's block of the step held at
  zero (its gradient block and its rows of J^T J v removed, so CG runs on the reduced normal
  equations) and norm balancing over the two free modes only;
* the CPD of the second core is oracle.cpd.solve (compression, dGN, uncompression) and its three
  unnormalised factors are used as (M^(1), W^(2), M^(2)).
"""
import numpy as np

from . import cpd as _cpd
from . import dgn as _dgn
from .mlsvd import canonical_signs


def tt_svd(T, R):
    """Alg. TT-SVD with TT-ranks min(R, rank): cores G^(1) (1 x I_1 x r_1), ..., G^(L) (r_{L-1} x I_L x 1)."""
    T = np.asarray(T, dtype=np.float64)
    dims = T.shape
    L = len(dims)
    cores = []
    r_prev = 1
    M = T.reshape(dims[0], -1)
    for l in range(L - 1):
        M = M.reshape(r_prev * dims[l], -1)
        U, s, _ = np.linalg.svd(M, full_matrices=False)
        r = min(R, len(s))
        U = canonical_signs(U[:, :r])
        cores.append(U.reshape(r_prev, dims[l], r))
        M = U.T @ M
        r_prev = r
    cores.append(M.reshape(r_prev, dims[-1], 1))
    return cores


def tt_full(cores):
    """T[i_1..i_L] = G^(1)(i_1) G^(2)(i_2) ... G^(L)(i_L), the contraction chain of the TT."""
    out = cores[0].reshape(cores[0].shape[1], cores[0].shape[2])      # I_1 x r_1
    shape = [cores[0].shape[1]]
    for G in cores[1:]:
        r0, I, r1 = G.shape
        out = out @ G.reshape(r0, I * r1)                              # (prod I) x (I r1)
        shape.append(I)
        out = out.reshape(-1, r1)
    return out.reshape(shape)


def cpd_train_cores(Ws):
    """Thm CPD_to_TT: G^(1) = W^(1), G^(l) = sum_r e_r (x) w_r^(l) (x) e_r, G^(L) = W^(L)T."""
    R = Ws[0].shape[1]
    cores = [Ws[0].reshape(1, Ws[0].shape[0], R)]
    for W in Ws[1:-1]:
        G = np.zeros((R, W.shape[0], R))
        for r in range(R):
            G[r, :, r] = W[:, r]
        cores.append(G)
    cores.append(Ws[-1].T.reshape(R, Ws[-1].shape[0], 1))
    return cores


def cpd_full_L(Ws):
    """sum_r w_r^(1) (x) ... (x) w_r^(L) for any order."""
    R = Ws[0].shape[1]
    out = Ws[0]
    for W in Ws[1:]:
        out = (out[:, None, :] * W[None, :, :]).reshape(-1, R)
    return out.sum(axis=1).reshape([W.shape[0] for W in Ws])


def _balance_free(Ws):
    """Norm balancing over modes 2 and 3 only (mode 1 is fixed): alpha_r = sqrt(n_r^(2) n_r^(3))."""
    Ws = [np.array(W, dtype=np.float64, copy=True) for W in Ws]
    n1 = np.sqrt(np.sum(Ws[1] ** 2, axis=0))
    n2 = np.sqrt(np.sum(Ws[2] ** 2, axis=0))
    for r in range(Ws[0].shape[1]):
        if n1[r] == 0.0 or n2[r] == 0.0:
            continue
        a = np.sqrt(n1[r] * n2[r])
        Ws[1][:, r] *= a / n1[r]
        Ws[2][:, r] *= a / n2[r]
    return Ws


def _pcg_fixed(Ws, pis, gammas, mu, rhs, M, cap, cg_tol):
    """oracle.dgn.pcg on the normal equations with block 1 removed: its right-hand side and its
    rows of the operator are zero, so every CG vector keeps a zero first block."""
    msq = [1.0 / np.sqrt(m) for m in M]
    msq[0] = np.zeros_like(msq[0])
    x = [np.zeros_like(W) for W in Ws]
    r = [b * s for b, s in zip(rhs, msq)]
    p = [v.copy() for v in r]
    rr = _dgn.dot(r, r)
    its = 0
    for _ in range(cap):
        if rr == 0.0:
            break
        z = [v * s for v, s in zip(p, msq)]
        jz = _dgn.jtj_v(Ws, pis, z)
        z = [(j + mu * g * v) * s for j, g, v, s in zip(jz, gammas, z, msq)]
        pz = _dgn.dot(p, z)
        if not pz > 0.0:
            break
        alpha = rr / pz
        x = [xv + alpha * pv for xv, pv in zip(x, p)]
        r = [rv - alpha * zv for rv, zv in zip(r, z)]
        eps = _dgn.dot(r, r)
        beta = eps / rr
        p = [rv + beta * pv for rv, pv in zip(r, p)]
        rr = eps
        its += 1
        if eps < cg_tol:
            break
    return [xv * s for xv, s in zip(x, msq)], its, rr


def bi_cpd_step(S, st, params, cap):
    """One dGN iteration with the first factor fixed (oracle.dgn.dgn_step restricted to modes 2, 3)."""
    S = np.asarray(S, dtype=np.float64)
    Ws = st.Ws
    k = st.k + 1
    pis = _dgn.grams(Ws)
    grad = _dgn.gradient(S, Ws, pis)
    grad[0] = np.zeros_like(grad[0])
    gammas = _dgn.regularization(Ws)
    M = _dgn.preconditioner(pis, gammas, st.mu)
    x, its, cg_res = _pcg_fixed(Ws, pis, gammas, st.mu, [-g for g in grad], M, cap, params.cg_tol_value())
    jx = _dgn.jtj_v(Ws, pis, x)
    f2_pred = st.f2 + 2.0 * _dgn.dot(grad, x) + _dgn.dot(x, jx)
    Wn = _balance_free([W + dx for W, dx in zip(Ws, x)])
    fn = _dgn.residual(S, Wn)
    f2_new = float(np.sum(fn * fn))
    err = np.sqrt(f2_new) / st.s_norm
    g = _dgn.gain_ratio(st.f2, f2_new, f2_pred)
    mu = _dgn.damping_update(st.mu, g)
    step = np.sqrt(_dgn.dot(x, x))
    grad_inf = max(float(np.max(np.abs(gv))) for gv in grad[1:])
    errs = st.errs + [err]
    stop = _dgn.stop_test(errs, k, step, grad_inf, params, st.div_ref)
    new = _dgn.State(Ws=Wn, mu=mu, k=k, f2=f2_new, s_norm=st.s_norm, div_ref=st.div_ref, errs=errs, stop=stop)
    return new, dict(k=k, cg_iters=its, rel_err=err, step_norm=step, grad_inf=grad_inf, gain=g, mu=mu, stop=stop)


def bi_cpd(F, S, W0, params, cg_uniforms):
    """Rank-R CPD (F, W2, W3) of the third-order S with the first factor fixed to F (Bi-CPD), from
    the start (F, W0[0], W0[1]); mu0 = tau mean|S| and the stopping rules of the dGN."""
    S = np.asarray(S, dtype=np.float64)
    Ws = _balance_free([np.asarray(F, dtype=np.float64), W0[0], W0[1]])
    f = _dgn.residual(S, Ws)
    f2 = float(np.sum(f * f))
    s_norm = float(np.sqrt(np.sum(S * S)))
    st = _dgn.State(Ws=Ws, mu=params.init_damp * float(np.mean(np.abs(S))), k=0, f2=f2, s_norm=s_norm,
                    div_ref=max(1.0, s_norm ** 2), errs=[np.sqrt(f2) / s_norm])
    infos = []
    while st.stop == _dgn.STOP_NONE:
        k = st.k + 1
        cap = params.cg_fixed if params.cg_fixed > 0 else _dgn.cg_cap(k, cg_uniforms[k - 1])
        st, info = bi_cpd_step(S, st, params, cap)
        infos.append(info)
    return st, infos


def cpd_ttd(T, R, params=None, W0=None, cg_uniforms=None):
    """Alg. CPD-TTD.  W0: initial factors for each third-order CPD, in order: for the second core
    the three core-dims x R matrices of oracle.cpd.solve, then for each core l = 3..L-1 the two
    free factors (I_l x R, R x R).  Returns the L factors (unnormalised), the cores and a log."""
    if params is None:
        params = _dgn.Params()
    T = np.asarray(T, dtype=np.float64)
    L = T.ndim
    assert L >= 4, "CPD-TTD is the route for orders above three"
    cores = tt_svd(T, R)
    assert all(G.shape[0] in (1, R) and G.shape[2] in (1, R) for G in cores), "TT-ranks below R"
    res2 = _cpd.solve(cores[1], R, params, W0=W0[0], cg_uniforms=cg_uniforms)
    M1, W2, M_prev = res2["W_unnormalized"]
    Ws = [None, W2]
    logs = [dict(iters=res2["iters"], stop=res2["stop"], rel_err=res2["rel_err_full"])]
    for l in range(2, L - 1):
        F = np.linalg.inv(M_prev).T
        st, infos = bi_cpd(F, cores[l], W0[l - 1], params, cg_uniforms)
        Ws.append(st.Ws[1])
        M_prev = st.Ws[2]
        logs.append(dict(iters=st.k, stop=st.stop, rel_err=st.errs[-1]))
    G1 = cores[0].reshape(cores[0].shape[1], R)
    GL = cores[-1].reshape(R, cores[-1].shape[1])
    Ws[0] = G1 @ M1
    Ws.append(GL.T @ M_prev)
    return Ws, cores, logs
