"""End-to-end Tensor Fox pipeline: Compress -> Initialize -> dGN -> Uncompress (oracle; test
infrastructure only).

Restates the flow chart of ch.4 "Tensor Fox" and its output format: factor
matrices with unit columns and a diagonal Lambda such that
T ~ sum_r lambda_r w_r^(1) (x) ... (x) w_r^(L).

Output reading (listed in the design doc): lambda_r >= 0, the columns of modes
1..L-1 are flipped so their largest-|.| entry is positive with the sign moved
into the last mode, and terms are sorted by decreasing lambda.
"""
import numpy as np

from . import dgn as _dgn
from .mlsvd import compress, compress_st, smart_init
from .multilinear import cpd_full, frob


def uncompress(Us, Ws):
    """W~^(l) = U^(l) W^(l) (ch.4 "Uncompression")."""
    return [U @ W for U, W in zip(Us, Ws)]


def normalize_output(Ws):
    """Unit columns plus lambda, with the sign and ordering reading described above."""
    Ws = [np.array(W, dtype=np.float64, copy=True) for W in Ws]
    L = len(Ws)
    R = Ws[0].shape[1]
    lam = np.ones(R)
    for l in range(L):
        n = np.sqrt(np.sum(Ws[l] ** 2, axis=0))
        lam *= n
        nz = n > 0
        Ws[l][:, nz] /= n[nz]
    for r in range(R):
        for l in range(L - 1):
            i = int(np.argmax(np.abs(Ws[l][:, r])))
            if Ws[l][i, r] < 0:
                Ws[l][:, r] = -Ws[l][:, r]
                Ws[L - 1][:, r] = -Ws[L - 1][:, r]
    order = np.argsort(-lam, kind="stable")
    return [W[:, order] for W in Ws], lam[order]


def refine(T, Wt, params, mu, k0, n_iters, cg_uniforms=None, tnorm2=None):
    """Refinement in the original space (the option ch.4 describes for Tensorlab and Tensor Fox:
    the compressed solution, uncompressed, starts iterations on T itself).  Reading: n_iters further
    iterations of the same dGN (oracle.dgn.dgn_step with T in place of the core), continuing the
    damping parameter mu and the iteration counter of the compressed run, so iteration j takes the
    CG cap of iteration k0 + j of the schedule (a fixed cap if params.cg_fixed); the stopping rules
    run with maxiter = n_iters and errors relative to ||T||.  Since W~^(l)T W~^(l) = W^(l)T W^(l)
    for orthonormal U^(l), the Grams, Pi, D and the preconditioner continue unchanged."""
    T = np.asarray(T, dtype=np.float64)
    p = _dgn.Params(maxiter=n_iters, tol=params.tol, mlsvd_tol=params.mlsvd_tol, init_damp=params.init_damp,
                    cg_tol=params.cg_tol, cg_fixed=params.cg_fixed)
    Ws = _dgn.norm_balance(Wt)
    f = _dgn.residual(T, Ws)
    f2 = float(np.sum(f * f))
    t_norm = float(np.sqrt(np.sum(T * T)))
    if tnorm2 is None:
        tnorm2 = t_norm ** 2
    st = _dgn.State(Ws=Ws, mu=mu, k=0, f2=f2, s_norm=t_norm, div_ref=max(1.0, tnorm2),
                    errs=[np.sqrt(f2) / t_norm])
    infos = []
    while st.stop == _dgn.STOP_NONE:
        k = k0 + st.k + 1
        if p.cg_fixed > 0:
            cap = p.cg_fixed
        else:
            cap = _dgn.cg_cap(k, cg_uniforms[min(k, len(cg_uniforms)) - 1])
        st, info = _dgn.dgn_step(T, st, p, cap)
        infos.append(info)
    return st, infos


def solve(T, R, params=None, init="random", W0=None, cg_uniforms=None, core_dims=None, log=None, st_mlsvd=False,
          refine_iters=0):
    """Full CPD of a third-order tensor.

    ``init``: "random" or "given" (W0 must hold R~_l x R matrices, drawn by
    the caller so that the GPU path can be fed the same numbers) or "mlsvd"
    (the MLSVD-energy initialisation).  ``cg_uniforms``: one uniform draw in
    [0, 1) per dGN iteration, mapped to the random CG cap.  ``st_mlsvd``: compress with the
    sequentially truncated MLSVD (ch.2 Alg. ST-MLSVD) instead of the classic one.
    """
    if params is None:
        params = _dgn.Params()
    T = np.asarray(T, dtype=np.float64)
    comp = compress_st if st_mlsvd else compress
    Us, sigmas, S = comp(T, R, params.mlsvd_tol, core_dims=core_dims)
    core = S.shape
    if init == "mlsvd":
        Ws0 = smart_init(S, R, extra=W0)
    else:
        if W0 is None:
            raise ValueError("random/given init needs W0 of shape core_dims[l] x R")
        Ws0 = [np.asarray(W, dtype=np.float64) for W in W0]
        for l in range(3):
            assert Ws0[l].shape == (core[l], R)
    tn2 = float(np.sum(T * T))
    st, infos = _dgn.run_dgn(S, Ws0, params, cg_uniforms=cg_uniforms, tnorm2=tn2, log=log)
    Wt = uncompress(Us, st.Ws)
    ref_st, ref_infos = None, []
    if refine_iters > 0:
        ref_st, ref_infos = refine(T, Wt, params, st.mu, st.k, refine_iters, cg_uniforms, tn2)
        Wt = ref_st.Ws
    Wn, lam = normalize_output(Wt)
    that = cpd_full(Wt)
    return dict(U=Us, sigma=sigmas, S=S, core_dims=core, W_core=st.Ws, W=Wn, lam=lam,
                W_unnormalized=Wt, iters=st.k, stop=st.stop, errs=st.errs, infos=infos,
                rel_err_core=st.errs[-1], rel_err_full=frob(T - that) / frob(T),
                mu=st.mu, refine_iters=len(ref_infos), refine_infos=ref_infos,
                refine_stop=ref_st.stop if ref_st is not None else 0)


def time_to_tol_iter(errs, tol):
    """First iteration k (1-based) whose core relative error is below tol, or None."""
    for k, e in enumerate(errs[1:], start=1):
        if e < tol:
            return k
    return None
