"""GPU parity of the robustness variants of the dGN (block-Jacobi preconditioner, draw-back with a
dogleg step) against the FP64 oracle, through the C ABI.

Tolerances follow the dGN step tests: with a fixed CG cap and a vanishing CG tolerance both sides
run the same number of CG iterations, and per-iteration quantities agree to relative 1e-8 (the
two sides differ only in summation order, amplified by the conditioning of the damped system).
"""
import dataclasses
import math

import numpy as np
import pytest
import torch

import synth
from oracle import cpd as ocpd
from oracle import dgn as odgn
from oracle import mlsvd as omlsvd
from oracle import multilinear as ml

pytestmark = pytest.mark.gpu

DEV = "cuda"
RTOL = 1e-8


def cp():
    import paper_2110_05997_amd as cp_
    return cp_


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=DEV, dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().double().numpy()


def log(*a):
    print(*a, flush=True)


def same_step(ig, io, rtol=RTOL):
    assert ig["k"] == io["k"]
    assert ig["cg_iters"] == io["cg_iters"], (ig, io)
    assert ig["drew_back"] == int(io["drew_back"])
    for key in ("rel_err", "step_norm", "grad_inf", "mu"):
        assert abs(ig[key] - io[key]) <= rtol * max(abs(io[key]), 1e-300), (io["k"], key, ig[key], io[key])
    assert abs(ig["gain"] - io["gain"]) <= 1e-7 * max(1.0, abs(io["gain"])), (ig["gain"], io["gain"])
    assert ig["stop"] == io["stop"]


# (12, 9, 10) R = 6 runs with the core in LDS; (20, 20, 20) R = 20 leaves no room for the core next
# to the block factors (core read from global memory)
@pytest.mark.parametrize("dims,R,seed", [((12, 9, 10), 6, 1), ((20, 20, 20), 20, 2)])
def test_block_jacobi_steps_match_oracle(dims, R, seed):
    log("block-Jacobi steps", dims, R)
    rng = np.random.default_rng(seed)
    Fs = [rng.standard_normal((d, R)) for d in dims]
    S = ml.cpd_full(Fs) + 1e-3 * rng.standard_normal(dims)
    W0 = synth.init_factors(dims, R, seed)
    cap = 6
    p = cp().params(maxiter=50, cg_fixed=cap, cg_tol=1e-300, precond="block")
    state = cp().DgnState(dev(S), R, p, W0=[dev(w) for w in W0])
    po = odgn.Params(maxiter=50, cg_fixed=cap, cg_tol=1e-300, block_precond=True)
    st = odgn.init_state(S, W0, po)
    for _ in range(6):
        st, io = odgn.dgn_step(S, st, po, cap)
        ig = state.step()
        same_step(ig, io)
        if st.stop:
            break
    Wg = [host(w) for w in state.factors()]
    for l in range(3):
        assert np.max(np.abs(Wg[l] - st.Ws[l])) <= 1e-8 * np.max(np.abs(st.Ws[l]))


def test_block_jacobi_random_caps_match_oracle():
    """The thesis's random CG cap and CG tolerance: the same trajectory over the first steps."""
    dims, R, seed = (12, 11, 10), 5, 3
    log("block-Jacobi random caps", dims, R)
    rng = np.random.default_rng(seed)
    Fs = [rng.standard_normal((d, R)) for d in dims]
    S = ml.cpd_full(Fs) + 1e-3 * rng.standard_normal(dims)
    W0 = synth.init_factors(dims, R, seed)
    U = synth.cg_uniforms(50, seed)
    state = cp().DgnState(dev(S), R, cp().params(maxiter=50, cg_uniforms=U, precond="block"),
                          W0=[dev(w) for w in W0])
    po = odgn.Params(maxiter=50, block_precond=True)
    st = odgn.init_state(S, W0, po)
    for _ in range(5):
        st, io = odgn.dgn_step(S, st, po, odgn.cg_cap(st.k + 1, U[st.k]))
        same_step(state.step(), io)
        if st.stop:
            break


def reconstruct(res):
    W = [host(w) for w in res["W"]]
    lam = host(res["lam"])
    return ml.cpd_full([W[0] * lam[None, :], W[1], W[2]])


@pytest.mark.parametrize("precond,drawback", [("block", False), ("block", True), ("jacobi", True)])
def test_solve_with_robustness_options_matches_oracle(precond, drawback):
    """Whole solves on a planted 23 x 31 x 17 rank-4 tensor: the reconstruction matches the
    oracle's to relative 1e-6 and the stop and iteration count agree."""
    log("solve", precond, drawback)
    T, _, _ = synth.planted((23, 31, 17), 4, seed=5, noise_rel=1e-5)
    R, maxiter, seed = 4, 200, 5
    U = synth.cg_uniforms(maxiter, seed)
    _, _, So = omlsvd.compress(T, R)
    W0 = synth.init_factors(So.shape, R, seed)
    po = odgn.Params(maxiter=maxiter, block_precond=(precond == "block"), drawback=drawback)
    ref = ocpd.solve(T, R, po, W0=W0, cg_uniforms=U)
    p = cp().params(maxiter=maxiter, cg_uniforms=U, precond=precond, drawback=drawback)
    res = cp().solve(dev(T), R, p, W0=[dev(w) for w in W0])
    info = res["info"]
    log(info, "oracle", ref["iters"], ref["stop"], ref["rel_err_full"])
    That = reconstruct(res)
    Tref = ml.cpd_full(ref["W_unnormalized"])
    assert ml.frob(That - Tref) / ml.frob(Tref) < 1e-6
    assert info["stop_reason"] == ref["stop"]
    assert abs(info["iters"] - ref["iters"]) <= 1


def drawback_case(seed, damp, eps):
    """A state one step from a planted rank-4 tensor (relative error about 1e-3 after it), then
    factors replaced by the planted ones with column 2 of every factor moved onto column 1 plus
    eps-sized noise: the next iteration's error jumps more than 100-fold."""
    dims, R = (10, 9, 8), 4
    rng = np.random.default_rng(seed)
    Fs = [rng.standard_normal((d, R)) for d in dims]
    T0 = ml.cpd_full(Fs)
    S = T0 + 1e-6 * ml.frob(T0) / math.sqrt(np.prod(dims)) * rng.standard_normal(dims)
    W0 = [F + 1e-3 * rng.standard_normal(F.shape) for F in Fs]
    far = [F.copy() for F in Fs]
    for f in far:
        f[:, 1] = f[:, 0] + eps * rng.standard_normal(f.shape[0])
    return S, W0, far, R


# (seed, tau, eps) chosen so that the dogleg takes each of its three branches on the oracle with
# a wide margin (branch asserted below): the cut steepest-descent step, the point on the segment,
# the Gauss-Newton step itself
@pytest.mark.parametrize("seed,damp,eps,branch", [(0, 1.0, 1e-3, "sd"), (0, 1e-3, 0.1, "seg"),
                                                  (2, 1e-3, 0.1, "gn")])
@pytest.mark.parametrize("precond", ["jacobi", "block"])
def test_drawback_step_matches_oracle(seed, damp, eps, branch, precond):
    log("draw-back", seed, damp, eps, branch, precond)
    S, W0, far, R = drawback_case(seed, damp, eps)
    cap = 8
    blk = precond == "block"
    po = odgn.Params(maxiter=20, drawback=True, cg_fixed=cap, cg_tol=1e-300, init_damp=damp, block_precond=blk)
    p = cp().params(maxiter=20, drawback=True, cg_fixed=cap, cg_tol=1e-300, init_damp=damp, precond=precond)
    state = cp().DgnState(dev(S), R, p, W0=[dev(w) for w in W0])
    st = odgn.init_state(S, W0, po)
    st, io = odgn.dgn_step(S, st, po, cap)
    same_step(state.step(), io)
    assert not io["drew_back"]
    # replace the factors on both sides: the next step starts from `far` with the residual there
    f = odgn.residual(S, far)
    st = dataclasses.replace(st, Ws=[w.copy() for w in far], f2=float(np.sum(f * f)))
    state.set_factors([dev(w) for w in far])
    seen = {}
    orig = odgn.dogleg

    def traced(h, g, jg2, delta):
        ngn = math.sqrt(odgn.dot(h, h))
        gg = odgn.dot(g, g)
        na = gg / jg2 * math.sqrt(gg)
        seen["branch"] = "gn" if ngn <= delta else ("sd" if na >= delta else "seg")
        return orig(h, g, jg2, delta)

    odgn.dogleg = traced
    try:
        st, io = odgn.dgn_step(S, st, po, cap)
    finally:
        odgn.dogleg = orig
    assert io["drew_back"]
    if not blk:
        assert seen["branch"] == branch
    ig = state.step()
    log(ig, io)
    same_step(ig, io)
    # and the iteration goes on from there identically
    st, io = odgn.dgn_step(S, st, po, cap)
    same_step(state.step(), io)


def test_set_factors_recomputes_the_residual():
    """Without the draw-back option a replaced point is iterated from like any other: the step
    from `far` matches the oracle's step from the same state."""
    S, W0, far, R = drawback_case(1, 1.0, 0.1)
    p = cp().params(maxiter=20, cg_fixed=5, cg_tol=1e-300)
    po = odgn.Params(maxiter=20, cg_fixed=5, cg_tol=1e-300)
    state = cp().DgnState(dev(S), R, p, W0=[dev(w) for w in W0])
    st = odgn.init_state(S, W0, po)
    st, _ = odgn.dgn_step(S, st, po, 5)
    state.step()
    f = odgn.residual(S, far)
    st = dataclasses.replace(st, Ws=[w.copy() for w in far], f2=float(np.sum(f * f)))
    state.set_factors([dev(w) for w in far])
    st, io = odgn.dgn_step(S, st, po, 5)
    same_step(state.step(), io)


def test_options_outside_their_support_are_rejected():
    lib = cp()
    # a core whose working set does not fit in one workgroup's LDS
    rng = np.random.default_rng(0)
    S = dev(rng.standard_normal((50, 50, 50)))
    for kw in ({"precond": "block"}, {"drawback": True}):
        p = lib.params(maxiter=5, **kw)
        state = lib.DgnState(S, 50, p, W0=[dev(rng.standard_normal((50, 50))) for _ in range(3)])
        with pytest.raises(RuntimeError, match="LDS"):
            state.step()
    # the refinement, the batched solver and the tensor-train route run the plain dGN
    T = dev(rng.standard_normal((12, 11, 10)))
    with pytest.raises(RuntimeError, match="refinement"):
        lib.solve(T, 3, lib.params(maxiter=5, refine_iters=2, drawback=True))
    T4 = dev(rng.standard_normal((6, 5, 4, 3)))
    with pytest.raises(RuntimeError, match="tensor-train"):
        lib.solve_tt(T4, 2, lib.params(maxiter=5, precond="block"))
