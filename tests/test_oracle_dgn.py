"""Pins of the oracle's dGN / PCG pieces against brute force, textbook routines and the thesis's
theorems (CPU only)."""
import itertools
import math

import numpy as np
import pytest

from conftest import read_golden_table
import synth
from oracle import dgn, cpd, mlsvd
from oracle import multilinear as ml


def vec_blocks(Vs):
    """w = [vec(W1); vec(W2); vec(W3)] with column stacking (ch.3 definition of w)."""
    return np.concatenate([V.flatten(order="F") for V in Vs])


def unvec_blocks(v, shapes):
    out, o = [], 0
    for (I, R) in shapes:
        out.append(v[o:o + I * R].reshape((I, R), order="F"))
        o += I * R
    return out


def explicit_jacobian(Ws):
    """Dense J_f from Lemma partialf: d f_{i1 i2 i3} / d w^(l)_{i' r} = -delta(i_l, i') prod_{m != l} w^(m)_{i_m r}.
    Rows in C order of the multi-index, columns in the order of vec_blocks."""
    dims = [W.shape[0] for W in Ws]
    R = Ws[0].shape[1]
    offs = np.cumsum([0] + [d * R for d in dims])
    J = np.zeros((int(np.prod(dims)), int(offs[-1])))
    for row, idx in enumerate(itertools.product(*[range(d) for d in dims])):
        for l in range(3):
            for r in range(R):
                val = -1.0
                for m in range(3):
                    if m != l:
                        val *= Ws[m][idx[m], r]
                J[row, offs[l] + r * dims[l] + idx[l]] = val
    return J


def F_of(S, Ws):
    f = dgn.residual(S, Ws)
    return 0.5 * float(np.sum(f * f))


CASES = [((4, 3, 2), 2, 0), ((5, 4, 3), 3, 1), ((3, 6, 4), 4, 2)]


@pytest.mark.parametrize("dims,R,seed", CASES)
def test_explicit_jacobian_matches_kronecker_lemma(dims, R, seed):
    """Columns of J for w_r^(l) equal -w_r^(1) (x) .. I .. (x) w_r^(L) (Lemma kronecker)."""
    rng = np.random.default_rng(seed)
    Ws = [rng.standard_normal((d, R)) for d in dims]
    J = explicit_jacobian(Ws)
    offs = np.cumsum([0] + [d * R for d in dims])
    for l in range(3):
        for r in range(R):
            parts = [Ws[m][:, r:r + 1] if m != l else np.eye(dims[l]) for m in range(3)]
            K = np.kron(np.kron(parts[0], parts[1]), parts[2])
            np.testing.assert_allclose(J[:, offs[l] + r * dims[l]: offs[l] + (r + 1) * dims[l]], -K, atol=1e-14)


@pytest.mark.parametrize("dims,R,seed", CASES)
def test_jtj_v_matches_explicit_jacobian(dims, R, seed):
    rng = np.random.default_rng(seed + 10)
    Ws = [rng.standard_normal((d, R)) for d in dims]
    Vs = [rng.standard_normal((d, R)) for d in dims]
    J = explicit_jacobian(Ws)
    ref = J.T @ (J @ vec_blocks(Vs))
    got = vec_blocks(dgn.jtj_v(Ws, dgn.grams(Ws), Vs))
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))


def test_jtj_v_transposed_variant_is_wrong():
    """Guards the orientation of V^(l'')T W^(l''): using W^T V instead fails against J^T J v."""
    rng = np.random.default_rng(3)
    Ws = [rng.standard_normal((d, 3)) for d in (4, 3, 5)]
    Vs = [rng.standard_normal(W.shape) for W in Ws]
    J = explicit_jacobian(Ws)
    ref = J.T @ (J @ vec_blocks(Vs))
    pis = dgn.grams(Ws)
    wrong = []
    for a in range(3):
        blk = Vs[a] @ dgn.pi_own(pis, a)
        for b in range(3):
            if b != a:
                blk = blk + Ws[a] @ (dgn.pi_pair(pis, a, b) * (Ws[b].T @ Vs[b]))
        wrong.append(blk)
    assert np.max(np.abs(vec_blocks(wrong) - ref)) > 1e-3 * np.max(np.abs(ref))


@pytest.mark.parametrize("dims,R,seed", CASES)
def test_gradient_is_jt_f_and_finite_differences(dims, R, seed):
    rng = np.random.default_rng(seed + 20)
    S = rng.standard_normal(dims)
    Ws = [rng.standard_normal((d, R)) for d in dims]
    J = explicit_jacobian(Ws)
    f = dgn.residual(S, Ws).ravel(order="C")
    g = vec_blocks(dgn.gradient(S, Ws))
    np.testing.assert_allclose(g, J.T @ f, rtol=1e-12, atol=1e-12)
    # central finite differences of F = 1/2 ||S - [[W]]||^2
    h = 1e-6
    shapes = [W.shape for W in Ws]
    w = vec_blocks(Ws)
    fd = np.zeros_like(w)
    for i in range(len(w)):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd[i] = (F_of(S, unvec_blocks(wp, shapes)) - F_of(S, unvec_blocks(wm, shapes))) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-6 * np.max(np.abs(g)))


def test_mttkrp_brute_force():
    rng = np.random.default_rng(4)
    S = rng.standard_normal((5, 4, 3))
    Ws = [rng.standard_normal((d, 2)) for d in S.shape]
    ref = [np.einsum("ijk,jr,kr->ir", S, Ws[1], Ws[2]),
           np.einsum("ijk,ir,kr->jr", S, Ws[0], Ws[2]),
           np.einsum("ijk,ir,jr->kr", S, Ws[0], Ws[1])]
    for l in range(3):
        np.testing.assert_allclose(dgn.mttkrp(S, Ws, l), ref[l], rtol=1e-12, atol=1e-12)


def test_block_structure_of_jtj():
    """H_{l'l'} = Pi^(l') (x) I and off-diagonal blocks from Thm JfT_Jf."""
    rng = np.random.default_rng(9)
    dims, R = (3, 4, 2), 2
    Ws = [rng.standard_normal((d, R)) for d in dims]
    J = explicit_jacobian(Ws)
    H = J.T @ J
    pis = dgn.grams(Ws)
    offs = np.cumsum([0] + [d * R for d in dims])
    for a in range(3):
        blk = H[offs[a]:offs[a + 1], offs[a]:offs[a + 1]]
        np.testing.assert_allclose(blk, np.kron(dgn.pi_own(pis, a), np.eye(dims[a])), atol=1e-12)
        for b in range(3):
            if b == a:
                continue
            blk = H[offs[a]:offs[a + 1], offs[b]:offs[b + 1]]
            P = dgn.pi_pair(pis, a, b)
            for r1 in range(R):
                for r2 in range(R):
                    sub = blk[r1 * dims[a]:(r1 + 1) * dims[a], r2 * dims[b]:(r2 + 1) * dims[b]]
                    np.testing.assert_allclose(sub, P[r1, r2] * np.outer(Ws[a][:, r2], Ws[b][:, r1]), atol=1e-12)


def test_scale_indeterminacy_null_vector():
    """u = (w_r^(1), -w_r^(2), 0) is in the kernel of J, so J^T J is singular."""
    rng = np.random.default_rng(6)
    Ws = [rng.standard_normal((d, 3)) for d in (5, 4, 6)]
    Us = [np.zeros_like(W) for W in Ws]
    Us[0][:, 1] = Ws[0][:, 1]
    Us[1][:, 1] = -Ws[1][:, 1]
    out = dgn.jtj_v(Ws, dgn.grams(Ws), Us)
    assert max(np.max(np.abs(o)) for o in out) < 1e-12 * max(np.max(np.abs(W)) for W in Ws) ** 5
    J = explicit_jacobian(Ws)
    assert np.linalg.matrix_rank(J.T @ J) < J.shape[1]


def test_regularization_dominates_offdiagonal():
    """diag(J^T J) + gamma >= every |off-diagonal| entry of its row (ch.4 Diagonal regularization)."""
    rng = np.random.default_rng(8)
    for trial in range(5):
        Ws = [rng.standard_normal((d, 3)) * rng.uniform(0.2, 3.0) for d in (3, 4, 2)]
        J = explicit_jacobian(Ws)
        H = J.T @ J
        gam = vec_blocks([np.ones((W.shape[0], 1)) * g[None, :] for W, g in zip(Ws, dgn.regularization(Ws))])
        A = H + np.diag(gam)
        off = np.abs(A - np.diag(np.diag(A)))
        assert np.all(np.diag(A)[:, None] >= off - 1e-12)
        # M is the diagonal of J^T J + mu D
        mu = 0.7
        M = dgn.preconditioner(dgn.grams(Ws), dgn.regularization(Ws), mu)
        Mv = vec_blocks([np.ones((W.shape[0], 1)) * m[None, :] for W, m in zip(Ws, M)])
        np.testing.assert_allclose(Mv, np.diag(H + mu * np.diag(gam)), rtol=1e-13)


def dense_system(S, Ws, mu):
    J = explicit_jacobian(Ws)
    gam = vec_blocks([np.ones((W.shape[0], 1)) * g[None, :] for W, g in zip(Ws, dgn.regularization(Ws))])
    A = J.T @ J + mu * np.diag(gam)
    g = vec_blocks(dgn.gradient(S, Ws))
    return A, g


@pytest.mark.parametrize("dims,R,seed", CASES)
def test_pcg_full_run_equals_cholesky(dims, R, seed):
    rng = np.random.default_rng(seed + 30)
    S = rng.standard_normal(dims)
    Ws = [rng.standard_normal((d, R)) for d in dims]
    mu = 0.3
    A, g = dense_system(S, Ws, mu)
    C = np.linalg.cholesky(A)
    ref = np.linalg.solve(C.T, np.linalg.solve(C, -g))
    pis = dgn.grams(Ws)
    gam = dgn.regularization(Ws)
    M = dgn.preconditioner(pis, gam, mu)
    x, its, res = dgn.pcg(Ws, pis, gam, mu, [-v for v in dgn.gradient(S, Ws)], M, 10 * len(g), 1e-28)
    np.testing.assert_allclose(vec_blocks(x), ref, rtol=1e-7, atol=1e-9 * np.max(np.abs(ref)))


@pytest.mark.parametrize("cap", [1, 2, 3, 5])
def test_truncated_pcg_descent_and_positive_prediction(cap):
    rng = np.random.default_rng(cap)
    dims, R = (5, 4, 6), 3
    S = rng.standard_normal(dims)
    Ws = [rng.standard_normal((d, R)) for d in dims]
    mu = 0.5
    pis = dgn.grams(Ws)
    gam = dgn.regularization(Ws)
    M = dgn.preconditioner(pis, gam, mu)
    grad = dgn.gradient(S, Ws, pis)
    x, its, _ = dgn.pcg(Ws, pis, gam, mu, [-v for v in grad], M, cap, 0.0)
    assert its == cap
    # descent direction (damped GN theorem, item 2) and positive predicted reduction
    assert dgn.dot(grad, x) < 0
    f2 = float(np.sum(dgn.residual(S, Ws) ** 2))
    f2_pred = f2 + 2 * dgn.dot(grad, x) + dgn.dot(x, dgn.jtj_v(Ws, pis, x))
    assert f2_pred < f2
    # the linearised residual computed explicitly agrees
    J = explicit_jacobian(Ws)
    flin = dgn.residual(S, Ws).ravel() + J @ vec_blocks(x)
    assert abs(float(flin @ flin) - f2_pred) < 1e-9 * f2


def test_pcg_a_norm_error_is_monotone():
    rng = np.random.default_rng(12)
    dims, R = (4, 5, 3), 3
    S = rng.standard_normal(dims)
    Ws = [rng.standard_normal((d, R)) for d in dims]
    mu = 0.2
    A, g = dense_system(S, Ws, mu)
    xs = np.linalg.solve(A, -g)
    pis, gam = dgn.grams(Ws), dgn.regularization(Ws)
    M = dgn.preconditioner(pis, gam, mu)
    prev = np.inf
    for cap in range(1, 12):
        x, _, _ = dgn.pcg(Ws, pis, gam, mu, [-v for v in dgn.gradient(S, Ws)], M, cap, 0.0)
        e = vec_blocks(x) - xs
        # preconditioned CG minimises the A-norm error over the Krylov space
        en = float(e @ A @ e)
        assert en <= prev * (1 + 1e-10) + 1e-20
        prev = en


def test_norm_balance_invariance():
    rng = np.random.default_rng(13)
    Ws = [rng.standard_normal((d, 4)) * s for d, s in zip((5, 6, 7), (0.1, 3.0, 10.0))]
    Wb = dgn.norm_balance(Ws)
    np.testing.assert_allclose(ml.cpd_full(Wb), ml.cpd_full(Ws), rtol=1e-12, atol=1e-12)
    n = dgn.column_norms(Wb)
    np.testing.assert_allclose(n[0], n[1], rtol=1e-12)
    np.testing.assert_allclose(n[0], n[2], rtol=1e-12)


def test_gain_ratio_and_damping_rule():
    assert dgn.gain_ratio(10.0, 4.0, 2.0) == pytest.approx(0.75)
    assert dgn.gain_ratio(10.0, 12.0, 2.0) < 0
    assert dgn.gain_ratio(10.0, 5.0, 10.0) == 0.0     # guard
    assert dgn.damping_update(1.0, 0.1) == 3.0
    assert dgn.damping_update(1.0, 0.8) == pytest.approx(1.0 / 3.0)
    assert dgn.damping_update(1.0, 0.5) == 1.0
    assert dgn.damping_update(1.0, 0.25) == 1.0
    assert dgn.damping_update(1.0, 0.75) == 1.0
    assert dgn.damping_update(1.0, -3.0) == 3.0


def test_cg_cap_bounds():
    assert dgn.cg_cap_bounds(1) == (2, 3)
    assert dgn.cg_cap_bounds(200) == (1 + 9, 2 + 118)
    assert dgn.cg_cap_bounds(32) == (1 + 4, 2 + 23)       # 32^0.4 = 4 exactly
    for k in range(1, 3000):
        lo, hi = dgn.cg_cap_bounds(k)
        a, b = k ** 0.4, k ** 0.9
        # agrees with the floating ceiling wherever k^p is not within rounding of an integer
        if abs(a - round(a)) > 1e-9:
            assert lo == 1 + math.ceil(a)
        if abs(b - round(b)) > 1e-9:
            assert hi == 2 + math.ceil(b)
    assert dgn.cg_cap(1, 0.0) == 2 and dgn.cg_cap(1, 0.9999) == 3
    assert dgn.cg_cap(200, 0.0) == 10 and dgn.cg_cap(200, 0.999999999) == 120
    # thesis: E(i_CG) ~ half the interval width at k = 200 (55)
    lo, hi = dgn.cg_cap_bounds(200)
    assert (hi - lo) // 2 == 55


def scripted_stop(errs, step=1.0, grad=1.0, maxiter=200, div_ref=1.0, tol=1e-6):
    p = dgn.Params(maxiter=maxiter, tol=tol)
    k = len(errs) - 1
    return dgn.stop_test(list(errs), k, step, grad, p, div_ref)


def test_stopping_conditions_in_order():
    assert scripted_stop([1.0, 5e-7]) == dgn.STOP_REL_ERR
    assert scripted_stop([1.0, 0.5], step=1e-7) == dgn.STOP_STEP
    assert scripted_stop([0.5, 0.5 - 1e-7]) == dgn.STOP_IMPROVEMENT
    assert scripted_stop([1.0, 0.5], grad=1e-8) == dgn.STOP_GRAD
    assert scripted_stop([1.0, 2e7], div_ref=1.0) == dgn.STOP_DIVERGED
    assert scripted_stop([1.0, 0.5], maxiter=1) == dgn.STOP_MAXITER
    # rule 1 wins over rule 2
    assert scripted_stop([1.0, 5e-7], step=0.0) == dgn.STOP_REL_ERR
    assert scripted_stop([1.0, 0.5]) == dgn.STOP_NONE


def test_windowed_stopping_conditions():
    maxiter = 200
    c = dgn.window_c(maxiter)
    assert c == 21
    # oscillating errors with no overall decrease -> average-error rule at k = 3c
    errs = [1.0] + [0.1 + (0.01 if j % 2 else -0.01) for j in range(1, 3 * c + 1)]
    assert scripted_stop(errs[:3 * c]) == dgn.STOP_NONE          # k = 3c-1 is not a check point
    assert scripted_stop(errs) == dgn.STOP_AVG_ERR
    # steadily decreasing errors with tiny improvements -> average-improvement rule
    errs = [1.0] + [0.5 - 2e-6 * j for j in range(1, 3 * c + 1)]
    assert scripted_stop(errs) == dgn.STOP_AVG_IMPR
    # healthy decrease keeps going
    errs = [1.0] + [0.5 * 0.97 ** j for j in range(1, 3 * c + 1)]
    assert scripted_stop(errs) == dgn.STOP_NONE


def forward_error(Ws_est, Fs):
    """min over permutations of the rank-one terms of sqrt(sum ||T_r' - T_sigma(r)||^2) (ch.4 conditioning section)."""
    R = Fs[0].shape[1]
    terms_est = [ml.cpd_full([W[:, r:r + 1] for W in Ws_est]) for r in range(R)]
    terms_ref = [ml.cpd_full([F[:, r:r + 1] for F in Fs]) for r in range(R)]
    D = np.array([[ml.frob(a - b) ** 2 for b in terms_ref] for a in terms_est])
    best = min(sum(D[r, p[r]] for r in range(R)) for p in itertools.permutations(range(R)))
    return math.sqrt(best)


@pytest.mark.parametrize("dims,R,seed", [((12, 10, 8), 4, 1), ((9, 9, 9), 3, 2), ((15, 7, 11), 5, 3)])
def test_planted_exact_recovery(dims, R, seed):
    T, Fs, T0 = synth.planted(dims, R, seed=seed)
    p = dgn.Params(tol=1e-13, maxiter=400)
    Us, _, S = mlsvd.compress(T, R)
    res = cpd.solve(T, R, p, W0=synth.init_factors(S.shape, R, seed), cg_uniforms=synth.cg_uniforms(400, seed))
    assert res["rel_err_full"] < 1e-10
    Wt = res["W_unnormalized"]
    assert forward_error(Wt, Fs) < 1e-8 * ml.frob(T0)


def test_warmup_recovers_factor_functions_and_printed_factors():
    T = synth.warmup_tensor()
    # the warm-up CPD is ill-conditioned: at tol = 1e-6 the improvement test stops near 3e-4,
    # so the recovery check runs with a tight tolerance
    p = dgn.Params(tol=1e-12, maxiter=200)
    res = cpd.solve(T, 3, p, init="mlsvd", cg_uniforms=synth.cg_uniforms(200, 0))
    assert res["rel_err_full"] < 1e-5
    Wt = res["W"]
    funcs = synth.warmup_factor_functions()
    printed = {"X": [], "Y": [], "Z": []}
    for row in read_golden_table("warmup_factors.txt"):
        printed[row[0]].append([float(v) for v in row[2:]])
    printed = [np.array(printed[n]) for n in "XYZ"]

    def cos(a, b):
        return abs(a @ b) / (np.linalg.norm(a) * np.linalg.norm(b))

    # each computed rank-one term matches one term of phi in every mode (up to scaling), and
    # each column the thesis printed is collinear with the matching computed column
    for r in range(3):
        best = max(range(3), key=lambda t: cos(Wt[0][:, r], funcs[0][:, t]))
        for l in range(3):
            assert cos(Wt[l][:, r], funcs[l][:, best]) > 1 - 1e-6
        pr = max(range(3), key=lambda t: cos(Wt[0][:, r], printed[0][:, t]))
        for l in range(3):
            assert cos(Wt[l][:, r], printed[l][:, pr]) > 1 - 1e-6
    # the printed factors are themselves collinear with phi's terms (8 printed digits)
    for l in range(3):
        for c in range(3):
            assert max(cos(printed[l][:, c], funcs[l][:, t]) for t in range(3)) > 1 - 1e-7


def test_config1_reaches_tolerance():
    T, Fs, T0 = synth.config1()
    Us, _, S = mlsvd.compress(T, 5)
    assert S.shape == (5, 5, 5)
    res = cpd.solve(T, 5, dgn.Params(), W0=synth.init_factors(S.shape, 5, 0), cg_uniforms=synth.cg_uniforms(200, 0))
    assert res["stop"] == dgn.STOP_REL_ERR
    assert res["rel_err_core"] < 1e-6
    assert cpd.time_to_tol_iter(res["errs"], 1e-6) == res["iters"]


def test_output_normalization():
    rng = np.random.default_rng(21)
    Ws = [rng.standard_normal((d, 4)) for d in (5, 6, 7)]
    Wn, lam = cpd.normalize_output(Ws)
    assert np.all(lam >= 0) and np.all(np.diff(lam) <= 0)
    for W in Wn:
        np.testing.assert_allclose(np.linalg.norm(W, axis=0), 1.0, rtol=1e-13)
    for l in range(2):
        for r in range(4):
            assert Wn[l][np.argmax(np.abs(Wn[l][:, r])), r] > 0
    rec = ml.cpd_full([Wn[0] * lam[None, :], Wn[1], Wn[2]])
    np.testing.assert_allclose(rec, ml.cpd_full(Ws), rtol=1e-12, atol=1e-12)


def test_initial_damping_is_tau_times_mean_abs_core():
    """ch.4 "Main parameters": mu0 = tau * E(|S|), the mean of the core's entries in absolute value
    (not tau * max_i a_ii of the damped Gauss-Newton section, not the mean of S, not max |S|).
    Hand-written 2x2x2 core: sum |s| = 1+2+...+8 = 36, mean 4.5; tau = 2 gives 9 exactly."""
    S = np.array([[[1.0, -2.0], [3.0, -4.0]], [[5.0, -6.0], [7.0, -8.0]]])
    W0 = [np.eye(2), np.eye(2), np.eye(2)]
    st = dgn.init_state(S, W0, dgn.Params(init_damp=2.0))
    assert st.mu == 9.0
    st1 = dgn.init_state(S, W0, dgn.Params())          # tau = 1 is the thesis default
    assert st1.mu == 4.5
    # a start whose J^T J diagonal is not 1 leaves mu0 unchanged (it depends on S only)
    st2 = dgn.init_state(S, [3.0 * np.eye(2), np.eye(2), np.eye(2)], dgn.Params())
    assert st2.mu == 4.5


def test_divergence_threshold_uses_max_one_and_tensor_norm_squared():
    """ch.4 "Stopping conditions", rule 7: stop when the relative error exceeds
    max{1, ||T||^2} / (1e-16 + tol).  The reference value is ||T||^2 of the input tensor (passed
    in by the driver), not ||S||^2 and not ||T||; below 1 it is clamped to 1."""
    S = np.array([[[1.0, -2.0], [3.0, -4.0]], [[5.0, -6.0], [7.0, -8.0]]])
    W0 = [np.eye(2), np.eye(2), np.eye(2)]
    p = dgn.Params()
    assert dgn.init_state(S, W0, p, tnorm2=16.0).div_ref == 16.0
    assert dgn.init_state(S, W0, p, tnorm2=0.25).div_ref == 1.0
    assert dgn.init_state(S, W0, p).div_ref == pytest.approx(204.0, rel=1e-15)   # no T given: ||S||^2 = 204
    # literal threshold with ||T||^2 = 16 and tol = 1e-6: 16 / (1e-16 + 1e-6)
    thr = 16.0 / (1e-16 + 1e-6)
    assert scripted_stop([1.0, thr * (1 + 1e-12)], div_ref=16.0) == dgn.STOP_DIVERGED
    assert scripted_stop([1.0, thr * (1 - 1e-12)], div_ref=16.0) == dgn.STOP_NONE
    # with ||T|| = 4 (not squared) the threshold would be 4e6; an error of 5e6 must not stop
    assert scripted_stop([1.0, 5e6], div_ref=16.0) == dgn.STOP_NONE


def test_windowed_rules_compare_disjoint_batches_of_c():
    """ch.4 "Stopping conditions", rules 5 and 6 are checked every c iterations and compare "the
    average of a batch with the next one"; the printed sums run over c + 1 indices that share the
    endpoint k0 - c while dividing by c.  Reading kept: two disjoint batches of c errors,
    err[k-2c+1..k-c] and err[k-c+1..k].  The sequence below separates the readings: the two batches
    hold the same values (rule 5 fires), while the literal sums also take err[k-2c] into the old
    batch and err[k-c] into the new one, which differ by 0.6, so the literal averages differ by
    0.6/c and rule 5 would not fire."""
    maxiter = 200
    c = dgn.window_c(maxiter)
    k = 3 * c
    errs = [1.0] + [0.2 + 0.01 * (j % c) for j in range(1, k + 1)]   # sawtooth of period c
    errs[k - 2 * c] = 0.8                                            # outside both kept batches
    old = errs[k - 2 * c + 1:k - c + 1]
    new = errs[k - c + 1:k + 1]
    assert len(old) == len(new) == c and sorted(old) == sorted(new)
    literal_old = sum(errs[k - 2 * c:k - c + 1]) / c
    literal_new = sum(errs[k - c:k + 1]) / c
    assert literal_old - literal_new > 0.6 / c - 1e-12
    assert scripted_stop(errs, maxiter=maxiter) == dgn.STOP_AVG_ERR
    # a lower new batch (mean 0.05 below the old one) keeps going
    errs2 = errs[:k - c + 1] + [e - 0.05 for e in new]
    assert scripted_stop(errs2, maxiter=maxiter) == dgn.STOP_NONE


def test_fixed_cg_cap_replaces_random_schedule():
    """cg_fixed > 0 (ch.4 "Conditioning": a large fixed cg_maxiter for hard tensors) sets the
    CG cap of every iteration; with cg_tol = 0 every iteration runs exactly that many CG
    iterations, and no uniforms are needed.  With the cap at n_p the step is the exact solution of
    the damped normal equations (CG finite termination), checked against a dense Cholesky solve."""
    T, _, _ = synth.planted((6, 5, 4), 3, seed=7, noise_rel=1e-2)
    S = np.asarray(T)
    W0 = synth.init_factors(S.shape, 3, 7)
    p = dgn.Params(maxiter=6, cg_fixed=3, cg_tol=0.0)
    st, infos = dgn.run_dgn(S, W0, p)
    assert len(infos) == 6 and all(i["cg_iters"] == 3 for i in infos)
    # exact step with cap = n_p
    n_p = 3 * (6 + 5 + 4)
    p2 = dgn.Params(maxiter=1, cg_fixed=n_p, cg_tol=0.0)
    st0 = dgn.init_state(S, W0, p2)
    Ws = st0.Ws
    pis = dgn.grams(Ws)
    grad = dgn.gradient(S, Ws, pis)
    gam = dgn.regularization(Ws)
    J = explicit_jacobian(Ws)
    D = np.concatenate([np.repeat(g, W.shape[0]) for g, W in zip(gam, Ws)])   # column-stacked blocks
    A = J.T @ J + st0.mu * np.diag(D)
    x_ref = np.linalg.solve(A, -vec_blocks(grad))
    st1, info = dgn.dgn_step(S, st0, p2, n_p)
    # the step is w1 - w0 before balancing; recover it from the logged norm and the direction
    M = dgn.preconditioner(pis, gam, st0.mu)
    x, its, _ = dgn.pcg(Ws, pis, gam, st0.mu, [-g for g in grad], M, n_p, 0.0)
    assert np.max(np.abs(vec_blocks(x) - x_ref)) < 1e-8 * np.max(np.abs(x_ref))
    assert abs(info["step_norm"] - np.linalg.norm(x_ref)) < 1e-8 * np.linalg.norm(x_ref)


# ---------------------------------------------------------------------------------------------
# Refinement in the original space
def test_full_space_gradient_is_the_lifted_core_gradient():
    """For T = (U1, U2, U3) . S with orthonormal U^(l), the gradient of the full-space problem at
    W~^(l) = U^(l) W^(l) is U^(l) times the core problem's gradient at W (the MTTKRP of T against
    the lifted factors is U^(l) S_(l) KR and the Grams of W~ equal those of W), which is what lets
    the refinement continue the compressed iteration."""
    rng = np.random.default_rng(31)
    S = rng.standard_normal((4, 3, 5))
    Us = [np.linalg.qr(rng.standard_normal((d, r)))[0] for d, r in zip((9, 7, 8), S.shape)]
    T = ml.multilinear(S, Us)
    W = [rng.standard_normal((r, 3)) for r in S.shape]
    g_core = dgn.gradient(S, W)
    g_full = dgn.gradient(T, [U @ w for U, w in zip(Us, W)])
    for l in range(3):
        assert np.max(np.abs(g_full[l] - Us[l] @ g_core[l])) < 1e-12 * np.max(np.abs(g_full[l]))


def test_refinement_keeps_an_exact_solution_and_improves_a_truncated_one():
    """Noiseless planted tensor: the compressed solve is exact, and the full-space refinement keeps it
    (error stays at rounding, steps vanish).  A compression forced below the tensor's multilinear
    rank loses signal; the refinement, working on T itself, lowers the full error."""
    T, _, _ = synth.planted((12, 10, 8), 3, seed=32)
    W0 = synth.init_factors((3, 3, 3), 3, 32)
    U = synth.cg_uniforms(200, 32)
    p = dgn.Params(tol=1e-13, maxiter=300)
    r0 = cpd.solve(T, 3, p, W0=W0, cg_uniforms=U, refine_iters=0)
    r1 = cpd.solve(T, 3, p, W0=W0, cg_uniforms=U, refine_iters=2)
    assert r0["rel_err_full"] < 1e-10 and r1["rel_err_full"] < 1e-10
    assert all(i["step_norm"] < 1e-8 for i in r1["refine_infos"])
    # rank 3 in a 2 x 2 x 2 core: the compression cannot hold the tensor
    Tn, _, _ = synth.planted((12, 10, 8), 3, seed=33, noise_rel=1e-3)
    W0n = synth.init_factors((2, 2, 2), 3, 33)
    pn = dgn.Params()
    c0 = cpd.solve(Tn, 3, pn, W0=W0n, cg_uniforms=U, core_dims=(2, 2, 2))
    c1 = cpd.solve(Tn, 3, pn, W0=W0n, cg_uniforms=U, core_dims=(2, 2, 2), refine_iters=8)
    assert c1["refine_iters"] >= 1
    assert c1["rel_err_full"] < 0.5 * c0["rel_err_full"]


# ---------------------------------------------------------------------------------------------
# Robustness variants: block-Jacobi preconditioner, draw-back + dogleg
def test_block_jacobi_split_has_identity_diagonal_blocks():
    """L = C (x) I with K_l = C_l C_l^T the diagonal blocks of J^T J + mu D: the preconditioned
    operator L^{-1} (J^T J + mu D) L^{-T} has identity diagonal blocks (explicit Jacobian)."""
    rng = np.random.default_rng(41)
    dims, R = (4, 3, 5), 3
    Ws = [rng.standard_normal((d, R)) for d in dims]
    mu = 0.3
    A, _ = dense_system(np.zeros(dims), Ws, mu)
    Ci = dgn.block_factors(dgn.grams(Ws), dgn.regularization(Ws), mu)
    # dense L^{-1} in the column-stacked order: block l is C_l^{-1} (x) I_{d_l}
    blocks = [np.kron(c, np.eye(d)) for c, d in zip(Ci, dims)]
    Linv = np.zeros_like(A)
    o = 0
    for B in blocks:
        Linv[o:o + B.shape[0], o:o + B.shape[0]] = B
        o += B.shape[0]
    P = Linv @ A @ Linv.T
    o = 0
    for d in dims:
        n = d * R
        assert np.max(np.abs(P[o:o + n, o:o + n] - np.eye(n))) < 1e-12
        o += n


def test_block_jacobi_pcg_full_run_equals_cholesky():
    rng = np.random.default_rng(42)
    dims, R = (5, 4, 3), 3
    Ws = [rng.standard_normal((d, R)) for d in dims]
    S = rng.standard_normal(dims)
    mu = 0.7
    pis = dgn.grams(Ws)
    gam = dgn.regularization(Ws)
    grad = dgn.gradient(S, Ws, pis)
    A, _ = dense_system(S, Ws, mu)
    x_ref = np.linalg.solve(A, -vec_blocks(grad))
    n_p = sum(dims) * R
    x, its, _ = dgn.pcg_block(Ws, pis, gam, mu, [-g for g in grad], dgn.block_factors(pis, gam, mu), n_p, 0.0)
    assert np.max(np.abs(vec_blocks(x) - x_ref)) < 1e-9 * np.max(np.abs(x_ref))


def test_dogleg_step_cases():
    """Madsen-Nielsen-Tingleff dogleg: h_gn inside the radius; the cut steepest-descent step when
    the Cauchy point is outside; otherwise a point of the segment [a, h_gn] on the radius."""
    g = [np.array([[1.0, 2.0]])]
    jg2 = 2.5                                  # |Jg|^2 -> Cauchy point a = -(5 / 2.5) g = -2 g, |a| = 2 sqrt(5)
    h = [np.array([[-10.0, 1.0]])]
    assert dgn.dogleg(h, g, jg2, 100.0) is h
    small = dgn.dogleg(h, g, jg2, 1.0)
    assert np.allclose(small[0], -g[0] / np.sqrt(5.0))
    delta = 6.0
    mid = dgn.dogleg(h, g, jg2, delta)
    assert abs(np.linalg.norm(mid[0]) - delta) < 1e-12
    a = -2.0 * g[0]
    t = (mid[0] - a) / (h[0] - a)
    assert np.allclose(t, t[0, 0]) and 0.0 <= t[0, 0] <= 1.0


def test_drawback_fires_only_on_a_hundredfold_error_jump():
    """Without a jump the draw-back option changes nothing; with the previous error recorded as
    tiny (a hundredfold jump) the iteration is redone from N(w_k) - x with a dogleg step no longer
    than half the failed one."""
    T, _, _ = synth.planted((8, 7, 6), 3, seed=43, noise_rel=1e-2)
    S = np.asarray(T)
    W0 = synth.init_factors(S.shape, 3, 43)
    U = synth.cg_uniforms(50, 43)
    p0, p1 = dgn.Params(maxiter=10), dgn.Params(maxiter=10, drawback=True)
    st0, inf0 = dgn.run_dgn(S, W0, p0, cg_uniforms=U)
    st1, inf1 = dgn.run_dgn(S, W0, p1, cg_uniforms=U)
    assert not any(i["drew_back"] for i in inf1)
    assert [i["rel_err"] for i in inf0] == [i["rel_err"] for i in inf1]
    st = dgn.init_state(S, W0, p1)
    st.errs = [1e-12]                          # plant a tiny previous error: the next step is a jump
    cap = dgn.cg_cap(1, U[0])
    _, plain = dgn.dgn_step(S, dgn.init_state(S, W0, p0), p0, cap)
    _, info = dgn.dgn_step(S, st, p1, cap)
    assert info["drew_back"]
    assert info["step_norm"] <= 0.5 * plain["step_norm"] * (1 + 1e-12)


def test_block_jacobi_dgn_reaches_the_noise_floor():
    """On a planted rank-4 tensor with 1e-4 relative noise the block-Jacobi dGN reaches the
    noise floor like the diagonal one."""
    T, _, _ = synth.planted((12, 11, 10), 4, seed=5, noise_rel=1e-4)
    S = np.asarray(T)
    W0 = synth.init_factors(S.shape, 4, 5)
    _, info = dgn.run_dgn(S, W0, dgn.Params(maxiter=100, block_precond=True),
                          cg_uniforms=synth.cg_uniforms(200, 5))
    assert info[-1]["rel_err"] < 1.5e-4
