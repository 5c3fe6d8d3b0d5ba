"""Pins of the tensor-train route (ch.4 "Tensor train and the CPD"): Alg. TT-SVD, Thm CPD_to_TT,
the Bi-CPD with a fixed first factor and Alg. CPD-TTD (CPU only)."""
import itertools

import numpy as np
import pytest

import synth
from oracle import dgn, tt


def planted_L(dims, R, seed):
    rng = np.random.default_rng(seed)
    Fs = [rng.standard_normal((d, R)) for d in dims]
    return tt.cpd_full_L(Fs), Fs


def test_cpd_full_matches_einsum():
    rng = np.random.default_rng(1)
    Fs = [rng.standard_normal((d, 2)) for d in (3, 4, 2, 5)]
    ref = np.einsum("ar,br,cr,dr->abcd", *Fs)
    assert np.max(np.abs(tt.cpd_full_L(Fs) - ref)) < 1e-14


def test_cpd_train_theorem():
    """Thm CPD_to_TT: the cores W^(1), (I, W^(l), I) . I, W^(L)T contract to the CPD."""
    T, Fs = planted_L((4, 5, 3, 6, 2), 3, 2)
    assert np.max(np.abs(tt.tt_full(tt.cpd_train_cores(Fs)) - T)) < 1e-12 * np.max(np.abs(T))


def test_tt_svd_exact_at_the_tt_ranks():
    """Alg. TT-SVD on a rank-3 tensor of order 5: every TT-rank is 3 (the CPD-train bounds them),
    the truncation loses nothing, and each core's (r_{l-1} I_l) x r_l reshape has orthonormal
    columns."""
    T, _ = planted_L((6, 7, 5, 8, 4), 3, 3)
    cores = tt.tt_svd(T, 3)
    assert [G.shape for G in cores] == [(1, 6, 3), (3, 7, 3), (3, 5, 3), (3, 8, 3), (3, 4, 1)]
    assert np.max(np.abs(tt.tt_full(cores) - T)) < 1e-12 * np.max(np.abs(T))
    for G in cores[:-1]:
        U = G.reshape(-1, G.shape[2])
        assert np.max(np.abs(U.T @ U - np.eye(U.shape[1]))) < 1e-13


def test_bi_cpd_with_the_true_first_factor():
    """S = (F, B, C) . I: with the first factor fixed to F the Bi-CPD fits S exactly and never moves
    F; B and C are recovered up to column scaling (their rank-one terms with F are exact)."""
    rng = np.random.default_rng(4)
    R = 3
    F, B, C = rng.standard_normal((R, R)), rng.standard_normal((7, R)), rng.standard_normal((R, R))
    S = tt.cpd_full_L([F, B, C])
    W0 = [rng.standard_normal((7, R)), rng.standard_normal((R, R))]
    st, infos = tt.bi_cpd(F, S, W0, dgn.Params(tol=1e-14, maxiter=300), synth.cg_uniforms(300, 4))
    assert np.array_equal(st.Ws[0], F)
    assert st.errs[-1] < 1e-10
    # each free column pair is the planted pair up to a scale (F's columns are independent)
    for r in range(R):
        best = max(range(R), key=lambda q: abs(np.dot(st.Ws[1][:, r], B[:, q])) /
                   (np.linalg.norm(st.Ws[1][:, r]) * np.linalg.norm(B[:, q])))
        c = abs(np.dot(st.Ws[1][:, r], B[:, best])) / (np.linalg.norm(st.Ws[1][:, r]) * np.linalg.norm(B[:, best]))
        assert c > 1 - 1e-9


def forward_error_L(Ws, Fs):
    R = Fs[0].shape[1]
    terms_e = [tt.cpd_full_L([W[:, r:r + 1] for W in Ws]) for r in range(R)]
    terms_r = [tt.cpd_full_L([F[:, r:r + 1] for F in Fs]) for r in range(R)]
    D = np.array([[np.linalg.norm(a - b) ** 2 for b in terms_r] for a in terms_e])
    return np.sqrt(min(sum(D[r, p[r]] for r in range(R)) for p in itertools.permutations(range(R))))


@pytest.mark.parametrize("dims,R,seed", [((8, 9, 10, 7), 3, 5), ((6, 7, 5, 8, 6), 4, 6), ((5, 5, 5, 5, 5, 5), 2, 7)])
def test_cpd_ttd_recovers_planted_tensors(dims, R, seed):
    """Alg. CPD-TTD on noiseless planted rank-R tensors of orders 4 to 6 recovers the rank-one terms
    (forward error up to permutation and scaling) and the tensor."""
    T, Fs = planted_L(dims, R, seed)
    W0 = tt_start(dims, R, seed)
    Ws, cores, logs = tt.cpd_ttd(T, R, dgn.Params(tol=1e-13, maxiter=400), W0=W0,
                                 cg_uniforms=synth.cg_uniforms(400, seed))
    assert np.linalg.norm(tt.cpd_full_L(Ws) - T) / np.linalg.norm(T) < 1e-9
    assert forward_error_L(Ws, Fs) < 1e-7 * np.linalg.norm(T)


def tt_start(dims, R, seed):
    """Start points of the third-order CPDs inside CPD-TTD (the seeded generator of synth)."""
    return synth.tt_init_factors(dims, R, seed)


def test_cpd_ttd_needs_order_four():
    T, _ = planted_L((4, 5, 6), 2, 8)
    with pytest.raises(AssertionError):
        tt.cpd_ttd(T, 2, W0=None)
