"""Pins of the oracle's multilinear primitives and MLSVD compression against the thesis's worked
examples, its theorems, and textbook routines (CPU only)."""
import itertools

import numpy as np
import pytest

from conftest import read_golden_matrices, read_golden_table
import synth
from oracle import multilinear as ml
from oracle import mlsvd


def example_tensor():
    T = np.zeros((3, 4, 2))
    v = 1
    for k in range(2):
        for j in range(4):
            for i in range(3):
                T[i, j, k] = v
                v += 1
    return T


def test_unfoldings_match_worked_example():
    g = read_golden_matrices("unfolding_3x4x2.txt")
    T = example_tensor()
    for l, name in enumerate(["T1", "T2", "T3"]):
        np.testing.assert_array_equal(ml.unfold(T, l), g[name])
        np.testing.assert_array_equal(ml.fold(g[name], l, T.shape), T)


def test_mode_product_matches_worked_example():
    g = read_golden_matrices("unfolding_3x4x2.txt")
    T = example_tensor()
    P = ml.mode_product(T, g["M"], 0)
    assert P.shape == (2, 4, 2)
    np.testing.assert_array_equal(ml.unfold(P, 0), g["MT1"])
    # multilinear multiplication with identities in the other modes is the same product
    np.testing.assert_array_equal(ml.multilinear(T, [g["M"], np.eye(4), np.eye(2)]), P)


def test_khatri_rao_gram_identity():
    rng = np.random.default_rng(5)
    A, B = rng.standard_normal((7, 4)), rng.standard_normal((5, 4))
    K = ml.khatri_rao(A, B)
    np.testing.assert_allclose(K.T @ K, (A.T @ A) * (B.T @ B), rtol=1e-13, atol=1e-13)


def test_cpd_unfolding_formula():
    """T_(l) = W^(l) (KR of the others)^T for a rank-R tensor (ch.2 unfolding formula)."""
    rng = np.random.default_rng(2)
    Ws = [rng.standard_normal((d, 3)) for d in (4, 5, 6)]
    T = ml.cpd_full(Ws)
    for l in range(3):
        np.testing.assert_allclose(ml.unfold(T, l), Ws[l] @ ml.khatri_rao_except(Ws, l).T, rtol=1e-12, atol=1e-12)
    # brute force entry check
    i, j, k = 3, 1, 4
    assert abs(T[i, j, k] - sum(Ws[0][i, r] * Ws[1][j, r] * Ws[2][k, r] for r in range(3))) < 1e-12


def test_warmup_table_4_5():
    T = synth.warmup_tensor()
    _, _, S = mlsvd.compress(T, 3)
    assert S.shape == (3, 3, 3)
    tab = mlsvd.truncation_error_table(S)
    rows = read_golden_table("warmup_table45.txt")
    assert len(rows) == 27
    for i, j, k, v in rows:
        got = tab[(int(i), int(j), int(k))]
        # the table prints 8 decimals
        assert abs(got - float(v)) <= 6e-9, (i, j, k, got, v)


def test_warmup_truncation_is_exact():
    """The 3x3x3 truncation reproduces T to roundoff (printed 3.85e-14)."""
    T = synth.warmup_tensor()
    Us, _, S = mlsvd.compress(T, 3)
    err = ml.frob(T - ml.multilinear(S, Us)) / ml.frob(T)
    assert err < 1e-12


def test_warmup_core_magnitudes():
    T = synth.warmup_tensor()
    _, _, S = mlsvd.compress(T, 3)
    for i, j, k, v in read_golden_table("warmup_core.txt"):
        decimals = len(v.split(".")[1]) if "." in v else 0
        unit = 10.0 ** (-decimals)           # one unit in the last printed digit
        got = abs(S[int(i) - 1, int(j) - 1, int(k) - 1])
        # printed values are rounded or truncated to that digit
        assert abs(got - abs(float(v))) <= unit, (i, j, k, got, v)


def test_warmup_smart_init():
    T = synth.warmup_tensor()
    Us, _, S = mlsvd.compress(T, 3)
    picks = mlsvd.smart_init_entries(S, 3)
    assert set(picks) == {(0, 0, 0), (1, 0, 1), (0, 1, 1)}
    Ws = mlsvd.smart_init(S, 3)
    err = mlsvd.uncompressed_error(T, Us, Ws)
    # printed as 0.0153 (4 decimals, truncated): within one unit of the last digit
    assert 0.0153 <= err < 0.0154


@pytest.mark.parametrize("dims,R", [((6, 5, 4), 3), ((9, 7, 8), 4), ((12, 5, 7), 6)])
def test_svd_route_matches_gram_route(dims, R):
    rng = np.random.default_rng(sum(dims))
    T = rng.standard_normal(dims)
    for l in range(3):
        P = min(dims[l], R)
        U1, s1 = mlsvd.left_singular_svd(T, l, P)
        U2, s2 = mlsvd.left_singular_gram(T, l, P)
        np.testing.assert_allclose(s1, s2, rtol=1e-10)
        # principal angles between the subspaces
        cosines = np.linalg.svd(U1.T @ U2, compute_uv=False)
        assert np.min(cosines) > 1 - 1e-10
        # with the same sign convention the vectors themselves agree
        np.testing.assert_allclose(U1, U2, atol=1e-8)


def test_mlsvd_theorem_properties():
    rng = np.random.default_rng(11)
    T = rng.standard_normal((5, 6, 4))
    Us, sig, S = mlsvd.full_mlsvd(T)
    # T = (U1, U2, U3) . S
    np.testing.assert_allclose(ml.multilinear(S, Us), T, atol=1e-12)
    # ||T|| = ||S|| = sqrt(sum sigma^2) in every mode
    for l in range(3):
        assert abs(np.sqrt(np.sum(sig[l] ** 2)) - ml.frob(T)) < 1e-12
    assert abs(ml.frob(S) - ml.frob(T)) < 1e-12
    # all-orthogonality and ordering of the hyperslices
    for l in range(3):
        Sl = ml.unfold(S, l)
        G = Sl @ Sl.T
        np.testing.assert_allclose(G - np.diag(np.diag(G)), 0, atol=1e-12)
        norms = np.sqrt(np.diag(G))
        np.testing.assert_allclose(norms, sig[l][:len(norms)], atol=1e-12)
        assert np.all(np.diff(norms) <= 1e-12)


def test_truncation_bound():
    """||T - T~||^2 <= sum of the discarded sigma^2 over all modes (ch.2 truncation theorem)."""
    rng = np.random.default_rng(3)
    T = rng.standard_normal((6, 7, 5))
    Us, sig, S = mlsvd.full_mlsvd(T)
    for ranks in [(2, 3, 2), (4, 4, 4), (1, 7, 3)]:
        St = np.zeros_like(S)
        St[:ranks[0], :ranks[1], :ranks[2]] = S[:ranks[0], :ranks[1], :ranks[2]]
        err2 = ml.frob(T - ml.multilinear(St, Us)) ** 2
        bound = sum(np.sum(sig[l][ranks[l]:] ** 2) for l in range(3))
        assert err2 <= bound + 1e-10


def test_order_two_reduces_to_matrix_svd():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((6, 9))
    U, s, Vt = np.linalg.svd(A)
    Us, sig, S = mlsvd.full_mlsvd(A)
    np.testing.assert_allclose(sig[0], s, rtol=1e-12)
    np.testing.assert_allclose(np.abs(S[:6, :6]), np.diag(s), atol=1e-12)


def test_truncation_rank_rule():
    # tail energy ratio must drop below tol / L
    s = np.array([10.0, 1.0, 1e-4, 1e-6])
    assert mlsvd.truncation_rank(s, 1e-6, 3) == 2      # tail 1e-8/101 < 3.3e-7
    s = np.array([10.0, 1.0, 1e-2, 1e-6])
    assert mlsvd.truncation_rank(s, 1e-6, 3) == 3      # tail at i=2 is 1e-4/101 > 3.3e-7
    assert mlsvd.truncation_rank(s, 1e-1, 3) == 1
    assert mlsvd.truncation_rank(np.zeros(3), 1e-6, 3) == 3
    assert mlsvd.truncation_rank(np.array([1.0, 1.0]), 1e-6, 3) == 2


def test_compress_planted_rank_and_core():
    T, Fs, T0 = synth.planted((14, 11, 9), 4, seed=7)
    Us, sig, S = mlsvd.compress(T, 4)
    assert S.shape == (4, 4, 4)
    np.testing.assert_allclose(ml.multilinear(S, Us), T, atol=1e-10 * ml.frob(T))
    for U in Us:
        np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)


def test_canonical_signs():
    U = np.array([[0.1, -0.9], [-0.8, 0.2], [0.3, 0.9]])
    V = mlsvd.canonical_signs(U)
    np.testing.assert_array_equal(V[:, 0], -U[:, 0])
    # tie on |.|: the lowest index decides (-0.9 at row 0) -> flipped
    np.testing.assert_array_equal(V[:, 1], -U[:, 1])


# ---------------------------------------------------------------------------------------------
# Sequentially truncated MLSVD (ch.2 Alg. ST-MLSVD)
def test_st_mlsvd_untruncated_equals_mlsvd():
    """Without truncation every U^(l) is square orthogonal, and multiplying an unfolding on the right
    by an orthogonal matrix keeps its left singular vectors and values: ST-MLSVD then equals the
    MLSVD of Thm MLSVD (bases, singular values and core)."""
    rng = np.random.default_rng(21)
    T = rng.standard_normal((5, 4, 3))
    Uc, sc, Sc = mlsvd.full_mlsvd(T)
    Us, ss, Ss = mlsvd.compress_st(T, 5, core_dims=(5, 4, 3))
    for l in range(3):
        assert np.allclose(Us[l], Uc[l], atol=1e-12)
        assert np.allclose(ss[l], sc[l], rtol=1e-12)
    assert np.allclose(Ss, Sc, atol=1e-12)


def test_st_mlsvd_recovers_exact_multilinear_rank():
    """A tensor of multilinear rank (3, 4, 2) (random Tucker core, orthonormal bases): the truncation
    rule keeps exactly (3, 4, 2) and the sequential truncation reconstructs T to rounding; its bases
    span the same subspaces as the classic compression's."""
    rng = np.random.default_rng(22)
    G = rng.standard_normal((3, 4, 2))
    Qs = [np.linalg.qr(rng.standard_normal((d, r)))[0] for d, r in zip((10, 9, 8), (3, 4, 2))]
    T = ml.multilinear(G, Qs)
    Us, _, S = mlsvd.compress_st(T, 4)
    assert S.shape == (3, 4, 2)
    That = ml.multilinear(S, Us)
    assert ml.frob(T - That) < 1e-13 * ml.frob(T)
    Uc, _, _ = mlsvd.compress(T, 4)
    for l in range(3):
        # equal subspaces: the projector difference vanishes
        assert np.max(np.abs(Us[l] @ Us[l].T - Uc[l] @ Uc[l].T)) < 1e-12


def test_st_mlsvd_error_within_truncation_bound_and_last_mode_orthogonal():
    """ST-MLSVD satisfies the truncation bound of ch.2 (Thm energy-mlsvd, the sum of the discarded
    squared singular values of the classic unfoldings), and its last core unfolding has orthogonal
    rows whose norms are the last mode's singular values (S_(3) = U^(3)T S^(2)_(3))."""
    T, _, _ = synth.planted((14, 12, 10), 6, seed=23, noise_rel=0.05)
    core = (4, 5, 3)
    Us, ss, S = mlsvd.compress_st(T, 6, core_dims=core)
    err2 = ml.frob(T - ml.multilinear(S, Us)) ** 2
    _, sc, _ = mlsvd.full_mlsvd(T)
    bound = sum(float(np.sum(sc[l][core[l]:] ** 2)) for l in range(3))
    assert err2 <= bound * (1 + 1e-12)
    S3 = ml.unfold(S, 2)
    Gm = S3 @ S3.T
    assert np.allclose(Gm, np.diag(ss[2][:core[2]] ** 2), atol=1e-10 * Gm.max())


def test_st_mlsvd_truncation_rule_on_planted_tensor():
    """Noisy planted rank-4 tensor, R = 4: the sequential and classic compressions keep the same core
    size, their bases agree to the noise level and the cores have equal norm within it."""
    T, _, _ = synth.planted((20, 18, 16), 4, seed=24, noise_rel=1e-8)
    Us, _, S = mlsvd.compress_st(T, 4)
    Uc, _, Sc = mlsvd.compress(T, 4)
    assert S.shape == Sc.shape == (4, 4, 4)
    for l in range(3):
        assert np.max(np.abs(Us[l] @ Us[l].T - Uc[l] @ Uc[l].T)) < 1e-6
    assert abs(ml.frob(S) - ml.frob(Sc)) < 1e-6 * ml.frob(Sc)
