"""Truncated MLSVD compression and the MLSVD-based initialisation (oracle; test infrastructure only).

Restates ch.2 "Multilinear singular value decomposition" (Thm MLSVD,
Alg. MLSVD, the truncation bound, Alg. ST-MLSVD), the Gram-eigenvector route of App. B
(lemma relating the SVD of M to the eigendecomposition of M M^T) and ch.4
section "Compression" (Alg. Compression, P_l = min(I_l, R)) and section
"Initialization".

Readings taken where the thesis is silent (each listed in the design doc):
* singular-vector signs: each column of U^(l) is flipped so that its entry of
  largest magnitude is positive (ties: lowest row index);
* the truncation test compares the squared tail energy ratio with
  mlsvd_tol / L, and R~_l is the first i (1-based) that passes;
* MLSVD-energy init: the R entries of largest magnitude, ties broken by the
  lexicographically smallest multi-index.
"""
import numpy as np

from .multilinear import unfold, multilinear, mode_product, cpd_full, frob


def canonical_signs(U):
    """Flip columns so the largest-|.| entry of each is positive (sign reading; ties -> lowest index)."""
    U = np.array(U, dtype=np.float64, copy=True)
    for j in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, j])))
        if U[i, j] < 0:
            U[:, j] = -U[:, j]
    return U


def left_singular_svd(T, l, P):
    """Leading P left singular vectors / values of T_(l) by the SVD itself (Alg. MLSVD)."""
    U, s, _ = np.linalg.svd(unfold(T, l), full_matrices=False)
    return canonical_signs(U[:, :P]), s[:P].copy()


def left_singular_gram(T, l, P):
    """Same quantities through the eigendecomposition of the Gram T_(l) T_(l)^T (App. B lemma):
    its eigenvectors are the left singular vectors and sigma = sqrt(lambda)."""
    A = unfold(T, l)
    lam, V = np.linalg.eigh(A @ A.T)
    order = np.argsort(lam)[::-1][:P]
    lam = np.clip(lam[order], 0.0, None)
    return canonical_signs(V[:, order]), np.sqrt(lam)


def truncation_rank(sigma, mlsvd_tol, L):
    """Smallest i with sum_{r>i} sigma_r^2 / sum_r sigma_r^2 < mlsvd_tol / L (ch.4 Alg. Compression).

    At i = P the tail is empty, so the loop always ends.
    """
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    total = s2.sum()
    P = len(s2)
    if total == 0.0:
        return P
    for i in range(1, P + 1):
        if s2[i:].sum() / total < mlsvd_tol / L:
            return i
    return P


def compress(T, R, mlsvd_tol=1e-6, core_dims=None, route="svd"):
    """Tensor Fox compression (ch.4 Alg. Compression).

    Returns ``(U, sigma, S)``: truncated orthonormal bases U^(l) (I_l x R~_l),
    the P_l leading mode-l singular values, and the core
    S = (U^(1)T, ..., U^(L)T) . T of shape R~_1 x ... x R~_L.
    ``core_dims`` overrides the truncation rule with fixed R~_l (used by the
    learned initialiser, which needs a fixed-size core).
    """
    T = np.asarray(T, dtype=np.float64)
    L = T.ndim
    Us, sigmas = [], []
    for l in range(L):
        P = min(T.shape[l], R) if core_dims is None else core_dims[l]
        if route == "svd":
            U, s = left_singular_svd(T, l, P)
        else:
            U, s = left_singular_gram(T, l, P)
        Us.append(U)
        sigmas.append(s)
    if core_dims is None:
        ranks = [truncation_rank(s, mlsvd_tol, L) for s in sigmas]
    else:
        ranks = list(core_dims)
    Us = [U[:, :r] for U, r in zip(Us, ranks)]
    S = multilinear(T, [U.T for U in Us])
    return Us, sigmas, S


def compress_st(T, R, mlsvd_tol=1e-6, core_dims=None):
    """Sequentially truncated MLSVD (ch.2 Alg. ST-MLSVD, the variant Tensor Fox can switch to):
    S^(0) = T; for l = 1..L the leading left singular vectors of the mode-l unfolding of the current
    S^(l-1) (P_l = min(I_l, R) of them, signs canonical), the truncation rule of Alg. Compression on
    those singular values, and S^(l) = S^(l-1) x_l U^(l)T, so each later mode works on the shrunk
    tensor.  Returns ``(U, sigma, S)`` as ``compress``; sigma^(l) are the singular values of the
    unfolding of S^(l-1)."""
    S = np.asarray(T, dtype=np.float64)
    L = S.ndim
    Us, sigmas = [], []
    for l in range(L):
        P = min(S.shape[l], R) if core_dims is None else core_dims[l]
        U, sg = left_singular_svd(S, l, P)
        r = truncation_rank(sg, mlsvd_tol, L) if core_dims is None else core_dims[l]
        U = U[:, :r]
        Us.append(U)
        sigmas.append(sg)
        S = mode_product(S, U.T, l)
    return Us, sigmas, S


def full_mlsvd(T):
    """Untruncated MLSVD of Thm MLSVD: U^(l) square orthogonal, S = (U^(1)T, ..., U^(L)T) . T."""
    T = np.asarray(T, dtype=np.float64)
    Us, sigmas = [], []
    for l in range(T.ndim):
        U, s, _ = np.linalg.svd(unfold(T, l), full_matrices=True)
        Us.append(canonical_signs(U))
        sigmas.append(s)
    return Us, sigmas, multilinear(T, [U.T for U in Us])


def smart_init_entries(S, R):
    """Multi-indices of the R core entries of largest magnitude (ch.4 "Initialization", MLSVD-energy
    reading: ties go to the lexicographically smallest multi-index)."""
    S = np.asarray(S, dtype=np.float64)
    flat = np.abs(S).ravel(order="C")
    # stable sort on -|s| keeps C-order (lexicographic) among equal magnitudes
    order = np.argsort(-flat, kind="stable")[:R]
    return [tuple(int(v) for v in np.unravel_index(i, S.shape)) for i in order]


def smart_init(S, R, extra=None):
    """MLSVD-energy initial point: W^(1)[:, r] = s_j e_{j1}, W^(l)[:, r] = e_{jl} for l > 1.

    If R exceeds the number of core entries the remaining columns are taken
    from ``extra`` (a list of R~_l x R matrices supplied by the caller).
    Norm balancing is applied by the caller (see dgn.norm_balance).
    """
    S = np.asarray(S, dtype=np.float64)
    Ws = [np.zeros((d, R)) for d in S.shape]
    idx = smart_init_entries(S, R)
    for r, j in enumerate(idx):
        Ws[0][j[0], r] = S[j]
        for l in range(1, S.ndim):
            Ws[l][j[l], r] = 1.0
    if len(idx) < R:
        if extra is None:
            raise ValueError("R exceeds the number of core entries; extra columns required")
        for l in range(S.ndim):
            Ws[l][:, len(idx):] = extra[l][:, len(idx):]
    return Ws


def truncation_error_table(S):
    """Relative error of every truncation S[:i, :j, :k] of an MLSVD core (ch.4 warm-up, Table 4.5)."""
    nS = frob(S)
    out = {}
    for i in range(1, S.shape[0] + 1):
        for j in range(1, S.shape[1] + 1):
            for k in range(1, S.shape[2] + 1):
                St = np.zeros_like(S)
                St[:i, :j, :k] = S[:i, :j, :k]
                out[(i, j, k)] = frob(S - St) / nS
    return out


def uncompressed_error(T, Us, Ws):
    """||T - (U^(1) W^(1), ..., U^(L) W^(L)) . I|| / ||T|| (ch.4 "Uncompression")."""
    return frob(np.asarray(T) - cpd_full([U @ W for U, W in zip(Us, Ws)])) / frob(T)
