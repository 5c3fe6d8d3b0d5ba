"""Multilinear-algebra primitives in FP64 (oracle; test infrastructure only).

Restates ch.2 "Multilinear multiplication" (definition of the multilinear
product, Alg. "Unfolding", definition of the mode-l product) and App. B
(Kronecker, Khatri-Rao and Hadamard products) of the thesis.

Conventions
-----------
* A tensor is a C-ordered ``numpy`` array ``T[i1, i2, ..., iL]``.
* ``unfold(T, l)`` follows Alg. "Unfolding": the mode-l fibres become the
  columns, ordered with the lowest remaining index running fastest
  (i1 fastest, then i2, ...).
* Factor matrices are ``I_l x R`` with the rank-one terms as columns.
"""
import numpy as np


def unfold(T, l):
    """Mode-``l`` unfolding T_(l), shape I_l x prod_{j != l} I_j (ch.2, Alg. Unfolding).

    Columns are the mode-l fibres taken with i1 varying fastest, which is a
    Fortran-order flattening of the remaining indices.
    """
    T = np.asarray(T)
    return np.reshape(np.moveaxis(T, l, 0), (T.shape[l], -1), order="F")


def fold(M, l, shape):
    """Inverse of :func:`unfold` for a tensor of the given ``shape``."""
    shape = tuple(shape)
    rest = shape[:l] + shape[l + 1:]
    A = np.reshape(np.asarray(M), (shape[l],) + rest, order="F")
    return np.moveaxis(A, 0, l)


def mode_product(T, M, l):
    """Mode-l product T x_l M, defined by (T x_l M)_(l) = M T_(l) (ch.2, definition of the product mode-l)."""
    T = np.asarray(T, dtype=np.float64)
    shape = list(T.shape)
    shape[l] = M.shape[0]
    return fold(np.asarray(M, dtype=np.float64) @ unfold(T, l), l, shape)


def multilinear(T, Ms):
    """Multilinear multiplication (M1, ..., ML) . T written out as a chain of mode products (ch.2)."""
    S = np.asarray(T, dtype=np.float64)
    for l, M in enumerate(Ms):
        S = mode_product(S, M, l)
    return S


def khatri_rao(A, B):
    """Column-wise Kronecker product A (.) B (App. B): column r is kron(A[:, r], B[:, r])."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    assert A.shape[1] == B.shape[1]
    out = np.empty((A.shape[0] * B.shape[0], A.shape[1]))
    for r in range(A.shape[1]):
        out[:, r] = np.kron(A[:, r], B[:, r])
    return out


def khatri_rao_except(Ws, l):
    """W^(L) (.) ... (.) W^(l+1) (.) W^(l-1) (.) ... (.) W^(1), the product paired with T_(l)
    in the gradient theorem of ch.4 (section "Computing the gradient")."""
    others = [Ws[j] for j in reversed(range(len(Ws))) if j != l]
    out = others[0]
    for W in others[1:]:
        out = khatri_rao(out, W)
    return out


def cpd_full(Ws):
    """Sum over r of w_r^(1) (x) ... (x) w_r^(L), the rank-R tensor of eq. (compute_cpd) in ch.3."""
    Ws = [np.asarray(W, dtype=np.float64) for W in Ws]
    R = Ws[0].shape[1]
    out = np.zeros(tuple(W.shape[0] for W in Ws))
    for r in range(R):
        term = Ws[0][:, r]
        for W in Ws[1:]:
            term = np.multiply.outer(term, W[:, r])
        out += term
    return out


def frob(T):
    """Frobenius norm (ch.1 inner product on tensors)."""
    return float(np.sqrt(np.sum(np.asarray(T, dtype=np.float64) ** 2)))
