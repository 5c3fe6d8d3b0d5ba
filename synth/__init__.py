"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and assembles input tensors; it holds
none of the CPD method's arithmetic.  Random numbers the method itself
consumes (the initial factors and the uniform draws behind the random CG
iteration cap) are produced here and passed to both the oracle and the HIP
library as inputs.

Workload shapes and distributions follow the thesis's synthetic tensors:
N(0,1) factor entries (random rank-R tensors of ch.4), factors with
prescribed pairwise column correlation through the Cholesky construction of
ch.4 "A special family of tensors", additive Gaussian noise scaled to a
target Frobenius ratio, and the separable function of the ch.4 warm-up.

Draw order (numpy ``default_rng``):
* tensor stream ``default_rng(seed)``: factor 1, factor 2, factor 3 (each
  ``standard_normal((I_l, R))``), then the noise ``standard_normal(dims)``;
* initial factors: ``default_rng([seed, 1])``, one ``standard_normal((d_l, R))``
  per mode in order;
* CG-cap uniforms: ``default_rng([seed, 2]).random(maxiter)``.
"""
import math

import numpy as np


def warmup_tensor():
    """T_ijk = phi(x_i, y_j, z_k) on the 6 x 5 x 4 grid of the ch.4 warm-up section."""
    x = np.linspace(0.0, 1.0, 6)
    y = np.linspace(0.0, 1.0, 5)
    z = np.linspace(0.0, 1.0, 4)
    X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
    return (np.cos(1 - X) * np.sin(1 + Y ** 2)
            - np.sin(1 + X ** 2) * np.exp(X ** 2 + Y ** 2 + Z ** 2)
            - np.cos(X) * np.log(1 + Z))


def warmup_factor_functions():
    """The three separable terms of the warm-up function, sampled on the grids (mode, term) -> vector."""
    x = np.linspace(0.0, 1.0, 6)
    y = np.linspace(0.0, 1.0, 5)
    z = np.linspace(0.0, 1.0, 4)
    X = np.stack([np.cos(1 - x), -np.sin(1 + x ** 2) * np.exp(x ** 2), -np.cos(x)], axis=1)
    Y = np.stack([np.sin(1 + y ** 2), np.exp(y ** 2), np.ones_like(y)], axis=1)
    Z = np.stack([np.ones_like(z), np.exp(z ** 2), np.log(1 + z)], axis=1)
    return [X, Y, Z]


def correlation_mixer(R, c):
    """Upper-triangular R_c with R_c^T R_c = c 11^T + (1 - c) I (ch.4 special family)."""
    G = c * np.ones((R, R)) + (1.0 - c) * np.eye(R)
    return np.linalg.cholesky(G).T


def outer3(A, B, C):
    """sum_r a_r (x) b_r (x) c_r assembled as A (C (.) B)^T, C-ordered."""
    I, J, K = A.shape[0], B.shape[0], C.shape[0]
    R = A.shape[1]
    KR = (B[:, None, :] * C[None, :, :]).reshape(J * K, R)   # row index j*K + k
    return (A @ KR.T).reshape(I, J, K)


def planted(dims, R, seed=0, snr_db=None, noise_rel=None, corr=None, dtype=np.float64):
    """Rank-R tensor with N(0,1) factors (optionally column-correlated) plus scaled Gaussian noise.

    Returns ``(T, factors, T0)``: the noisy tensor in ``dtype``, the planted
    factors and the noiseless tensor (FP64).  Noise is scaled to
    ||E|| = noise_rel ||T0|| or to the SNR 20 log10(||T0|| / ||E||) = snr_db.
    """
    rng = np.random.default_rng(seed)
    Fs = [rng.standard_normal((d, R)) for d in dims]
    if corr is not None:
        Rc = correlation_mixer(R, corr)
        Fs = [F @ Rc for F in Fs]
    T0 = outer3(*Fs)
    rel = None
    if noise_rel is not None:
        rel = noise_rel
    elif snr_db is not None:
        rel = 10.0 ** (-snr_db / 20.0)
    T = T0
    if rel is not None and rel > 0:
        E = rng.standard_normal(tuple(dims))
        T = T0 + (rel * math.sqrt(np.sum(T0 * T0)) / math.sqrt(np.sum(E * E))) * E
    return np.ascontiguousarray(T.astype(dtype)), Fs, T0


def init_factors(core_dims, R, seed=0):
    """Random N(0,1) initial factors W^(l) in R^{d_l x R} (ch.4 "Initialization", random approach)."""
    rng = np.random.default_rng([seed, 1])
    return [rng.standard_normal((d, R)) for d in core_dims]


def cg_uniforms(maxiter, seed=0):
    """One uniform draw in [0, 1) per dGN iteration; the method maps it to the random CG cap."""
    return np.random.default_rng([seed, 2]).random(maxiter)


def batch_shapes(n, seed=0, lo=10, hi=64, rlo=2, rhi=12):
    """Shapes and ranks of a batch of small CPDs: each mode ~ U{lo..hi}, rank ~ U{rlo..rhi}."""
    rng = np.random.default_rng([seed, 3])
    dims = rng.integers(lo, hi + 1, size=(n, 3))
    ranks = rng.integers(rlo, rhi + 1, size=n)
    return [tuple(int(v) for v in d) for d in dims], [int(r) for r in ranks]


def batch_members(n, seed=0, snr_db=50.0, dtype=np.float64):
    """Members of a batch of small planted CPDs (shapes and ranks from ``batch_shapes``); member b
    is ``planted(dims_b, R_b, seed=seed * 1000003 + b + 1, snr_db)`` with initial core factors
    ``init_factors(P_b, R_b, seed=seed * 1000003 + b + 1)``, P_b,l = min(dims_b,l, R_b).
    Returns (tensors, ranks, initial factors)."""
    shapes, ranks = batch_shapes(n, seed)
    Ts, W0s = [], []
    for b, (dims, R) in enumerate(zip(shapes, ranks)):
        s = seed * 1000003 + b + 1
        T, _, _ = planted(dims, R, seed=s, snr_db=snr_db, dtype=dtype)
        Ts.append(T)
        W0s.append(init_factors([min(d, R) for d in dims], R, s))
    return Ts, ranks, W0s


# Named workloads (the shapes of the five benchmark configurations)
def config1(seed=0):
    """50^3 FP64, R = 5, N(0,1) factors, noise at 1e-6 relative Frobenius norm."""
    return planted((50, 50, 50), 5, seed=seed, noise_rel=1e-6, dtype=np.float64)


def config2(seed=0):
    """200^3 FP32, R = 20, factor columns with pairwise correlation 0.5, SNR 40 dB."""
    return planted((200, 200, 200), 20, seed=seed, snr_db=40.0, corr=0.5, dtype=np.float32)


def config3(seed=0, dtype=np.float32):
    """600^3, R = 50, N(0,1) factors, SNR 60 dB."""
    return planted((600, 600, 600), 50, seed=seed, snr_db=60.0, dtype=dtype)


def tt_init_factors(dims, R, seed=0):
    """Start points of the third-order CPDs of the tensor-train route for an order-L tensor with
    every TT-rank R: for the second core (R x I_2 x R, compressed to P = (R, min(I_2, R), R)) three
    P_l x R matrices, then for cores l = 3..L-1 the free factors (I_l x R, R x R); N(0,1) entries
    from ``default_rng([seed, 4])`` in that order."""
    rng = np.random.default_rng([seed, 4])
    out = [[rng.standard_normal((p, R)) for p in (R, min(dims[1], R), R)]]
    for d in dims[2:-1]:
        out.append([rng.standard_normal((d, R)), rng.standard_normal((R, R))])
    return out


def planted_order_L(dims, R, seed=0, noise_rel=None, dtype=np.float64):
    """Rank-R tensor of any order with N(0,1) factors (drawn in mode order from
    ``default_rng(seed)``) plus optional Gaussian noise of relative Frobenius norm noise_rel."""
    rng = np.random.default_rng(seed)
    Fs = [rng.standard_normal((d, R)) for d in dims]
    out = Fs[0]
    for F in Fs[1:]:
        out = (out[:, None, :] * F[None, :, :]).reshape(-1, R)
    T0 = out.sum(axis=1).reshape(dims)
    T = T0
    if noise_rel:
        E = rng.standard_normal(tuple(dims))
        T = T0 + (noise_rel * math.sqrt(np.sum(T0 * T0)) / math.sqrt(np.sum(E * E))) * E
    return np.ascontiguousarray(T.astype(dtype)), Fs
