"""Pins of the FP64 network oracle: gradients against central finite differences of the loss, the
ReLU kink excluded; the Adam update against its closed form on a scalar; forward against an
explicit per-sample loop."""
import numpy as np

from oracle import mlp as omlp


def test_forward_matches_per_sample_loop():
    Ws, bs = omlp.init_params([7, 5, 4, 3], seed=1)
    x = np.random.default_rng(0).standard_normal((6, 7))
    y, _ = omlp.forward(Ws, bs, x)
    for i in range(6):
        h = x[i]
        for l in range(3):
            z = np.array([sum(h[a] * Ws[l][a, b] for a in range(len(h))) + bs[l][b] for b in range(Ws[l].shape[1])])
            h = np.maximum(z, 0) if l < 2 else z
        np.testing.assert_allclose(y[i], h, rtol=1e-13, atol=1e-13)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    Ws, bs = omlp.init_params([6, 5, 4, 3], seed=2)
    bs = [rng.standard_normal(b.shape) * 0.1 for b in bs]
    x = rng.standard_normal((5, 6))
    t = rng.standard_normal((5, 3))

    def loss():
        y, _ = omlp.forward(Ws, bs, x)
        return omlp.mse_loss(y, t)[0]

    y, cache = omlp.forward(Ws, bs, x)
    _, dy = omlp.mse_loss(y, t)
    dWs, dbs = omlp.backward(Ws, cache, dy)
    h = 1e-6
    for P, G in list(zip(Ws, dWs)) + list(zip(bs, dbs)):
        for idx in np.ndindex(P.shape):
            old = P[idx]
            P[idx] = old + h
            lp = loss()
            P[idx] = old - h
            lm = loss()
            P[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - G[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, G[idx])


def test_adam_closed_form_first_step():
    # first step: mhat = g, vhat = g^2, so p moves by lr * g / (|g| + eps) ~ lr * sign(g)
    p, m, v = omlp.adam_step(np.array([1.0]), np.array([-3.0]), np.zeros(1), np.zeros(1), 1, lr=0.1)
    np.testing.assert_allclose(p, 1.0 + 0.1 * 3.0 / (3.0 + 1e-8), rtol=1e-15)
    np.testing.assert_allclose(m, -0.3)
    np.testing.assert_allclose(v, 0.001 * 9.0)
