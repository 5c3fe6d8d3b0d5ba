"""FP64 reference of the learned-initialisation network (test infrastructure only).

A plain multilayer perceptron x -> relu(x W1 + b1) -> relu(. W2 + b2) -> . W3 + b3, the squared-
error loss it is trained with, its gradients by the chain rule and the Adam update (Kingma & Ba,
2015, Algorithm 1).  The thesis has no learned component; this module pins the GPU kernels of
that extension.  Row-major layouts as in the library: W_l is n_in x n_out, a batch of inputs is
B x n_in.  Parity: pinned by central finite differences of the loss (tests), not by the thesis.
"""
import numpy as np


def init_params(sizes, seed=0):
    """He-normal weights N(0, 2 / fan_in), zero biases; sizes = [n_in, h1, h2, n_out]."""
    rng = np.random.default_rng([seed, 5])
    Ws, bs = [], []
    for a, b in zip(sizes[:-1], sizes[1:]):
        Ws.append(rng.standard_normal((a, b)) * np.sqrt(2.0 / a))
        bs.append(np.zeros(b))
    return Ws, bs


def forward(Ws, bs, x):
    """Returns the output and the list of layer inputs / pre-activations needed by backward."""
    acts = [x]
    pre = []
    h = x
    L = len(Ws)
    for l in range(L):
        z = h @ Ws[l] + bs[l]
        pre.append(z)
        h = np.maximum(z, 0.0) if l < L - 1 else z
        acts.append(h)
    return h, (acts, pre)


def mse_loss(y, t):
    """Mean over all entries of (y - t)^2, and its gradient with respect to y."""
    n = y.size
    d = y - t
    return float(np.sum(d * d) / n), 2.0 * d / n


def backward(Ws, cache, dy):
    """Gradients (dWs, dbs) of a scalar loss whose gradient with respect to the output is dy."""
    acts, pre = cache
    L = len(Ws)
    dWs, dbs = [None] * L, [None] * L
    g = dy
    for l in range(L - 1, -1, -1):
        if l < L - 1:
            g = g * (pre[l] > 0.0)
        dWs[l] = acts[l].T @ g
        dbs[l] = np.sum(g, axis=0)
        g = g @ Ws[l].T
    return dWs, dbs


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of parameter p with gradient g at step t (1-based); returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
