"""Learned starting point for the dGN on a fixed-size compressed core (an extension: the thesis
initialises with random or MLSVD-energy points, ch.4 "Initialization").

A network maps the compressed core S (fixed core dims, e.g. 16^3), normalised to unit Frobenius
norm, to the R-term factors of S, balanced (equal column norms across modes), sign-fixed (modes 1
and 2 have a positive largest entry) and ordered by decreasing weight, scaled by ||S||^{-1/3}.
Training pairs come from the library itself: each planted tensor is compressed by cpd_compress,
and the factors of its core are the batched solver's converged CPD of that core.  All arithmetic
runs in libcpd (cpd_compress, cpd_solve_batched, cpd_mlp_*); this module only moves tensors and
calls the C ABI.
"""
import ctypes
import math

import torch

from . import _lib
from . import Batch, compress, params, _stream


class MLP:
    """x -> relu(x W1 + b1) -> relu(. W2 + b2) -> . W3 + b3 in FP32 on the GPU (libcpd kernels)."""

    def __init__(self, sizes, seed=0, device="cuda"):
        self.sizes = list(sizes)
        g = torch.Generator(device="cpu").manual_seed(int(seed))
        self.W, self.b = [], []
        for a, c in zip(self.sizes[:-1], self.sizes[1:]):
            w = torch.randn((a, c), generator=g, dtype=torch.float32) * math.sqrt(2.0 / a)   # He-normal
            self.W.append(w.to(device).contiguous())
            self.b.append(torch.zeros(c, dtype=torch.float32, device=device))
        self.gW = [torch.zeros_like(w) for w in self.W]
        self.gb = [torch.zeros_like(b) for b in self.b]
        self.mW = [torch.zeros_like(w) for w in self.W]
        self.vW = [torch.zeros_like(w) for w in self.W]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        P = lambda ts: (ctypes.c_void_p * 3)(*[t.data_ptr() for t in ts])
        self.net = _lib.Mlp(*self.sizes, P(self.W), P(self.b))
        self.grads = _lib.MlpGrads(P(self.gW), P(self.gb))
        self.adam = _lib.Adam(1e-3, 0.9, 0.999, 1e-8, 0, P(self.mW), P(self.mb), P(self.vW), P(self.vb))
        self.device = device
        self._ws = {}
        self._mse_ws = torch.empty(8192, dtype=torch.uint8, device=device)
        self._loss = torch.zeros(1, dtype=torch.float32, device=device)

    def _workspace(self, B):
        if B not in self._ws:
            n = _lib.lib().cpd_mlp_workspace_bytes(ctypes.byref(self.net), B)
            self._ws[B] = torch.empty(max(n, 256), dtype=torch.uint8, device=self.device)
        return self._ws[B]

    def forward(self, x):
        x = x.contiguous()
        B = x.shape[0]
        y = torch.empty((B, self.sizes[-1]), dtype=torch.float32, device=self.device)
        ws = self._workspace(B)
        _lib.check(_lib.lib().cpd_mlp_forward(ctypes.byref(self.net), x.data_ptr(), y.data_ptr(), B, ws.data_ptr(),
                                               ws.numel(), _stream()), "cpd_mlp_forward")
        return y

    def train_step(self, x, t, lr=1e-3):
        """One Adam step on the mean squared error of a batch; returns the loss (a device tensor)."""
        L = _lib.lib()
        x, t = x.contiguous(), t.contiguous()
        B = x.shape[0]
        y = self.forward(x)
        dy = torch.empty_like(y)
        _lib.check(L.cpd_mlp_mse(y.data_ptr(), t.data_ptr(), y.numel(), dy.data_ptr(), self._loss.data_ptr(),
                                 self._mse_ws.data_ptr(), self._mse_ws.numel(), _stream()), "cpd_mlp_mse")
        ws = self._workspace(B)
        _lib.check(L.cpd_mlp_backward(ctypes.byref(self.net), x.data_ptr(), dy.data_ptr(), ctypes.byref(self.grads),
                                      B, ws.data_ptr(), ws.numel(), _stream()), "cpd_mlp_backward")
        self.adam.lr = float(lr)
        _lib.check(L.cpd_mlp_adam_step(ctypes.byref(self.net), ctypes.byref(self.grads), ctypes.byref(self.adam),
                                       _stream()), "cpd_mlp_adam_step")
        return self._loss


def core_feature(S):
    """(x, scale): the core flattened and normalised to unit norm, and its norm."""
    nrm = float(torch.linalg.vector_norm(S))
    return (S.reshape(-1) / nrm).to(torch.float32), nrm


def factor_target(W, lam, scale):
    """Flattened balanced factors (modes stacked, each core_dim x R row-major) scaled by scale^{-1/3}."""
    c = lam.clamp(min=0.0) ** (1.0 / 3.0)
    return torch.cat([(w * c[None, :]).reshape(-1) for w in W]).to(torch.float32) / scale ** (1.0 / 3.0)


def factors_from_output(y, core, R, scale):
    """Inverse of factor_target: the three core_dims[l] x R initial factors (FP64)."""
    y = y.to(torch.float64) * scale ** (1.0 / 3.0)
    out, o = [], 0
    for d in core:
        out.append(y[o:o + d * R].reshape(d, R).contiguous())
        o += d * R
    return out


def planted_device(dims, R, gen, device="cuda"):
    """Noiseless planted tensor with N(0,1) factors, formed on the device (input generation)."""
    F = [torch.randn((d, R), generator=gen, dtype=torch.float64, device="cpu").to(device) for d in dims]
    KR = (F[1][:, None, :] * F[2][None, :, :]).reshape(dims[1] * dims[2], R)
    return (F[0] @ KR.T).reshape(dims).contiguous()


def make_dataset(n, seed, dims=(100, 100, 100), R=8, core=(16, 16, 16), chunk=512, device="cuda", progress=None):
    """n training pairs (x, t) from planted tensors: core of cpd_compress with fixed core dims, target
    the batched solver's CPD of that core (pairs whose solve did not reach rel. err 1e-6 are dropped).
    progress(done, n) is called after each chunk.  Returns (X, T, kept)."""
    gen = torch.Generator(device="cpu").manual_seed(int(seed))
    pc = params(core_dims=core)
    X, Tt = [], []
    done = 0
    while done < n:
        m = min(chunk, n - done)
        cores = []
        for _ in range(m):
            Td = planted_device(dims, R, gen, device)
            _, _, S, _ = compress(Td, R, pc)
            cores.append(S.reshape(core))
        scales = torch.stack([torch.linalg.vector_norm(S) for S in cores]).cpu().tolist()
        X.extend([(S.reshape(-1) / sc).to(torch.float32) for S, sc in zip(cores, scales)])
        b = Batch(cores, [R] * m, params(seed=seed * 7919 + done), graph=False)
        infos = b.run()
        for j in range(m):
            Tt.append(factor_target(b.W[j], b.lam[j], scales[j]) if infos[j]["rel_err_full"] < 1e-6 else None)
        b.close()
        done += m
        if progress is not None:
            progress(done, n)
    keep = [i for i, t in enumerate(Tt) if t is not None]
    X = torch.stack([X[i] for i in keep])
    T = torch.stack([Tt[i] for i in keep])
    return X, T, len(keep)


def train(X, T, sizes=None, epochs=10, batch=512, lr=1e-3, seed=0, progress=None):
    """Adam on the squared error over the shuffled training set; returns (network, loss history).
    progress(epoch, loss) is called after each epoch."""
    sizes = sizes or [X.shape[1], 1024, 1024, T.shape[1]]
    net = MLP(sizes, seed=seed, device=X.device)
    g = torch.Generator(device="cpu").manual_seed(int(seed) + 1)
    hist = []
    n = X.shape[0]
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        tot = 0.0
        nb = 0
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            loss = net.train_step(X[idx], T[idx], lr)
            tot += float(loss.item()) if (i // batch) % 16 == 0 else 0.0
            nb += 1 if (i // batch) % 16 == 0 else 0
        hist.append(tot / max(nb, 1))
        if progress is not None:
            progress(ep, hist[-1])
    return net, hist


def evaluate(net, n_test, seed, dims=(100, 100, 100), R=8, core=(16, 16, 16), maxiter=200, progress=None):
    """Solves n_test new planted tensors from the starting points
      learned  - the network's prediction for the compressed core,
      fallback - the prediction unless the MLSVD-energy point has a smaller core residual
                 (the dGN residual judges the network; the MLSVD point is the fallback),
      mlsvd    - the MLSVD-energy point (ch.4 "Initialization"),
      random   - N(0,1) factors,
    and records per solve: first iteration with core rel. error below 1e-6 (0 if none), iterations
    run, wall time of the whole cpd_solve (compression included), final and initial core error."""
    import time
    from . import residual_norm2, solve, DgnState
    gen = torch.Generator(device="cpu").manual_seed(int(seed))
    out = {"learned": [], "fallback": [], "mlsvd": [], "random": []}
    for i in range(n_test):
        Td = planted_device(dims, R, gen, net.device)
        _, _, S, _ = compress(Td, R, params(core_dims=core))
        S3 = S.reshape(core).contiguous()
        x, s = core_feature(S3)
        W_l = factors_from_output(net.forward(x[None, :])[0], core, R, s)
        st = DgnState(S3, R, params(core_dims=core, init="mlsvd"))
        W_m = [w.clone() for w in st.factors()]
        W_r = [torch.randn((d, R), generator=gen, dtype=torch.float64).to(net.device) for d in core]
        e = {k: float(residual_norm2(S3, W)[0]) ** 0.5 / s for k, W in (("learned", W_l), ("mlsvd", W_m), ("random", W_r))}
        use_l = e["learned"] <= e["mlsvd"]
        runs = [("learned", W_l, e["learned"]), ("fallback", W_l if use_l else W_m, min(e["learned"], e["mlsvd"])),
                ("mlsvd", W_m, e["mlsvd"]), ("random", W_r, e["random"])]
        for name, W0, e0 in runs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = solve(Td, R, params(core_dims=core, init="given", maxiter=maxiter), W0=W0)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            inf = r["info"]
            out[name].append((max(inf["tol_iter"], 0), inf["iters"], dt, inf["rel_err_core"], e0))
        if progress is not None and (i + 1) % 100 == 0:
            progress(i + 1, n_test)
    return out


def summarize(results):
    """Per starting point: fraction reaching 1e-6, median iterations and time to 1e-6 over those,
    median initial core error."""
    import statistics
    summ = {}
    for name, rows in results.items():
        ok = [r for r in rows if r[0] > 0]
        summ[name] = {"reached_1e-6": len(ok) / max(len(rows), 1),
                      "median_iters_to_1e-6": statistics.median([r[0] for r in ok]) if ok else None,
                      "median_s_to_1e-6": statistics.median([r[2] for r in ok]) if ok else None,
                      "median_initial_core_err": statistics.median([r[4] for r in rows]) if rows else None}
    return summ


if __name__ == "__main__":
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser(description="train and evaluate the learned starting point")
    ap.add_argument("--n-train", type=int, default=100000)
    ap.add_argument("--n-test", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch", type=int, default=256)
    a = ap.parse_args()

    def say(*args):
        print(*args, flush=True)

    t0 = time.perf_counter()
    X, T, kept = make_dataset(a.n_train, seed=0, progress=lambda d, n: say(f"data {d}/{n}"))
    t1 = time.perf_counter()
    net, hist = train(X, T, epochs=a.epochs, batch=a.batch, progress=lambda e, l: say(f"epoch {e} loss {l:.5f}"))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    res = evaluate(net, a.n_test, seed=1, progress=lambda d, n: say(f"eval {d}/{n}"))
    print(json.dumps({"n_train": a.n_train, "kept": kept, "data_s": t1 - t0, "train_s": t2 - t1,
                      "loss": hist, "eval": summarize(res)}), flush=True)
