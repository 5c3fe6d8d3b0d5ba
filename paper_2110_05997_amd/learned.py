"""Learned starting point for the dGN on a fixed-size compressed core (an extension: the thesis
initialises with random or MLSVD-energy points, ch.4 "Initialization").

A network maps the compressed core S (fixed core dims, e.g. 16^3), normalised to unit Frobenius
norm, to the R-term factors of S, balanced (equal column norms across modes) and scaled by
||S||^{-1/3} (cpd_learned_features / cpd_learned_target).  Training pairs come from the library
itself: each planted tensor is compressed by cpd_compress, and the factors of its core are the
batched solver's converged CPD of that core.  Inference is one call, cpd_learned_start: feature,
forward pass, rescaling and, optionally, the judge (a few dGN iterations from the network's start
and from the fallback N(0,1) start; the better one is kept).  All arithmetic runs in libcpd; this
module moves tensors, draws the planted inputs and calls the C ABI.
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


def features(cores):
    """(X, norms): FP32 features x = S / ||S|| of a list of equal-shape FP64 device cores, and their
    norms (cpd_learned_features)."""
    Sb = torch.stack([S.reshape(-1) for S in cores]).contiguous()
    n_items, n = Sb.shape
    X = torch.empty((n_items, n), dtype=torch.float32, device=Sb.device)
    norms = torch.empty(n_items, dtype=torch.float64, device=Sb.device)
    _lib.check(_lib.lib().cpd_learned_features(Sb.data_ptr(), n_items, n, X.data_ptr(), norms.data_ptr(), _stream()),
               "cpd_learned_features")
    return X, norms


def factor_target(W, lam, core, R, s_norm):
    """FP32 target of one core's CPD (unit-column factors W, weights lam) with core norm s_norm
    (cpd_learned_target)."""
    t = torch.empty(sum(core) * R, dtype=torch.float32, device=lam.device)
    Wp = (ctypes.c_void_p * 3)(*[w.contiguous().data_ptr() for w in W])
    _lib.check(_lib.lib().cpd_learned_target(Wp, lam.data_ptr(), (ctypes.c_int32 * 3)(*core), R, float(s_norm),
                                             t.data_ptr(), _stream()), "cpd_learned_target")
    return t


def learned_start(net, S, R, judge_iters=0, p=None, W_fallback=None, margin=1.0):
    """The starting point for the core S from the network (cpd_learned_start).  judge_iters > 0:
    judge_iters dGN iterations from the network's start and from the fallback (W_fallback, else the
    library's N(0,1) start for p.seed); the fallback is returned when the network's error after
    them exceeds margin times the fallback's.  Returns (W, chosen, judge_err) with W the three
    core_dims[l] x R factors, chosen 0 (network) or 1 (fallback)."""
    L = _lib.lib()
    core = tuple(int(d) for d in S.shape)
    cd = (ctypes.c_int32 * 3)(*core)
    S = S.contiguous()
    p = p if p is not None else params()
    n = L.cpd_learned_start_workspace_bytes(ctypes.byref(net.net), cd, R, judge_iters)
    if n == 0:
        raise ValueError("learned_start: the network does not map this core size and rank")
    ws = torch.empty(n, dtype=torch.uint8, device=S.device)
    W = torch.empty(sum(core) * R, dtype=torch.float64, device=S.device)
    wf = None
    if W_fallback is not None:
        wf = torch.cat([w.reshape(-1) for w in W_fallback]).to(device=S.device, dtype=torch.float64).contiguous()
    chosen = ctypes.c_int32()
    errs = (ctypes.c_double * 2)()
    _lib.check(L.cpd_learned_start(ctypes.byref(net.net), S.data_ptr(), cd, R, judge_iters, float(margin),
                                   ctypes.byref(p),
                                   wf.data_ptr() if wf is not None else None, W.data_ptr(), ctypes.byref(chosen),
                                   errs, ws.data_ptr(), n, _stream()), "cpd_learned_start")
    out, o = [], 0
    for d in core:
        out.append(W[o:o + d * R].view(d, R))
        o += d * R
    return out, chosen.value, (errs[0], errs[1])


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
        Xc, norms = features(cores)
        scales = norms.cpu().tolist()
        X.extend(list(Xc))
        b = Batch(cores, [R] * m, params(seed=seed * 7919 + done), graph=False)
        infos = b.run()
        for j in range(m):
            ok = infos[j]["rel_err_full"] < 1e-6 and scales[j] > 0.0
            Tt.append(factor_target(b.W[j], b.lam[j], core, R, scales[j]) if ok else None)
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


JUDGES = ((3, 1.0), (3, 2.0), (10, 1.0), (10, 2.0))   # (dGN iterations, margin) of the judge rules


def evaluate(net, n_test, seed, dims=(100, 100, 100), R=8, core=(16, 16, 16), maxiter=200, progress=None):
    """Solves n_test new planted tensors from the starting points
      learned - the network's start (cpd_learned_start without the judge),
      random  - the library's N(0,1) start (cpd_solve's default for the same seed),
      mlsvd   - the MLSVD-energy point (ch.4 "Initialization"),
    all with the same CG-cap stream (params seed), and records per solve: the first iteration with
    core rel. error below 1e-6 (0 if none), iterations run, the device time from the solve's first
    kernel to that iteration (in-kernel clock, compression included; -1 if none) and the device
    time of the start's own inference call (cuda events; 0 for the plain starts).
    For every judge rule (k, margin) in JUDGES, cpd_learned_start with the judge is run too and its
    choice recorded in results["judge"][(k, margin)]: the judged start is bit-identical to the
    network's or to the random start, so its solve is the corresponding row's."""
    from . import solve
    gen = torch.Generator(device="cpu").manual_seed(int(seed))
    out = {"learned": [], "random": [], "mlsvd": [], "judge": {j: [] for j in JUDGES}}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for i in range(n_test):
        Td = planted_device(dims, R, gen, net.device)
        _, _, S, _ = compress(Td, R, params(core_dims=core))
        S3 = S.reshape(core).contiguous()
        sd = int(seed) * 1000003 + i
        pc = params(core_dims=core, seed=sd)
        ev0.record()
        W_l, _, _ = learned_start(net, S3, R, p=pc)
        ev1.record()
        ev1.synchronize()
        t_l = ev0.elapsed_time(ev1)
        for (k, m) in JUDGES:
            ev0.record()
            _, chosen, errs = learned_start(net, S3, R, judge_iters=k, p=pc, margin=m)
            ev1.record()
            ev1.synchronize()
            out["judge"][(k, m)].append((chosen, errs[0], errs[1], ev0.elapsed_time(ev1)))
        for name, W0, init, t_ms in (("learned", W_l, "given", t_l), ("random", None, "random", 0.0),
                                     ("mlsvd", None, "mlsvd", 0.0)):
            r = solve(Td, R, params(core_dims=core, init=init, maxiter=maxiter, seed=sd), W0=W0)
            inf = r["info"]
            out[name].append((max(inf["tol_iter"], 0), inf["iters"], inf["time_to_tol_ns"], t_ms))
        if progress is not None and (i + 1) % 100 == 0:
            progress(i + 1, n_test)
    return out


def summarize(results):
    """Per starting point: fraction reaching 1e-6; over those, the median iterations and device ms
    to 1e-6 of the solve, and the median total with the start's inference.  Per judge rule the
    same figures for the start it picks, and the share of network starts it keeps."""
    import statistics

    def stats(rows):
        ok = [r for r in rows if r[0] > 0]
        return {"reached_1e-6": len(ok) / max(len(rows), 1),
                "median_iters_to_1e-6": statistics.median([r[0] for r in ok]) if ok else None,
                "median_solve_ms_to_1e-6": statistics.median([r[2] * 1e-6 for r in ok]) if ok else None,
                "median_total_ms_to_1e-6": statistics.median([r[2] * 1e-6 + r[3] for r in ok]) if ok else None,
                "median_start_ms": statistics.median([r[3] for r in rows]) if rows else None}

    summ = {name: stats(results[name]) for name in ("learned", "random", "mlsvd")}
    for (k, m), picks in results["judge"].items():
        rows = [(results["learned"][i] if c == 0 else results["random"][i])[:3] + (t,)
                for i, (c, _, _, t) in enumerate(picks)]
        st = stats(rows)
        st["network_kept"] = sum(1 for c, _, _, _ in picks if c == 0) / max(len(picks), 1)
        summ["judged k=%d margin=%g" % (k, m)] = st
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
