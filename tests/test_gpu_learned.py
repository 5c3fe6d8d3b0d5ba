"""Learned starting point, end to end on the GPU (an extension: the thesis has no learned part, so
its parity is unpinned by the thesis; the inference call is checked against the FP64 network of
oracle/mlp.py and the oracle's dGN).  Training pairs come from the library: planted 100^3 rank-8
tensors compressed to a fixed 16^3 core, with the batched solver's CPD of each core as target.
The network is trained by the library's MLP kernels and judged by the dGN on new tensors."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import dgn as odgn
from oracle import mlp as omlp
from oracle import multilinear as ml

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


def small_net(core, R, seed):
    """A library network whose weights are the oracle's He-normal draw rounded to FP32 (the oracle
    sees the same rounded values)."""
    from paper_2110_05997_amd import learned as lr
    sizes = [int(np.prod(core)), 48, 40, sum(core) * R]
    Ws, bs = omlp.init_params(sizes, seed=seed)
    rng = np.random.default_rng(seed)
    bs = [rng.standard_normal(b.shape) * 0.1 for b in bs]
    net = lr.MLP(sizes, seed=0)
    for l in range(3):
        net.W[l].copy_(torch.as_tensor(Ws[l], dtype=torch.float32))
        net.b[l].copy_(torch.as_tensor(bs[l], dtype=torch.float32))
    Ws = [w.double().cpu().numpy() for w in net.W]
    bs = [b.double().cpu().numpy() for b in net.b]
    return net, Ws, bs


def oracle_start(Ws, bs, S, R):
    """x = S / ||S||, y = network(x), W = y ||S||^{1/3}, split into the three factors."""
    s = float(np.sqrt(np.sum(S * S)))
    y, _ = omlp.forward(Ws, bs, (S.reshape(-1) / s)[None, :])
    y = y[0] * s ** (1.0 / 3.0)
    out, o = [], 0
    for d in S.shape:
        out.append(y[o:o + d * R].reshape(d, R))
        o += d * R
    return out


def test_features_and_targets_match_their_definition():
    from paper_2110_05997_amd import learned as lr
    rng = np.random.default_rng(3)
    core, R = (5, 4, 6), 3
    cores = [rng.standard_normal(core) * (i + 1) for i in range(3)]
    X, norms = lr.features([torch.as_tensor(c, device="cuda") for c in cores])
    for i, c in enumerate(cores):
        s = np.sqrt(np.sum(c * c))
        assert abs(norms[i].item() - s) <= 1e-14 * s
        np.testing.assert_allclose(X[i].cpu().double().numpy(), (c.reshape(-1) / s), rtol=0, atol=1e-7)
    W = [rng.standard_normal((d, R)) for d in core]
    lam = np.array([2.0, 0.5, -1.0])
    t = lr.factor_target([torch.as_tensor(w, device="cuda") for w in W], torch.as_tensor(lam, device="cuda"),
                         core, R, 8.0)
    ref = np.concatenate([(w * np.cbrt(np.maximum(lam, 0.0))[None, :]).reshape(-1) for w in W]) / 2.0
    np.testing.assert_allclose(t.cpu().double().numpy(), ref, rtol=1e-6, atol=1e-7)


def test_learned_start_matches_oracle_network():
    from paper_2110_05997_amd import learned as lr
    core, R = (6, 5, 4), 2
    net, Ws, bs = small_net(core, R, 11)
    S = synth.planted(core, R, seed=4, noise_rel=1e-2)[0]
    W, chosen, errs = lr.learned_start(net, torch.as_tensor(S, device="cuda"), R)
    assert chosen == 0 and errs == (0.0, 0.0)
    Wo = oracle_start(Ws, bs, S, R)
    for l in range(3):
        got = W[l].cpu().numpy()
        # FP32 network: relative 1e-5 of the largest entry
        assert np.max(np.abs(got - Wo[l])) <= 1e-5 * np.max(np.abs(Wo[l])), l


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_learned_start_judge_matches_oracle(seed):
    """judge_iters dGN iterations from the network's start and from a given fallback start: the
    errors after them match the oracle's runs from the same starts, and the choice is the smaller
    error (where the two differ by more than the FP32 network's perturbation can move them)."""
    from paper_2110_05997_amd import learned as lr
    from paper_2110_05997_amd import params
    core, R, k = (6, 5, 4), 2, 3
    net, Ws, bs = small_net(core, R, 20 + seed)
    S = synth.planted(core, R, seed=seed, noise_rel=1e-3)[0]
    Wf = synth.init_factors(core, R, seed)
    U = synth.cg_uniforms(k, seed)
    p = params(maxiter=k, cg_uniforms=U)
    W, chosen, errs = lr.learned_start(net, torch.as_tensor(S, device="cuda"), R, judge_iters=k, p=p,
                                       W_fallback=[torch.as_tensor(w, device="cuda") for w in Wf])
    e = []
    for W0 in (oracle_start(Ws, bs, S, R), Wf):
        _, infos = odgn.run_dgn(S, W0, odgn.Params(maxiter=k), cg_uniforms=U)
        e.append(infos[-1]["rel_err"])
    log(seed, errs, e, chosen)
    for a, b in zip(errs, e):
        assert abs(a - b) <= 1e-3 * b
    if abs(e[0] - e[1]) > 1e-2 * max(e):
        assert chosen == (0 if e[0] <= e[1] else 1)
    if chosen == 0:
        ref = [w.cpu().numpy() for w in lr.learned_start(net, torch.as_tensor(S, device="cuda"), R)[0]]
    else:
        ref = Wf
    for l in range(3):
        np.testing.assert_array_equal(W[l].cpu().numpy(), ref[l])
    # a margin above the ratio of the two errors keeps the network's start
    _, kept, _ = lr.learned_start(net, torch.as_tensor(S, device="cuda"), R, judge_iters=k, p=p,
                                  W_fallback=[torch.as_tensor(w, device="cuda") for w in Wf],
                                  margin=1.01 * max(1.0, e[0] / e[1]))
    assert kept == 0


def test_learned_init_trains_and_is_recorded():
    from paper_2110_05997_amd import learned as lr
    X, T, kept = lr.make_dataset(2048, seed=0)
    log("kept", kept, "of 2048")
    assert kept > 1024
    net, hist = lr.train(X, T, epochs=20, batch=256)
    log("loss", hist[0], "->", hist[-1])
    assert hist[-1] < 0.5 * hist[0]
    summ = lr.summarize(lr.evaluate(net, 64, seed=1))
    for k, v in summ.items():
        log(k, v)
    # what the network gains over the method without it: reach rate against the MLSVD-energy point
    # and against the library's default N(0,1) start (same CG caps), the latter within three of the
    # 64 test tensors (the network here is trained on 2048 pairs only)
    assert summ["learned"]["reached_1e-6"] >= summ["mlsvd"]["reached_1e-6"]
    assert summ["learned"]["reached_1e-6"] >= summ["random"]["reached_1e-6"] - 3 / 64
    for (k, m) in lr.JUDGES:
        assert 0.0 <= summ["judged k=%d margin=%g" % (k, m)]["network_kept"] <= 1.0
