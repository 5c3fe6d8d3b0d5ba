"""Full-size parity of the 600^3 workload (R = 50, N(0,1) factors, 60 dB; FP32 tensor) against the
FP64 oracle's solve of the same input, start point and CG caps.  The oracle's results are stored,
sampled, by tests/golden/make_config3.py (oracle and synth only; three SVDs of 600 x 360000
unfoldings take minutes on the host).

* FP64 Grams (cpd_solve): singular values to 1e-10 relative, entries of U^(l) and of the core S to
  1e-8 / 1e-10 of the largest (sign-canonical bases; eigenvectors of the Gram vs the SVD), the
  reconstruction T^ at 400 sampled positions to 1e-6 of the largest sampled entry, the same stop
  reason and the iteration count within one.
* BF16 Grams (cpd_solve_mixed): the bases come from a BF16 Gram, and the dGN's end point at R = 50
  depends chaotically on such perturbations, so the distance to the oracle is reported, not bounded
  (see the test's docstring).
"""
import os

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config3_oracle.txt")
R, INIT_SEED, CG_SEED = 50, 2, 0


def log(*a):
    print(*a, flush=True)


def read_golden():
    g = {"U": [], "S": [], "That": [], "sigma": {}}
    with open(GOLD) as fh:
        for line in fh:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "summary":
                kv = dict(zip(t[1::2], t[2::2]))
                g["core"] = (int(t[2]), int(t[3]), int(t[4]))
                g["iters"] = int(kv["iters"])
                g["stop"] = int(kv["stop"])
                g["rel_err_full"] = float(kv["rel_err_full"])
                g["rel_err_core"] = float(kv["rel_err_core"])
            elif t[0] == "sigma":
                g["sigma"][int(t[1])] = np.array([float(v) for v in t[2:]])
            elif t[0] == "lambda":
                g["lambda"] = np.array([float(v) for v in t[1:]])
            elif t[0] == "U":
                g["U"].append((int(t[1]), int(t[2]), int(t[3]), float(t[4])))
            elif t[0] == "S":
                g["S"].append((int(t[1]), int(t[2]), int(t[3]), float(t[4])))
            elif t[0] == "That":
                g["That"].append((int(t[1]), int(t[2]), int(t[3]), float(t[4])))
    return g


@pytest.fixture(scope="module")
def c3():
    import paper_2110_05997_amd as cp
    log("config3 inputs")
    T, _, _ = synth.config3()
    Td = torch.as_tensor(T).to("cuda")
    del T
    W0 = cp.flat_w0([torch.as_tensor(w).to("cuda") for w in synth.init_factors((R, R, R), R, INIT_SEED)], Td.device)
    p = cp.params(cg_uniforms=synth.cg_uniforms(200, CG_SEED))
    return cp, Td, W0, p, read_golden()


def that_at(res, idx):
    W = [w.cpu().numpy() for w in res["W"]]
    lam = res["lam"].cpu().numpy()
    return np.array([float(np.sum(lam * W[0][i] * W[1][j] * W[2][k])) for i, j, k in idx])


def test_config3_fp64_grams_match_oracle(c3):
    cp, Td, W0, p, g = c3
    log("config3 FP64 Grams: compression")
    Us, sg, S, core = cp.compress(Td, R, p)
    assert tuple(core) == g["core"]
    for l in range(3):
        s = sg[l].cpu().numpy()
        assert np.max(np.abs(s - g["sigma"][l]) / g["sigma"][l][0]) < 1e-10, l
    Uh = [u.cpu().numpy() for u in Us]
    umax = max(abs(v) for *_, v in g["U"])
    du = max(abs(Uh[l][i, r] - v) for l, i, r, v in g["U"])
    Sh = S.cpu().numpy()
    smax = max(abs(v) for *_, v in g["S"])
    ds = max(abs(Sh[a, b, c] - v) for a, b, c, v in g["S"])
    log("U max diff", du, "S max diff / max", ds / smax)
    assert du < 1e-8 * umax
    assert ds < 1e-10 * smax
    log("config3 FP64 Grams: solve")
    res = cp.solve(Td, R, p, W0=W0)
    info = res["info"]
    idx = [(i, j, k) for i, j, k, _ in g["That"]]
    ref = np.array([v for *_, v in g["That"]])
    d = np.max(np.abs(that_at(res, idx) - ref)) / np.max(np.abs(ref))
    log("solve", info, "oracle iters", g["iters"], "stop", g["stop"], "That sampled max diff", d)
    assert info["stop_reason"] == g["stop"]
    assert abs(info["iters"] - g["iters"]) <= 1
    assert d < 1e-6
    assert abs(info["rel_err_full"] - g["rel_err_full"]) <= 1e-6 * g["rel_err_full"]
    lam = res["lam"].cpu().numpy()
    assert np.max(np.abs(lam - g["lambda"])) < 1e-6 * g["lambda"][0]


def test_config3_bf16_grams_error_vs_oracle(c3):
    """The BF16-Gram solve from the same start.  At R = 50 the dGN's path is chaotic (from eleven of
    twelve N(0,1) starts the oracle itself stops in a swamp near 0.14), so the BF16 perturbation of
    the bases can send it to another end point: its distance to the oracle's reconstruction is
    printed (and reported by the benchmark), and the result is checked for validity: a stopping rule
    fired, finite errors no better than the noise allows, and a full error either at the noise floor
    or at a swamp level the oracle's own starts also reach (< 0.2)."""
    cp, Td, W0, p, g = c3
    log("config3 BF16 Grams")
    Tlo = Td.to(torch.bfloat16).contiguous()
    res = cp.solve_mixed(Tlo, Td, R, p, W0=W0)
    info = res["info"]
    idx = [(i, j, k) for i, j, k, _ in g["That"]]
    ref = np.array([v for *_, v in g["That"]])
    d = np.max(np.abs(that_at(res, idx) - ref)) / np.max(np.abs(ref))
    floor = 10 ** (-60 / 20)
    log("mixed", info, "That sampled max diff vs oracle", d, "oracle rel_err_full", g["rel_err_full"])
    assert tuple(info["core_dims"]) == g["core"]
    assert 1 <= info["stop_reason"] <= 8
    assert np.isfinite(d) and np.isfinite(info["rel_err_full"])
    assert 0.99 * floor < info["rel_err_full"] < 0.2
