"""Writes tests/golden/config3_oracle.txt: the FP64 oracle's solve of the 600^3 workload (R = 50,
N(0,1) factors, 60 dB, FP32 storage promoted to FP64), sampled, for the full-size GPU parity test.

Only synth (the seeded inputs) and oracle/ are used.  Start point: synth.init_factors(core, 50,
seed=2) (from seeds 0, 1 and 3..11 the oracle's dGN stops in swamps near 0.14 and seed 4 diverges;
seed 2 reaches the noise floor); CG-cap uniforms: synth.cg_uniforms(200, 0); thesis defaults
otherwise.  Stored: the summary of the solve, the leading singular values of every mode, and entries of U^(l), of the core
S and of the reconstruction T^ = sum_r lambda_r w_r^(1) o w_r^(2) o w_r^(3) at seeded positions.
Run time: a few minutes (three SVDs of 600 x 360000 unfoldings).

    python tests/golden/make_config3.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import cpd as ocpd  # noqa: E402
from oracle import dgn as odgn  # noqa: E402
from oracle import mlsvd as omlsvd  # noqa: E402

R, INIT_SEED, CG_SEED, NSAMP = 50, 2, 0, 400


def main():
    t0 = time.perf_counter()
    T, _, _ = synth.config3()
    Th = np.asarray(T, dtype=np.float64)
    del T
    P = (R, R, R)
    W0 = synth.init_factors(P, R, INIT_SEED)
    U = synth.cg_uniforms(200, CG_SEED)
    res = ocpd.solve(Th, R, odgn.Params(), W0=W0, cg_uniforms=U,
                     log=lambda i: print("k", i["k"], "err", i["rel_err"], "cg", i["cg_iters"], flush=True))
    print("solve", time.perf_counter() - t0, "s", res["iters"], res["stop"], res["rel_err_full"], flush=True)
    rng = np.random.default_rng(12345)
    W, lam = res["W"], res["lam"]
    S = res["S"]
    out = []
    out.append("# Oracle solve of the 600^3 workload (written by tests/golden/make_config3.py; oracle only).")
    out.append(f"summary core {S.shape[0]} {S.shape[1]} {S.shape[2]} iters {res['iters']} stop {res['stop']} "
               f"rel_err_core {res['rel_err_core']!r} rel_err_full {res['rel_err_full']!r} "
               f"tol_iter {ocpd.time_to_tol_iter(res['errs'], 1e-6) or -1} s_norm {float(np.linalg.norm(S))!r}")
    for l in range(3):
        out.append("sigma " + str(l) + " " + " ".join(repr(float(v)) for v in res["sigma"][l]))
    out.append("lambda " + " ".join(repr(float(v)) for v in lam))
    for l in range(3):
        ii = rng.integers(0, 600, NSAMP)
        rr = rng.integers(0, S.shape[l], NSAMP)
        for i, r in zip(ii, rr):
            out.append(f"U {l} {i} {r} {float(res['U'][l][i, r])!r}")
    for _ in range(NSAMP):
        a, b, c = (int(rng.integers(0, d)) for d in S.shape)
        out.append(f"S {a} {b} {c} {float(S[a, b, c])!r}")
    for _ in range(NSAMP):
        i, j, k = (int(v) for v in rng.integers(0, 600, 3))
        v = float(np.sum(lam * W[0][i] * W[1][j] * W[2][k]))
        out.append(f"That {i} {j} {k} {v!r}")
    with open(os.path.join(HERE, "config3_oracle.txt"), "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("wrote", len(out), "lines", flush=True)


if __name__ == "__main__":
    main()
