"""GPU parity of the tensor-train route (cpd_solve_tt; ch.4 "Tensor train and the CPD") against
the oracle's Alg. CPD-TTD on the same seeded tensors, start points and CG caps.  The stopping
tolerance is 1e-10, below the 1e-6 noise, so the inner CPDs end on the improvement rule at their
minimisers instead of on an error test within rounding of the threshold (which could move the
stopping iteration by one between the two sides).  The reconstructions agree to 1e-6 relative (the
accuracy target of the path) and the full errors to within their distance (triangle inequality);
orders 4 to 6 exercise the CPD of the second core and one to three Bi-CPDs."""
import numpy as np
import pytest
import torch

import synth
from oracle import dgn as odgn
from oracle import tt as ott

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("dims,R,seed,dtype", [((8, 9, 10, 7), 3, 5, np.float64),
                                               ((6, 7, 5, 8, 6), 4, 6, np.float64),
                                               ((10, 10, 10, 10, 10, 10), 3, 8, np.float32)])
def test_cpd_tt_matches_oracle(dims, R, seed, dtype):
    import paper_2110_05997_amd as cp
    log("cpd tt", dims, R, dtype.__name__)
    T, _ = synth.planted_order_L(dims, R, seed=seed, noise_rel=1e-6, dtype=dtype)
    Td = torch.as_tensor(T).to("cuda")
    Th = Td.double().cpu().numpy()
    U = synth.cg_uniforms(200, seed)
    W0 = synth.tt_init_factors(dims, R, seed)
    Ws, _, logs = ott.cpd_ttd(Th, R, odgn.Params(tol=1e-10), W0=W0, cg_uniforms=U)
    ref = ott.cpd_full_L(Ws)
    res = cp.solve_tt(Td, R, cp.params(cg_uniforms=U, tol=1e-10), W0=W0)
    W = [w.cpu().numpy() for w in res["W"]]
    lam = res["lam"].cpu().numpy()
    got = ott.cpd_full_L([W[0] * lam[None, :]] + W[1:])
    d = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    e_ref = np.linalg.norm(Th - ref) / np.linalg.norm(Th)
    log(res["info"], "oracle logs", logs, "That diff", d, "oracle err", e_ref)
    assert d < 1e-6
    assert abs(res["info"]["rel_err_full"] - e_ref) <= 1.01 * d * np.linalg.norm(ref) / np.linalg.norm(Th) + 1e-12
    for w in W:
        np.testing.assert_allclose(np.linalg.norm(w, axis=0), 1.0, rtol=1e-12)
    assert np.all(lam >= 0) and np.all(np.diff(lam) <= 0)


def test_cpd_tt_rejects_unsupported_shapes():
    import paper_2110_05997_amd as cp
    T = torch.ones((4, 5, 6), dtype=torch.float64, device="cuda")
    with pytest.raises(Exception):
        cp.solve_tt(T, 2)                              # order 3: use cpd_solve
    T4 = torch.ones((2, 5, 6, 7), dtype=torch.float64, device="cuda")
    with pytest.raises(Exception):
        cp.solve_tt(T4, 3)                             # R > I_1: a TT-rank cannot reach R
