"""FP64 CPU oracle for the Tensor Fox CPD hot path (test infrastructure only).

This package is the plain, slow, obviously-correct reference that the HIP
library is checked against.  It is test infrastructure: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (``paper_2110_05997_amd``) never imports it and
shares no code with it; the two meet only through the seeded input generators
in ``synth``.

Every function cites the passage of F. B. Diniz, "Tensor decompositions and
algorithms, with applications to tensor learning" (thesis, 2019;
arXiv:2110.05997) that it restates.  Section numbers are the thesis's own
(ch. 2 = multilinear algebra, ch. 3 = Gauss-Newton, ch. 4 = Tensor Fox,
App. A = conjugate gradient / preconditioning, App. B = special products).

Parity status of each part is listed in ``PARITY``; every entry is pinned by a
``-m "not gpu"`` test against something other than the oracle itself.
"""

PARITY = {
    "multilinear.unfold": "pinned: ch.2 Unfolding worked example (3x4x2 integer tensor)",
    "multilinear.mode_product": "pinned: ch.2 mode-1 product worked example",
    "multilinear.khatri_rao": "pinned: App.B special-products identity (A.B)^T(A.B)=A^TA*B^TB",
    "mlsvd.compress": "pinned: ch.4 warm-up Table 4.5 (27 truncation errors), core magnitudes, "
                      "MLSVD theorems (norm, all-orthogonality), L=2 reduces to matrix SVD",
    "mlsvd.smart_init": "pinned: ch.4 warm-up picks s111, s212, s122 with init error 0.0153",
    "dgn.gradient": "pinned: brute-force J^T f from Lemma partialf, finite differences of F",
    "dgn.jtj_v": "pinned: explicit dense Jacobian (Lemma kronecker), scale-indeterminacy null vector",
    "dgn.regularization": "pinned: off-diagonal domination bound of ch.4 Regularization section",
    "dgn.pcg": "pinned: CG finite termination equals a dense Cholesky solve (App. A)",
    "dgn.solve": "pinned: exact recovery of planted low-rank tensors; warm-up factor functions",
}
