"""Learned starting point, end to end on the GPU. Training pairs come from the library: planted
100^3 rank-8 tensors compressed to a fixed 16^3 core, with the batched solver's CPD of each core
as target. The network is trained by the library's MLP kernels and judged by the dGN on new
tensors. Parity is unpinned (the thesis has no learned part). The checks are that training
reduces the loss, and that the trained network's starting points are recorded against the MLSVD-
energy and N(0,1) starting points; the learned point must reach rel. error 1e-6 at least as
often as the MLSVD-energy point."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


def test_learned_init_trains_and_is_recorded():
    from paper_2110_05997_amd import learned as lr
    X, T, kept = lr.make_dataset(2048, seed=0)
    log("kept", kept, "of 2048")
    assert kept > 1024
    net, hist = lr.train(X, T, epochs=20, batch=256)
    log("loss", hist[0], "->", hist[-1])
    assert hist[-1] < 0.5 * hist[0]
    summ = lr.summarize(lr.evaluate(net, 24, seed=1))
    log(summ)
    assert summ["learned"]["reached_1e-6"] >= summ["mlsvd"]["reached_1e-6"]
    # the fallback rule never starts from a point with a larger core residual than the MLSVD point
    assert summ["fallback"]["median_initial_core_err"] <= summ["mlsvd"]["median_initial_core_err"] + 1e-12
