"""GPU parity of the learned-initialisation network kernels (FP32 matrix cores) against the FP64
oracle of oracle/mlp.py.  Tolerance: FP32 GEMMs over K <= 4096 terms carry a relative error of about
sqrt(K) * 2^-24 < 1e-5 of the largest entry; the bound used is 1e-4.  The Adam update is compared
through the step it takes (p_new - p) on the kernels' own gradients; its FP32 evaluation loses
about 2^-24 |p| / lr relative."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def lib():
    from paper_2110_05997_amd import _lib
    return _lib


def log(*a):
    print(*a, flush=True)


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


# B <= 8 takes the small-batch (split-K matrix-vector) forward, larger batches the tiled GEMM
@pytest.mark.parametrize("dims,B", [([37, 70, 33, 19], 45), ([4096, 1024, 1024, 384], 256),
                                    ([37, 70, 33, 19], 5), ([4096, 1024, 1024, 384], 1),
                                    ([4096, 1024, 1024, 384], 8)])
def test_mlp_forward_backward_adam_match_oracle(dims, B):
    log("mlp", dims, B)
    L = lib()
    rng = np.random.default_rng(4)
    Ws, bs = omlp.init_params(dims, seed=3)
    bs = [rng.standard_normal(b.shape) * 0.1 for b in bs]
    x = rng.standard_normal((B, dims[0]))
    t = rng.standard_normal((B, dims[3]))
    f32 = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float32)).cuda().contiguous()
    Wd, bd, xd, td = [f32(w) for w in Ws], [f32(b) for b in bs], f32(x), f32(t)
    # the oracle sees the same FP32-rounded values
    Ws = [w.double().cpu().numpy() for w in Wd]
    bs = [b.double().cpu().numpy() for b in bd]
    x, t = xd.double().cpu().numpy(), td.double().cpu().numpy()
    net = L.Mlp(dims[0], dims[1], dims[2], dims[3], (ctypes.c_void_p * 3)(*[w.data_ptr() for w in Wd]),
                (ctypes.c_void_p * 3)(*[b.data_ptr() for b in bd]))
    gW = [torch.zeros_like(w) for w in Wd]
    gb = [torch.zeros_like(b) for b in bd]
    grads = L.MlpGrads((ctypes.c_void_p * 3)(*[g.data_ptr() for g in gW]), (ctypes.c_void_p * 3)(*[g.data_ptr() for g in gb]))
    mW, vW = [torch.zeros_like(w) for w in Wd], [torch.zeros_like(w) for w in Wd]
    mb, vb = [torch.zeros_like(b) for b in bd], [torch.zeros_like(b) for b in bd]
    P = lambda ts: (ctypes.c_void_p * 3)(*[q.data_ptr() for q in ts])
    adam = L.Adam(1e-3, 0.9, 0.999, 1e-8, 0, P(mW), P(mb), P(vW), P(vb))
    lb = L.lib()
    ws = torch.empty(lb.cpd_mlp_workspace_bytes(ctypes.byref(net), B), dtype=torch.uint8, device="cuda")
    ws2 = torch.empty(8192, dtype=torch.uint8, device="cuda")
    y = torch.empty((B, dims[3]), dtype=torch.float32, device="cuda")
    dy = torch.empty_like(y)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L.check(lb.cpd_mlp_forward(ctypes.byref(net), xd.data_ptr(), y.data_ptr(), B, ws.data_ptr(), ws.numel(), s), "fwd")
    L.check(lb.cpd_mlp_mse(y.data_ptr(), td.data_ptr(), y.numel(), dy.data_ptr(), loss.data_ptr(), ws2.data_ptr(),
                           ws2.numel(), s), "mse")
    L.check(lb.cpd_mlp_backward(ctypes.byref(net), xd.data_ptr(), dy.data_ptr(), ctypes.byref(grads), B,
                                ws.data_ptr(), ws.numel(), s), "bwd")
    W_before = [w.clone() for w in Wd]
    b_before = [b.clone() for b in bd]
    net_before = L.Mlp(dims[0], dims[1], dims[2], dims[3], P(W_before), P(b_before))
    L.check(lb.cpd_mlp_adam_step(ctypes.byref(net), ctypes.byref(grads), ctypes.byref(adam), s), "adam")
    torch.cuda.synchronize()
    yo, cache = omlp.forward(Ws, bs, x)
    lo, dyo = omlp.mse_loss(yo, t)
    # The ReLU masks are decisions taken in floating point: a pre-activation within rounding of 0
    # may have different signs in FP32 and FP64. The oracle backward therefore takes the kernel's
    # masks. The hidden activations are the first two regions of the workspace, 256-byte aligned.
    off2 = (B * dims[1] * 4 + 255) // 256 * 256
    H1 = ws[:B * dims[1] * 4].view(torch.float32).reshape(B, dims[1]).double().cpu().numpy()
    H2 = ws[off2:off2 + B * dims[2] * 4].view(torch.float32).reshape(B, dims[2]).double().cpu().numpy()
    acts, pre = cache
    masked = (acts, [np.where(H1 > 0, np.abs(pre[0]) + 1.0, 0.0), np.where(H2 > 0, np.abs(pre[1]) + 1.0, 0.0), pre[2]])
    flip1 = (H1 > 0) != (pre[0] > 0)
    flip2 = (H2 > 0) != (pre[1] > 0)
    flips = int(np.sum(flip1) + np.sum(flip2))
    log("relu decisions that differ between FP32 and FP64:", flips)
    # a decision can differ only where the FP64 pre-activation is within FP32 rounding of zero: at
    # most one hidden entry in 10^4
    assert flips <= 1e-4 * B * (dims[1] + dims[2]), flips
    dWo, dbo = omlp.backward(Ws, masked, dyo)
    # the oracle's own masks, on the rows where every decision agrees: the backward kernel is run
    # again on those rows only (same dy rows), and compared with the oracle's backward on them
    ok = ~(flip1.any(axis=1) | flip2.any(axis=1))
    assert ok.sum() >= B // 2
    rows = torch.as_tensor(np.nonzero(ok)[0], device="cuda")
    xk, dyk = xd[rows].contiguous(), dy[rows].contiguous()
    Bk = int(ok.sum())
    gWk = [torch.zeros_like(w) for w in Wd]
    gbk = [torch.zeros_like(b) for b in bd]
    gradsk = L.MlpGrads(P(gWk), P(gbk))
    wsk = torch.empty(lb.cpd_mlp_workspace_bytes(ctypes.byref(net_before), Bk), dtype=torch.uint8, device="cuda")
    yk = torch.empty((Bk, dims[3]), dtype=torch.float32, device="cuda")
    L.check(lb.cpd_mlp_forward(ctypes.byref(net_before), xk.data_ptr(), yk.data_ptr(), Bk, wsk.data_ptr(),
                               wsk.numel(), s), "fwd rows")
    L.check(lb.cpd_mlp_backward(ctypes.byref(net_before), xk.data_ptr(), dyk.data_ptr(), ctypes.byref(gradsk), Bk,
                                wsk.data_ptr(), wsk.numel(), s), "bwd rows")
    torch.cuda.synchronize()
    _, cache_k = omlp.forward(Ws, bs, x[ok])
    dWk, dbk = omlp.backward(Ws, cache_k, dyk.double().cpu().numpy())
    for l in range(3):
        assert relmax(gWk[l].double().cpu().numpy(), dWk[l]) < 1e-4, ("own masks", l)
        assert relmax(gbk[l].double().cpu().numpy(), dbk[l]) < 1e-4, ("own masks", l)
    assert relmax(y.double().cpu().numpy(), yo) < 1e-4
    assert abs(float(loss.item()) - lo) <= 1e-5 * lo
    for l in range(3):
        assert relmax(gW[l].double().cpu().numpy(), dWo[l]) < 1e-4, l
        assert relmax(gb[l].double().cpu().numpy(), dbo[l]) < 1e-4, l
        # Adam normalises every entry (the first step is about lr * sign(g)), so it is checked on the
        # gradients the kernels produced: the oracle update of those gradients
        g = gW[l].double().cpu().numpy()
        p_ref, _, _ = omlp.adam_step(Ws[l], g, np.zeros_like(Ws[l]), np.zeros_like(Ws[l]), 1)
        step = (Wd[l].double() - W_before[l].double()).cpu().numpy()
        assert relmax(step, p_ref - Ws[l]) < 1e-3, l
    assert adam.step == 1
