"""The allocation-free fused residual (cpd_residual_norm2_noalloc) against the workspace entry point
cpd_residual_norm2 and the FP64 oracle, through the C ABI.  Both entry points run the same kernels
with the same fixed grid and summation order, so their results must be bit-identical; against the
oracle the bound is the FP64 rounding of the summation (relative 1e-12)."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import dgn as odgn

pytestmark = pytest.mark.gpu


def _call(noalloc, T, Ws, out):
    from paper_2110_05997_amd import _lib
    L = _lib.lib()
    dims = (ctypes.c_int64 * 3)(*T.shape)
    dt = {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2}[T.dtype]
    Wp = (ctypes.c_void_p * 3)(*[w.data_ptr() for w in Ws])
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    R = Ws[0].shape[1]
    if noalloc:
        return L.cpd_residual_norm2_noalloc(T.data_ptr(), dt, dims, Wp, R, out.data_ptr(), s)
    ws = torch.empty(L.cpd_residual_workspace_bytes(dims), dtype=torch.uint8, device="cuda")
    st = L.cpd_residual_norm2(T.data_ptr(), dt, dims, Wp, R, out.data_ptr(), ws.data_ptr(), ws.numel(), s)
    torch.cuda.synchronize()
    return st


def test_noalloc_residual_matches_workspace_entry_point():
    # two calls in a row, the second on a smaller input (the scratch keeps the first call's partials)
    for dims, R, dtype, seed in [((150, 90, 70), 9, torch.float32, 0), ((33, 20, 17), 4, torch.float64, 1)]:
        print("noalloc residual", dims, R, dtype, flush=True)
        rng = np.random.default_rng(seed)
        Fs = [rng.standard_normal((d, R)) for d in dims]
        T = torch.as_tensor(rng.standard_normal(dims)).to(device="cuda", dtype=dtype).contiguous()
        Ws = [torch.as_tensor(F, device="cuda") for F in Fs]
        a = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        b = torch.full((1,), -2.0, dtype=torch.float64, device="cuda")
        assert _call(True, T, Ws, a) == 0
        torch.cuda.synchronize()
        assert _call(False, T, Ws, b) == 0
        va, vb = float(a.item()), float(b.item())
        assert va == vb, (va, vb)
        f = odgn.residual(T.double().cpu().numpy(), Fs)
        ref = float(np.sum(f * f))
        assert abs(va - ref) <= 1e-12 * ref, (va, ref)


def test_noalloc_residual_rejects_bad_arguments():
    T = torch.ones((4, 5, 6), dtype=torch.float64, device="cuda")
    Ws = [torch.ones((d, 65), dtype=torch.float64, device="cuda") for d in (4, 5, 6)]
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert _call(True, T, Ws, out) == -1          # R = 65 > 64: CPD_E_INVALID, nothing launched
    torch.cuda.synchronize()
    assert float(out.item()) == 0.0
