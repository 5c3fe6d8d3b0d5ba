"""MI355X (gfx950) implementation of the Tensor Fox CPD hot path (thesis of F. B. Diniz, 2019):
truncated-MLSVD compression, damped Gauss-Newton with preconditioned CG on the core, and
uncompression.

The compute runs in ``lib/libcpd.so`` (HIP kernels behind the C ABI of ``include/cpd.h``); this
package only marshals arguments.  Tensors are ``torch`` CUDA (HIP) tensors; the work is enqueued
on ``torch.cuda.current_stream()``.
"""
import ctypes

import torch

from . import _lib
from ._lib import (CPD_BF16, CPD_F32, CPD_F64, CPD_INIT_GIVEN, CPD_INIT_MLSVD, CPD_INIT_RANDOM,
                   STOP_NAMES, CpdError, Params, SolveInfo, StepInfo)

__all__ = ["params", "gram", "eig_top", "compress", "DgnState", "solve", "flat_w0", "mttkrp", "residual_norm2",
           "jtj_v", "Batch", "solve_mixed", "CpdError", "STOP_NAMES"]

_DTYPES = {torch.float64: CPD_F64, torch.float32: CPD_F32, torch.bfloat16: CPD_BF16}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dims(T):
    return (ctypes.c_int64 * 3)(*T.shape)


def _dtype(T):
    if T.dtype not in _DTYPES:
        raise TypeError(f"unsupported dtype {T.dtype}")
    return _DTYPES[T.dtype]


def _check_tensor(T):
    if not (T.is_cuda and T.is_contiguous() and T.dim() == 3):
        raise ValueError("expected a contiguous 3-way tensor on the GPU")


def _ws(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def params(maxiter=200, tol=1e-6, mlsvd_tol=1e-6, init_damp=1.0, cg_tol=0.0, cg_fixed=0,
           cg_uniforms=None, seed=0, init="random", core_dims=None, compute_dtype=CPD_F64, st_mlsvd=False,
           refine_iters=0, precond="jacobi", drawback=False):
    """Build a cpd_params struct (defaults are the thesis's).  ``cg_uniforms`` (host floats) must
    outlive the call that uses the struct; it is kept on the returned object.  ``precond``:
    "jacobi" (diagonal) or "block" (block-Jacobi); ``drawback``: redo a step whose error jumps
    100-fold from the drawn-back point with a dogleg step."""
    p = Params()
    _lib.lib().cpd_default_params(ctypes.byref(p))
    p.maxiter, p.tol, p.mlsvd_tol, p.init_damp = int(maxiter), float(tol), float(mlsvd_tol), float(init_damp)
    p.cg_tol, p.cg_fixed, p.seed = float(cg_tol), int(cg_fixed), int(seed)
    p.init = {"random": CPD_INIT_RANDOM, "mlsvd": CPD_INIT_MLSVD, "given": CPD_INIT_GIVEN}[init]
    if core_dims is not None:
        p.core_dims = (ctypes.c_int32 * 3)(*core_dims)
    p.compute_dtype = int(compute_dtype)
    p.st_mlsvd = 1 if st_mlsvd else 0
    p.refine_iters = int(refine_iters)
    p.precond = {"jacobi": 0, "block": 1}[precond]
    p.drawback = 1 if drawback else 0
    if cg_uniforms is not None:
        arr = (ctypes.c_double * len(cg_uniforms))(*[float(u) for u in cg_uniforms])
        if len(cg_uniforms) < maxiter:
            raise ValueError("cg_uniforms needs maxiter entries")
        p.cg_uniforms = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
        p._keep = arr
    return p


def gram(T, mode, compute_dtype=CPD_F64):
    """G = T_(mode) T_(mode)^T in FP64."""
    _check_tensor(T)
    L = _lib.lib()
    dims = _dims(T)
    ws = _ws(L.cpd_gram_workspace_bytes(dims, mode), T.device)
    G = torch.empty((T.shape[mode], T.shape[mode]), dtype=torch.float64, device=T.device)
    _lib.check(L.cpd_gram(_ptr(T), _dtype(T), dims, mode, compute_dtype, _ptr(G), _ptr(ws), ws.numel(),
                          _stream()), "cpd_gram")
    return G


def eig_top(G, P):
    """Leading P eigenpairs (U n x P, lam P) of a symmetric FP64 matrix."""
    n = G.shape[0]
    L = _lib.lib()
    ws = _ws(L.cpd_eig_workspace_bytes(n, P), G.device)
    U = torch.empty((n, P), dtype=torch.float64, device=G.device)
    lam = torch.empty(P, dtype=torch.float64, device=G.device)
    _lib.check(L.cpd_eig_top(_ptr(G.contiguous()), n, P, _ptr(U), _ptr(lam), _ptr(ws), ws.numel(), _stream()),
               "cpd_eig_top")
    return U, lam


def compress(T, R, p=None):
    """Truncated MLSVD: returns (U list, sigma list, S, core_dims)."""
    _check_tensor(T)
    L = _lib.lib()
    if p is None:
        p = params()
    dims = _dims(T)
    fixed = all(p.core_dims[l] > 0 for l in range(3))
    P = [p.core_dims[l] if fixed else min(T.shape[l], R) for l in range(3)]
    ws = _ws(L.cpd_workspace_bytes(dims, R, ctypes.byref(p)), T.device)
    Uf = [torch.empty(T.shape[l] * P[l], dtype=torch.float64, device=T.device) for l in range(3)]
    sg = [torch.empty(P[l], dtype=torch.float64, device=T.device) for l in range(3)]
    S = torch.empty(P[0] * P[1] * P[2], dtype=torch.float64, device=T.device)
    core = (ctypes.c_int32 * 3)()
    _lib.check(L.cpd_compress(_ptr(T), _dtype(T), dims, R, ctypes.byref(p),
                              (ctypes.c_void_p * 3)(*[u.data_ptr() for u in Uf]),
                              (ctypes.c_void_p * 3)(*[s.data_ptr() for s in sg]), _ptr(S), core,
                              _ptr(ws), ws.numel(), _stream()), "cpd_compress")
    cd = tuple(int(c) for c in core)
    Us = [Uf[l][: T.shape[l] * cd[l]].view(T.shape[l], cd[l]) for l in range(3)]
    S = S[: cd[0] * cd[1] * cd[2]].view(*cd)
    return Us, sg, S, cd


class DgnState:
    """Device-resident dGN state for a core S (see cpd_state_init / cpd_dgn_step / cpd_dgn_run)."""

    def __init__(self, S, R, p=None, W0=None, t_norm2=0.0):
        L = _lib.lib()
        self.p = p if p is not None else params()
        self.S = S.contiguous()
        self.core = tuple(int(d) for d in S.shape)
        self.R = int(R)
        cd = (ctypes.c_int32 * 3)(*self.core)
        nbytes = L.cpd_state_bytes(cd, self.R, ctypes.byref(self.p))
        self.buf = torch.zeros(nbytes, dtype=torch.uint8, device=S.device)
        w0 = None
        if W0 is not None:
            w0 = torch.cat([w.reshape(-1) for w in W0]).to(device=S.device, dtype=torch.float64).contiguous()
        self._w0 = w0
        _lib.check(L.cpd_state_init(_ptr(self.buf), _ptr(self.S), cd, self.R, _ptr(w0), float(t_norm2),
                                    ctypes.byref(self.p), _stream()), "cpd_state_init")

    def step(self):
        info = StepInfo()
        _lib.check(_lib.lib().cpd_dgn_step(_ptr(self.buf), _ptr(self.S), ctypes.byref(self.p), ctypes.byref(info),
                                           _stream()), "cpd_dgn_step")
        return info.as_dict()

    def run(self):
        it, st = ctypes.c_int32(), ctypes.c_int32()
        log = (StepInfo * self.p.maxiter)()
        _lib.check(_lib.lib().cpd_dgn_run(_ptr(self.buf), _ptr(self.S), ctypes.byref(self.p), ctypes.byref(it),
                                          ctypes.byref(st), log, self.p.maxiter, _stream()), "cpd_dgn_run")
        return it.value, st.value, [log[i].as_dict() for i in range(it.value)]

    def set_factors(self, W):
        """Overwrite the state's current factors (three core_dims[l] x R matrices); the header
        (mu, residual, error history) is left as it is."""
        w = _flat_w0(W, self.S.device)
        if w.numel() != sum(self.core) * self.R:
            raise ValueError("set_factors: expected %d entries" % (sum(self.core) * self.R))
        _lib.check(_lib.lib().cpd_state_factors(_ptr(self.buf), _ptr(w), 1, _stream()), "cpd_state_factors")
        torch.cuda.current_stream().synchronize()

    def factors(self):
        n = sum(self.core) * self.R
        W = torch.empty(n, dtype=torch.float64, device=self.S.device)
        _lib.check(_lib.lib().cpd_state_factors(_ptr(self.buf), _ptr(W), 0, _stream()), "cpd_state_factors")
        out, o = [], 0
        for d in self.core:
            out.append(W[o:o + d * self.R].view(d, self.R))
            o += d * self.R
        return out


def workspace_bytes(shape, R, p=None):
    if p is None:
        p = params()
    return _lib.lib().cpd_workspace_bytes((ctypes.c_int64 * 3)(*shape), R, ctypes.byref(p))


def _flat_w0(W0, device):
    """The three initial core factors as one contiguous FP64 device vector (a tensor that already is
    one is used as it is, so repeated calls need no concatenation)."""
    if W0 is None:
        return None
    if isinstance(W0, torch.Tensor):
        if W0.dtype != torch.float64 or not W0.is_contiguous() or W0.device != device:
            raise ValueError("a flat W0 must be a contiguous FP64 tensor on the tensor's device")
        return W0
    return torch.cat([w.reshape(-1) for w in W0]).to(device=device, dtype=torch.float64).contiguous()


def flat_w0(W0, device):
    """Concatenate initial core factors once, for repeated solve() calls with the same start."""
    return _flat_w0(W0, device)


def solve(T, R, p=None, W0=None, ws=None):
    """Full CPD.  Returns dict(W=[3 x (I_l x R)], lam, info) with the C struct's fields.  W0: the three
    initial core factors, or one flat FP64 tensor holding them in order (see flat_w0)."""
    _check_tensor(T)
    L = _lib.lib()
    if p is None:
        p = params()
    dims = _dims(T)
    if ws is None:
        ws = _ws(L.cpd_workspace_bytes(dims, R, ctypes.byref(p)), T.device)
    W = [torch.empty((T.shape[l], R), dtype=torch.float64, device=T.device) for l in range(3)]
    lam = torch.empty(R, dtype=torch.float64, device=T.device)
    w0 = _flat_w0(W0, T.device)
    info = SolveInfo()
    _lib.check(L.cpd_solve(_ptr(T), _dtype(T), dims, R, ctypes.byref(p), _ptr(w0),
                           (ctypes.c_void_p * 3)(*[w.data_ptr() for w in W]), _ptr(lam), ctypes.byref(info),
                           _ptr(ws), ws.numel(), _stream()), "cpd_solve")
    d = {f: getattr(info, f) for f, _ in SolveInfo._fields_}
    d["core_dims"] = tuple(info.core_dims)
    return dict(W=W, lam=lam, info=d)


def solve_tt(T, R, p=None, W0=None, ws=None):
    """Rank-R CPD of a tensor of order >= 4 through the tensor train (cpd_solve_tt).  W0: None or
    the nested start points of synth.tt_init_factors (host arrays), packed here in that order.
    Returns dict(W=[L x (I_l x R)], lam, info)."""
    if not (T.is_cuda and T.is_contiguous()):
        raise ValueError("expected a contiguous tensor on the GPU")
    L = _lib.lib()
    if p is None:
        p = params()
    Lord = T.dim()
    dims = (ctypes.c_int64 * Lord)(*T.shape)
    if ws is None:
        nb = L.cpd_tt_workspace_bytes(Lord, dims, R, ctypes.byref(p))
        if nb == 0:
            raise ValueError("cpd_solve_tt: shape outside the supported limits")
        ws = _ws(nb, T.device)
    W = [torch.empty((T.shape[l], R), dtype=torch.float64, device=T.device) for l in range(Lord)]
    lam = torch.empty(R, dtype=torch.float64, device=T.device)
    w0 = None
    if W0 is not None:
        flat = [torch.as_tensor(m, dtype=torch.float64).reshape(-1) for grp in W0 for m in grp]
        w0 = torch.cat(flat).to(T.device)
    info = SolveInfo()
    Wp = (ctypes.c_void_p * Lord)(*[w.data_ptr() for w in W])
    _lib.check(L.cpd_solve_tt(_ptr(T), _dtype(T), Lord, dims, R, ctypes.byref(p), _ptr(w0) if w0 is not None else None,
                              Wp, _ptr(lam), ctypes.byref(info), _ptr(ws), ws.numel(), _stream()), "cpd_solve_tt")
    return dict(W=W, lam=lam, info=_info_dict(info))


def _info_dict(info):
    d = {f: getattr(info, f) for f, _ in SolveInfo._fields_}
    d["core_dims"] = tuple(info.core_dims)
    return d


class Batch:
    """Many small CPDs solved together (every mode <= 64).  ``Ts``: list of contiguous 3-way
    tensors on the GPU, all FP64 or all FP32; ``Rs``: ranks; ``W0``: optional list (per member) of
    three P_l x R initial core factors.  Outputs ``W`` / ``lam`` are allocated once and refilled by
    every run.  With ``graph=True`` a plan is built (Gram variant autotuned, launches captured in
    a hipGraph) and :meth:`run` replays it."""

    def __init__(self, Ts, Rs, p=None, W0=None, graph=True):
        L = _lib.lib()
        if len(Ts) != len(Rs) or not Ts:
            raise ValueError("need one rank per tensor")
        dt = Ts[0].dtype
        for T in Ts:
            _check_tensor(T)
            if T.dtype != dt:
                raise TypeError("all members must share one dtype")
        self.p = p if p is not None else params()
        self.n = len(Ts)
        self.dtype = _dtype(Ts[0])
        self._keep = list(Ts)
        dev = Ts[0].device
        self.W, self.lam = [], []
        items = (_lib.BatchItem * self.n)()
        for b, (T, R) in enumerate(zip(Ts, Rs)):
            it = items[b]
            it.T = T.data_ptr()
            for l in range(3):
                it.dims[l] = T.shape[l]
            it.R = int(R)
            Wb = [torch.empty((T.shape[l], R), dtype=torch.float64, device=dev) for l in range(3)]
            lb = torch.empty(R, dtype=torch.float64, device=dev)
            self.W.append(Wb)
            self.lam.append(lb)
            for l in range(3):
                it.W[l] = Wb[l].data_ptr()
            it.lam = lb.data_ptr()
            if W0 is not None:
                w0 = [torch.as_tensor(w, dtype=torch.float64).to(dev).contiguous() for w in W0[b]]
                self._keep.extend(w0)
                for l in range(3):
                    it.W0[l] = w0[l].data_ptr()
        self.items = items
        nb = L.cpd_batch_workspace_bytes(items, self.n, ctypes.byref(self.p))
        if nb == 0:
            raise ValueError("invalid batch (modes must be 1..64, R 1..64)")
        self.ws = _ws(nb, dev)
        self.plan = None
        if graph:
            h = ctypes.c_void_p()
            _lib.check(L.cpd_batch_plan_create(items, self.n, self.dtype, ctypes.byref(self.p), _ptr(self.ws),
                                               self.ws.numel(), _stream(), ctypes.byref(h)), "cpd_batch_plan_create")
            self.plan = h

    def run(self, read_info=True):
        L = _lib.lib()
        infos = (SolveInfo * self.n)() if read_info else None
        if self.plan is not None:
            _lib.check(L.cpd_batch_plan_run(self.plan, infos, _stream()), "cpd_batch_plan_run")
        else:
            _lib.check(L.cpd_solve_batched(self.items, self.n, self.dtype, ctypes.byref(self.p), infos,
                                           _ptr(self.ws), self.ws.numel(), _stream()), "cpd_solve_batched")
        return [_info_dict(i) for i in infos] if read_info else None

    def variant(self):
        """(chosen Gram variant, time of each candidate in ms)."""
        ms = (ctypes.c_float * 4)()
        v = _lib.lib().cpd_batch_plan_variant(self.plan, ms) if self.plan is not None else -1
        return v, list(ms)

    def close(self):
        if self.plan is not None:
            _lib.lib().cpd_batch_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_mixed(T_lo, T, R, p=None, W0=None, ws=None):
    """cpd_solve with the compression Grams from the BF16 copy T_lo on the BF16 matrix cores and
    everything else from T.  Returns dict(W, lam, info) like :func:`solve`."""
    _check_tensor(T)
    _check_tensor(T_lo)
    if T_lo.dtype != torch.bfloat16 or tuple(T_lo.shape) != tuple(T.shape):
        raise ValueError("T_lo must be a BF16 copy of T")
    L = _lib.lib()
    if p is None:
        p = params()
    dims = _dims(T)
    if ws is None:
        ws = _ws(L.cpd_workspace_bytes(dims, R, ctypes.byref(p)), T.device)
    W = [torch.empty((T.shape[l], R), dtype=torch.float64, device=T.device) for l in range(3)]
    lam = torch.empty(R, dtype=torch.float64, device=T.device)
    w0 = _flat_w0(W0, T.device)
    info = SolveInfo()
    _lib.check(L.cpd_solve_mixed(_ptr(T_lo), CPD_BF16, _ptr(T), _dtype(T), dims, R, ctypes.byref(p), _ptr(w0),
                                 (ctypes.c_void_p * 3)(*[w.data_ptr() for w in W]), _ptr(lam), ctypes.byref(info),
                                 _ptr(ws), ws.numel(), _stream()), "cpd_solve_mixed")
    return dict(W=W, lam=lam, info=_info_dict(info))


def mttkrp(T, Ws, mode, compute_dtype=CPD_F64):
    """M = T_(mode) (Khatri-Rao of the other two factors), FP64 result; compute_dtype picks the
    FP64, FP32 or BF16 matrix-core path (see cpd_mttkrp in cpd.h)."""
    _check_tensor(T)
    L = _lib.lib()
    R = Ws[0].shape[1]
    dims = _dims(T)
    ws = _ws(L.cpd_mttkrp_workspace_bytes(dims, R, mode), T.device)
    M = torch.empty((T.shape[mode], R), dtype=torch.float64, device=T.device)
    Wc = [w.contiguous().to(torch.float64) for w in Ws]
    _lib.check(L.cpd_mttkrp(_ptr(T), _dtype(T), dims, (ctypes.c_void_p * 3)(*[w.data_ptr() for w in Wc]), R, mode,
                            compute_dtype, _ptr(M), _ptr(ws), ws.numel(), _stream()), "cpd_mttkrp")
    return M


def residual_norm2(T, Ws):
    _check_tensor(T)
    L = _lib.lib()
    R = Ws[0].shape[1]
    dims = _dims(T)
    ws = _ws(L.cpd_residual_workspace_bytes(dims), T.device)
    out = torch.empty(1, dtype=torch.float64, device=T.device)
    Wc = [w.contiguous().to(torch.float64) for w in Ws]
    _lib.check(L.cpd_residual_norm2(_ptr(T), _dtype(T), dims, (ctypes.c_void_p * 3)(*[w.data_ptr() for w in Wc]),
                                    R, _ptr(out), _ptr(ws), ws.numel(), _stream()), "cpd_residual_norm2")
    return out


def profile_enable(on=True, kernels=None):
    """Record HIP events around the path's main kernels (see cpd_profile_* in cpd.h); ``kernels``: a
    list of names from _lib.PROFILE_KERNELS to time (default: all)."""
    L = _lib.lib()
    mask = 0xFFFFFFFF if kernels is None else sum(1 << _lib.PROFILE_KERNELS.index(k) for k in kernels)
    L.cpd_profile_select(mask)
    L.cpd_profile_enable(1 if on else 0)


def block_sum_ns(nthreads=512, reps=20000):
    """Device time of one block-wide sum (one barrier + LDS round trip) in a workgroup of nthreads."""
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    out = ctypes.c_double()
    _lib.check(_lib.lib().cpd_profile_block_sum_ns(nthreads, reps, _ptr(ws), 16, ctypes.byref(out), _stream()),
               "cpd_profile_block_sum_ns")
    return out.value


def profile_reset():
    _lib.lib().cpd_profile_reset()


def profile_read():
    """{kernel: (launches, total_ms)} accumulated since the last reset."""
    out = (_lib.KernelTime * len(_lib.PROFILE_KERNELS))()
    _lib.check(_lib.lib().cpd_profile_read(out), "cpd_profile_read")
    return {name: (int(out[i].launches), float(out[i].total_ms)) for i, name in enumerate(_lib.PROFILE_KERNELS)}


def jtj_v(Ws, Vs):
    L = _lib.lib()
    R = Ws[0].shape[1]
    Wc = [w.contiguous().to(torch.float64) for w in Ws]
    Vc = [v.contiguous().to(torch.float64) for v in Vs]
    out = [torch.empty_like(w) for w in Wc]
    dims = (ctypes.c_int32 * 3)(*[w.shape[0] for w in Wc])
    _lib.check(L.cpd_jtj_v((ctypes.c_void_p * 3)(*[w.data_ptr() for w in Wc]),
                           (ctypes.c_void_p * 3)(*[v.data_ptr() for v in Vc]), dims, R,
                           (ctypes.c_void_p * 3)(*[o.data_ptr() for o in out]), _stream()), "cpd_jtj_v")
    return out
