"""The C-ABI library loads and exports every function include/cpd.h declares (CPU only: no compute)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "cpd.h")
LIB = os.path.join(ROOT, "paper_2110_05997_amd", "lib", "libcpd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(cpd_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ["cpd_compress", "cpd_dgn_step", "cpd_solve", "cpd_state_init", "cpd_dgn_run", "cpd_gram",
                 "cpd_eig_top", "cpd_mttkrp", "cpd_residual_norm2", "cpd_jtj_v"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcpd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcpd.so not built")
def test_binding_signatures_cover_the_header():
    from paper_2110_05997_amd import _lib
    bound = {n for n, _, _ in _lib.SIGNATURES}
    assert set(declared_functions()) <= bound


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcpd.so not built")
def test_host_only_queries():
    """Workspace and state-size queries run on the host and need no GPU."""
    from paper_2110_05997_amd import _lib
    L = _lib.lib()
    p = _lib.Params()
    L.cpd_default_params(ctypes.byref(p))
    assert p.maxiter == 200 and p.tol == 1e-6 and p.init_damp == 1.0
    dims = (ctypes.c_int64 * 3)(200, 200, 200)
    assert L.cpd_workspace_bytes(dims, 20, ctypes.byref(p)) > 200 ** 3 * 8 // 10
    assert L.cpd_workspace_bytes((ctypes.c_int64 * 3)(0, 2, 2), 2, ctypes.byref(p)) == 0
    assert L.cpd_state_bytes((ctypes.c_int32 * 3)(20, 20, 20), 20, ctypes.byref(p)) > 0
    assert L.cpd_gram_workspace_bytes(dims, 0) > 0
    assert L.cpd_eig_workspace_bytes(200, 20) > 0
    assert b"gfx950" in L.cpd_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcpd.so not built")
def test_batch_workspace_query():
    """The batch workspace query reads only shapes, ranks and which pointers are set."""
    from paper_2110_05997_amd import _lib
    L = _lib.lib()
    p = _lib.Params()
    L.cpd_default_params(ctypes.byref(p))
    items = (_lib.BatchItem * 3)()
    for b, (dims, R) in enumerate([((10, 20, 30), 4), ((64, 64, 64), 12), ((11, 9, 10), 12)]):
        it = items[b]
        it.T = 0x1000
        for l in range(3):
            it.dims[l] = dims[l]
            it.W[l] = 0x1000
        it.R = R
        it.lam = 0x1000
    n_ok = L.cpd_batch_workspace_bytes(items, 3, ctypes.byref(p))
    assert n_ok > 12 * 64 * 64 * 8        # at least the first projection of the 64^3 member
    items[1].dims[0] = 65                                   # modes are limited to 64
    assert L.cpd_batch_workspace_bytes(items, 3, ctypes.byref(p)) == 0
    items[1].dims[0] = 64
    items[2].W0[0] = 0x1000                                 # W0 must be all or none
    assert L.cpd_batch_workspace_bytes(items, 3, ctypes.byref(p)) == 0
