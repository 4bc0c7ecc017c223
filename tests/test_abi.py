"""The C-ABI library loads on the CPU, exports every symbol the header declares, and rejects
invalid arguments before touching the GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "seedcg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(seedcg_[A-Za-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_0901_3512_amd.seedcg import LIB_PATH, load_library
    if not os.path.exists(LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return load_library()


def test_exports_every_declared_symbol(lib):
    from paper_0901_3512_amd.seedcg import exported_symbols
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(exported_symbols()) == names


def test_create_rejects_bad_arguments_on_host(lib):
    from paper_0901_3512_amd.seedcg import Params
    p = Params()
    lib.seedcg_default_params(ctypes.byref(p))
    assert p.t_bc == -1 and p.reorth_k == 10 and abs(p.past_factor - 1.5) < 1e-15 and p.tol == 1e-10
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    for dims in ((3, 4, 4, 4), (4, 4, 0, 4), (4, 4, 4, 5)):
        for d in range(4):
            p.dims[d] = dims[d]
        rc = lib.seedcg_create(ctypes.byref(p), dummy, ctypes.byref(h))
        assert rc == -1
        assert b"even" in lib.seedcg_last_error(None)
    for d in range(4):
        p.dims[d] = 4
    p.t_bc = 0
    assert lib.seedcg_create(ctypes.byref(p), dummy, ctypes.byref(h)) == -1
    p.t_bc = -1
    p.basis_fp32 = 3   # 0, 1 or 2
    assert lib.seedcg_create(ctypes.byref(p), dummy, ctypes.byref(h)) == -1
    assert b"basis_fp32" in lib.seedcg_last_error(None)
    p.basis_fp32 = 0
    p.tol = 0.0
    assert lib.seedcg_create(ctypes.byref(p), dummy, ctypes.byref(h)) == -1
    assert lib.seedcg_create(None, dummy, ctypes.byref(h)) == -1
    # the roofline probes refuse bad arguments before any GPU call
    d = ctypes.c_double()
    assert lib.seedcg_probe_bandwidth(3, 1 << 20, 1, None, ctypes.byref(d)) == -1
    assert lib.seedcg_probe_bandwidth(0, 1000, 1, None, ctypes.byref(d)) == -1
    assert lib.seedcg_probe_mfma(2, 10, None, ctypes.byref(d)) == -1
    assert lib.seedcg_probe_mfma(0, 0, None, ctypes.byref(d)) == -1
    assert lib.seedcg_apply_M(None, None, None, 1) == -1
    assert lib.seedcg_solve_seed(None, None, None, 1, None) == -1


def test_create_batch_rejects_bad_arguments_on_host(lib):
    from paper_0901_3512_amd.seedcg import Params
    p = Params()
    lib.seedcg_default_params(ctypes.byref(p))
    assert p.autotune == 1
    h = ctypes.c_void_p()
    dims = (ctypes.c_int32 * 8)(4, 4, 4, 4, 4, 4, 4, 4)
    kap = (ctypes.c_double * 2)(0.12, 0.13)
    links = (ctypes.c_void_p * 2)(16, 32)   # never dereferenced: validation fails first
    assert lib.seedcg_create_batch(0, dims, kap, links, 4, ctypes.byref(p), ctypes.byref(h)) == -1
    assert lib.seedcg_create_batch(2, dims, kap, links, 26, ctypes.byref(p), ctypes.byref(h)) == -1
    assert b"nrhs" in lib.seedcg_batch_last_error(None)
    bad = (ctypes.c_int32 * 8)(4, 4, 4, 4, 4, 3, 4, 4)
    assert lib.seedcg_create_batch(2, bad, kap, links, 4, ctypes.byref(p), ctypes.byref(h)) == -1
    nolink = (ctypes.c_void_p * 2)(16, None)
    assert lib.seedcg_create_batch(2, dims, kap, nolink, 4, ctypes.byref(p), ctypes.byref(h)) == -1
    p.precond = 1
    assert lib.seedcg_create_batch(2, dims, kap, links, 4, ctypes.byref(p), ctypes.byref(h)) == -1
    assert lib.seedcg_solve_batch(None, None, None, None) == -1
    lib.seedcg_destroy_batch(None)
