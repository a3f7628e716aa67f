"""Host-side checks of the C ABI: the library loads, exports every function the
public header declares, and rejects invalid arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "qdd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qdd_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def Q():
    from paper_1011_0911_amd import qdd

    if not os.path.exists(qdd.LIB_PATH):
        pytest.fail("libqdd.so not built (run __graft_entry__.build())")
    qdd.lib()
    return qdd


def test_header_declares_the_boundary():
    names = header_functions()
    for must in ("qdd_create", "qdd_set_gauge", "qdd_set_params", "qdd_dw_hat", "qdd_dw", "qdd_sap",
                 "qdd_dfl_build", "qdd_solve"):
        assert must in names


def test_library_exports_every_declared_symbol(Q):
    L = Q.lib()
    for name in header_functions():
        assert hasattr(L, name), name
        assert name in Q.SIGNATURES, f"binding lacks {name}"


def test_invalid_geometry_and_config_rejected_on_host(Q):
    cfg = Q.default_config()
    assert Q.workspace_bytes((4, 4, 4, 4), cfg) > 0
    assert Q.workspace_bytes((5, 4, 4, 4), cfg) == 0          # odd extent
    assert Q.workspace_bytes((8, 8, 8, 6), Q.default_config(precond=Q.PRECOND_SAP)) == 0  # 4 does not divide 6
    assert Q.workspace_bytes((8, 8, 8, 6), cfg) > 0           # blocks unused without SAP
    assert Q.workspace_bytes((4, 4, 4, 4), Q.default_config(max_nrhs=0)) == 0
    assert Q.workspace_bytes((12, 8, 8, 8), Q.default_config(precond=Q.PRECOND_SAP)) == 0  # 3 blocks in time
    assert Q.workspace_bytes((8, 8, 8, 8), Q.default_config(precond=Q.PRECOND_DFL)) == 0  # no Ns
    assert Q.workspace_bytes((8, 8, 8, 8), Q.default_config(nkv=33)) == 0
    net = dict(precond=Q.PRECOND_DFL, dfl_Ns=4, dfl_bs=(2, 2, 2, 2), sap_bs=(2, 2, 2, 2), use_net=1)
    assert cfg.net_terms == 3
    assert Q.workspace_bytes((8, 8, 8, 8), Q.default_config(**net)) > 0
    assert Q.workspace_bytes((8, 8, 8, 8), Q.default_config(net_terms=1, **net)) > 0
    assert Q.workspace_bytes((8, 8, 8, 8), Q.default_config(net_terms=0, **net)) == 0
    assert Q.workspace_bytes((8, 8, 8, 8), Q.default_config(net_terms=4, **net)) == 0
    g = Q.make_geom((5, 4, 4, 4))
    h = ctypes.c_void_p()
    st = Q.lib().qdd_create(ctypes.byref(g), ctypes.byref(cfg), None, 0, None, ctypes.byref(h))
    assert st == Q.QDD_EINVAL and not h.value
    assert b"even" in Q.lib().qdd_last_error(None)
    g = Q.make_geom((4, 4, 4, 4))
    st = Q.lib().qdd_create(ctypes.byref(g), ctypes.byref(cfg), None, 0, None, ctypes.byref(h))
    assert st == Q.QDD_ENOWS


def test_workspace_grows_with_batch_and_krylov_space(Q):
    a = Q.workspace_bytes((8, 8, 8, 8), Q.default_config())
    b = Q.workspace_bytes((8, 8, 8, 8), Q.default_config(max_nrhs=4))
    c = Q.workspace_bytes((8, 8, 8, 8), Q.default_config(nkv=24))
    assert b > a and c > a
