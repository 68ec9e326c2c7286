"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol that include/ctbop.h declares, and rejects bad arguments before any
device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(ctbop_[a-z_0-9]+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def L():
    import paper_1802_07871_amd as ct
    path = ct.LIB_PATH
    if not os.path.exists(path):
        from paper_1802_07871_amd import build
        build.build()
    return ct.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert "ctbop_compute_energy_forces_charges" in names
    for nm in sorted(names):
        assert hasattr(L, nm), nm


def test_binding_exports_match_header():
    import paper_1802_07871_amd as ct
    assert set(ct.EXPORTS) <= _declared()


def test_bad_arguments_rejected_on_host(L, theta):
    import paper_1802_07871_amd as ct
    h = ctypes.c_void_p()
    bad = theta.copy()
    assert L.ctbop_create(bad.ctypes.data, 55, None, ctypes.byref(h)) == ct.E_INVAL
    bad[6] = -1.0
    assert L.ctbop_create(bad.ctypes.data, 56, None, ctypes.byref(h)) == ct.E_INVAL
    assert b"sigma" in L.ctbop_last_error()
    assert L.ctbop_create(theta.ctypes.data, 56, None, ctypes.byref(h)) == 0
    nb = ctypes.c_size_t()
    box = np.ascontiguousarray(np.eye(3).ravel() * 2.0)
    pbc = np.ones(3, dtype=np.int32)
    # periodic cell narrower than a third of the Coulomb-list radius
    assert L.ctbop_system_bytes(h, 10, box.ctypes.data, pbc.ctypes.data, ctypes.byref(nb)) == ct.E_INVAL
    box = np.ascontiguousarray(np.diag([20.0, 20.0, -20.0]).ravel())
    assert L.ctbop_system_bytes(h, 10, box.ctypes.data, pbc.ctypes.data, ctypes.byref(nb)) == ct.E_INVAL
    box = np.ascontiguousarray(np.eye(3).ravel() * 20.0)
    assert L.ctbop_system_bytes(h, 0, box.ctypes.data, pbc.ctypes.data, ctypes.byref(nb)) == ct.E_INVAL
    assert L.ctbop_system_bytes(h, 1000, box.ctypes.data, pbc.ctypes.data, ctypes.byref(nb)) == 0
    assert nb.value > 1000 * 512 * 8
    # the system buffer must be at least that large
    rc = L.ctbop_compute_energy_forces_charges(h, 1000, ctypes.c_void_p(8), ctypes.c_void_p(8), box.ctypes.data,
                                               pbc.ctypes.data, 0.0, 0, ctypes.c_void_p(256), nb.value - 1,
                                               None, ctypes.c_void_p(8), ctypes.c_void_p(8), None, None)
    assert rc == ct.E_NOMEM
    # parameter replacement: the same checks as create
    assert L.ctbop_set_params(h, bad.ctypes.data, 56) == ct.E_INVAL
    assert L.ctbop_set_params(h, theta.ctypes.data, 56) == 0
    # the adjoint: workspace size, and no preceding evaluation on this buffer
    ab = ctypes.c_size_t()
    assert L.ctbop_param_grad_bytes(h, 1000, box.ctypes.data, pbc.ctypes.data, ctypes.byref(ab)) == 0
    assert ab.value > 1000 * 32 * 6 * 8          # dual bond coefficients, 32 bonds per row
    g = np.zeros(56)
    rc = L.ctbop_param_grad(h, 1000, box.ctypes.data, pbc.ctypes.data, ctypes.c_void_p(256), nb.value,
                            ctypes.c_void_p(256), ab.value, 1.0, ctypes.c_void_p(8), None, g.ctypes.data, None,
                            None)
    assert rc == ct.E_INVAL and b"preceding evaluation" in L.ctbop_last_error()
    L.ctbop_destroy(h)
