"""CPU checks of the C-ABI library: it loads and exports every declared symbol,
and its header and binding agree.  No compute calls (no GPU here)."""

import ctypes
import os
import re

import pytest

from paper_2209_04015_amd import afqmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "afqmc.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(afqmc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(afqmc.LIB_PATH):
        pytest.fail("libafqmc.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(afqmc.LIB_PATH)


def test_header_declares_the_binding_entry_points():
    assert _declared() == sorted(afqmc.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_version_and_error_string(lib):
    lib.afqmc_version.restype = ctypes.c_int
    assert lib.afqmc_version() >= 1
    lib.afqmc_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.afqmc_last_error(), bytes)


def test_param_struct_layout_matches_header():
    # int N, na, nb, K; double dt; int taylor_order, precision, max_walkers; double mu, e_shift;
    # int exchange
    assert ctypes.sizeof(afqmc._Params) == 64
    assert afqmc._Params.mu.offset == 40
    assert afqmc._Params.exchange.offset == 56
    assert ctypes.sizeof(afqmc._Walkers) == 32


def test_init_rejects_bad_arguments_without_touching_the_device(lib):
    afqmc.load()
    p = afqmc._Params(0, 1, 1, 1, 0.01, 6, 0, 1, float("nan"), float("nan"))
    h = ctypes.c_void_p()
    import numpy as np

    z = np.zeros(4)
    rc = afqmc._lib.afqmc_init_hamiltonian(ctypes.byref(p), z.ctypes.data, z.ctypes.data,
                                           z.ctypes.data, z.ctypes.data, None, ctypes.byref(h))
    assert rc == 1
    assert b"bad sizes" in afqmc._lib.afqmc_last_error()
    p = afqmc._Params(4, 50, 1, 1, 0.01, 6, 0, 1, float("nan"), float("nan"))
    rc = afqmc._lib.afqmc_init_hamiltonian(ctypes.byref(p), z.ctypes.data, z.ctypes.data,
                                           z.ctypes.data, z.ctypes.data, None, ctypes.byref(h))
    assert rc in (1, 4)
    p = afqmc._Params(4, 2, 2, 1, -1.0, 6, 0, 1, float("nan"), float("nan"))
    rc = afqmc._lib.afqmc_init_hamiltonian(ctypes.byref(p), z.ctypes.data, z.ctypes.data,
                                           z.ctypes.data, z.ctypes.data, None, ctypes.byref(h))
    assert rc == 1
    assert not h.value
