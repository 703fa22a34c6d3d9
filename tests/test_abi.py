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
    # int exchange, flags
    assert ctypes.sizeof(afqmc._Params) == 64
    assert afqmc._Params.mu.offset == 40
    assert afqmc._Params.exchange.offset == 56
    assert afqmc._Params.flags.offset == 60
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
    p = afqmc._Params(4, 2, 2, 1, 0.01, 6, 0, 1, float("nan"), float("nan"), 0, 6)
    rc = afqmc._lib.afqmc_init_hamiltonian(ctypes.byref(p), z.ctypes.data, z.ctypes.data,
                                           z.ctypes.data, z.ctypes.data, None, ctypes.byref(h))
    assert rc == 1 and b"flags" in afqmc._lib.afqmc_last_error()
    assert not h.value


def test_msd_create_rejects_bad_arguments_without_touching_the_device(lib):
    """Sizes, null pointers and the excitation format are checked on the host
    before any device call (so this runs without a GPU)."""
    import numpy as np

    afqmc.load()
    N, na, nb, ndet = 10, 3, 2, 3
    C = np.eye(N)
    coeff = np.ones(ndet)
    rank = np.zeros((ndet, 2), np.int32)
    orbs = np.full((ndet, 2, 2, afqmc.MSD_MAX_RANK), -1, np.int32)

    def create(N=N, na=na, nb=nb, ndet=ndet, rank=rank, orbs=orbs, coeff=coeff, C=C):
        h = ctypes.c_void_p()
        rc = afqmc._lib.afqmc_msd_create(N, na, nb, C.ctypes.data, C.ctypes.data, ndet, coeff.ctypes.data,
                                         rank.ctypes.data, orbs.ctypes.data, 4, None, ctypes.byref(h))
        return rc, afqmc._lib.afqmc_last_error().decode(), h.value

    assert create(N=0)[0] == 1
    assert create(na=11)[0] == 1                    # more electrons than orbitals
    assert create(na=46, N=60)[0] == 4              # beyond the kernels' electron limit
    assert create(ndet=0)[0] == 1
    bad = rank.copy(); bad[1, 0] = 7
    rc, msg, h = create(rank=bad)
    assert rc == 1 and "determinant 1" in msg and h is None
    r2, o2 = rank.copy(), orbs.copy()
    r2[2, 1] = 1; o2[2, 1, 0, 0] = 0; o2[2, 1, 1, 0] = 1     # particle inside the reference
    rc, msg, h = create(rank=r2, orbs=o2)
    assert rc == 1 and "determinant 2 spin 1" in msg and h is None


def test_msd_calls_reject_a_null_handle(lib):
    afqmc.load()
    w = afqmc._Walkers()
    assert afqmc._lib.afqmc_msd_overlap(None, ctypes.byref(w), 1, ctypes.c_void_p(1), None) == 1
    assert afqmc._lib.afqmc_msd_green_function(None, ctypes.byref(w), 1, ctypes.c_void_p(1), None) == 1
    assert afqmc._lib.afqmc_msd_force_bias(None, None, ctypes.byref(w), 1, ctypes.c_void_p(1), None) == 1
    assert afqmc._lib.afqmc_msd_propagate(None, None, ctypes.byref(w), 1, ctypes.c_void_p(1), None) == 1
    afqmc._lib.afqmc_msd_destroy(None)              # no-op


def test_noalloc_comb_rejects_bad_arguments_without_touching_the_device(lib):
    afqmc.load()
    w = afqmc._Walkers()
    f = afqmc._lib.afqmc_population_control_noalloc
    assert f(0, 1, 1, ctypes.byref(w), 4, 0.5, None, None, None) == 1
    assert f(4, 5, 1, ctypes.byref(w), 4, 0.5, None, None, None) == 1
    assert f(4, 2, 2, ctypes.byref(w), 65537, 0.5, None, None, None) == 1
    assert b"65536" in afqmc._lib.afqmc_last_error()
    assert f(4, 2, 2, ctypes.byref(w), 4, 0.5, None, None, None) == 1     # null walker arrays
    assert f(4, 2, 2, ctypes.byref(w), 0, 0.5, None, None, None) == 0     # nothing to do
