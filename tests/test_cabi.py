"""Host-only checks of the C-ABI library: it builds, loads, and exports every
function include/dmrg.h declares; option defaults and status strings.  No
compute call is made (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmrg.h")


@pytest.fixture(scope="module")
def lib():
    import paper_1507_00161_amd as pk
    if not os.path.exists(pk.LIB_PATH):
        from paper_1507_00161_amd import build
        build.build()
    return pk.declare(ctypes.CDLL(pk.LIB_PATH))


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmrg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("dmrg_load_hamiltonian", "dmrg_sweep", "dmrg_heff_layout", "dmrg_heff_apply",
              "dmrg_energy", "dmrg_sweep_many", "dmrg_create", "dmrg_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_default_options(lib):
    import paper_1507_00161_amd as pk
    o = pk.Options()
    lib.dmrg_default_options(ctypes.byref(o))
    assert o.precision == 0 and o.seed == 1507
    assert o.davidson_tol == 1e-7 and o.davidson_max_iter == 100 and o.davidson_max_subspace == 24
    assert o.tie_tol == 1e-13 and o.noise == 0.0 and o.select_basis == 0
    assert o.trunc_eps == 0.0 and o.d_min == 0 and o.n_states == 1


def test_status_strings(lib):
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        s = lib.dmrg_status_string(code)
        assert isinstance(s, bytes) and len(s) > 0
    assert lib.dmrg_status_string(-6) == b"device error"


def test_bad_options_rejected_before_any_device_call(lib):
    import paper_1507_00161_amd as pk
    o = pk.Options()
    lib.dmrg_default_options(ctypes.byref(o))
    o.davidson_max_subspace = 64
    h = ctypes.c_void_p()
    assert lib.dmrg_create(ctypes.byref(o), ctypes.byref(h)) == -1
    assert h.value is None
    for field, value in (("trunc_eps", -1e-6), ("d_min", -1), ("n_states", 0), ("n_states", 3)):
        lib.dmrg_default_options(ctypes.byref(o))
        setattr(o, field, value)
        assert lib.dmrg_create(ctypes.byref(o), ctypes.byref(h)) == -1, field
        assert h.value is None


def test_null_context_arguments(lib):
    assert lib.dmrg_sweep(None, None, 8, None) == -1
    assert lib.dmrg_energy(None, None) == -1
    lib.dmrg_destroy(None)


def test_sweep_many_rejects_null_and_repeated_contexts(lib):
    """Argument checks happen before any context is touched (the pointers
    below are never dereferenced)."""
    fake = ctypes.c_void_p(0x1000)
    D = (ctypes.c_int32 * 2)(8, 8)
    two = (ctypes.c_void_p * 2)(fake.value, fake.value)
    assert lib.dmrg_sweep_many(two, 2, None, D, None) == -1
    with_null = (ctypes.c_void_p * 2)(fake.value, None)
    assert lib.dmrg_sweep_many(with_null, 2, None, D, None) == -1
    assert lib.dmrg_sweep_many(None, 2, None, D, None) == -1
