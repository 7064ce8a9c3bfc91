"""Host-only checks of the C-ABI library: it builds, loads, and exports every
function include/dmrg.h declares; option defaults and status strings; the
host-only ordering entry point against the oracle.  No device call is made
(no GPU here)."""
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
    assert o.trunc_eps == 0.0 and o.d_min == 0 and o.n_states == 1 and o.measure == 0 and o.graph == 0
    assert o.group_products == 1


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
    for field, value in (("trunc_eps", -1e-6), ("d_min", -1), ("n_states", 0), ("n_states", 3),
                         ("measure", 2), ("measure", -1), ("graph", 2), ("group_products", 2),
                         ("group_products", -1)):
        lib.dmrg_default_options(ctypes.byref(o))
        setattr(o, field, value)
        assert lib.dmrg_create(ctypes.byref(o), ctypes.byref(h)) == -1, field
        assert h.value is None


def test_null_context_arguments(lib):
    assert lib.dmrg_sweep(None, None, 8, None) == -1
    assert lib.dmrg_energy(None, None) == -1
    assert lib.dmrg_orbital_entropies(None, None, None, None, None, None) == -1
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


# ------------------------------- entropy-based ordering (host-only entry point)
def _fiedler(lib, I):
    import paper_1507_00161_amd as pk
    return pk.fiedler_ordering(I, lib=lib)


def test_fiedler_ordering_matches_the_oracle(lib):
    """dmrg_fiedler_ordering (cyclic Jacobi in the library) against the oracle's
    LAPACK-based definition: same ordering and Fiedler value, on random
    non-negative symmetric matrices, a hidden seriation, and the oracle's
    mutual information of the pf 8p+8n workload."""
    import json
    import numpy as np
    from oracle import entropy
    rng = np.random.default_rng(11)
    mats = []
    for n in (2, 3, 5, 12, 40, 60, 120):
        a = rng.uniform(0.0, 1.0, (n, n)) ** 3
        a = np.triu(a, 1)
        mats.append(a + a.T)
    n = 24
    pos = np.empty(n, int)
    pos[rng.permutation(n)] = np.arange(n)
    d = np.abs(pos[:, None] - pos[None, :])
    mats.append(np.exp(-0.5 * d) * (d > 0))
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_energies.json")))
    mats.append(np.array(gold["cases"]["pf_8p8n_ent"]["mutual"]))
    for I in mats:
        order, val = _fiedler(lib, I)
        want_val, _ = entropy.fiedler_vector(I)
        assert np.array_equal(order, entropy.fiedler_ordering(I)), I.shape
        assert abs(val - want_val) <= 1e-10 * max(1.0, abs(want_val))
        assert sorted(order.tolist()) == list(range(I.shape[0]))


def test_fiedler_ordering_edge_cases(lib):
    import numpy as np
    import paper_1507_00161_amd as pk
    order, val = _fiedler(lib, np.zeros((1, 1)))
    assert order.tolist() == [0] and val == 0.0
    # two sites: the Fiedler vector is (-1, 1)/sqrt 2 after the sign rule
    order, val = _fiedler(lib, np.array([[0.0, 0.3], [0.3, 0.0]]))
    assert order.tolist() == [0, 1] and abs(val - 0.6) < 1e-15
    out = np.empty(3, np.int32)
    bad = [np.array([[0.0, 1.0, 0.0], [0.5, 0.0, 1.0], [0.0, 1.0, 0.0]]),
           np.array([[0.0, np.nan, 0.0], [np.nan, 0.0, 1.0], [0.0, 1.0, 0.0]])]
    for m in bad:
        with pytest.raises(pk.DMRGError):
            _fiedler(lib, m)
    m = np.ones((3, 3))
    assert lib.dmrg_fiedler_ordering(None, 3, out.ctypes.data_as(ctypes.c_void_p), None) == -1
    assert lib.dmrg_fiedler_ordering(m.ctypes.data_as(ctypes.c_void_p), 0,
                                     out.ctypes.data_as(ctypes.c_void_p), None) == -1
    assert lib.dmrg_fiedler_ordering(m.ctypes.data_as(ctypes.c_void_p), 3, None, None) == -1
