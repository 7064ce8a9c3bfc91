"""Error paths of the C ABI (forced from the host; every kernel exits normally)."""
import numpy as np
import pytest

from workloads import WORKLOADS, make_hamiltonian, make_space

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00161_amd as pk
    pk.library()
    return pk


def _h():
    return WORKLOADS["p_2p2n"].hamiltonian()


def _load(c, h, **over):
    sp = h.space
    args = dict(species=sp.species, two_m=sp.two_m, eps=h.eps, V=h.V.ravel(), n_p=h.n_p, n_n=h.n_n,
                two_M=h.two_M)
    args.update(over)
    c.load_hamiltonian(**args)


def test_invalid_hamiltonian_rejected(pk):
    h = _h()
    c = pk.Context()
    V = h.V.copy()
    i, j, k, l = np.argwhere(V != 0)[0]
    V[i, j, k, l] += 0.5              # breaks antisymmetry / (ij)<->(kl) symmetry
    with pytest.raises(pk.DMRGError) as e:
        _load(c, h, V=V.ravel())
    assert e.value.status == -2 and "(i,j,k,l)" in str(e.value)
    # a consistently (anti)symmetrised element that violates the 2M selection rule
    V = h.V.copy()
    a, b = 0, 1                       # p3/2 protons with 2m = -3, -1
    cc, d = 2, 3                      # p3/2 protons with 2m = 1, 3
    for (p, q, r, s_, v) in ((a, b, cc, d, 1.0), (b, a, cc, d, -1.0), (a, b, d, cc, -1.0), (b, a, d, cc, 1.0)):
        V[p, q, r, s_] = v
        V[r, s_, p, q] = v
    with pytest.raises(pk.DMRGError) as e:
        _load(c, h, V=V.ravel())
    assert e.value.status == -2 and "selection rule" in str(e.value)


def test_unreachable_target(pk):
    h = _h()
    c = pk.Context()
    with pytest.raises(pk.DMRGError) as e:
        _load(c, h, n_p=2, n_n=1, two_M=0)          # odd particle number cannot have 2M = 0
    assert e.value.status == -3
    with pytest.raises(pk.DMRGError) as e:
        _load(c, h, n_p=7, n_n=2, two_M=0)          # more protons than proton sites
    assert e.value.status == -3


def test_calls_out_of_order_and_bad_arguments(pk):
    h = _h()
    c = pk.Context()
    with pytest.raises(pk.DMRGError) as e:
        c.sweep(8)
    assert e.value.status == -4                      # no Hamiltonian
    _load(c, h)
    with pytest.raises(pk.DMRGError) as e:
        c.energy()
    assert e.value.status == -4
    with pytest.raises(pk.DMRGError) as e:
        c.heff_layout()
    assert e.value.status == -4
    with pytest.raises(pk.DMRGError) as e:
        c.sweep(0)
    assert e.value.status == -1
    with pytest.raises(pk.DMRGError) as e:
        c.sweep(8, ordering=[0] * 12)
    assert e.value.status == -1
    with pytest.raises(pk.DMRGError) as e:
        c.heff_configs()
    assert e.value.status == -4


def test_invalid_truncation_options_rejected(pk):
    for kw in ({"trunc_eps": -1e-6}, {"d_min": -1}):
        with pytest.raises(pk.DMRGError) as e:
            pk.Context(**kw)
        assert e.value.status == -1


def test_orbital_entropies_need_a_measuring_sweep(pk):
    """dmrg_orbital_entropies: DMRG_ERR_STATE without measure = 1, before the
    first measuring sweep has completed, and after the ordering changed until
    the next sweep completes."""
    h = _h()
    c = pk.Context()
    _load(c, h)
    c.sweep(16)
    with pytest.raises(pk.DMRGError) as e:
        c.orbital_entropies()
    assert e.value.status == -4
    c = pk.Context(measure=1)
    _load(c, h)
    with pytest.raises(pk.DMRGError) as e:
        c.orbital_entropies()
    assert e.value.status == -4
    c.sweep_steps(16, 3)              # a partial sweep measures nothing complete
    with pytest.raises(pk.DMRGError) as e:
        c.orbital_entropies()
    assert e.value.status == -4
    c.sweep(16)
    m = c.orbital_entropies()
    assert np.all(np.isfinite(m["s1"])) and np.all(m["s1"] >= 0)
    order = np.arange(12)[::-1].copy()
    c.sweep_steps(16, 1, ordering=order)
    with pytest.raises(pk.DMRGError) as e:
        c.orbital_entropies()
    assert e.value.status == -4
    with pytest.raises(pk.DMRGError) as e:
        pk.Context(measure=2)
    assert e.value.status == -1


def test_not_converged_warning_keeps_valid_results(pk):
    h = _h()
    c = pk.Context(davidson_max_iter=1)
    _load(c, h)
    r = c.sweep(16)
    assert r["code"] == 1 and r["not_converged"] > 0
    assert np.isfinite(r["energy"]) and c.energy() == r["energy"]


def test_memory_cap_reports_out_of_memory(pk):
    h = WORKLOADS["sd_4p4n"].hamiltonian()
    c = pk.Context(mem_cap_bytes=1 << 20)
    _load(c, h)
    with pytest.raises(pk.DMRGError) as e:
        c.sweep(64)
    assert e.value.status == -5
    # the context is still usable for a fresh load
    _load(c, _h())


def test_check_fp64_rejects_bad_argument(pk):
    c = pk.Context(precision=1)
    assert c._lib.dmrg_check_fp64(c._h, 2) == -1
    assert c._lib.dmrg_check_fp64(None, 1) == -1
    c.check_fp64(True)
    c.check_fp64(False)


def test_set_cideas_errors(pk):
    h = _h()
    c = pk.Context()
    s = np.full(h.space.n_sites, 0.3)
    n = np.full(h.space.n_sites, 0.5)
    sa, na = pk._f64(s), pk._f64(n)
    assert c._lib.dmrg_set_cideas(c._h, pk._ptr(sa), pk._ptr(na)) == -4    # no Hamiltonian yet
    _load(c, h)
    assert c._lib.dmrg_set_cideas(c._h, pk._ptr(pk._f64(s)), None) == -1
    bad = s.copy()
    bad[3] = -1.0
    with pytest.raises(pk.DMRGError) as e:
        c.set_cideas(bad, n)
    assert e.value.status == -1
    c.set_cideas(s, n)
    c.set_cideas(None, None)
