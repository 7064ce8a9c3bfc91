"""dmrg_heff_apply_noalloc (fixed device scratch, no allocation) against
dmrg_heff_apply, through the C ABI: two calls in a row, the second on a
smaller bond, in every precision, and the size check on a bond whose
intermediates do not fit the fixed array."""
import numpy as np
import pytest

from workloads import WORKLOADS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00161_amd as pk
    pk.library()
    return pk


def _ctx(pk, name, **kw):
    h = WORKLOADS[name].hamiltonian()
    sp = h.space
    c = pk.Context(**kw)
    c.load_hamiltonian(sp.species, sp.two_m, h.eps, h.V.ravel(), h.n_p, h.n_n, h.two_M)
    return c


def _both(c, x, prec):
    import torch
    xt = torch.tensor(x, device="cuda:0")
    y1 = torch.full_like(xt, np.nan)
    y2 = torch.full_like(xt, np.nan)
    c.heff_apply(xt, y1, prec)
    c.heff_apply_noalloc(xt, y2, prec)
    torch.cuda.synchronize()
    return y1.cpu().numpy(), y2.cpu().numpy()


def test_noalloc_matches_apply_two_calls(pk):
    # first call: sd 4p+4n at a middle bond (larger); second: p 2p+2n (smaller)
    big = _ctx(pk, "sd_4p4n", precision=1, davidson_tol=1e-8, noise=1e-4, noise_sweeps=1, seed=3)
    big.sweep(48)
    big.sweep_steps(48, 11)
    small = _ctx(pk, "p_2p2n", precision=2, davidson_tol=1e-8, seed=3)
    small.sweep(16)
    small.sweep_steps(16, 5)
    _, d_big, _, _ = big.heff_layout()
    _, d_small, _, _ = small.heff_layout()
    assert d_small < d_big
    rng = np.random.default_rng(0)
    for prec in (0, 1, 2):
        for c, d in ((big, d_big), (small, d_small)):
            x = rng.normal(size=d)
            y1, y2 = _both(c, x, prec)
            assert np.all(np.isfinite(y1)) and np.all(np.isfinite(y2))
            # same plans and kernels: the same values
            assert np.array_equal(y1, y2), (prec, d, float(np.abs(y1 - y2).max()))


def test_noalloc_rejects_a_bond_beyond_the_array(pk):
    import torch
    c = _ctx(pk, "pf_8p8n", davidson_tol=1e-6, select_basis=1, seed=3)
    c.sweep_steps(1024, 19)
    _, dim, _, _ = c.heff_layout()
    x = torch.zeros(dim, dtype=torch.float64, device="cuda:0")
    y = torch.zeros_like(x)
    with pytest.raises(pk.DMRGError) as e:
        c.heff_apply_noalloc(x, y, 1)
    assert e.value.status == -5 and "static scratch" in str(e.value)
    # the context stays usable
    c.heff_apply(x, y, 1)
    torch.cuda.synchronize()
