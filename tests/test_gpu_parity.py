"""Parity of the HIP path (through the C ABI) with the CPU oracle.

* H_eff psi equals the Hamiltonian applied to determinants, element by
  element, at every bond of full sweeps (determinant-selection mode, where
  every block state is one determinant and the oracle's Slater-Condon rows
  are the expected values), including the full 56Ni-sized pf 8p+8n space at
  D = 2048 on sampled rows;
* sweep energies equal the oracle's (tests/golden, written by the oracle
  alone) to 1e-8 relative in FP64 and 1e-6 in the mixed modes;
* exact diagonalisation and closed forms: p shell at exact D, the degenerate
  pairing model at the pf 8p+8n size;
* orbital correlations, entropies and mutual information of measuring sweeps
  equal the oracle's, the exact ground vector's at full rank, and the
  pairing closed form at the pf 8p+8n size.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import ed
from workloads import (WORKLOADS, make_hamiltonian, make_pairing, make_space, random_ordering)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_energies.json")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def pk():
    import paper_1507_00161_amd as pk
    pk.library()   # raises if the HIP library is missing: no fallback
    return pk


def _ctx(pk, h, **kw):
    c = pk.Context(**kw)
    sp = h.space
    c.load_hamiltonian(sp.species, sp.two_m, h.eps, h.V.ravel(), h.n_p, h.n_n, h.two_M)
    return c


def _apply(c, x, torch_dev, prec=0):
    import torch
    xt = torch.tensor(x, device=torch_dev)
    yt = torch.zeros_like(xt)
    c.heff_apply(xt, yt, prec)
    torch.cuda.synchronize()
    return yt.cpu().numpy()


def _chain(h, order):
    return h.eps[order], h.V[np.ix_(order, order, order, order)]


# Element-wise bounds of the reduced-precision products.  With u the unit
# roundoff of the operand type (2^-24 FP32, 2^-8 BF16), a product of an
# operator entry, a psi entry and a second operator entry picks up at most
# five roundings of relative size u/2 (psi, both operators, the alpha scaling
# and the intermediate Z), so the input part of the error of output row r is
# at most 2.5 u S_r, S_r = sum over the row's Slater-Condon terms of
# |term| |x| (ed.abs_apply_rows, >= (|H||x|)_r), since every GEMM product is
# bounded by one such term in a determinant basis.  FP32 accumulation adds
# roundings of the running sums; these are sums of terms of both signs, and
# their rounding errors stay of the order of u S_r.  The bounds below are
# c u S_r with c = 4 (BF16: inputs only; its FP32 accumulation is 2^16 finer)
# and c = 64 (FP32: inputs plus accumulation, with a wide margin).
U_LOW = {1: 2.0 ** -24, 2: 2.0 ** -8}
C_LOW = {1: 64.0, 2: 4.0}


def _check_low(y_low, ref, scale, prec):
    err = np.abs(y_low - ref)
    bound = C_LOW[prec] * U_LOW[prec] * scale + 1e-300
    assert np.all(err <= bound), (prec, float((err / bound).max()))
    return float((err / (U_LOW[prec] * np.maximum(scale, 1e-300))).max())


@pytest.mark.parametrize("space,n_p,n_n,two_M,D,rand", [
    ("p", 2, 2, 0, 6, False),
    ("sd", 2, 3, 1, 10, True),
    ("pf", 3, 2, 1, 12, True),
])
def test_heff_equals_slater_condon_every_bond(pk, torch_dev, space, n_p, n_n, two_M, D, rand):
    sp = make_space(space)
    h = make_hamiltonian(sp, 31, n_p, n_n, two_M)
    order = random_ordering(sp.n_sites, 2) if rand else np.arange(sp.n_sites)
    eps_c, V_c = _chain(h, order)
    c = _ctx(pk, h, davidson_tol=1e-9, select_basis=1, seed=99)
    rng = np.random.default_rng(0)
    nsteps = 2 * (sp.n_sites - 1)
    worst = 0.0
    for st in range(nsteps):
        c.sweep_steps(D, 0 if st == 0 else 1, order)
        bond, dim, qn, dims = c.heff_layout()
        assert dims.prod(axis=1).sum() == dim
        cfg = c.heff_configs()
        assert len(set(cfg.tolist())) == dim
        x = rng.normal(size=dim)
        y = _apply(c, x, torch_dev)
        rows = np.arange(dim) if dim <= 300 else rng.choice(dim, 300, replace=False)
        ref = ed.apply_rows(eps_c, V_c, cfg, x, rows)
        worst = max(worst, np.abs(y[rows] - ref).max() / max(1.0, np.abs(ref).max()))
        scale = ed.abs_apply_rows(eps_c, V_c, cfg, x, rows)
        for prec in (1, 2):
            _check_low(_apply(c, x, torch_dev, prec)[rows], ref, scale, prec)
    assert worst < 1e-12


def test_heff_full_size_pf_8p8n_D2048_sampled_rows(pk, torch_dev):
    """The 56Ni-sized space at the benchmark's bond dimension and precisions:
    sampled output rows of H_eff psi against Slater-Condon rows."""
    h = WORKLOADS["pf_8p8n"].hamiltonian()
    c = _ctx(pk, h, davidson_tol=1e-6, select_basis=1, seed=3)
    c.sweep_steps(2048, 19)          # to the middle of the chain
    bond, dim, qn, dims = c.heff_layout()
    assert bond == 19 and dim > 10000
    cfg = c.heff_configs()
    rng = np.random.default_rng(1)
    x = rng.normal(size=dim)
    rows = rng.choice(dim, 120, replace=False)
    ref = ed.apply_rows(h.eps, h.V, cfg, x, rows)
    y64 = _apply(c, x, torch_dev, 0)
    assert np.abs(y64[rows] - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())
    scale = ed.abs_apply_rows(h.eps, h.V, cfg, x, rows)
    for prec in (1, 2):
        _check_low(_apply(c, x, torch_dev, prec)[rows], ref, scale, prec)


@pytest.mark.parametrize("name,D", [("pfg9_12p12n", 2048), ("pfg9_12p12n_M2", 1024)])
def test_heff_full_size_pfg9_sampled_rows(pk, torch_dev, name, D):
    """The 64Ge-sized pf + g9/2 space (60 sites, 12p + 12n, 2M = 0 and 4) at
    the middle bond: sampled output rows of H_eff psi against Slater-Condon
    rows, FP64 to 1e-11, and the mixed products within their precision."""
    h = WORKLOADS[name].hamiltonian()
    c = _ctx(pk, h, davidson_tol=1e-6, select_basis=1, seed=5)
    c.sweep_steps(D, 29)
    bond, dim, qn, dims = c.heff_layout()
    assert bond == 29 and dim > 10000
    cfg = c.heff_configs()
    rng = np.random.default_rng(2)
    x = rng.normal(size=dim)
    rows = rng.choice(dim, 80, replace=False)
    ref = ed.apply_rows(h.eps, h.V, cfg, x, rows)
    y64 = _apply(c, x, torch_dev, 0)
    assert np.abs(y64[rows] - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())
    scale = ed.abs_apply_rows(h.eps, h.V, cfg, x, rows)
    for prec in (1, 2):
        _check_low(_apply(c, x, torch_dev, prec)[rows], ref, scale, prec)


def test_heff_is_symmetric_and_linear(pk, torch_dev):
    h = WORKLOADS["sd_4p4n"].hamiltonian()
    c = _ctx(pk, h, davidson_tol=1e-8, noise=1e-4, noise_sweeps=1, seed=2)
    c.sweep(24)
    c.sweep_steps(24, 11)
    bond, dim, _, _ = c.heff_layout()
    rng = np.random.default_rng(3)
    x1, x2 = rng.normal(size=dim), rng.normal(size=dim)
    y1, y2 = _apply(c, x1, torch_dev), _apply(c, x2, torch_dev)
    assert abs(x2 @ y1 - x1 @ y2) < 1e-11 * abs(x2 @ y1) + 1e-11
    y12 = _apply(c, 2.0 * x1 - 3.0 * x2, torch_dev)
    assert np.abs(y12 - (2 * y1 - 3 * y2)).max() < 1e-11 * np.abs(y12).max()


@pytest.mark.parametrize("precision", [1, 2])
def test_mixed_davidson_at_the_product_limit_returns_the_fp64_rayleigh_quotient(pk, torch_dev, precision):
    """A mixed solve stopped by davidson_max_iter with reduced-precision
    columns in its subspace still reports the FP64 Rayleigh quotient of the
    vector it returns.  The state at the turning point (bond N - 2) is the
    solve's own result, so theta = psi . H64 psi there."""
    h = WORKLOADS["sd_4p4n"].hamiltonian()
    c = _ctx(pk, h, precision=precision, davidson_tol=1e-12, davidson_max_iter=3, seed=4)
    r = c.sweep_steps(64, h.space.n_sites - 1)
    assert r["code"] == 1 and r["not_converged"] > 0
    bond, dim, _, _ = c.heff_layout()
    assert bond == h.space.n_sites - 2
    psi = c.get_psi()
    assert abs(psi @ psi - 1.0) < 1e-12
    th = psi @ _apply(c, psi, torch_dev, 0)
    assert abs(r["last_theta"] - th) <= 1e-13 * abs(th), (r["last_theta"], th)


@pytest.mark.parametrize("name,D", [("sd_4p4n", 48), ("pf_8p8n", 64)])
def test_fp64_check_leaves_the_run_unchanged(pk, name, D):
    """dmrg_check_fp64 repeats every mixed solve in FP64 from the same guess:
    the energies of the run are bit-identical to a run without it, every solve
    is paired, and the paired energies agree within the mixed tolerance."""
    h = WORKLOADS[name].hamiltonian()
    opts = dict(precision=1, davidson_tol=1e-7, noise=1e-4, noise_sweeps=1, seed=5)
    a, b = _ctx(pk, h, **opts), _ctx(pk, h, **opts)
    b.check_fp64(True)
    for _ in range(2):
        ra, rb = a.sweep(D), b.sweep(D)
        assert ra["energy"] == rb["energy"] and ra["last_theta"] == rb["last_theta"]
        assert ra["check_solves"] == 0 and rb["check_solves"] == rb["solves"] > 0
        assert rb["check_max_rel"] <= 1e-6
    b.check_fp64(False)
    assert b.sweep(D)["check_solves"] == 0


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _golden_ham(spec):
    if isinstance(spec, str):
        return WORKLOADS[spec].hamiltonian()
    space, seed, n_p, n_n, two_M = spec
    return make_hamiltonian(make_space(space), seed, n_p, n_n, two_M)


@pytest.mark.parametrize("name", ["p_2p2n_D64", "p_2p2n_M2_D16", "sd_4p4n_D32", "sd_3p2n_M1_rand_D24",
                                  "pf_8p8n_D32", "pfg9_12p12n_D16", "pfg9_12p12n_M2_D16",
                                  "pfg9_12p12n_D64", "pfg9_12p12n_M2_D64"])
@pytest.mark.parametrize("precision,rtol", [(0, 1e-8), (1, 1e-6), (2, 1e-6)])
def test_sweep_energies_match_oracle(pk, name, precision, rtol):
    g = _golden()
    case = g["cases"][name]
    h = _golden_ham(case["workload"])
    sp = h.space
    order = None if case["ordering_seed"] is None else random_ordering(sp.n_sites, case["ordering_seed"])
    c = _ctx(pk, h, precision=precision, **g["options"])
    prev = None
    for D, e_ref in zip(case["D"], case["energies"]):
        r = c.sweep(D, order)
        assert r["code"] == 0
        assert abs(r["energy"] - e_ref) <= rtol * abs(e_ref), (D, r["energy"], e_ref)
        if "exact" in case:
            assert r["energy"] >= case["exact"] - 1e-9        # variational bound
        # the energy change between sweeps that the paper's stopping rule reads
        if prev is None:
            assert math.isnan(r["delta_energy"])
        else:
            assert r["delta_energy"] == r["energy"] - prev
        prev = r["energy"]
    assert c.energy() == r["energy"]


@pytest.mark.parametrize("precision,rtol", [(0, 1e-8), (1, 1e-6)])
def test_benchmark_schedule_matches_oracle(pk, precision, rtol):
    """The benchmark's own workload and schedule (pf 8p+8n, the 56Ni-sized
    space; D = 512, 512, 1024, 1024, then 2048; the benchmark's options):
    every sweep energy against the oracle's on the same schedule
    (tests/golden/oracle_bench_schedule.json), FP64 to 1e-8 and mixed FP32
    to 1e-6 relative."""
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_bench_schedule.json")
    with open(path) as f:
        g = json.load(f)
    assert g["workload"] == "pf_8p8n" and len(g["D"]) >= 5
    h = WORKLOADS["pf_8p8n"].hamiltonian()
    c = _ctx(pk, h, precision=precision, **g["options"])
    for k, (D, e_ref) in enumerate(zip(g["D"], g["energies"])):
        r = c.sweep(D)
        assert r["code"] in (0, 1)       # the first sweep from the hash start may hit the product limit
        assert abs(r["energy"] - e_ref) <= rtol * abs(e_ref), (k, D, r["energy"], e_ref)


@pytest.mark.parametrize("name", ["p_2p2n_cideas", "sd_4p4n_cideas", "pf_8p8n_cideas"])
@pytest.mark.parametrize("precision,rtol", [(0, 1e-8), (1, 1e-6)])
def test_cideas_sweeps_match_oracle(pk, name, precision, rtol):
    """The CI-DEAS start (environment blocks from the CI spaces of an active
    space grown by the entropy profile of a measuring run, the profile stored
    with the case): sweep energies equal the oracle's."""
    g = _golden()
    case = g["cases"][name]
    h = _golden_ham(case["workload"])
    sp = h.space
    order = None if case["ordering_seed"] is None else random_ordering(sp.n_sites, case["ordering_seed"])
    opts = {k: v for k, v in case["options"].items() if k != "cideas"}
    c = _ctx(pk, h, precision=precision, **g["options"], **opts)
    c.set_cideas(case["cideas_s1"], case["cideas_n1"])
    for D, e_ref in zip(case["D"], case["energies"]):
        r = c.sweep(D, order)
        assert r["code"] in (0, 1)
        assert abs(r["energy"] - e_ref) <= rtol * abs(e_ref), (D, r["energy"], e_ref)


@pytest.mark.parametrize("name", ["p_2p2n_dbss", "sd_4p4n_dbss"])
@pytest.mark.parametrize("precision,rtol", [(0, 1e-8), (1, 1e-6)])
def test_dbss_sweeps_match_oracle(pk, name, precision, rtol):
    """Dynamic block-state selection (kept count from the truncation error,
    within [d_min, D]): sweep energies and, in FP64, the largest kept count of
    each sweep equal the oracle's."""
    g = _golden()
    case = g["cases"][name]
    h = _golden_ham(case["workload"])
    c = _ctx(pk, h, precision=precision, **g["options"], **case["options"])
    for D, e_ref, k_ref in zip(case["D"], case["energies"], case["kept_max"]):
        r = c.sweep(D)
        assert r["code"] == 0
        assert abs(r["energy"] - e_ref) <= rtol * abs(e_ref), (D, r["energy"], e_ref)
        if precision == 0:
            assert r["kept_max"] == k_ref
        assert r["discarded_max"] <= case["options"]["trunc_eps"] or r["kept_max"] == D


@pytest.mark.parametrize("name", ["p_2p2n_two", "sd_4p4n_two"])
@pytest.mark.parametrize("precision,rtol", [(0, 1e-8), (1, 1e-6)])
def test_two_state_sweeps_match_oracle(pk, name, precision, rtol):
    """The two lowest states targeted at once: both sweep energies equal the
    oracle's (and at full rank, p shell, the two lowest ED eigenvalues)."""
    g = _golden()
    case = g["cases"][name]
    h = _golden_ham(case["workload"])
    c = _ctx(pk, h, precision=precision, **g["options"], **case["options"])
    for D, e0, e1 in zip(case["D"], case["energies"], case["energies_excited"]):
        r = c.sweep(D)
        # 1 = a solve stopped at the product limit; the oracle stops at the
        # same limit (the second state from the random start, first sweep)
        assert r["code"] in (0, 1)
        assert abs(r["energy"] - e0) <= rtol * abs(e0), (D, r["energy"], e0)
        assert abs(r["energy_excited"] - e1) <= rtol * abs(e1), (D, r["energy_excited"], e1)
        assert r["energy_excited"] >= r["energy"]
    assert c.energy() == r["energy"]


@pytest.mark.parametrize("name", ["pfg9_12p12n", "pfg9_12p12n_M2"])
def test_pfg9_ramp_lowers_the_energy(pk, name):
    """The 60-site pf + g9/2 space (12p + 12n, J_z = 0 and 2) on a short ramp
    in mixed FP32: each sweep stays at or below the previous one and below
    the oracle's D = 16 energies."""
    g = _golden()["cases"][name + "_D16"]
    h = WORKLOADS[name].hamiltonian()
    c = _ctx(pk, h, precision=1, davidson_tol=1e-7, noise=1e-4, noise_sweeps=1, seed=7)
    prev = None
    for D in (32, 64, 128):
        r = c.sweep(D)
        assert r["code"] in (0, 1) and np.isfinite(r["energy"])
        if prev is not None:
            assert r["energy"] <= prev + 1e-7
        prev = r["energy"]
    assert prev < min(g["energies"])


def test_p_shell_exact_bond_dimension_equals_ed(pk):
    h = WORKLOADS["p_2p2n"].hamiltonian()
    e0 = ed.ground_energy(h.eps, h.V, h.space.species, h.space.two_m, 2, 2, 0)[0]
    for order in (None, random_ordering(12, 4)):
        c = _ctx(pk, h, davidson_tol=1e-10, noise=1e-4, noise_sweeps=1)
        for _ in range(2):
            r = c.sweep(64, order)
        assert abs(r["energy"] - e0) < 1e-10


def test_pairing_closed_form_pf_8p8n(pk):
    """Degenerate pairing in the 56Ni-sized space (pf, 8p + 8n):
    E = 16 eps - G [4 (10 - 4 + 1) * 2] = 16 eps - 56 G.  The state has large
    exactly degenerate density-matrix multiplets (dropped whole at the cut),
    so it needs D = 1024 here; smaller D stays in a trapped state."""
    sp = make_space("pf")
    G, eps0 = 0.35, -1.25
    h = make_pairing(sp, G, eps0, 8, 8)
    c = _ctx(pk, h, davidson_tol=1e-9, noise=1e-4, noise_sweeps=2, seed=5)
    for _ in range(2):
        r = c.sweep(1024)
    assert abs(r["energy"] - (16 * eps0 - 56 * G)) < 1e-8


# ------------------------------------ orbital correlations and entropies
def _chain_view(m, order, n):
    """Library outputs (site indices) viewed in chain positions, as the oracle
    stores its raw correlations."""
    o = np.arange(n) if order is None else np.asarray(order)
    return m["n1"][o], m["nn"][np.ix_(o, o)], m["hop"][np.ix_(o, o)]


# Entropy tolerance: the golden states are converged to a Davidson residual of
# 1e-9, so with gaps above 0.01 MeV the correlations (quadratic in psi) agree
# to ~1e-7, and entropies (slope |ln(n/(1-n))| < 10 for these occupations) to
# ~1e-6.
@pytest.mark.parametrize("name", ["p_2p2n_ent", "sd_4p4n_ent", "sd_3p2n_M1_rand_ent", "pf_8p8n_ent",
                                  "sd_4p4n_two_ent", "sd_4p4n_dbss_ent"])
@pytest.mark.parametrize("precision,rtol", [(0, 1e-8), (1, 1e-6)])
def test_entropies_match_oracle(pk, name, precision, rtol):
    """Measuring sweeps (also with two targeted states, where the first state is
    measured, and with dynamic block states): energies, the correlations
    <n_i>, <n_i n_j>, <c+_i c_j> and the one-orbital entropies and mutual
    information equal the oracle's."""
    g = _golden()
    case = g["cases"][name]
    h = _golden_ham(case["workload"])
    n = h.space.n_sites
    order = None if case["ordering_seed"] is None else random_ordering(n, case["ordering_seed"])
    opts = dict(case["options"], measure=1)
    c = _ctx(pk, h, precision=precision, **g["options"], **opts)
    for D, e_ref in zip(case["D"], case["energies"]):
        r = c.sweep(D, order)
        # 1 = a solve stopped at the product limit, as the oracle's does (second state, first sweep)
        assert r["code"] == 0 or (r["code"] == 1 and opts.get("n_states") == 2)
        assert abs(r["energy"] - e_ref) <= rtol * abs(e_ref), (D, r["energy"], e_ref)
    m = c.orbital_entropies()
    assert np.abs(m["s1"] - np.array(case["s1"])).max() < 1e-6
    assert np.abs(m["mutual"] - np.array(case["mutual"])).max() < 1e-6
    assert np.array_equal(m["mutual"], m["mutual"].T) and np.all(np.diag(m["mutual"]) == 0.0)
    n1, nn, hop = _chain_view(m, order, n)
    cor = case["correlations"]
    iu = np.triu_indices(n, 1)
    assert np.abs(n1 - np.array(cor["n1"])).max() < 1e-7
    assert np.abs(nn[iu] - np.array(cor["nn"])[iu]).max() < 1e-7
    assert np.abs(hop[iu] - np.array(cor["hop"])[iu]).max() < 1e-7


def test_entropies_at_full_rank_equal_ed(pk):
    """p shell at a bond dimension above the exact Schmidt rank: entropies and
    mutual information equal those of the exact ground vector, brute force
    over determinants, in any chain ordering."""
    from oracle import entropy
    h = WORKLOADS["p_2p2n"].hamiltonian()
    sp = h.space
    E0, basis, vec = ed.ground_state(h.eps, h.V, sp.species, sp.two_m, 2, 2, 0)
    s1e, Ie = entropy.entropies_of_vector(basis, vec, sp.n_sites)
    n, nn, hop = entropy.correlations_from_vector(basis, vec, sp.n_sites)
    for order in (None, random_ordering(12, 4)):
        c = _ctx(pk, h, davidson_tol=1e-10, noise=1e-4, noise_sweeps=1, measure=1)
        for _ in range(2):
            r = c.sweep(64, order)
        assert abs(r["energy"] - E0) < 1e-10
        m = c.orbital_entropies()
        assert np.abs(m["s1"] - s1e).max() < 1e-8 and np.abs(m["mutual"] - Ie).max() < 1e-8
        assert np.abs(m["n1"] - n).max() < 1e-9
        iu = np.triu_indices(sp.n_sites, 1)
        assert np.abs(m["nn"][iu] - nn[iu]).max() < 1e-9
        if order is None:   # <c+_i c_j> carries the Jordan-Wigner order of the chain
            assert np.abs(m["hop"][iu] - hop[iu]).max() < 1e-9


def test_entropies_pairing_closed_form_pf_8p8n(pk):
    """Degenerate pairing in the 56Ni-sized space (pf, 40 sites, 8p + 8n):
    the ground state is the product of the seniority-zero states of 4 pairs in
    Omega = 10 for each species, so <n_i> = 2/5; time-reversed partners have
    rho = diag(3/5, 0, 0, 2/5); other like-particle pairs have
    <n_i n_j> = 4*3/(10*9) = 2/15 and no hopping; protons and neutrons are
    uncorrelated.  Every entropy and mutual information at full size."""
    import math
    sp = make_space("pf")
    h = make_pairing(sp, 0.35, -1.25, 8, 8)
    c = _ctx(pk, h, davidson_tol=1e-9, noise=1e-4, noise_sweeps=2, seed=5, measure=1)
    for _ in range(2):
        r = c.sweep(1024)
    assert abs(r["energy"] - (16 * -1.25 - 56 * 0.35)) < 1e-8
    m = c.orbital_entropies()

    def ent(ws):
        return -sum(w * math.log(w) for w in ws if w > 0)

    h1 = ent([0.4, 0.6])
    other = 2 * h1 - ent([1 / 3, 4 / 15, 4 / 15, 2 / 15])
    assert np.abs(m["n1"] - 0.4).max() < 1e-7
    assert np.abs(m["s1"] - h1).max() < 1e-6
    n = sp.n_sites
    want = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i == j or sp.species[i] != sp.species[j]:
                continue
            partner = sp.shell[i] == sp.shell[j] and sp.two_m[i] == -sp.two_m[j]
            want[i, j] = h1 if partner else other
    assert np.abs(m["mutual"] - want).max() < 1e-6
    assert np.abs(m["hop"]).max() < 1e-7


def test_entropies_full_size_pf_8p8n_D2048(pk):
    """The benchmark's workload and schedule (pf 8p+8n, D = 512, 512, 1024,
    1024, 2048) with measuring sweeps: mixed FP32 and FP64 give the same
    energy (1e-6) and the same entropies and mutual information (1e-5); at
    this size 0 <= s_i <= ln 2, 0 <= I_ij <= 2 ln 2 (subadditivity, which a
    pair's rho_ij from one normalised state obeys), occupations in [0, 1]
    summing to about 8 per species (each from its own bond), and
    |<c+_i c_j>| <= 1/2."""
    import math
    h = WORKLOADS["pf_8p8n"].hamiltonian()
    out = {}
    for prec in (1, 0):
        c = _ctx(pk, h, precision=prec, davidson_tol=1e-7, noise=1e-4, noise_sweeps=2, seed=1507, measure=1)
        for D in (512, 512, 1024, 1024, 2048):
            r = c.sweep(D)
            assert r["code"] in (0, 1)
        out[prec] = (r["energy"], c.orbital_entropies())
        c.close()
    (e32, m32), (e64, m64) = out[1], out[0]
    assert abs(e32 - e64) <= 1e-6 * abs(e64)
    assert np.abs(m32["s1"] - m64["s1"]).max() < 1e-5
    assert np.abs(m32["mutual"] - m64["mutual"]).max() < 1e-5
    for m in (m32, m64):
        s1, I, n1, nn, hop = m["s1"], m["mutual"], m["n1"], m["nn"], m["hop"]
        assert s1.min() >= 0.0 and s1.max() <= math.log(2) + 1e-12
        assert I.min() >= -1e-9 and I.max() <= 2 * math.log(2) + 1e-12
        assert np.array_equal(I, I.T)
        assert n1.min() >= -1e-12 and n1.max() <= 1.0 + 1e-12
        assert abs(n1[:20].sum() - 8.0) < 0.05 and abs(n1[20:].sum() - 8.0) < 0.05
        assert (np.abs(hop) <= 0.5 + 1e-12).all()   # |<c+_i c_j>| <= sqrt(<n_i><1 - n_j>)-type bound


@pytest.mark.parametrize("precision,rtol,group,graph", [
    (0, 1e-8, 1, 0), (1, 1e-6, 1, 0), (1, 1e-6, 0, 0),
    pytest.param(1, 1e-6, 0, 1, marks=pytest.mark.skip(
        reason="captured-graph products in concurrent contexts ended the process with a host segmentation "
               "fault (cause not found); dmrg_sweep_many now launches every product directly"))])
def test_sweep_many_matches_oracle_batched(pk, precision, rtol, group, graph):
    """The independent small solves of the batched workload (seeded p, sd and
    pf instances, 2..8 particles per species, D from 64 to 512), advanced
    together by dmrg_sweep_many with their products launched in groups
    (group_products = 1) or each context on its own stream (0): the
    first-sweep energy of every instance the oracle has
    (tests/golden/oracle_batched.json: p and sd at every D, pf at D <= 128)."""
    from workloads import batched_instances
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_batched.json")
    with open(path) as f:
        g = json.load(f)
    ws = batched_instances(g["count"])
    idx = sorted(int(i) for i in g["instances"])
    assert len(idx) >= 20
    ctxs = [_ctx(pk, ws[i].hamiltonian(), precision=precision, group_products=group, graph=graph, **g["options"])
            for i in idx]
    st, out = pk.sweep_many(ctxs, [ws[i].D_schedule[0] for i in idx])
    assert st in (0, 1)
    for i, o in zip(idx, out):
        e_ref = g["instances"][str(i)]["energy"]
        assert o["status"] in (0, 1)
        assert abs(o["energy"] - e_ref) <= rtol * abs(e_ref), (i, o["energy"], e_ref)


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_products_match_direct_launches(pk, torch_dev, precision):
    """Option graph (each bond's product captured once in a HIP graph and
    replayed): sweeps are bit-identical to direct launches, and repeated
    products at one bond, with eager work and synchronisations between the
    replays, each equal the direct product exactly."""
    import torch
    h = WORKLOADS["sd_4p4n"].hamiltonian()
    opts = dict(precision=precision, davidson_tol=1e-8, noise=1e-4, noise_sweeps=1, seed=4)
    a, b = _ctx(pk, h, **opts), _ctx(pk, h, graph=1, **opts)
    for D in (32, 48):
        ra, rb = a.sweep(D), b.sweep(D)
        assert ra["energy"] == rb["energy"] and ra["products_low"] == rb["products_low"]
    a.sweep_steps(48, 9)
    b.sweep_steps(48, 9)
    _, dim, _, _ = a.heff_layout()
    rng = np.random.default_rng(5)
    for k in range(4):
        x = torch.tensor(rng.normal(size=dim), device=torch_dev)
        ya, yb = torch.empty_like(x), torch.empty_like(x)
        a.heff_apply(x, ya, precision)
        b.heff_apply(x, yb, precision)
        z = (x * 2.0).sum()            # eager work between the replays
        torch.cuda.synchronize()
        assert torch.isfinite(z)
        assert torch.equal(ya, yb), k


def test_sweep_many_matches_single_contexts(pk):
    """Concurrent sweeps of independent contexts (several host threads, one
    stream each) give the results of one-at-a-time sweeps."""
    from workloads import batched_instances
    hs = [WORKLOADS["p_2p2n"].hamiltonian(), make_hamiltonian(make_space("sd"), 5, 2, 2, 0)]
    hs += [w.hamiltonian() for w in batched_instances(6)]
    precs = [0, 1] * (len(hs) // 2)
    single = []
    for h, p in zip(hs, precs):
        c = _ctx(pk, h, davidson_tol=1e-9, seed=3, precision=p)
        single.append(c.sweep(24)["energy"])
        c.close()
    ctxs = [_ctx(pk, h, davidson_tol=1e-9, seed=3, precision=p) for h, p in zip(hs, precs)]
    st, out = pk.sweep_many(ctxs, [24] * len(hs))
    assert st == 0
    for o, e in zip(out, single):
        assert o["status"] == 0 and abs(o["energy"] - e) <= 1e-12 * abs(e)
    for c in ctxs:
        c.close()


def test_sweep_many_measuring_contexts_match_single(pk):
    """Measuring sweeps of independent contexts advanced together (one host
    thread and stream each) give the entropies of one-at-a-time sweeps."""
    from workloads import batched_instances
    hs = [WORKLOADS["p_2p2n"].hamiltonian()] + [w.hamiltonian() for w in batched_instances(4)]
    single = []
    for h in hs:
        c = _ctx(pk, h, davidson_tol=1e-9, seed=3, measure=1)
        c.sweep(24)
        single.append(c.orbital_entropies())
        c.close()
    ctxs = [_ctx(pk, h, davidson_tol=1e-9, seed=3, measure=1) for h in hs]
    st, out = pk.sweep_many(ctxs, [24] * len(hs))
    assert st in (0, 1)
    for c, ref in zip(ctxs, single):
        m = c.orbital_entropies()
        assert np.abs(m["s1"] - ref["s1"]).max() <= 1e-12
        assert np.abs(m["mutual"] - ref["mutual"]).max() <= 1e-12
        c.close()
