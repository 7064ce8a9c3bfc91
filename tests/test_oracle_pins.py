"""Pins of the CPU oracle against facts it does not compute itself.

* m-scheme dimensions quoted by the paper (1.1e9 for 56Ni in the pf shell;
  1.7e14 for 64Ge in pf+g9/2, which is the positive-parity count);
* a brute-force Fock-space Hamiltonian built from Jordan-Wigner matrices
  (a construction independent of the determinant code);
* closed forms: the degenerate pairing model, V = 0, two particles;
* the DMRG projection identity H_eff = P^T H P with P a selection of
  determinants, checked element by element against Slater-Condon rules;
* DMRG at a bond dimension that holds the exact state equals ED;
* the dynamic block-state count against a search over its definition;
* orbital correlations and entropies against brute force on the exact ground
  vector, the pairing closed form and one determinant; spectral seriation of
  Robinson matrices for the ordering.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dmrg, ed, entropy, hashrand
from workloads import (WORKLOADS, make_hamiltonian, make_one_body, make_pairing, make_space,
                       random_ordering)


# ---------------------------------------------------------------- dimensions
def _parity_dim(space, n_p, n_n, two_M, l_of_shell):
    """Count determinants of positive parity: DP over sites with parity bit."""
    counts = {(0, 0, 0, 0): 1}
    for s, m, sh in zip(space.species, space.two_m, space.shell):
        l = l_of_shell[space.shells[sh]]
        nxt = dict(counts)
        for (a, b, t, p), c in counts.items():
            key = (a + (s == 0), b + (s == 1), t + int(m), (p + l) % 2)
            if key[0] <= n_p and key[1] <= n_n:
                nxt[key] = nxt.get(key, 0) + c
        counts = nxt
    return counts.get((n_p, n_n, two_M, 0), 0)


def test_mscheme_dimensions_paper():
    pf = make_space("pf")
    # 56Ni, pf shell, J_z = 0: the paper quotes 1.1e9
    d = ed.mscheme_dimension(pf.species, pf.two_m, 8, 8, 0)
    assert d == 1_087_455_228
    assert round(d / 1e9, 1) == 1.1
    pfg = make_space("pfg9")
    tot = ed.mscheme_dimension(pfg.species, pfg.two_m, 12, 12, 0)
    assert tot == 345_133_964_269_907
    l_of = {"f7/2": 3, "p3/2": 1, "f5/2": 3, "p1/2": 1, "g9/2": 4}
    pos = _parity_dim(pfg, 12, 12, 0, l_of)
    # 64Ge in pf+g9/2: the paper's 1.7e14 is the positive-parity dimension
    assert pos == 172_566_984_081_435
    assert round(pos / 1e14, 1) == 1.7


def test_mscheme_dimensions_small():
    p, sd = make_space("p"), make_space("sd")
    assert len(ed.mscheme_basis(p.species, p.two_m, 2, 2, 0)) == 51
    assert ed.mscheme_dimension(p.species, p.two_m, 2, 2, 0) == 51
    assert len(ed.mscheme_basis(sd.species, sd.two_m, 4, 4, 0)) == 28_503
    assert ed.mscheme_dimension(sd.species, sd.two_m, 4, 4, 0) == 28_503
    assert ed.mscheme_dimension(sd.species, sd.two_m, 6, 6, 0) == 93_710    # 28Si
    assert ed.mscheme_dimension(p.species, p.two_m, 2, 2, 4) == 29


# ------------------------------------------------- brute-force Fock space
def _jw_annihilators(n):
    """Dense-free sparse c_i on the 2^n Fock space, bit i = site i,
    |c> = prod_{i in c ascending} c+_i |0>."""
    dim = 1 << n
    states = np.arange(dim)
    ops = []
    for i in range(n):
        occ = (states >> i) & 1
        src = states[occ == 1]
        below = np.array([bin(s & ((1 << i) - 1)).count("1") for s in src])
        sign = np.where(below % 2, -1.0, 1.0)
        ops.append(sp.csr_matrix((sign, (src ^ (1 << i), src)), shape=(dim, dim)))
    return ops


def _fock_hamiltonian(eps, V):
    n = len(eps)
    c = _jw_annihilators(n)
    cd = [x.T.tocsr() for x in c]
    H = sum(eps[i] * (cd[i] @ c[i]) for i in range(n))
    for i, j, k, l in itertools.product(range(n), repeat=4):
        v = V[i, j, k, l]
        if v != 0.0:
            H = H + 0.25 * v * (cd[i] @ cd[j] @ c[l] @ c[k])
    return H.tocsr()


def _small_space(n_per_species=4):
    """A 2 x 4-site space (p3/2-like) for brute force."""
    from workloads import Space
    sp_ = np.array([0] * n_per_species + [1] * n_per_species, np.int32)
    tm = np.array([-3, -1, 1, 3] * 2, np.int32)
    sh = np.zeros(2 * n_per_species, np.int32)
    return Space("p32", ("p3/2",), sp_, tm, sh)


def test_hamiltonian_generator_symmetries():
    h = WORKLOADS["sd_4p4n"].hamiltonian()
    V = h.V
    assert np.allclose(V, -V.transpose(1, 0, 2, 3))
    assert np.allclose(V, -V.transpose(0, 1, 3, 2))
    assert np.allclose(V, V.transpose(2, 3, 0, 1))
    s, m = h.space.species, h.space.two_m
    nz = np.argwhere(V != 0)
    assert np.all(m[nz[:, 0]] + m[nz[:, 1]] == m[nz[:, 2]] + m[nz[:, 3]])
    assert np.all(np.sort(s[nz[:, :2]], 1) == np.sort(s[nz[:, 2:]], 1))


@pytest.mark.parametrize("target", [(1, 1, 0), (2, 1, 1), (2, 2, 0), (2, 2, 2)])
def test_ed_matches_fock_bruteforce(target):
    space = _small_space()
    h = make_hamiltonian(space, 77, *target)
    Hf = _fock_hamiltonian(h.eps, h.V)
    basis = ed.mscheme_basis(space.species, space.two_m, *target)
    Hd = ed.hamiltonian_matrix(h.eps, h.V, basis).toarray()
    ref = Hf.toarray()[np.ix_(basis.astype(np.int64), basis.astype(np.int64))]
    assert np.abs(Hd - ref).max() < 1e-13
    # H is block diagonal in (n_p, n_n, 2M): no leakage out of the sector
    others = np.setdiff1d(np.arange(Hf.shape[0]), basis.astype(np.int64))
    assert abs(Hf.toarray()[np.ix_(others, basis.astype(np.int64))]).max() < 1e-14
    e = ed.ground_energy(h.eps, h.V, space.species, space.two_m, *target)
    assert abs(e[0] - np.linalg.eigvalsh(ref)[0]) < 1e-12


def test_ed_apply_rows_matches_matrix():
    space = _small_space()
    h = make_hamiltonian(space, 5, 2, 2, 0)
    basis = ed.mscheme_basis(space.species, space.two_m, 2, 2, 0)
    H = ed.hamiltonian_matrix(h.eps, h.V, basis)
    psi = np.random.default_rng(0).normal(size=len(basis))
    rows = [0, 3, len(basis) - 1]
    assert np.allclose(ed.apply_rows(h.eps, h.V, basis, psi, rows), (H @ psi)[rows], atol=1e-12)


def test_ed_abs_apply_rows_bounds_abs_matrix():
    """abs_apply_rows >= |H| |psi| row by row (from the sparse matrix), with
    equality for one proton and one neutron, where every off-diagonal element
    is a single Vbar and the diagonal is eps_i + eps_j + Vbar_ijij."""
    space = _small_space()
    for target, equal in (((2, 2, 0), False), ((1, 1, 0), True)):
        h = make_hamiltonian(space, 6, *target)
        basis = ed.mscheme_basis(space.species, space.two_m, *target)
        H = ed.hamiltonian_matrix(h.eps, h.V, basis)
        psi = np.random.default_rng(2).normal(size=len(basis))
        rows = range(len(basis))
        ref = abs(H) @ np.abs(psi)
        got = ed.abs_apply_rows(h.eps, h.V, basis, psi, rows)
        assert np.all(got >= ref - 1e-12)
        if equal:
            # the diagonal may cancel between eps and Vbar_ijij: compare off it
            off = abs(H - sp.diags(H.diagonal())) @ np.abs(psi)
            dia = np.abs(psi) * np.array([abs(h.eps[i]) + abs(h.eps[j]) + abs(h.V[i, j, i, j])
                                          for i, j in (sorted(b for b in range(8) if (int(c) >> b) & 1)
                                                       for c in basis)])
            assert np.allclose(got, off + dia, rtol=0, atol=1e-12)
        else:
            assert np.any(got > ref + 1e-9)      # one-body-like elements add several terms


# ---------------------------------------------------------- closed forms
def _pairing_energy(eps0, G, space, n_p, n_n):
    omega = int(np.sum(space.species == 0)) // 2
    e = eps0 * (n_p + n_n)
    for n in (n_p, n_n):
        e -= G * (n // 2) * (omega - n // 2 + 1)
    return e


@pytest.mark.parametrize("name,n_p,n_n", [("p", 2, 2), ("sd", 2, 2), ("sd", 4, 2), ("p", 4, 2)])
def test_ed_pairing_closed_form(name, n_p, n_n):
    space = make_space(name)
    h = make_pairing(space, 0.7, -1.3, n_p, n_n)
    e = ed.ground_energy(h.eps, h.V, space.species, space.two_m, n_p, n_n, 0)[0]
    assert abs(e - _pairing_energy(-1.3, 0.7, space, n_p, n_n)) < 1e-10


def test_ed_one_body_closed_form():
    space = make_space("sd")
    h = make_one_body(space, 11, 3, 2, 1)
    e = ed.ground_energy(h.eps, h.V, space.species, space.two_m, 3, 2, 1)[0]
    prot = [i for i in range(space.n_sites) if space.species[i] == 0]
    neut = [i for i in range(space.n_sites) if space.species[i] == 1]
    best = math.inf
    for a in itertools.combinations(prot, 3):
        for b in itertools.combinations(neut, 2):
            if sum(space.two_m[list(a + b)]) == 1:
                best = min(best, sum(h.eps[list(a + b)]))
    assert abs(e - best) < 1e-12


def test_ed_two_particles_direct():
    """1p + 1n: the Hamiltonian matrix is eps_i + eps_j + Vbar_ijij on the
    diagonal and Vbar_ijkl off it, in the basis c+_i c+_j |0> (i proton, j neutron)."""
    space = make_space("p")
    h = make_hamiltonian(space, 3, 1, 1, 0)
    prot = [i for i in range(12) if space.species[i] == 0]
    neut = [i for i in range(12) if space.species[i] == 1]
    pairs = [(i, j) for i in prot for j in neut if space.two_m[i] + space.two_m[j] == 0]
    M = np.array([[h.V[i, j, k, l] + (h.eps[i] + h.eps[j]) * ((i, j) == (k, l))
                   for (k, l) in pairs] for (i, j) in pairs])
    e = ed.ground_energy(h.eps, h.V, space.species, space.two_m, 1, 1, 0)[0]
    assert abs(e - np.linalg.eigvalsh(M)[0]) < 1e-12


# ------------------------------------------------------------------ hashing
def test_splitmix64_reference_sequence():
    # SplitMix64 from state 0 (Steele, Lea, Flood 2014; reference code output)
    outs, x = [], 0
    for _ in range(3):
        outs.append(hashrand.splitmix64(x))
        x = (x + 0x9E3779B97F4A7C15) & hashrand.M64
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert 0.0 <= hashrand.u01(hashrand.hkey(1, 2, 3)) < 1.0


# ----------------------------------------------------------------- DMRG
def _dmrg(h, D, sweeps, ordering=None, **kw):
    sp_ = h.space
    opts = dmrg.Options(davidson_tol=kw.pop("tol", 1e-10), noise=kw.pop("noise", 1e-4),
                        noise_sweeps=kw.pop("noise_sweeps", 2), seed=kw.pop("seed", 1507), **kw)
    o = dmrg.DMRG(h.eps, h.V, sp_.species, sp_.two_m, h.n_p, h.n_n, h.two_M, ordering, opts)
    res = [o.sweep(D) for _ in range(sweeps)]
    return o, res


def test_dmrg_exact_bond_dimension_equals_ed():
    h = WORKLOADS["p_2p2n"].hamiltonian()
    e0 = ed.ground_energy(h.eps, h.V, h.space.species, h.space.two_m, 2, 2, 0)[0]
    o, res = _dmrg(h, 64, 2)
    assert abs(res[-1]["energy"] - e0) < 1e-10
    # ordering invariance at exact D
    o2, res2 = _dmrg(h, 64, 2, ordering=random_ordering(12, 9))
    assert abs(res2[-1]["energy"] - e0) < 1e-10


def test_dmrg_variational_and_monotone_in_D():
    space = make_space("sd")
    h = make_hamiltonian(space, 21, 2, 2, 0)
    e0 = ed.ground_energy(h.eps, h.V, space.species, space.two_m, 2, 2, 0)[0]
    energies = []
    for D in (4, 8, 16):
        o, res = _dmrg(h, D, 3)
        assert all(r.theta >= e0 - 1e-10 for r in o.records)
        energies.append(res[-1]["energy"])
    assert energies[0] >= energies[1] - 1e-9 >= energies[2] - 2e-9
    assert energies[2] - e0 < energies[0] - e0


def test_dmrg_pairing_closed_form():
    space = make_space("sd")
    h = make_pairing(space, 0.5, -1.0, 2, 2)
    o, res = _dmrg(h, 64, 2)
    assert abs(res[-1]["energy"] - _pairing_energy(-1.0, 0.5, space, 2, 2)) < 1e-9


def test_dmrg_one_body_closed_form():
    space = make_space("p")
    h = make_one_body(space, 4, 3, 2, 1)
    e0 = ed.ground_energy(h.eps, h.V, space.species, space.two_m, 3, 2, 1)[0]
    o, res = _dmrg(h, 16, 2)
    assert abs(res[-1]["energy"] - e0) < 1e-10


def _check_projection(o, bond, setup, rng):
    """H_eff (from block operators) equals <c'|H|c> on the determinants that
    label the superblock basis, for a random vector, all rows."""
    enlL, Sops, enlR, Eops, terms = setup
    cfg = o.psi_configs(enlL, enlR)
    assert cfg is not None
    layout = o.psi_layout(enlL, enlR)
    psi = {q: rng.normal(size=s) for q, s in layout.items()}
    y = o.heff_apply(terms, psi)
    keys = sorted(psi)
    flat_c = np.concatenate([cfg[q].ravel() for q in keys])
    flat_psi = np.concatenate([psi[q].ravel() for q in keys])
    flat_y = np.concatenate([y[q].ravel() for q in keys])
    assert len(set(flat_c.tolist())) == len(flat_c)        # a basis of distinct determinants
    ref = ed.apply_rows(o.eps, o.V, flat_c, flat_psi, range(len(flat_c)))
    assert np.abs(flat_y - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())
    # symmetric: x^T H y == y^T H x
    x2 = {q: rng.normal(size=s) for q, s in layout.items()}
    y2 = o.heff_apply(terms, x2)
    assert abs(o.vdot(x2, y) - o.vdot(psi, y2)) < 1e-10 * max(1.0, abs(o.vdot(x2, y)))
    # conservation: every block couples S and E sectors adding up to the target
    for q in keys:
        assert q in enlL.dims and dmrg.qsub(o.T, q) in enlR.dims


@pytest.mark.parametrize("name,n_p,n_n,two_M,D", [("p", 2, 2, 0, 6), ("sd", 2, 3, 1, 10)])
def test_dmrg_projection_identity_selected_basis(name, n_p, n_n, two_M, D):
    space = make_space(name)
    h = make_hamiltonian(space, 31, n_p, n_n, two_M)
    opts = dmrg.Options(davidson_tol=1e-9, select_basis=True, seed=99)
    o = dmrg.DMRG(h.eps, h.V, space.species, space.two_m, n_p, n_n, two_M,
                  random_ordering(space.n_sites, 2), opts)
    rng = np.random.default_rng(1)
    seen = []

    def hook(oo, bond, direction, setup):
        seen.append((bond, direction))
        _check_projection(oo, bond, setup, rng)

    o.sweep(D, on_step=hook)
    o.sweep(D, on_step=hook)
    assert len(seen) == 4 * (space.n_sites - 1)
    # truncation really happened somewhere
    assert any(sum(b.dims.values()) == D for b in o.L.values())


# ------------------------------------------ dynamic block-state selection
def test_dbss_count_against_search():
    """The DBSS count against its definition by search: the smallest n whose
    discarded weight (1 - the fresh sum of the n largest weights) is at most
    eps, then clamped to [d_min, D], on random weight spectra."""
    rng = np.random.default_rng(5)
    checked = 0
    for _ in range(300):
        w = np.sort(rng.dirichlet(np.full(int(rng.integers(1, 40)), 0.3)))[::-1]
        eps = float(10.0 ** rng.uniform(-8, -0.3))
        d_min, D = int(rng.integers(0, 6)), int(rng.integers(1, 50))
        disc = [1.0 - math.fsum(w[:n]) for n in range(len(w) + 1)]
        if any(abs(d - eps) < 1e-12 for d in disc):
            continue                                    # a rounding tie at the threshold
        n = next(n for n in range(len(w) + 1) if disc[n] <= eps)
        assert dmrg.dbss_count(list(w), D, eps, d_min) == min(max(n, d_min), D, len(w))
        checked += 1
    assert checked > 250


def test_dbss_truncations_meet_the_error():
    """Along a DBSS run every truncation keeps D states or discards at most
    eps, and the count moves with eps (fewer states for a looser error)."""
    h = WORKLOADS["sd_4p4n"].hamiltonian()
    sp_ = h.space

    class Rec(dmrg.DMRG):
        def density_iso(self, rho, D):
            iso, disc = super().density_iso(rho, D)
            self.log.append((sum(U.shape[1] for U in iso.values()), disc, D))
            return iso, disc

    kept = {}
    for eps in (1e-2, 1e-3):
        o = Rec(h.eps, h.V, sp_.species, sp_.two_m, h.n_p, h.n_n, h.two_M, None,
                dmrg.Options(davidson_tol=1e-8, noise=1e-4, noise_sweeps=1, seed=7, trunc_eps=eps, d_min=4))
        o.log = []
        for _ in range(2):
            o.sweep(96)
        assert o.log and all(d <= eps + 1e-12 or n == D for n, d, D in o.log)
        kept[eps] = sum(n for n, _, _ in o.log)
    assert kept[1e-2] < kept[1e-3]


def test_dbss_exact_at_full_rank():
    """With a bond dimension above the exact Schmidt rank and a tiny error,
    DBSS reproduces exact diagonalisation."""
    h = WORKLOADS["p_2p2n"].hamiltonian()
    e0 = ed.ground_energy(h.eps, h.V, h.space.species, h.space.two_m, 2, 2, 0)[0]
    o, res = _dmrg(h, 64, 3, trunc_eps=1e-10, d_min=1)
    assert abs(res[-1]["energy"] - e0) < 1e-10
    assert res[-1]["discarded_max"] <= 1e-10


# ------------------------------------------ two lowest states at once
def test_two_state_exact_bond_dimension_equals_ed():
    """Targeting the two lowest states with their averaged density matrix:
    at a bond dimension above the exact Schmidt rank both energies are the
    two lowest eigenvalues of exact diagonalisation."""
    h = WORKLOADS["p_2p2n"].hamiltonian()
    e = ed.ground_energy(h.eps, h.V, h.space.species, h.space.two_m, 2, 2, 0, nroots=2)
    o, res = _dmrg(h, 64, 2, n_states=2)
    assert abs(res[-1]["energy"] - e[0]) < 1e-10
    assert abs(res[-1]["energy_excited"] - e[1]) < 1e-10


def test_two_state_energies_are_upper_bounds():
    """Truncated two-state runs: every step's two Ritz values bound the two
    lowest exact eigenvalues from above (Hylleraas-Undheim), and more block
    states never raise the pair."""
    space = make_space("sd")
    h = make_hamiltonian(space, 21, 2, 2, 0)
    e = ed.ground_energy(h.eps, h.V, space.species, space.two_m, 2, 2, 0, nroots=2)
    last = None
    for D in (8, 16):
        o, res = _dmrg(h, D, 3, n_states=2)
        r = res[-1]
        assert r["energy"] >= e[0] - 1e-10 and r["energy_excited"] >= e[1] - 1e-10
        assert r["energy_excited"] >= r["energy"] - 1e-10
        if last:
            assert r["energy"] <= last[0] + 1e-8 and r["energy_excited"] <= last[1] + 1e-8
        last = (r["energy"], r["energy_excited"])


# ------------------------------- orbital entropies, mutual information, ordering
def _h2(x):
    return -x * math.log(x) - (1 - x) * math.log(1 - x)


def test_correlations_from_vector_two_particles():
    """Two protons in four sites, psi = a|{0,1}> + b|{2,3}> + c|{0,2}>
    (determinants as ascending creation products): <n_i>, <n_i n_j> and the
    signed hopping element <c+_1 c_2>, worked out by hand."""
    basis = np.array(sorted([0b0011, 0b1100, 0b0101]), dtype=np.uint64)   # 3, 5, 12
    a, b, c = 0.6, 0.0, 0.8
    amp = {0b0011: a, 0b1100: b, 0b0101: c}
    vec = np.array([amp[int(x)] for x in basis])
    n, nn, hop = entropy.correlations_from_vector(basis, vec, 4)
    assert np.allclose(n, [a * a + c * c, a * a, c * c + b * b, b * b])
    assert abs(nn[0, 1] - a * a) < 1e-15 and abs(nn[0, 2] - c * c) < 1e-15 and nn[1, 2] == 0.0
    # c_2 c+_0 c+_2 |0> = -c+_0 |0> and c+_1 c+_0 |0> = -c+_0 c+_1 |0>, so
    # c+_1 c_2 |{0,2}> = +|{0,1}> and <c+_1 c_2> = a * c
    assert abs(hop[1, 2] - a * c) < 1e-15 and abs(hop[2, 1] - a * c) < 1e-15
    assert abs(hop[0, 3]) < 1e-15


@pytest.mark.parametrize("name,n_p,n_n,D,ordered", [("p", 2, 2, 64, False), ("p", 2, 2, 64, True),
                                                     ("sd", 2, 1, 128, False)])
def test_entropies_at_full_rank_equal_ed(name, n_p, n_n, D, ordered):
    """DMRG at a bond dimension above the exact Schmidt rank: the measured
    correlations and the entropies and mutual information built from them
    equal those of the exact ground vector, in any site ordering."""
    space = make_space(name)
    h = make_hamiltonian(space, 31, n_p, n_n, 1 if n_p + n_n == 3 else 0)
    E0, basis, vec = ed.ground_state(h.eps, h.V, space.species, space.two_m, h.n_p, h.n_n, h.two_M)
    n, nn, hop = entropy.correlations_from_vector(basis, vec, space.n_sites)
    s1e, Ie = entropy.entropies_of_vector(basis, vec, space.n_sites)
    ordering = random_ordering(space.n_sites, 5) if ordered else None
    o, res = _dmrg(h, D, 3, ordering=ordering, measure=True)
    assert abs(res[-1]["energy"] - E0) < 1e-10
    s1, I, m = o.entropies()
    assert np.abs(s1 - s1e).max() < 1e-9 and np.abs(I - Ie).max() < 1e-9
    assert np.abs(res[-1]["s1"] - s1).max() == 0.0
    if not ordered:
        iu = np.triu_indices(space.n_sites, 1)
        assert np.abs(m["n1"] - n).max() < 1e-9
        assert np.abs(m["nn"][iu] - nn[iu]).max() < 1e-9
        assert np.abs(m["hop"][iu] - hop[iu]).max() < 1e-9
        assert np.count_nonzero(np.abs(hop[iu]) > 1e-6) > 0


def test_entropies_pairing_closed_form():
    """Degenerate pairing with one proton pair and one neutron pair: the ground
    state is the product of the two uniform pair states, so <n_i> = 1/Omega,
    time-reversed partners share I = h(1/Omega), other like-particle pairs
    have rho_ij = diag(1 - 2/Omega, 1/Omega, 1/Omega, 0), and protons and
    neutrons are uncorrelated."""
    space = make_space("sd")
    h = make_pairing(space, 0.5, -1.0, 2, 2)
    o, res = _dmrg(h, 128, 3, measure=True)
    s1, I, _ = o.entropies()
    om = int(np.sum(space.species == 0)) // 2
    x = 1.0 / om
    s3 = -(1 - 2 * x) * math.log(1 - 2 * x) - 2 * x * math.log(x)
    N = space.n_sites
    assert np.abs(s1 - _h2(x)).max() < 1e-8
    for i in range(N):
        for j in range(i + 1, N):
            if space.species[i] != space.species[j]:
                want = 0.0
            elif space.shell[i] == space.shell[j] and space.two_m[i] == -space.two_m[j]:
                want = _h2(x)
            else:
                want = 2 * _h2(x) - s3
            assert abs(I[i, j] - want) < 1e-8, (i, j, I[i, j], want)


def test_entropies_vanish_for_one_determinant():
    """V = 0 with non-degenerate energies: the ground state is one determinant,
    so every orbital is pure and no two are correlated."""
    space = make_space("p")
    h = make_one_body(space, 4, 3, 2, 1)
    o, res = _dmrg(h, 64, 2, measure=True)
    s1, I, _ = o.entropies()
    assert np.abs(s1).max() < 1e-10 and np.abs(I).max() < 1e-10


def test_entropy_invariants_truncated():
    """At a truncated D: 0 <= s_i <= ln 2, I symmetric with zero diagonal and
    non-negative (each rho_ij comes from one normalised state)."""
    h = WORKLOADS["sd_4p4n"].hamiltonian()
    o, res = _dmrg(h, 24, 2, measure=True)
    s1, I, _ = o.entropies()
    assert s1.min() >= -1e-14 and s1.max() <= math.log(2) + 1e-14
    assert np.array_equal(I, I.T) and np.all(np.diag(I) == 0.0)
    assert I.min() >= -1e-12 and I.max() > 1e-3


def test_fiedler_ordering_recovers_a_hidden_seriation():
    """Spectral seriation: for a matrix whose entries fall off with the distance
    in a hidden order (a Robinson matrix, the case the eta = 2 spectral method
    solves exactly), the Fiedler ordering is that order or its reverse; for a
    weighted path it is the path."""
    rng = np.random.default_rng(3)
    for n in (5, 12, 40):
        hidden = rng.permutation(n)
        pos = np.empty(n, dtype=int)
        pos[hidden] = np.arange(n)
        d = np.abs(pos[:, None] - pos[None, :])
        for I in (np.exp(-0.7 * d) * (d > 0), (d == 1).astype(float) * 0.3):
            got = entropy.fiedler_ordering(I)
            assert np.array_equal(got, hidden) or np.array_equal(got, hidden[::-1])
            # the sign rule: the site listed first in site order sits in the first half
            f = entropy.fiedler_vector(I)[1]
            assert f[np.nonzero(f)[0][0]] < 0
    # the ordering lowers the entanglement distance of a scrambled path
    I = (d == 1).astype(float)
    assert entropy.entanglement_distance(I, entropy.fiedler_ordering(I)) == n - 1
