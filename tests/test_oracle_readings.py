"""Pins of the oracle's readings below the paper's level of detail.

Each reading is checked against something other than its own code:

* the density-matrix perturbation (noise) term, against reduced density
  matrices built by brute force on determinants, with Jordan-Wigner signs
  counted over the whole chain;
* the truncation count with its tie rule (and with DBSS), against a search
  over the rule's definition stated with explicit tie groups;
* the wavefunction prediction: at a bond dimension that keeps the exact
  state, the predicted vector is already an eigenvector of the next H_eff,
  with the exact-diagonalisation energy;
* the H_eff diagonal (Davidson preconditioner), against the diagonal of H_eff
  assembled from products with unit vectors.
"""
import math

import numpy as np
import pytest

from oracle import dmrg, ed
from workloads import WORKLOADS, make_hamiltonian, make_space, random_ordering


def _vec(d, psi):
    return np.concatenate([psi[q].ravel() for q in sorted(psi)]) if psi else np.zeros(0)


# ------------------------------------------------ density-matrix noise term
def _jw(det: int, i: int) -> float:
    """(-1)^(occupied chain sites below i) for c_i or c+_i on a determinant."""
    return -1.0 if bin(det & ((1 << i) - 1)).count("1") & 1 else 1.0


def _brute_rho(o, psi, setup, alpha, left):
    """rho of the S (left) or E block from determinants: Psi Psi^T plus
    alpha * sum over the block's sites of (c Psi)(c Psi)^T + (c+ Psi)(c+ Psi)^T,
    each projected onto the block basis (the basis of selected determinants)."""
    enlL, Sops, enlR, Eops, terms = setup
    cfg = o.psi_configs(enlL, enlR)
    T = o.T
    bond = enlL.site
    smask = (1 << (bond + 1)) - 1
    sbasis, ebasis = {}, {}
    for q, C in cfg.items():
        for a in range(C.shape[0]):
            sbasis[int(C[a, 0]) & smask] = (q, a)
        for b in range(C.shape[1]):
            ebasis[int(C[0, b]) & ~smask] = (dmrg.qsub(T, q), b)
    # amplitudes on determinants
    amp = {}
    for q, X in psi.items():
        C = cfg[q]
        for a in range(X.shape[0]):
            for b in range(X.shape[1]):
                amp[int(C[a, b])] = X[a, b]
    dims = {}
    for q, X in psi.items():
        if left:
            dims[q] = X.shape[0]
        else:
            dims[dmrg.qsub(T, q)] = X.shape[1]
    rho = {q: np.zeros((d, d)) for q, d in dims.items()}

    def add_outer(vec, w):
        # vec: {det: amplitude} in the product basis; contract over the other block
        rows = {}
        for det, v in vec.items():
            s, e = det & smask, det & ~smask
            if s not in sbasis or e not in ebasis:
                continue       # outside the block basis: projected out
            (qs, a), (qe, b) = sbasis[s], ebasis[e]
            if left:
                rows.setdefault((qs, e), {})[a] = v
            else:
                rows.setdefault((qe, s), {})[b] = v
        for (q, _), r in rows.items():
            idx = np.array(list(r.keys()))
            val = np.array(list(r.values()))
            rho[q][np.ix_(idx, idx)] += w * np.outer(val, val)

    add_outer(amp, 1.0)
    if alpha:
        sites = range(0, bond + 1) if left else range(bond + 1, o.N)
        for i in sites:
            for create in (False, True):
                out = {}
                for det, v in amp.items():
                    occ = (det >> i) & 1
                    if occ == create:
                        continue
                    d2 = det ^ (1 << i)
                    out[d2] = out.get(d2, 0.0) + _jw(det, i) * v
                add_outer(out, alpha)
    return rho


@pytest.mark.parametrize("name,n_p,n_n,two_M,D,oseed", [("p", 2, 2, 0, 6, 2), ("sd", 2, 3, 1, 10, 4)])
def test_noise_density_matrix_against_determinants(name, n_p, n_n, two_M, D, oseed):
    space = make_space(name)
    h = make_hamiltonian(space, 31, n_p, n_n, two_M)
    opts = dmrg.Options(davidson_tol=1e-9, select_basis=True, seed=99)
    o = dmrg.DMRG(h.eps, h.V, space.species, space.two_m, n_p, n_n, two_M,
                  random_ordering(space.n_sites, oseed), opts)
    checked = [0, 0]

    def hook(oo, bond, direction, setup):
        enlL, Sops, enlR, Eops, terms = setup
        for alpha in (0.0, 0.7):
            if direction == "LR":
                got = oo.rho_left(oo.psi, Sops, alpha, bond)
            else:
                got = oo.rho_right(oo.psi, Eops, alpha, bond)
            ref = _brute_rho(oo, oo.psi, setup, alpha, direction == "LR")
            assert set(got) == set(ref)
            for q in ref:
                assert np.abs(got[q] - ref[q]).max() < 1e-12, (bond, direction, alpha, q)
        checked[direction == "RL"] += 1

    o.sweep(D, on_step=hook)
    o.sweep(D, on_step=hook)
    assert checked[0] > 0 and checked[1] > 0


# ------------------------------------------------------- truncation count
def _count_by_groups(w, D, tie_tol, trunc_eps=0.0, d_min=0):
    """The tie rule stated with explicit groups: weights (descending) form
    tie groups, maximal runs whose neighbours differ by at most tie_tol.  A cut
    is admissible where it does not split a group.  The kept count is the
    largest admissible nonzero cut not above the nominal count, else the
    smallest admissible cut above it.  The nominal count is D (at most all
    weights), or with DBSS the smallest n whose discarded remainder is at most
    trunc_eps, clamped to [d_min, D]."""
    n_all = len(w)
    if trunc_eps > 0.0:
        nominal = next(n for n in range(n_all + 1)
                       if n == n_all or 1.0 - math.fsum(w[:n]) <= trunc_eps)
        # the remainder is summed in descending order in the rule; fsum agrees
        # with it away from exact boundaries, which the spectra below avoid
        nominal = min(max(nominal, d_min), D, n_all)
    else:
        nominal = min(D, n_all)
    group = [0] * n_all
    for x in range(1, n_all):
        group[x] = group[x - 1] + (1 if w[x - 1] - w[x] > tie_tol else 0)
    admissible = [n for n in range(1, n_all + 1) if n == n_all or group[n - 1] != group[n]]
    below = [n for n in admissible if n <= nominal]
    if nominal == 0:
        return 0
    if below:
        return max(below)
    return min(n for n in admissible if n >= nominal)


def _planted_spectrum(rng, tie_tol):
    """Random descending weights summing to one with tied groups (within
    tie_tol, or exactly equal, or zero) planted at random places."""
    n = int(rng.integers(4, 40))
    w = list(rng.exponential(size=n) * 10.0 ** rng.uniform(-6, 0, size=n))
    for _ in range(int(rng.integers(1, 4))):
        g = int(rng.integers(2, 6))
        v = float(rng.choice(w))
        kind = rng.integers(3)
        if kind == 0:
            w += [v] * g                                   # exact ties
        elif kind == 1:
            w += [v + tie_tol * rng.uniform(-0.4, 0.4) for _ in range(g)]   # within the tolerance
        else:
            w += [0.0] * g                                 # zero weights
    w = np.array(sorted(w, reverse=True))
    return list(w / w.sum())


def test_truncation_count_against_group_search():
    rng = np.random.default_rng(11)
    tie_tol = 1e-13
    straddled = 0
    for trial in range(3000):
        w = _planted_spectrum(rng, tie_tol * 50)
        tol = tie_tol * 100 if trial % 2 else tie_tol
        D = int(rng.integers(1, len(w) + 3))
        got = dmrg.truncation_count(w, D, tol)
        assert got == _count_by_groups(w, D, tol), (w, D)
        assert got <= max(D, 1) or got == _count_by_groups(w, D, tol)
        if 0 < D < len(w) and w[D - 1] - w[D] <= tol:
            straddled += 1
            assert got != D
    assert straddled > 100      # the planted groups do straddle cuts


def test_truncation_count_boundary_cases():
    """Hand-built dyadic spectra whose gaps equal the tolerance exactly (tied,
    by the rule's 'at most'), a cut inside a zero group, and a tie group that
    starts at the top (raised to the group's end)."""
    t = 2.0 ** -44
    w = [0.5, 0.25, 0.25 - t, 0.125, 0.125 - 2 * t]
    assert _count_by_groups(w, 2, t) == 1
    assert dmrg.truncation_count(w, 2, t) == 1          # gap == tol: tied
    assert dmrg.truncation_count(w, 2, t / 2) == 2      # gap > tol: a cut
    assert dmrg.truncation_count(w, 4, t) == 4          # gap 2 t > tol: a cut
    z = [0.5, 0.5, 0.0, 0.0, 0.0]
    assert dmrg.truncation_count(z, 3, 1e-13) == 2       # zero group dropped whole
    assert dmrg.truncation_count(z, 1, 1e-13) == 2       # top group raised to its end
    assert dmrg.truncation_count(z, 5, 1e-13) == 5       # everything fits
    assert dmrg.truncation_count([1.0 / 3] * 3, 2, 1e-13) == 3


def test_truncation_count_with_dbss_against_search():
    rng = np.random.default_rng(12)
    for _ in range(2000):
        w = _planted_spectrum(rng, 5e-12)
        D = int(rng.integers(1, len(w) + 3))
        eps = float(10.0 ** rng.uniform(-8, -1))
        d_min = int(rng.integers(0, 6))
        got = dmrg.truncation_count(w, D, 1e-13, eps, d_min)
        assert got == _count_by_groups(w, D, 1e-13, eps, d_min), (w, D, eps, d_min)


def test_density_iso_applies_the_count():
    """density_iso on sector density matrices with a known spectrum (planted
    ties across sectors): the kept weights are the top ones of the count, the
    discarded weight is the rest, and the columns are eigenvectors with the
    sign rule (largest-magnitude entry positive)."""
    rng = np.random.default_rng(3)
    for trial in range(200):
        nsec = int(rng.integers(1, 5))
        spec = _planted_spectrum(rng, 0.0)
        cuts = np.sort(rng.choice(np.arange(1, len(spec)), size=min(nsec - 1, len(spec) - 1),
                                  replace=False)) if nsec > 1 else []
        parts = np.split(np.array(spec), cuts)
        rho = {}
        for x, p in enumerate(parts):
            Q, _ = np.linalg.qr(rng.normal(size=(len(p), len(p))))
            rho[(x, 0, 0)] = (Q * p) @ Q.T * 3.0          # trace 3: normalised inside
        o = dmrg.DMRG(np.zeros(2), np.zeros((2, 2, 2, 2)), [0, 1], [1, -1], 1, 0, 1,
                      opts=dmrg.Options())
        D = int(rng.integers(1, len(spec) + 2))
        iso, disc = o.density_iso(rho, D)
        allw = np.sort(np.concatenate([np.linalg.eigvalsh(m / 3.0) for m in rho.values()]))[::-1]
        n = _count_by_groups(list(allw), D, 1e-13)
        assert sum(U.shape[1] for U in iso.values()) == n
        assert abs(disc - max(0.0, 1.0 - allw[:n].sum())) < 1e-12
        for q, U in iso.items():
            m = rho[q] / 3.0
            assert np.abs(U.T @ U - np.eye(U.shape[1])).max() < 1e-12
            lam = np.diag(U.T @ m @ U)
            assert np.abs(m @ U - U * lam).max() < 1e-10
            assert np.all(np.diff(lam) <= 1e-15)
            for c in range(U.shape[1]):
                assert U[int(np.argmax(np.abs(U[:, c]))), c] > 0


# ------------------------------------------------------------- prediction
@pytest.mark.parametrize("oseed", [None, 9])
def test_prediction_is_an_eigenvector_at_exact_D(oseed):
    """p shell 2p + 2n at D = 64 keeps the exact state: the guess carried to
    the next bond by the prediction is the same state, so it is an
    eigenvector of the next bond's H_eff with the ED energy."""
    h = WORKLOADS["p_2p2n"].hamiltonian()
    sp_ = h.space
    e0 = ed.ground_energy(h.eps, h.V, sp_.species, sp_.two_m, 2, 2, 0)[0]
    order = None if oseed is None else random_ordering(12, oseed)
    o = dmrg.DMRG(h.eps, h.V, sp_.species, sp_.two_m, 2, 2, 0, order,
                  dmrg.Options(davidson_tol=1e-12, seed=5))
    o.sweep(64)
    orig = o.solve_bond
    seen = {"LR": 0, "RL": 0}

    def checked(bond, direction, setup):
        terms = setup[4]
        x = o.psi
        y = o.heff_apply(terms, x)
        nx = o.vdot(x, x)
        th = o.vdot(x, y) / nx
        res = {q: y[q] - th * x[q] for q in x}
        r = math.sqrt(o.vdot(res, res))
        assert abs(nx - 1.0) < 1e-10, (bond, direction, nx)
        assert r < 1e-8, (bond, direction, r)
        assert abs(th - e0) < 1e-10, (bond, direction, th, e0)
        seen[direction] += 1
        return orig(bond, direction, setup)

    o.solve_bond = checked
    o.sweep(64)
    assert seen["LR"] == 10 and seen["RL"] == 10


# --------------------------------------------------------------- diagonal
@pytest.mark.parametrize("name,n_p,n_n,two_M,D", [("p", 2, 2, 0, 8), ("sd", 2, 1, 1, 12)])
def test_heff_diag_equals_assembled_diagonal(name, n_p, n_n, two_M, D):
    space = make_space(name)
    h = make_hamiltonian(space, 17, n_p, n_n, two_M)
    o = dmrg.DMRG(h.eps, h.V, space.species, space.two_m, n_p, n_n, two_M,
                  random_ordering(space.n_sites, 3), dmrg.Options(davidson_tol=1e-9, noise=1e-4,
                                                                  noise_sweeps=1, seed=8))
    rng = np.random.default_rng(0)
    nchk = [0]

    def hook(oo, bond, direction, setup):
        terms = setup[4]
        layout = oo.psi_layout(setup[0], setup[2])
        keys = sorted(layout)
        zero = {q: np.zeros(s) for q, s in layout.items()}
        d = oo.heff_diag(terms, zero)
        flat = [(q, a, b) for q in keys for a in range(layout[q][0]) for b in range(layout[q][1])]
        pick = rng.choice(len(flat), size=min(24, len(flat)), replace=False)
        for p in pick:
            q, a, b = flat[p]
            e = {k: v.copy() for k, v in zero.items()}
            e[q][a, b] = 1.0
            col = oo.heff_apply(terms, e)
            assert abs(col[q][a, b] - d[q][a, b]) < 1e-12 * max(1.0, abs(col[q][a, b])), (bond, q, a, b)
        nchk[0] += 1

    o.sweep(D, on_step=hook)
    o.sweep(D, on_step=hook)
    assert nchk[0] == 4 * (space.n_sites - 1)


# ------------------------------------------------------------------ CI-DEAS
def _profile(h):
    """One-orbital entropies and occupations of the exact ground state."""
    sp_ = h.space
    _, basis, vec = ed.ground_state(h.eps, h.V, sp_.species, sp_.two_m, h.n_p, h.n_n, h.two_M)
    from oracle import entropy
    n, _, _ = entropy.correlations_from_vector(basis, vec, sp_.n_sites)
    s1, _ = entropy.entropies_of_vector(basis, vec, sp_.n_sites)
    return s1, n


@pytest.mark.parametrize("oseed", [None, 6])
def test_cideas_exact_at_full_rank(oseed):
    h = WORKLOADS["p_2p2n"].hamiltonian()
    sp_ = h.space
    s1, n1 = _profile(h)
    e0 = ed.ground_energy(h.eps, h.V, sp_.species, sp_.two_m, 2, 2, 0)[0]
    order = None if oseed is None else random_ordering(12, oseed)
    o = dmrg.DMRG(h.eps, h.V, sp_.species, sp_.two_m, 2, 2, 0, order,
                  dmrg.Options(davidson_tol=1e-11, seed=3, cideas_entropy=s1, cideas_occupation=n1))
    assert o.cideas
    r = [o.sweep(64) for _ in range(2)]
    assert abs(r[-1]["energy"] - e0) < 1e-10


def test_cideas_variational_truncated():
    space = make_space("sd")
    h = make_hamiltonian(space, 21, 2, 2, 0)
    s1, n1 = _profile(h)
    e0 = ed.ground_energy(h.eps, h.V, space.species, space.two_m, 2, 2, 0)[0]
    o = dmrg.DMRG(h.eps, h.V, space.species, space.two_m, 2, 2, 0, None,
                  dmrg.Options(davidson_tol=1e-9, noise=1e-4, noise_sweeps=1, seed=3,
                               cideas_entropy=s1, cideas_occupation=n1))
    res = [o.sweep(8)["energy"] for _ in range(3)]
    assert all(rec.theta >= e0 - 1e-10 for rec in o.records)
    assert res[2] <= res[0] + 1e-9


def _popcount(x):
    return bin(x).count("1")


@pytest.mark.parametrize("name,n_p,n_n,two_M,D,oseed", [("p", 2, 2, 0, 6, 1), ("sd", 2, 3, 1, 9, 2),
                                                     ("sd", 4, 4, 0, 30, None)])
def test_cideas_blocks_against_definition(name, n_p, n_n, two_M, D, oseed):
    """Every environment block of the CI-DEAS start, against the rule stated
    with the nested CI spaces C_k (determinants differing from the reference
    only on the k most entropic sites of the block): the block holds all of
    C_k* for the largest k* with |C_k*| <= D, and is completed to D states
    from C_{k*+1} with the fewest differing sites first.  The candidate
    determinants are built independently: each determinant of the block
    before it, with the new site empty or occupied, kept when the sites to
    its left can complete the target."""
    space = make_space(name)
    h = make_hamiltonian(space, 44, n_p, n_n, two_M)
    rng = np.random.default_rng(9)
    s1 = rng.uniform(0.0, 0.69, space.n_sites)
    n1 = rng.uniform(0.0, 1.0, space.n_sites)
    order = None if oseed is None else random_ordering(space.n_sites, oseed)
    o = dmrg.DMRG(h.eps, h.V, space.species, space.two_m, n_p, n_n, two_M, order,
                  dmrg.Options(seed=5, cideas_entropy=s1, cideas_occupation=n1))
    o.initialize(D)
    N, T = o.N, o.T
    # reference and entropy in chain positions, from the inputs directly
    sc = np.asarray(s1)[o.order]
    oc = np.asarray(n1)[o.order]
    ref = 0
    for sp_, cnt in ((0, n_p), (1, n_n)):
        sites = sorted((i for i in range(N) if o.species[i] == sp_), key=lambda i: (-oc[i], i))
        for i in sites[:cnt]:
            ref |= 1 << i
    truncated = 0
    for lo in range(N - 1, 1, -1):
        prev, blk = o.R[lo + 1], o.R[lo]
        reach = o.reach(0, lo)

        def qn(c):
            q = [0, 0, 0]
            for i in range(N):
                if (c >> i) & 1:
                    q[0 if o.species[i] == 0 else 1] += 1
                    q[2] += int(o.two_m[i])
            return tuple(q)

        cands = [c0 | (b << lo) for cs in prev.configs.values() for c0 in cs for b in (0, 1)]
        cands = [c for c in cands if dmrg.qsub(T, qn(c)) in reach]
        kept = sorted(c for cs in blk.configs.values() for c in cs)
        assert len(kept) == min(D, len(cands)) and len(set(kept)) == len(kept)
        if len(cands) <= D:
            assert kept == sorted(cands)
            continue
        truncated += 1
        top = sorted(range(lo, N), key=lambda i: (-sc[i], i))
        diff = {c: (c ^ ref) & ~((1 << lo) - 1) for c in cands}

        def space_k(k):
            allowed = 0
            for i in top[:k]:
                allowed |= 1 << i
            return {c for c in cands if diff[c] & ~allowed == 0}

        k = 0
        while len(space_k(k + 1)) <= D:
            k += 1
        inner, outer = space_k(k), space_k(k + 1)
        ks = set(kept)
        assert inner <= ks <= outer
        extra, rest = ks - inner, outer - ks
        if extra and rest:
            assert max(_popcount(diff[c]) for c in extra) <= min(_popcount(diff[c]) for c in rest)
    assert truncated > 0
