"""Seeded synthetic shell-model inputs shared by the oracle and the GPU path.

This module only *draws inputs*: the m-scheme single-particle sites of a
valence space and a random one- plus two-body Hamiltonian on them.  It holds
none of the DMRG arithmetic; both the CPU oracle and the GPU library consume
what it returns (site quantum numbers, eps[N], Vbar[N,N,N,N]).

Physics conventions (paper Eq. 1 and the m-scheme basis it is written in):

* a site is one single-particle m-state alpha = (shell, 2m, species); protons
  (species 0) precede neutrons (species 1), and within a species the shells
  come in the listed order with 2m ascending ("natural order");
* H = sum_i eps_i n_i + 1/4 sum_ijkl Vbar_ijkl c+_i c+_j c_l c_k with Vbar
  antisymmetric in (ij) and in (kl), real and symmetric under (ij)<->(kl).
  Eq. 1 writes the same operator as -1/2 sum V c+c+cc; with a random V the
  overall sign is immaterial and both paths use this +1/4 Vbar form.

The synthetic workloads stand in for the paper's USD, KB3, GXPF1A and G-matrix
interactions, which are not available: only the valence spaces and particle
numbers are borrowed (sd: 28Si, pf: 56Ni / 64Ge, pf+g9/2: 64Ge).
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Dict, List, Sequence, Tuple

import numpy as np

# 2j of each j-shell used by the valence spaces below
SHELL_TWO_J: Dict[str, int] = {
    "s1/2": 1, "p1/2": 1, "p3/2": 3, "d3/2": 3, "d5/2": 5,
    "f5/2": 5, "f7/2": 7, "g9/2": 9,
}

SPACES: Dict[str, List[str]] = {
    "p": ["p3/2", "p1/2"],
    "sd": ["d5/2", "s1/2", "d3/2"],
    "pf": ["f7/2", "p3/2", "f5/2", "p1/2"],
    "pfg9": ["f7/2", "p3/2", "f5/2", "p1/2", "g9/2"],
}


@dataclasses.dataclass(frozen=True)
class Space:
    """m-scheme single-particle sites of a valence space, in natural order."""
    name: str
    shells: Tuple[str, ...]
    species: np.ndarray      # int32[N], 0 = proton, 1 = neutron
    two_m: np.ndarray        # int32[N]
    shell: np.ndarray        # int32[N], index into `shells`

    @property
    def n_sites(self) -> int:
        return int(self.species.shape[0])


def make_space(name: str) -> Space:
    shells = SPACES[name]
    sp, tm, sh = [], [], []
    for species in (0, 1):
        for s_idx, s in enumerate(shells):
            tj = SHELL_TWO_J[s]
            for m2 in range(-tj, tj + 1, 2):
                sp.append(species)
                tm.append(m2)
                sh.append(s_idx)
    return Space(name, tuple(shells), np.array(sp, np.int32),
                 np.array(tm, np.int32), np.array(sh, np.int32))


def allowed(space: Space, i: int, j: int, k: int, l: int) -> bool:
    """Selection rule of the two-body term: conserved 2M and charge multiset."""
    s, m = space.species, space.two_m
    if m[i] + m[j] != m[k] + m[l]:
        return False
    return sorted((int(s[i]), int(s[j]))) == sorted((int(s[k]), int(s[l])))


def canonical_elements(space: Space) -> List[Tuple[int, int, int, int]]:
    """Independent two-body elements: i<j, k<l, (i,j) <= (k,l), allowed.

    Listed in lexicographic (i, j, k, l) order, which is also the draw order.
    """
    n = space.n_sites
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    out = []
    for (i, j) in pairs:
        for (k, l) in pairs:
            if (i, j) <= (k, l) and allowed(space, i, j, k, l):
                out.append((i, j, k, l))
    return out


def _fill(V: np.ndarray, i: int, j: int, k: int, l: int, v: float) -> None:
    """Set one element and all partners fixed by antisymmetry and symmetry."""
    for (a, b, sab) in ((i, j, 1.0), (j, i, -1.0)):
        for (c, d, scd) in ((k, l, 1.0), (l, k, -1.0)):
            V[a, b, c, d] = sab * scd * v
            V[c, d, a, b] = sab * scd * v


@dataclasses.dataclass
class Hamiltonian:
    space: Space
    eps: np.ndarray          # float64[N]
    V: np.ndarray            # float64[N,N,N,N], Vbar_ijkl
    n_p: int
    n_n: int
    two_M: int
    label: str = ""

    def npz_dict(self) -> dict:
        return dict(species=self.space.species, two_m=self.space.two_m,
                    eps=self.eps, V=self.V,
                    target=np.array([self.n_p, self.n_n, self.two_M], np.int32))


def make_hamiltonian(space: Space, seed: int, n_p: int, n_n: int, two_M: int,
                     shell_offsets: Dict[str, float] | None = None,
                     per_species_eps: bool = False) -> Hamiltonian:
    """Random eps / Vbar draw.

    eps: one U(-2, 2) MeV draw per j-shell, shared by all its m-states and (by
    default) by protons and neutrons; `shell_offsets` adds a constant per shell
    (the pf+g9/2 workload lifts g9/2 by +3 MeV).  Vbar: one N(0, 1 MeV) draw
    per canonical element (see `canonical_elements`), partners filled by
    antisymmetry and (ij)<->(kl) symmetry.  Draw order: eps shell by shell
    (protons then neutrons if per species), then Vbar lexicographically.
    """
    rng = np.random.default_rng(seed)
    n = space.n_sites
    nsh = len(space.shells)
    if per_species_eps:
        e_sh = rng.uniform(-2.0, 2.0, size=(2, nsh))
    else:
        e1 = rng.uniform(-2.0, 2.0, size=nsh)
        e_sh = np.stack([e1, e1])
    if shell_offsets:
        for s_idx, s in enumerate(space.shells):
            e_sh[:, s_idx] += shell_offsets.get(s, 0.0)
    eps = e_sh[space.species, space.shell].astype(np.float64)
    canon = canonical_elements(space)
    vals = rng.normal(0.0, 1.0, size=len(canon))
    V = np.zeros((n, n, n, n))
    for (i, j, k, l), v in zip(canon, vals):
        _fill(V, i, j, k, l, float(v))
    return Hamiltonian(space, eps, V, n_p, n_n, two_M)


def make_pairing(space: Space, G: float, eps0: float, n_p: int, n_n: int,
                 two_M: int = 0) -> Hamiltonian:
    """Pure like-particle pairing with degenerate single-particle energies.

    Pairs are the time-reversed partners (2m < 0, -2m) of one shell and one
    species; Vbar_{(i_p j_p)(i_q j_q)} = -G for every two pairs p, q of the
    same species (the -m site precedes the +m site in natural order).
    """
    n = space.n_sites
    pairs = {0: [], 1: []}
    for i in range(n):
        if space.two_m[i] < 0:
            for j in range(n):
                if (space.species[j] == space.species[i] and space.shell[j] == space.shell[i]
                        and space.two_m[j] == -space.two_m[i]):
                    pairs[int(space.species[i])].append((i, j))
    V = np.zeros((n, n, n, n))
    for sp in (0, 1):
        for (i, j) in pairs[sp]:
            for (k, l) in pairs[sp]:
                _fill(V, i, j, k, l, -G)
    eps = np.full(n, eps0, np.float64)
    return Hamiltonian(space, eps, V, n_p, n_n, two_M, label="pairing")


def make_one_body(space: Space, seed: int, n_p: int, n_n: int, two_M: int = 0) -> Hamiltonian:
    """Vbar = 0 with random per-site single-particle energies U(-2, 2)."""
    rng = np.random.default_rng(seed)
    eps = rng.uniform(-2.0, 2.0, size=space.n_sites)
    n = space.n_sites
    return Hamiltonian(space, eps, np.zeros((n, n, n, n)), n_p, n_n, two_M, label="one-body")


# ---------------------------------------------------------------------------
# The named workloads (valence space, particle numbers, seed, D schedule)
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    space: str
    n_p: int
    n_n: int
    two_M: int
    seed: int
    D_schedule: Tuple[int, ...]
    shell_offsets: Tuple[Tuple[str, float], ...] = ()

    def hamiltonian(self) -> Hamiltonian:
        h = make_hamiltonian(make_space(self.space), self.seed, self.n_p, self.n_n,
                             self.two_M, dict(self.shell_offsets))
        h.label = self.name
        return h


WORKLOADS: Dict[str, Workload] = {
    # p shell, 2p + 2n, M = 0: the exact space (dimension 51) fits in D = 64.
    "p_2p2n": Workload("p_2p2n", "p", 2, 2, 0, 150701, (64,) * 4),
    # sd shell, 4p + 4n, M = 0 (dimension 28,503), D = 256.
    "sd_4p4n": Workload("sd_4p4n", "sd", 4, 4, 0, 150702, (256,) * 6),
    # pf shell, 8p + 8n, M = 0 (dimension 1,087,455,228; the 56Ni space), ramp to D = 2048.
    "pf_8p8n": Workload("pf_8p8n", "pf", 8, 8, 0, 150703,
                        (512, 512, 1024, 1024, 2048, 2048, 2048, 2048)),
    # pf + g9/2, 12p + 12n, M = 0 and 2M = 4, g9/2 lifted by 3 MeV (64Ge space).
    "pfg9_12p12n": Workload("pfg9_12p12n", "pfg9", 12, 12, 0, 150704,
                            (512,) * 2 + (1024,) * 2 + (2048,) * 2 + (3072,) * 2 + (4096,) * 2,
                            (("g9/2", 3.0),)),
    "pfg9_12p12n_M2": Workload("pfg9_12p12n_M2", "pfg9", 12, 12, 4, 150704,
                               (512,) * 2 + (1024,) * 2 + (2048,) * 2 + (3072,) * 2 + (4096,) * 2,
                               (("g9/2", 3.0),)),
}


def batched_instances(count: int = 64, base_seed: int = 150705) -> List[Workload]:
    """Independent small solves: space from {p, sd, pf}, 2..8 particles per
    species capped at the species' m-state count, even total (so that M = 0 is
    reachable), D from {64, 128, 256, 512}, 4 sweeps; instance i is seeded
    with base_seed * 1000 + i."""
    out = []
    for i in range(count):
        seed = base_seed * 1000 + i
        rng = np.random.default_rng(seed)
        space = ["p", "sd", "pf"][int(rng.integers(0, 3))]
        cap = make_space(space).n_sites // 2
        while True:
            n_p = int(rng.integers(2, 9))
            n_n = int(rng.integers(2, 9))
            if n_p <= cap and n_n <= cap and (n_p + n_n) % 2 == 0:
                break
        D = int([64, 128, 256, 512][int(rng.integers(0, 4))])
        out.append(Workload(f"batch_{i}", space, n_p, n_n, 0, seed, (D,) * 4))
    return out


def random_ordering(n: int, seed: int) -> np.ndarray:
    """A seeded permutation of the sites (for ordering-invariance checks)."""
    return np.random.default_rng(seed).permutation(n).astype(np.int32)
