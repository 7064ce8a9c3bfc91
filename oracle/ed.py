"""Exact diagonalisation in the m-scheme basis (test infrastructure only).

The many-body basis is the set of Slater determinants with fixed proton
number, neutron number and total 2M (the m-scheme of the paper's basis
dimension counts, e.g. 1.1e9 for 56Ni in the pf shell).  A determinant is a
bit mask over the sites; |c> = prod_{i in c, ascending} c+_i |0>, so the
Jordan-Wigner sign of c_p or c+_p on |c> is (-1)^(number of occupied sites
below p).  H (Eq. 1, written as sum eps n + sum_{i<j,k<l} Vbar c+_i c+_j c_l c_k)
is applied to determinants term by term.
"""
from __future__ import annotations

import itertools
from typing import Dict, Iterable, List, Sequence, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def mscheme_dimension(species: Sequence[int], two_m: Sequence[int], n_p: int, n_n: int,
                      two_M: int) -> int:
    """Number of determinants with (n_p, n_n, 2M): dynamic programming over sites."""
    counts: Dict[Tuple[int, int, int], int] = {(0, 0, 0): 1}
    for s, m in zip(species, two_m):
        nxt = dict(counts)
        for (a, b, t), c in counts.items():
            key = (a + (s == 0), b + (s == 1), t + int(m))
            if key[0] <= n_p and key[1] <= n_n:
                nxt[key] = nxt.get(key, 0) + c
        counts = nxt
    return counts.get((n_p, n_n, two_M), 0)


def mscheme_basis(species, two_m, n_p: int, n_n: int, two_M: int) -> np.ndarray:
    """All determinants of the sector as a sorted uint64 array of bit masks."""
    species = np.asarray(species)
    two_m = np.asarray(two_m)
    prot = [i for i in range(len(species)) if species[i] == 0]
    neut = [i for i in range(len(species)) if species[i] == 1]

    def by_m(sites, n):
        out: Dict[int, List[int]] = {}
        for comb in itertools.combinations(sites, n):
            m = int(sum(two_m[list(comb)])) if comb else 0
            mask = 0
            for i in comb:
                mask |= 1 << i
            out.setdefault(m, []).append(mask)
        return out

    pm, nm = by_m(prot, n_p), by_m(neut, n_n)
    states = []
    for mp, lp in pm.items():
        ln = nm.get(two_M - mp)
        if not ln:
            continue
        for a in lp:
            for b in ln:
                states.append(a | b)
    return np.array(sorted(states), dtype=np.uint64)


def _nonzero_two_body(V: np.ndarray, tol: float = 0.0):
    """List (i, j, k, l, Vbar_ijkl) with i<j, k<l and |Vbar| > tol."""
    n = V.shape[0]
    iu, ju = np.triu_indices(n, 1)
    sub = V[iu[:, None], ju[:, None], iu[None, :], ju[None, :]]
    a, b = np.nonzero(np.abs(sub) > tol)
    return [(int(iu[x]), int(ju[x]), int(iu[y]), int(ju[y]), float(sub[x, y]))
            for x, y in zip(a, b)]


def _sign_below(c: np.ndarray, p: int) -> np.ndarray:
    below = c & np.uint64((1 << p) - 1)
    return 1 - 2 * (np.bitwise_count(below).astype(np.int64) & 1)


def hamiltonian_matrix(eps, V, basis: np.ndarray) -> sp.csr_matrix:
    """Sparse H on the determinant list `basis` (must be closed under H)."""
    dim = basis.shape[0]
    eps = np.asarray(eps)
    n = len(eps)
    diag = np.zeros(dim)
    for i in range(n):
        diag += eps[i] * ((basis >> np.uint64(i)) & np.uint64(1)).astype(np.float64)
    rows, cols, vals = [np.arange(dim)], [np.arange(dim)], [diag]
    for (i, j, k, l, v) in _nonzero_two_body(V):
        c = basis
        bk, bl = np.uint64(1 << k), np.uint64(1 << l)
        bi, bj = np.uint64(1 << i), np.uint64(1 << j)
        ok = ((c & bk) != 0) & ((c & bl) != 0)
        if not ok.any():
            continue
        idx = np.nonzero(ok)[0]
        c0 = c[idx]
        s = _sign_below(c0, k)
        c1 = c0 ^ bk
        s = s * _sign_below(c1, l)
        c2 = c1 ^ bl
        ok2 = ((c2 & bj) == 0)
        s, c2, idx = s[ok2], c2[ok2], idx[ok2]
        s = s * _sign_below(c2, j)
        c3 = c2 | bj
        ok3 = ((c3 & bi) == 0)
        s, c3, idx = s[ok3], c3[ok3], idx[ok3]
        s = s * _sign_below(c3, i)
        c4 = c3 | bi
        tgt = np.searchsorted(basis, c4)
        if np.any(tgt >= dim) or np.any(basis[np.minimum(tgt, dim - 1)] != c4):
            raise ValueError("determinant list is not closed under H")
        rows.append(tgt)
        cols.append(idx)
        vals.append(v * s.astype(np.float64))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(dim, dim))


def ground_energy(eps, V, species, two_m, n_p: int, n_n: int, two_M: int,
                  nroots: int = 1) -> np.ndarray:
    """Lowest eigenvalue(s) of H in the (n_p, n_n, 2M) m-scheme sector."""
    basis = mscheme_basis(species, two_m, n_p, n_n, two_M)
    H = hamiltonian_matrix(eps, V, basis)
    if basis.shape[0] <= 2000:
        w = np.linalg.eigvalsh(H.toarray())
        return w[:nroots]
    w = spla.eigsh(H, k=nroots, which="SA", tol=1e-13, maxiter=20000,
                   return_eigenvectors=False)
    return np.sort(w)


def ground_state(eps, V, species, two_m, n_p: int, n_n: int, two_M: int):
    """(E0, basis, vector) of the lowest state in the (n_p, n_n, 2M) sector."""
    basis = mscheme_basis(species, two_m, n_p, n_n, two_M)
    H = hamiltonian_matrix(eps, V, basis)
    if basis.shape[0] <= 2000:
        w, v = np.linalg.eigh(H.toarray())
        return float(w[0]), basis, v[:, 0]
    w, v = spla.eigsh(H, k=1, which="SA", tol=1e-14, maxiter=20000)
    return float(w[0]), basis, v[:, 0]


def apply_rows(eps, V, configs: np.ndarray, psi: np.ndarray, rows: Iterable[int]) -> np.ndarray:
    """(H psi)[r] for selected positions r of a vector given on determinants.

    `configs[x]` is the determinant of component x of `psi` (any order, any
    subset of a sector); components of H psi outside that set are not needed
    because only the requested rows are returned.  Each row is computed on its
    own from <c_r| H |c'> = <c'| H |c_r> (H is real symmetric).
    """
    eps = np.asarray(eps)
    n = len(eps)
    index = {int(c): x for x, c in enumerate(configs)}
    terms = _nonzero_two_body(V)
    by_kl: Dict[Tuple[int, int], List[Tuple[int, int, float]]] = {}
    for (i, j, k, l, v) in terms:
        by_kl.setdefault((k, l), []).append((i, j, v))
    out = []
    for r in rows:
        c = int(configs[r])
        acc = psi[r] * sum(eps[i] for i in range(n) if (c >> i) & 1)
        occ = [i for i in range(n) if (c >> i) & 1]

        def sgn(cc, p):
            return -1 if bin(cc & ((1 << p) - 1)).count("1") & 1 else 1

        for a in range(len(occ)):
            for b in range(a + 1, len(occ)):
                k, l = occ[a], occ[b]
                lst = by_kl.get((k, l))
                if not lst:
                    continue
                s1 = sgn(c, k)
                c1 = c ^ (1 << k)
                s2 = sgn(c1, l)
                c2 = c1 ^ (1 << l)
                for (i, j, v) in lst:
                    if (c2 >> j) & 1:
                        continue
                    s3 = sgn(c2, j)
                    c3 = c2 | (1 << j)
                    if (c3 >> i) & 1:
                        continue
                    s4 = sgn(c3, i)
                    c4 = c3 | (1 << i)
                    x = index.get(c4)
                    if x is not None:
                        acc += v * s1 * s2 * s3 * s4 * psi[x]
        out.append(acc)
    return np.array(out)


def abs_apply_rows(eps, V, configs: np.ndarray, psi: np.ndarray, rows: Iterable[int]) -> np.ndarray:
    """Sum over the Slater-Condon terms of row r of |term| |psi|:
    |psi_r| sum_{i occupied} |eps_i| plus |Vbar_ijkl| |psi_x| for every term
    c+_i c+_j c_l c_k that connects the determinant of row r with component x.
    This bounds (|H| |psi|)_r from above (equal where every matrix element is
    a single term); it sets the scale of rounding errors in a product H psi
    computed in reduced precision."""
    eps = np.asarray(eps)
    n = len(eps)
    index = {int(c): x for x, c in enumerate(configs)}
    by_kl: Dict[Tuple[int, int], List[Tuple[int, int, float]]] = {}
    for (i, j, k, l, v) in _nonzero_two_body(V):
        by_kl.setdefault((k, l), []).append((i, j, abs(v)))
    out = []
    for r in rows:
        c = int(configs[r])
        occ = [i for i in range(n) if (c >> i) & 1]
        acc = abs(psi[r]) * sum(abs(eps[i]) for i in occ)
        for a in range(len(occ)):
            for b in range(a + 1, len(occ)):
                lst = by_kl.get((occ[a], occ[b]))
                if not lst:
                    continue
                c2 = c ^ (1 << occ[a]) ^ (1 << occ[b])
                for (i, j, v) in lst:
                    if (c2 >> i) & 1 or (c2 >> j) & 1:
                        continue
                    x = index.get(c2 | (1 << i) | (1 << j))
                    if x is not None:
                        acc += v * abs(psi[x])
        out.append(acc)
    return np.array(out)
