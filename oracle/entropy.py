"""Orbital entropies, mutual information and the entropy-based ordering.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The entropy paragraph defines the one-orbital entropy s_i = -Tr rho_i ln rho_i
from the reduced density matrix of orbital i, the two-orbital entropy s_ij from
that of the pair (i, j), their combination into the mutual information, and the
ordering that minimises the entanglement distance sum_ij I_ij |i - j|^eta,
with eta = 2 solved by spectral graph theory.  An orbital here is one site
(one m-state, local dimension 2, the C^2 paragraph).

Readings written out here:

* With the proton number, the neutron number and 2M fixed, rho_i is diagonal,
  diag(1 - <n_i>, <n_i>).  In the basis |00>, |01>, |10>, |11> of the
  occupations (n_i, n_j), rho_ij has the diagonal
  <(1-n_i)(1-n_j)>, <(1-n_i) n_j>, <n_i (1-n_j)>, <n_i n_j>, and its only
  off-diagonal pair couples |01> and |10> through <c+_i c_j>; that element is
  zero unless i and j are of one species with the same 2m (any other pairing
  of |01> with |10>, or of |00> with |11>, changes a conserved number).
* The paper prints I_ij as s_ij - s_i - s_j, which is never positive; the
  distance it minimises needs non-negative weights, so the mutual information
  here is I_ij = s_i + s_j - s_ij >= 0 (subadditivity), zero on the diagonal.
* The eta = 2 distance sum_ij I_ij (p_i - p_j)^2, relaxed from positions to real
  numbers with a fixed norm and orthogonal to the constant vector, is
  minimised by the eigenvector of the second smallest eigenvalue of the graph
  Laplacian L = diag(sum_j I_ij) - I (the Fiedler vector); the ordering sorts
  the sites by its components.  The vector's sign is fixed so that its first
  component (in site order) larger than 1e-9 of the largest magnitude is
  negative; components that agree to 1e-10 of the largest magnitude are
  ties and keep site order.  A disconnected graph (a zero Fiedler value of
  multiplicity two) has no unique Fiedler vector.
"""
from __future__ import annotations

import numpy as np


def correlations_from_vector(basis: np.ndarray, vec: np.ndarray, n_sites: int):
    """<n_i>, <n_i n_j> and <c+_i c_j> of a state given on determinants.

    `basis` is the sorted uint64 determinant list (bit i = site i occupied,
    |c> = prod over occupied sites in ascending order of c+ on |0>) and `vec`
    the real amplitudes.  Brute force over determinants, straight from the
    definitions: the Jordan-Wigner sign of c_p or c+_p on |c> is
    (-1)^(occupied sites below p)."""
    basis = np.asarray(basis, dtype=np.uint64)
    vec = np.asarray(vec, dtype=np.float64)
    w = vec * vec
    occ = np.stack([((basis >> np.uint64(i)) & np.uint64(1)).astype(np.float64)
                    for i in range(n_sites)])                       # (N, dim)
    n = occ @ w
    nn = (occ * w) @ occ.T
    index = {int(c): x for x, c in enumerate(basis)}
    hop = np.zeros((n_sites, n_sites))

    def below(c: int, p: int) -> int:
        return bin(c & ((1 << p) - 1)).count("1")

    for x, c in enumerate(basis.tolist()):
        if vec[x] == 0.0:
            continue
        for j in range(n_sites):
            if not (c >> j) & 1:
                continue
            s1 = -1.0 if below(c, j) & 1 else 1.0
            c1 = c ^ (1 << j)
            for i in range(n_sites):
                if (c1 >> i) & 1:
                    continue
                s2 = -1.0 if below(c1, i) & 1 else 1.0
                y = index.get(c1 | (1 << i))
                if y is not None:
                    hop[i, j] += vec[y] * s1 * s2 * vec[x]
    return n, nn, hop


def vn_entropy(w) -> float:
    """-sum w ln w over the eigenvalues w of a density matrix (0 ln 0 = 0)."""
    w = np.asarray(w, dtype=np.float64)
    w = w[w > 0.0]
    return float(-np.sum(w * np.log(w)))


def rho_one(n_i: float) -> np.ndarray:
    """rho_i in the basis |0>, |1>."""
    return np.diag([1.0 - n_i, n_i])


def rho_two(n_i: float, n_j: float, nn_ij: float, hop_ij: float) -> np.ndarray:
    """rho_ij in the basis |00>, |01>, |10>, |11> of (n_i, n_j); hop_ij = <c+_i c_j>."""
    r = np.zeros((4, 4))
    r[0, 0] = 1.0 - n_i - n_j + nn_ij
    r[1, 1] = n_j - nn_ij
    r[2, 2] = n_i - nn_ij
    r[3, 3] = nn_ij
    r[2, 1] = hop_ij
    r[1, 2] = hop_ij
    return r


def entropies(n1, pair_ni, pair_nj, nn, hop):
    """s_i from <n_i> (n1), and for i < j s_ij and I_ij = s_i + s_j - s_ij from
    the pair's own <n_i>, <n_j>, <n_i n_j>, <c+_i c_j> (pair_ni[i, j] etc., all
    taken from one state).  Returns (s1, I) with I symmetric, zero diagonal."""
    N = len(n1)
    s1 = np.array([vn_entropy(np.linalg.eigvalsh(rho_one(x))) for x in n1])
    I = np.zeros((N, N))
    for i in range(N):
        for j in range(i + 1, N):
            a, b = pair_ni[i, j], pair_nj[i, j]
            sij = vn_entropy(np.linalg.eigvalsh(rho_two(a, b, nn[i, j], hop[i, j])))
            si = vn_entropy(np.linalg.eigvalsh(rho_one(a)))
            sj = vn_entropy(np.linalg.eigvalsh(rho_one(b)))
            I[i, j] = I[j, i] = si + sj - sij
    return s1, I


def entropies_of_vector(basis, vec, n_sites: int):
    """(s1, I) of a state given on determinants (all from the one state)."""
    n, nn, hop = correlations_from_vector(basis, vec, n_sites)
    ni = np.repeat(n[:, None], n_sites, axis=1)
    return entropies(n, ni, ni.T, nn, hop)


def fiedler_vector(I):
    """Fiedler value and vector of L = diag(sum_j I_ij) - I, sign-fixed."""
    I = np.asarray(I, dtype=np.float64)
    L = np.diag(I.sum(axis=1)) - I
    w, v = np.linalg.eigh(L)
    f = v[:, 1].copy()
    tol = 1e-9 * np.max(np.abs(f))
    for x in f:
        if abs(x) > tol:
            if x > 0.0:
                f = -f
            break
    return float(w[1]), f


def fiedler_ordering(I) -> np.ndarray:
    """Ordering (chain position -> site) that sorts the sites by the Fiedler
    vector of the mutual-information Laplacian (eta = 2); stable in site order."""
    _, f = fiedler_vector(I)
    key = np.round(f / (1e-10 * np.max(np.abs(f))))
    return np.argsort(key, kind="stable").astype(np.int32)


def entanglement_distance(I, ordering, eta: float = 2.0) -> float:
    """sum_{i<j} I_ij |p_i - p_j|^eta with p the chain position of each site."""
    I = np.asarray(I, dtype=np.float64)
    pos = np.empty(len(ordering), dtype=np.int64)
    pos[np.asarray(ordering)] = np.arange(len(ordering))
    d = np.abs(pos[:, None] - pos[None, :]).astype(np.float64) ** eta
    return float(np.sum(np.triu(I * d, 1)))


__all__ = ["correlations_from_vector", "vn_entropy", "rho_one", "rho_two", "entropies",
           "entropies_of_vector", "fiedler_vector", "fiedler_ordering", "entanglement_distance"]
