"""Plain FP64 two-site DMRG for shell-model Hamiltonians (test infrastructure only).

What it follows:
* Eq. 1 - H = sum eps_i n_i + 1/4 sum Vbar_ijkl c+_i c+_j c_l c_k on m-scheme
  sites with occupation 0/1 (the C^2 representation, q = 2);
* the two-site superblock Xi(l) (x) Lambda (x) Lambda (x) Xi(r) on an ordered
  chain, basis truncation through the Schmidt (SVD) decomposition of the
  superblock state, sweeping left-to-right and back, a fixed number of block
  states M (called D here) per sweep, or dynamic block-state
  selection (DBSS) from a truncation error;
* the excitation-energy paragraph: the two lowest states targeted at once
  (n_states = 2), truncated with their averaged density matrix.
Below that level of detail the paper only cites the standard method; the
readings taken are: complementary operators for the two-body term (the
S|E split below), a Davidson eigensolver, density-matrix truncation with a
deterministic tie rule, and a deterministic configuration-selection start in
place of CI-DEAS.  Each is documented where it is coded.

Conventions
-----------
Chain sites 0..N-1 (after the ordering).  Jordan-Wigner order = chain order.
A block state is a combination of determinants of its sites, created in
chain order.  Quantum number q = (n_p, n_n, 2M).  For a left block X and a
right block Y, (O_X O_Y)|x,y> = (-1)^{p(O_Y) n(x)} O_X|x> (x) O_Y|y>, so the
superblock matrix of O_X O_Y is (O_X P^{p(O_Y)}) (x) O_Y with P = diag((-1)^n).

Enlarged blocks S = L*s (site s right of L) and E = s*R (site s left of R)
have merged sectors q whose states are ordered: site empty part first, then
site occupied part.

Two-body split between S and E (all indices summed over the set shown):
  H = H_S + H_E + T_AA + T_AA^T + T_BB + T_31 + T_31^T + T_13 + T_13^T
  T_AA = sum_{i<j in S, k<l in E} Vbar_ijkl (c+_i c+_j)_S (c_l c_k)_E
  T_BB = sum_{i,k in S, j,l in E} Vbar_ijkl (c+_i c_k)_S (c+_j c_l)_E
  T_31 = sum_{l in E} R^S_l (c_l)_E,   R^S_l = -sum_{i<j,k in S} Vbar_ijkl c+_i c+_j c_k
  T_13 = sum_{i in S} (c+_i)_S R^E_i,  R^E_i =  sum_{j, k<l in E} Vbar_ijkl c+_j c_l c_k
The V sums of T_AA / T_BB are carried by the larger side as complementary
operators P, Q indexed by the smaller side's sites.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import hashrand

QN = Tuple[int, int, int]


def qadd(a: QN, b: QN) -> QN:
    return (a[0] + b[0], a[1] + b[1], a[2] + b[2])


def qsub(a: QN, b: QN) -> QN:
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def qneg(a: QN) -> QN:
    return (-a[0], -a[1], -a[2])


def nparticles(q: QN) -> int:
    return q[0] + q[1]


ZERO: QN = (0, 0, 0)

# site operators as (sigma_out, sigma_in) -> value, with their parity
SITE_I = ({(0, 0): 1.0, (1, 1): 1.0}, 0)
SITE_CD = ({(1, 0): 1.0}, 1)     # c+
SITE_C = ({(0, 1): 1.0}, 1)      # c
SITE_N = ({(1, 1): 1.0}, 0)      # n


class Op:
    """Block-sparse operator with one quantum-number shift dq and parity par.

    blocks[q_in] is the dense (d(q_in + dq) x d(q_in)) matrix."""
    __slots__ = ("dq", "par", "blocks")

    def __init__(self, dq: QN, par: int, blocks: Optional[Dict[QN, np.ndarray]] = None):
        self.dq = dq
        self.par = par
        self.blocks = blocks if blocks is not None else {}

    def block(self, q_in: QN, trans: bool):
        """(q_out, matrix) of op or op^T acting on sector q_in, or None."""
        if not trans:
            b = self.blocks.get(q_in)
            return None if b is None else (qadd(q_in, self.dq), b)
        src = qsub(q_in, self.dq)
        b = self.blocks.get(src)
        return None if b is None else (src, b.T)

    def T(self) -> "Op":
        return Op(qneg(self.dq), self.par,
                  {qadd(q, self.dq): b.T.copy() for q, b in self.blocks.items()})


@dataclasses.dataclass
class Part:
    sigma: int
    qb: QN        # sector of the base block
    off: int
    dim: int


class Enlarged:
    """S = L*s (side 'L') or E = s*R (side 'R'): merged sectors with parts."""

    def __init__(self, side: str, site: int, dsite: QN, base_dims: Dict[QN, int],
                 keep) -> None:
        self.side, self.site, self.dsite = side, site, dsite
        parts: Dict[QN, List[Part]] = {}
        for sigma in (0, 1):
            for qb in sorted(base_dims):
                q = qadd(qb, dsite) if sigma else qb
                parts.setdefault(q, []).append(Part(sigma, qb, 0, base_dims[qb]))
        self.parts: Dict[QN, List[Part]] = {}
        self.dims: Dict[QN, int] = {}
        for q in sorted(parts):
            if not keep(q):
                continue
            ps = sorted(parts[q], key=lambda p: p.sigma)
            off = 0
            for p in ps:
                p.off = off
                off += p.dim
            self.parts[q] = ps
            self.dims[q] = off

    def part(self, q: QN, sigma: int) -> Optional[Part]:
        for p in self.parts.get(q, ()):
            if p.sigma == sigma:
                return p
        return None


class Block:
    """A stored (truncated) left or right block."""

    def __init__(self, side: str, lo: int, hi: int, dims: Dict[QN, int]):
        self.side, self.lo, self.hi = side, lo, hi        # sites lo..hi-1
        self.dims = dict(sorted(dims.items()))
        self.ops: Dict[tuple, Op] = {}
        self.iso: Dict[QN, np.ndarray] = {}               # rows: composite, cols: block states
        self.iso_parts: Dict[QN, List[Part]] = {}         # composite part layout per sector
        self.configs: Optional[Dict[QN, List[int]]] = None
        self.normal = True     # carries normal (A, B) rather than complementary (P, Q) pair ops

    @property
    def length(self) -> int:
        return self.hi - self.lo


def vacuum(side: str, lo: int) -> Block:
    b = Block(side, lo, lo, {ZERO: 1})
    b.ops[("H",)] = Op(ZERO, 0, {ZERO: np.zeros((1, 1))})
    b.configs = {ZERO: [0]}
    return b


def dbss_count(w_desc, D: int, eps: float, d_min: int) -> int:
    """Dynamic block-state selection (DBSS).  The paper's block-state
    paragraph (the method description after Eq. 1) has the number of block
    states set by an a priori truncation error delta eps_TR, with a minimum
    M_min in the production runs; the rule itself is only cited.  Reading: keep the fewest largest
    weights (w_desc, descending) whose discarded remainder 1 - sum(kept) is
    at most eps, then clamp to [d_min, D].  The remainder is formed by adding
    the weights in descending order.  The caller applies its tie rule to the
    count afterwards."""
    n, kept = 0, 0.0
    while n < len(w_desc) and 1.0 - kept > eps:
        kept += w_desc[n]
        n += 1
    return min(max(n, d_min), D, len(w_desc))


def truncation_count(w_desc, D: int, tie_tol: float, trunc_eps: float = 0.0, d_min: int = 0) -> int:
    """Number of density-matrix weights kept (w_desc: all weights, descending).

    The two-site paragraph truncates the block basis to the M (here D) states
    of largest weight; with DBSS the count comes from the truncation error
    (dbss_count).  Reading for ties: when the weights on both sides of the cut
    differ by at most tie_tol, the cut would split states the density matrix
    cannot tell apart, so the count is lowered to the end of the previous tie
    group (D_eff <= D); if no such end exists the count is raised to the end of
    the group that straddles the cut.  Zero weights form one such group."""
    n = min(D, len(w_desc))
    if trunc_eps > 0.0:
        n = dbss_count(w_desc, D, trunc_eps, d_min)
    n0 = n
    while 0 < n < len(w_desc) and w_desc[n - 1] - w_desc[n] <= tie_tol:
        n -= 1
    if n == 0:
        n = n0
        while n < len(w_desc) and w_desc[n - 1] - w_desc[n] <= tie_tol:
            n += 1
    return n


@dataclasses.dataclass
class Options:
    davidson_tol: float = 1e-7
    davidson_max_iter: int = 100
    davidson_max_subspace: int = 24
    tie_tol: float = 1e-13
    seed: int = 1507
    select_basis: bool = False   # truncate by configuration selection (tests)
    noise: float = 0.0           # density-matrix perturbation weight alpha ...
    noise_sweeps: int = 0        # ... applied during the first noise_sweeps sweeps
    trunc_eps: float = 0.0       # > 0: dynamic block-state selection (DBSS) to this truncation error
    d_min: int = 0               # DBSS: fewest block states kept (D is the most)
    n_states: int = 1            # 2: the two lowest states, truncated with their averaged density matrix
    measure: bool = False        # orbital correlations and entropies during the right-to-left half
    # CI-DEAS start (both given, site indices): one-orbital entropies and
    # occupations <n_i> of a preprocessing run, for the environment blocks
    cideas_entropy: Optional[np.ndarray] = None
    cideas_occupation: Optional[np.ndarray] = None


@dataclasses.dataclass
class StepRecord:
    bond: int
    direction: str
    theta: float
    nprod: int
    converged: bool
    discarded: float
    kept: int


class DMRG:
    def __init__(self, eps, V, species, two_m, n_p: int, n_n: int, two_M: int,
                 ordering=None, opts: Optional[Options] = None):
        n = len(eps)
        order = np.arange(n) if ordering is None else np.asarray(ordering)
        self.order = order
        self.N = n
        self.eps = np.asarray(eps, np.float64)[order]
        self.V = np.asarray(V, np.float64)[np.ix_(order, order, order, order)]
        self.species = np.asarray(species)[order]
        self.two_m = np.asarray(two_m)[order]
        self.T: QN = (n_p, n_n, two_M)
        self.opts = opts or Options()
        self.delta = [((1, 0, int(self.two_m[i])) if self.species[i] == 0 else
                       (0, 1, int(self.two_m[i]))) for i in range(n)]
        # reach[a][b]: quantum numbers reachable by occupying a subset of sites a..b-1
        self._reach_cache: Dict[Tuple[int, int], set] = {}
        self.L: Dict[int, Block] = {}
        self.R: Dict[int, Block] = {}
        self.psi: Optional[Dict[QN, np.ndarray]] = None
        self.psi2: Optional[Dict[QN, np.ndarray]] = None   # the second state (n_states = 2)
        self.theta2 = math.nan
        self.psi_bond: Optional[int] = None
        self.psi_fresh = False     # psi is the converged eigenvector at psi_bond
        self.theta = math.nan
        self.records: List[StepRecord] = []
        self.nprod_total = 0
        self.sweeps_done = 0
        self.heff_flops = 0.0      # matmul flops of all H_eff products (timing report only)
        self.heff_seconds = 0.0
        o = self.opts
        self.cideas = o.cideas_entropy is not None and o.cideas_occupation is not None
        if self.cideas:
            self.cd_s = np.asarray(o.cideas_entropy, np.float64)[order]
            occ = np.asarray(o.cideas_occupation, np.float64)[order]
            # reference determinant: per species the n_species sites of largest
            # <n_i> (ties to the lower chain position)
            ref = 0
            for sp_, n_sp in ((0, n_p), (1, n_n)):
                sites = [i for i in range(n) if self.species[i] == sp_]
                sites.sort(key=lambda i: (-occ[i], i))
                for i in sites[:n_sp]:
                    ref |= 1 << i
            self.cd_ref = ref

    # ------------------------------------------------------------------ sectors
    def reach(self, a: int, b: int) -> set:
        """Quantum numbers of all determinants of sites a..b-1 (exact DP)."""
        key = (a, b)
        if key not in self._reach_cache:
            cur = {ZERO}
            for i in range(a, b):
                cur = cur | {qadd(q, self.delta[i]) for q in cur}
            self._reach_cache[key] = cur
        return self._reach_cache[key]

    def normal_S(self, bond: int) -> bool:
        """S = sites 0..bond carries the normal pair operators iff |S| <= |E|."""
        return bond + 1 <= self.N - bond - 1

    def left_normal(self, length: int) -> bool:
        return self.normal_S(length)

    def right_normal(self, lo: int) -> bool:
        # R_lo builds E at bond lo-2, which is normal iff |E| < |S|
        return self.N - lo + 1 < lo - 1

    # ---------------------------------------------------------------- kron
    def kron(self, enl: Enlarged, base: Optional[Op], site, coef: float = 1.0,
             trans: bool = False) -> Op:
        """Matrix of (base op) x (site op) on an enlarged block (base=None: identity)."""
        smat, spar = site
        bdq = ZERO if base is None else (qneg(base.dq) if trans else base.dq)
        bpar = 0 if base is None else base.par
        dsig = 1 if (1, 0) in smat else (-1 if (0, 1) in smat else 0)
        dq = qadd(bdq, enl.dsite) if dsig == 1 else (qsub(bdq, enl.dsite) if dsig == -1 else bdq)
        out = Op(dq, (bpar + spar) % 2)
        for q_in, parts in enl.parts.items():
            q_out = qadd(q_in, dq)
            if q_out not in enl.parts:
                continue
            blk = None
            for p_in in parts:
                if base is None:
                    src = (p_in.qb, None)
                else:
                    src = base.block(p_in.qb, trans)
                    if src is None:
                        continue
                for (so, si), v in smat.items():
                    if si != p_in.sigma:
                        continue
                    p_out = enl.part(q_out, so)
                    if p_out is None or p_out.qb != src[0]:
                        continue
                    if enl.side == "L":
                        sign = -1.0 if (spar and nparticles(p_in.qb) % 2) else 1.0
                    else:
                        sign = -1.0 if (bpar and p_in.sigma) else 1.0
                    m = np.eye(p_in.dim) if src[1] is None else src[1]
                    if blk is None:
                        blk = np.zeros((enl.dims[q_out], enl.dims[q_in]))
                    blk[p_out.off:p_out.off + p_out.dim, p_in.off:p_in.off + p_in.dim] += coef * v * sign * m
            if blk is not None:
                out.blocks[q_in] = blk
        return out

    @staticmethod
    def accumulate(terms: List[Optional[Op]]) -> Optional[Op]:
        """Sum operators of equal dq/parity; None (= zero) entries are skipped."""
        res = None
        for t in terms:
            if t is None or not t.blocks:
                continue
            if res is None:
                res = Op(t.dq, t.par, {q: b.copy() for q, b in t.blocks.items()})
                continue
            assert res.dq == t.dq and res.par == t.par
            for q, b in t.blocks.items():
                if q in res.blocks:
                    res.blocks[q] += b
                else:
                    res.blocks[q] = b.copy()
        return res

    @staticmethod
    def lincomb(items) -> Optional[Op]:
        """sum coef * op (or op^T) over (coef, op, trans) items."""
        res = None
        for coef, op, trans in items:
            if op is None or coef == 0.0:
                continue
            t = op.T() if trans else op
            scaled = Op(t.dq, t.par, {q: coef * b for q, b in t.blocks.items()})
            res = DMRG.accumulate([res, scaled])
        return res

    # -------------------------------------------------- complementary helpers
    # For a left block L, P^L_kl = sum_{i<j in L} V_ijkl c+_i c+_j and
    # Q^L_jl = sum_{i,k in L} V_ijkl c+_i c_k, taken from L's stored
    # complementary operators or formed from its normal A_ij, B_ik.
    def PL(self, L: Block, k: int, l: int) -> Optional[Op]:
        if not L.normal:
            return L.ops.get(("P", k, l))
        V = self.V
        return self.lincomb([(V[i, j, k, l], L.ops.get(("A", i, j)), False)
                             for i in range(L.lo, L.hi) for j in range(i + 1, L.hi)])

    def QL(self, L: Block, j: int, l: int) -> Optional[Op]:
        if not L.normal:
            if j <= l:
                return L.ops.get(("Q", j, l))
            q = L.ops.get(("Q", l, j))
            return None if q is None else q.T()
        V = self.V
        items = []
        for i in range(L.lo, L.hi):
            for k in range(L.lo, L.hi):
                if i <= k:
                    items.append((V[i, j, k, l], L.ops.get(("B", i, k)), False))
                else:
                    items.append((V[i, j, k, l], L.ops.get(("B", k, i)), True))
        return self.lincomb(items)

    # For a right block R, P^R_ij = sum_{k<l in R} V_ijkl c_l c_k and
    # Q^R_ik = sum_{j,l in R} V_ijkl c+_j c_l.
    def PR(self, R: Block, i: int, j: int) -> Optional[Op]:
        if not R.normal:
            return R.ops.get(("P", i, j))
        V = self.V
        return self.lincomb([(V[i, j, k, l], R.ops.get(("A", k, l)), True)
                             for k in range(R.lo, R.hi) for l in range(k + 1, R.hi)])

    def QR(self, R: Block, i: int, k: int) -> Optional[Op]:
        if not R.normal:
            if i <= k:
                return R.ops.get(("Q", i, k))
            q = R.ops.get(("Q", k, i))
            return None if q is None else q.T()
        V = self.V
        items = []
        for j in range(R.lo, R.hi):
            for l in range(R.lo, R.hi):
                if j <= l:
                    items.append((V[i, j, k, l], R.ops.get(("B", j, l)), False))
                else:
                    items.append((V[i, j, k, l], R.ops.get(("B", l, j)), True))
        return self.lincomb(items)

    # --------------------------------------------------------------- blocking
    def enlarge_left(self, L: Block, keep) -> Tuple[Enlarged, Dict[tuple, Op]]:
        """Operators of S = L*s with s = L.hi, from L's operators."""
        s = L.hi
        N, V, eps = self.N, self.V, self.eps
        enl = Enlarged("L", s, self.delta[s], L.dims, keep)
        K = lambda op, site, coef=1.0, trans=False: (None if (op is None and site is None) else
                                                      self.kron(enl, op, site, coef, trans))
        ops: Dict[tuple, Op] = {}
        Lr = range(L.lo, L.hi)
        # H_S = H_L + eps_s n_s + Q^L_ss n_s + R^L_s c_s + h.c.
        Hx = self.accumulate([K(L.ops.get(("H",)), SITE_I), K(None, SITE_N, eps[s])])
        q_ss = self.QL(L, s, s)
        rs = L.ops.get(("R", s))
        t31 = None if rs is None else K(rs, SITE_C)
        H = self.accumulate([Hx, None if q_ss is None else K(q_ss, SITE_N),
                             t31, None if t31 is None else t31.T()])
        ops[("H",)] = H
        # creation operators
        for i in Lr:
            c = L.ops.get(("C", i))
            if c is not None:
                ops[("C", i)] = K(c, SITE_I)
        ops[("C", s)] = K(None, SITE_CD)
        if self.opts.measure:
            # occupation operators of every S site, for the orbital correlations
            for i in Lr:
                nb = L.ops.get(("N", i))
                if nb is not None:
                    ops[("N", i)] = K(nb, SITE_I)
            ops[("N", s)] = K(None, SITE_N)
        # R^S_l = R^L_l + Q^L_sl c+_s - P^L_sl c_s - (sum_i V_issl c+_i) n_s
        for l in range(s + 1, N):
            pieces = [None if L.ops.get(("R", l)) is None else K(L.ops[("R", l)], SITE_I)]
            q = self.QL(L, s, l)
            if q is not None:
                pieces.append(K(q, SITE_CD))
            p = self.PL(L, s, l)
            if p is not None:
                pieces.append(K(p, SITE_C, -1.0))
            cn = self.lincomb([(-V[i, s, s, l], L.ops.get(("C", i)), False) for i in Lr])
            if cn is not None:
                pieces.append(K(cn, SITE_N))
            r = self.accumulate(pieces)
            if r is not None:
                ops[("R", l)] = r
        if self.normal_S(s):
            # normal pair operators on S
            for i in Lr:
                for j in range(i + 1, L.hi):
                    a = L.ops.get(("A", i, j))
                    if a is not None:
                        ops[("A", i, j)] = K(a, SITE_I)
                c = L.ops.get(("C", i))
                if c is not None:
                    ops[("A", i, s)] = K(c, SITE_CD)
                for k in range(i, L.hi):
                    b = L.ops.get(("B", i, k))
                    if b is not None:
                        ops[("B", i, k)] = K(b, SITE_I)
                if c is not None:
                    ops[("B", i, s)] = K(c, SITE_C)
            ops[("B", s, s)] = K(None, SITE_N)
        else:
            # complementary operators on S, indexed by the sites right of s
            for k in range(s + 1, N):
                for l in range(k + 1, N):
                    pieces = []
                    p = self.PL(L, k, l)
                    if p is not None:
                        pieces.append(K(p, SITE_I))
                    cs = self.lincomb([(V[i, s, k, l], L.ops.get(("C", i)), False) for i in Lr])
                    if cs is not None:
                        pieces.append(K(cs, SITE_CD))
                    r = self.accumulate(pieces)
                    if r is not None:
                        ops[("P", k, l)] = r
            for j in range(s + 1, N):
                for l in range(j, N):
                    pieces = []
                    q = self.QL(L, j, l)
                    if q is not None:
                        pieces.append(K(q, SITE_I))
                    a = self.lincomb([(V[i, j, s, l], L.ops.get(("C", i)), False) for i in Lr])
                    if a is not None:
                        pieces.append(K(a, SITE_C))
                    b = self.lincomb([(-V[s, j, k, l], L.ops.get(("C", k)), True) for k in Lr])
                    if b is not None:
                        pieces.append(K(b, SITE_CD))
                    if V[s, j, s, l] != 0.0:
                        pieces.append(K(None, SITE_N, V[s, j, s, l]))
                    r = self.accumulate(pieces)
                    if r is not None:
                        ops[("Q", j, l)] = r
        return enl, ops

    def enlarge_right(self, R: Block, keep) -> Tuple[Enlarged, Dict[tuple, Op]]:
        """Operators of E = s*R with s = R.lo - 1, from R's operators."""
        s = R.lo - 1
        V, eps = self.V, self.eps
        enl = Enlarged("R", s, self.delta[s], R.dims, keep)
        K = lambda op, site, coef=1.0, trans=False: self.kron(enl, op, site, coef, trans)
        ops: Dict[tuple, Op] = {}
        Rr = range(R.lo, R.hi)
        bond = s - 1
        # H_E = H_R + eps_s n_s + n_s Q^R_ss + c+_s R^R_s + h.c.
        q_ss = self.QR(R, s, s)
        rs = R.ops.get(("R", s))
        t13 = None if rs is None else K(rs, SITE_CD)
        ops[("H",)] = self.accumulate([K(R.ops.get(("H",)), SITE_I), K(None, SITE_N, eps[s]),
                                       None if q_ss is None else K(q_ss, SITE_N),
                                       t13, None if t13 is None else t13.T()])
        ops[("C", s)] = K(None, SITE_CD)
        for j in Rr:
            c = R.ops.get(("C", j))
            if c is not None:
                ops[("C", j)] = K(c, SITE_I)
        # R^E_i = R^R_i + c+_s P^R_is + c_s Q^R_is - n_s (sum_l V_issl c_l)
        for i in range(0, s):
            pieces = [None if R.ops.get(("R", i)) is None else K(R.ops[("R", i)], SITE_I)]
            p = self.PR(R, i, s)
            if p is not None:
                pieces.append(K(p, SITE_CD))
            q = self.QR(R, i, s)
            if q is not None:
                pieces.append(K(q, SITE_C))
            cn = self.lincomb([(-V[i, s, s, l], R.ops.get(("C", l)), True) for l in Rr])
            if cn is not None:
                pieces.append(K(cn, SITE_N))
            r = self.accumulate(pieces)
            if r is not None:
                ops[("R", i)] = r
        if not self.normal_S(bond):
            # E carries normal pair operators (E is the smaller side)
            for l in Rr:
                c = R.ops.get(("C", l))
                if c is not None:
                    ops[("A", s, l)] = K(c, SITE_CD)
                    ops[("B", s, l)] = K(c, SITE_CD, trans=True)
            for k in Rr:
                for l in range(k + 1, R.hi):
                    a = R.ops.get(("A", k, l))
                    if a is not None:
                        ops[("A", k, l)] = K(a, SITE_I)
                for l in range(k, R.hi):
                    b = R.ops.get(("B", k, l))
                    if b is not None:
                        ops[("B", k, l)] = K(b, SITE_I)
            ops[("B", s, s)] = K(None, SITE_N)
        else:
            # complementary operators on E, indexed by the sites left of s
            for i in range(0, s):
                for j in range(i + 1, s):
                    pieces = []
                    p = self.PR(R, i, j)
                    if p is not None:
                        pieces.append(K(p, SITE_I))
                    cl = self.lincomb([(-V[i, j, s, l], R.ops.get(("C", l)), True) for l in Rr])
                    if cl is not None:
                        pieces.append(K(cl, SITE_C))
                    r = self.accumulate(pieces)
                    if r is not None:
                        ops[("P", i, j)] = r
            for i in range(0, s):
                for k in range(i, s):
                    pieces = []
                    q = self.QR(R, i, k)
                    if q is not None:
                        pieces.append(K(q, SITE_I))
                    if V[i, s, k, s] != 0.0:
                        pieces.append(K(None, SITE_N, V[i, s, k, s]))
                    a = self.lincomb([(V[i, s, k, l], R.ops.get(("C", l)), True) for l in Rr])
                    if a is not None:
                        pieces.append(K(a, SITE_CD))
                    b = self.lincomb([(-V[i, j, k, s], R.ops.get(("C", j)), False) for j in Rr])
                    if b is not None:
                        pieces.append(K(b, SITE_C))
                    r = self.accumulate(pieces)
                    if r is not None:
                        ops[("Q", i, k)] = r
        return enl, ops

    # ----------------------------------------------------------- H_eff terms
    def heff_terms(self, bond: int, Sops, Eops):
        """(coef, A, transA, B, transB, sign_on_output, parity) per term.

        A term adds coef * sgn * op(A) psi op(B)^T; the fermion sign
        (-1)^{p n(q_S)} is taken on the input S sector, or on the output S
        sector for the transposed (h.c.) partners."""
        s_sites = range(0, bond + 1)
        e_sites = range(bond + 1, self.N)
        terms = [(1.0, Sops[("H",)], False, None, False, False, 0),
                 (1.0, None, False, Eops[("H",)], False, False, 0)]

        def pair(a, ta, b, tb, par, with_hc):
            if a is None or b is None:
                return
            terms.append((1.0, a, ta, b, tb, False, par))
            if with_hc:
                terms.append((1.0, a, not ta, b, not tb, True, par))

        if self.normal_S(bond):
            for i in s_sites:
                for j in range(i + 1, bond + 1):
                    pair(Sops.get(("A", i, j)), False, Eops.get(("P", i, j)), False, 0, True)
                for k in range(i, bond + 1):
                    pair(Sops.get(("B", i, k)), False, Eops.get(("Q", i, k)), False, 0, i < k)
        else:
            for k in e_sites:
                for l in range(k + 1, self.N):
                    pair(Sops.get(("P", k, l)), False, Eops.get(("A", k, l)), True, 0, True)
                for l in range(k, self.N):
                    pair(Sops.get(("Q", k, l)), False, Eops.get(("B", k, l)), False, 0, k < l)
        for l in e_sites:
            pair(Sops.get(("R", l)), False, Eops.get(("C", l)), True, 1, True)
        for i in s_sites:
            pair(Sops.get(("C", i)), False, Eops.get(("R", i)), False, 1, True)
        return terms

    def heff_apply(self, terms, psi: Dict[QN, np.ndarray]) -> Dict[QN, np.ndarray]:
        t0 = time.perf_counter()
        T = self.T
        y = {q: np.zeros_like(b) for q, b in psi.items()}
        flops = 0.0
        for coef, A, tA, B, tB, sign_out, par in terms:
            for q_in, X in psi.items():
                if A is None:
                    q_out, Am = q_in, None
                else:
                    r = A.block(q_in, tA)
                    if r is None:
                        continue
                    q_out, Am = r
                if q_out not in y:
                    continue
                if B is None:
                    Bm = None
                else:
                    r = B.block(qsub(T, q_in), tB)
                    if r is None:
                        continue
                    Bm = r[1]
                sg = 1.0
                if par:
                    sg = -1.0 if nparticles(q_out if sign_out else q_in) % 2 else 1.0
                if Bm is not None:
                    flops += 2.0 * X.shape[0] * X.shape[1] * Bm.shape[0]
                    Z = X @ Bm.T
                else:
                    Z = X
                if Am is not None:
                    flops += 2.0 * Am.shape[0] * Am.shape[1] * Z.shape[1]
                    Z = Am @ Z
                y[q_out] += (coef * sg) * Z
        self.heff_flops += flops
        self.heff_seconds += time.perf_counter() - t0
        return y

    def heff_diag(self, terms, psi) -> Dict[QN, np.ndarray]:
        T = self.T
        d = {q: np.zeros_like(b) for q, b in psi.items()}
        for coef, A, tA, B, tB, sign_out, par in terms:
            if (A is not None and A.dq != ZERO) or (B is not None and B.dq != ZERO):
                continue
            for q in psi:
                da = np.ones(psi[q].shape[0]) if A is None else (
                    np.diag(A.blocks[q]) if q in A.blocks else None)
                qe = qsub(T, q)
                db = np.ones(psi[q].shape[1]) if B is None else (
                    np.diag(B.blocks[qe]) if qe in B.blocks else None)
                if da is None or db is None:
                    continue
                d[q] += coef * np.outer(da, db)
        return d

    # ----------------------------------------------------------- vectors
    @staticmethod
    def vdot(a, b) -> float:
        return float(sum(np.vdot(a[q], b[q]) for q in a))

    @staticmethod
    def vcomb(coefs, vecs):
        out = {q: np.zeros_like(b) for q, b in vecs[0].items()}
        for c, v in zip(coefs, vecs):
            for q in out:
                out[q] += c * v[q]
        return out

    def davidson(self, apply, diag, x0, lock=None):
        """Lowest eigenpair of the symmetric operator `apply` (Davidson).

        Subspace V starts from the normalised guess; the correction is the
        residual divided by (diag - theta), magnitudes below 1e-12 clamped;
        two passes of classical Gram-Schmidt; restart to [x] at the maximum
        subspace size; converged when ||H x - theta x|| <= tol.  With `lock`
        (a normalised vector) the search runs in its orthogonal complement:
        the guess and every correction are orthogonalised against it and the
        residual is projected, which gives the next eigenpair."""
        o = self.opts

        def deflate(v):
            if lock is None:
                return v
            c = self.vdot(lock, v)
            return {q: v[q] - c * lock[q] for q in v}

        x0 = deflate(x0)
        nx = math.sqrt(self.vdot(x0, x0))
        x0 = {q: b / nx for q, b in x0.items()}
        Vs, Ws = [x0], [apply(x0)]
        nprod = 1
        converged = False
        while True:
            k = len(Vs)
            G = np.array([[self.vdot(Vs[a], Ws[b]) for b in range(k)] for a in range(k)])
            G = 0.5 * (G + G.T)
            w, U = np.linalg.eigh(G)
            theta, s = float(w[0]), U[:, 0]
            x = self.vcomb(s, Vs)
            hx = self.vcomb(s, Ws)
            r = deflate({q: hx[q] - theta * x[q] for q in x})
            rn = math.sqrt(self.vdot(r, r))
            if rn <= o.davidson_tol:
                converged = True
                break
            if nprod >= o.davidson_max_iter:
                break
            t = {}
            for q in r:
                den = diag[q] - theta
                den = np.where(np.abs(den) < 1e-12, np.where(den < 0, -1e-12, 1e-12), den)
                t[q] = r[q] / den
            if k >= o.davidson_max_subspace:
                nx = math.sqrt(self.vdot(x, x))
                Vs = [{q: b / nx for q, b in x.items()}]
                Ws = [{q: b / nx for q, b in hx.items()}]
            tn = math.sqrt(self.vdot(t, t))
            t = {q: b / tn for q, b in t.items()}
            for _ in range(2):
                t = deflate(t)
                c = [self.vdot(v, t) for v in Vs]
                proj = self.vcomb(c, Vs)
                t = {q: t[q] - proj[q] for q in t}
            tn = math.sqrt(self.vdot(t, t))
            if tn < 1e-12:
                break
            t = {q: b / tn for q, b in t.items()}
            Vs.append(t)
            Ws.append(apply(t))
            nprod += 1
        return theta, x, nprod, converged

    # ----------------------------------------------------------- truncation
    def select_counts(self, dims: Dict[QN, int], D: int) -> Dict[QN, int]:
        """Share D across sectors in proportion to their dimension (integer
        largest remainder, ties to the smaller q), capped at the dimension."""
        total = sum(dims.values())
        if total <= D:
            return dict(dims)
        keep = {q: (D * d) // total for q, d in dims.items()}
        rem = sorted(dims, key=lambda q: (-((D * dims[q]) % total), q))
        left = D - sum(keep.values())
        for q in rem:
            if left == 0:
                break
            if keep[q] < dims[q]:
                keep[q] += 1
                left -= 1
        return keep

    def selection_iso(self, dims: Dict[QN, int], D: int, tag: int, pos: int, mix: bool = False):
        """Selection isometry: per sector the kept states are those with the
        smallest SplitMix64 key (seed, tag, pos, q, index), in index order.

        With mix=True the selection S is multiplied by the Householder
        reflection I - 2 v v^T / |v|^2 of a hash-random vector v (entries
        2u - 1 keyed by (seed, 4, pos, q, row)): still an isometry, but every
        kept state then overlaps every configuration of its sector, so no
        symmetry sector of the Hamiltonian is missing from the start."""
        keep = self.select_counts(dims, D)
        iso = {}
        seed = self.opts.seed
        for q, d in dims.items():
            k = keep[q]
            if k == 0:
                continue
            keys = sorted(range(d), key=lambda x: (hashrand.hkey(seed, tag, pos, q[0], q[1],
                                                                 q[2], x), x))
            chosen = sorted(keys[:k])
            U = np.zeros((d, k))
            U[chosen, np.arange(k)] = 1.0
            if mix and d > 1:
                v = np.array([2.0 * hashrand.u01(hashrand.hkey(seed, 4, pos, q[0], q[1], q[2], x)) - 1.0
                              for x in range(d)])
                U = U - (2.0 / float(v @ v)) * np.outer(v, v @ U)
            iso[q] = U
        return iso

    def cideas_iso(self, enl: Enlarged, base: Block, D: int, lo: int):
        """CI-DEAS environment block (the block-state paragraph cites the
        procedure: a CI-based, dynamically extended active space grown by the
        orbital entropy profile).  Reading: the block R = sites lo..N-1 keeps
        determinants of its composite basis (site lo times the block R_{lo+1}
        built before it).  Its active space is the first k of its sites in
        decreasing one-orbital entropy (ties to the lower position); a
        determinant belongs to the CI space of that active space when it
        differs from the reference determinant only on those k sites.  The
        block keeps the CI space of the largest k that holds at most D
        determinants, then fills up to D from the next space's new members,
        fewest differing sites first, then by the SplitMix64 key
        (seed, 5, lo, low and high 32 bits of the determinant).  The active
        space grows as the blocks are built from the right end toward the
        left: the extension is dynamic."""
        N, seed, ref = self.N, self.opts.seed, self.cd_ref
        mask = ((1 << N) - 1) & ~((1 << lo) - 1)
        order = sorted(range(lo, N), key=lambda i: (-self.cd_s[i], i))
        rank = {site: k + 1 for k, site in enumerate(order)}
        cand = []   # (level, differing sites, key, sector, row)
        for q, parts in enl.parts.items():
            row = 0
            for p in parts:
                bit = (1 << enl.site) if p.sigma else 0
                for c0 in base.configs[p.qb]:
                    c = c0 | bit
                    d = (c ^ ref) & mask
                    lev = max((rank[i] for i in range(lo, N) if (d >> i) & 1), default=0)
                    key = hashrand.hkey(seed, 5, lo, c & 0xFFFFFFFF, c >> 32)
                    cand.append((lev, bin(d).count("1"), key, q, row))
                    row += 1
        if len(cand) <= D:
            kept = cand
        else:
            count = {}
            for t in cand:
                count[t[0]] = count.get(t[0], 0) + 1
            kstar, cum = -1, 0
            for k in range(0, N - lo + 1):
                if cum + count.get(k, 0) > D:
                    break
                cum += count.get(k, 0)
                kstar = k
            kept = [t for t in cand if t[0] <= kstar]
            nxt = sorted((t for t in cand if t[0] == kstar + 1), key=lambda t: (t[1], t[2]))
            kept += nxt[:D - len(kept)]
        rows = {}
        for t in kept:
            rows.setdefault(t[3], []).append(t[4])
        iso = {}
        for q in enl.dims:
            if q not in rows:
                continue
            r = sorted(rows[q])
            U = np.zeros((enl.dims[q], len(r)))
            U[r, np.arange(len(r))] = 1.0
            iso[q] = U
        return iso

    def dbss_count(self, w_desc, D: int) -> int:
        return dbss_count(w_desc, D, self.opts.trunc_eps, self.opts.d_min)

    def density_iso(self, rho: Dict[QN, np.ndarray], D: int):
        """Keep the D largest density-matrix weights over all sectors.

        If the weights at the cut differ by no more than tie_tol the whole
        tied group is dropped (kept if that would leave nothing); zero weights
        are such a group, so they are kept only when all of them fit.  Columns are eigenvectors in descending weight order
        with their largest-magnitude entry made positive."""
        o = self.opts
        tr = sum(float(np.trace(m)) for m in rho.values())
        eig = {}
        allw = []
        for q, m in rho.items():
            w, U = np.linalg.eigh(m / tr)
            eig[q] = (w, U)
            for x in range(len(w)):
                allw.append((float(w[x]), q, x))
        allw.sort(key=lambda t: -t[0])
        n = truncation_count([t[0] for t in allw], D, o.tie_tol, o.trunc_eps, o.d_min)
        kept = allw[:n]
        disc = 1.0 - sum(t[0] for t in kept)
        iso = {}
        for q in rho:
            idx = [x for (w, qq, x) in kept if qq == q]
            if not idx:
                continue
            w, U = eig[q]
            idx.sort(key=lambda x: -w[x])
            M = U[:, idx].copy()
            for c in range(M.shape[1]):
                a = int(np.argmax(np.abs(M[:, c])))
                if M[a, c] < 0:
                    M[:, c] = -M[:, c]
            iso[q] = M
        return iso, max(disc, 0.0)

    # ----------------------------------------------------------- renormalise
    def new_block(self, side, lo, hi, enl: Enlarged, ops: Dict[tuple, Op], iso, base: Block) -> Block:
        blk = Block(side, lo, hi, {q: U.shape[1] for q, U in iso.items()})
        blk.iso = iso
        blk.iso_parts = {q: enl.parts[q] for q in iso}
        for key, op in ops.items():
            nb = {}
            for q_in, m in op.blocks.items():
                q_out = qadd(q_in, op.dq)
                if q_in in iso and q_out in iso:
                    nb[q_in] = iso[q_out].T @ m @ iso[q_in]
            if nb:
                blk.ops[key] = Op(op.dq, op.par, nb)
        if base.configs is not None and all(np.all((U == 0) | (U == 1)) for U in iso.values()):
            blk.configs = {}
            for q, U in iso.items():
                comp = []
                for p in enl.parts[q]:
                    bit = (1 << enl.site) if p.sigma else 0
                    comp += [c | bit for c in base.configs[p.qb]]
                blk.configs[q] = [comp[int(np.argmax(U[:, c]))] for c in range(U.shape[1])]
        # switch from normal to complementary pair operators where required
        if side == "L":
            blk.normal = self.normal_S(hi - 1)
            if blk.normal and not self.left_normal(blk.length):
                self._to_complementary_left(blk)
        else:
            blk.normal = not self.normal_S(lo - 1)
            if blk.normal and not self.right_normal(blk.lo):
                self._to_complementary_right(blk)
        return blk

    def _to_complementary_left(self, blk: Block) -> None:
        N = self.N
        P = {(k, l): self.PL(blk, k, l) for k in range(blk.hi, N) for l in range(k + 1, N)}
        Q = {(j, l): self.QL(blk, j, l) for j in range(blk.hi, N) for l in range(j, N)}
        for key in [k for k in blk.ops if k[0] in "AB"]:
            del blk.ops[key]
        blk.normal = False
        for (k, l), op in P.items():
            if op is not None:
                blk.ops[("P", k, l)] = op
        for (j, l), op in Q.items():
            if op is not None:
                blk.ops[("Q", j, l)] = op

    def _to_complementary_right(self, blk: Block) -> None:
        P = {(i, j): self.PR(blk, i, j) for i in range(blk.lo) for j in range(i + 1, blk.lo)}
        Q = {(i, k): self.QR(blk, i, k) for i in range(blk.lo) for k in range(i, blk.lo)}
        for key in [k for k in blk.ops if k[0] in "AB"]:
            del blk.ops[key]
        blk.normal = False
        for (i, j), op in P.items():
            if op is not None:
                blk.ops[("P", i, j)] = op
        for (i, k), op in Q.items():
            if op is not None:
                blk.ops[("Q", i, k)] = op

    # ------------------------------------------------- perturbed density matrix
    def rho_left(self, psi, Sops, alpha: float, bond: int):
        """rho_S = Psi Psi^T per S sector, plus alpha * sum_O (O Psi)(O Psi)^T over
        O = c+_i, c_i of every S site (White's density-matrix perturbation);
        it gives weight to block states one particle away from the current
        state, which a plain truncation would discard."""
        rho = {q: X @ X.T for q, X in psi.items()}
        if alpha == 0.0:
            return rho
        for i in range(0, bond + 1):
            C = Sops.get(("C", i))
            if C is None:
                continue
            for trans in (False, True):
                for q_in, X in psi.items():
                    r = C.block(q_in, trans)
                    if r is None or r[0] not in rho:
                        continue
                    Phi = r[1] @ X
                    rho[r[0]] += alpha * (Phi @ Phi.T)
        return rho

    def rho_right(self, psi, Eops, alpha: float, bond: int):
        """rho_E = Psi^T Psi per E sector, perturbed by c+_j, c_j of every E site."""
        T = self.T
        rho = {qsub(T, q): X.T @ X for q, X in psi.items()}
        if alpha == 0.0:
            return rho
        for j in range(bond + 1, self.N):
            C = Eops.get(("C", j))
            if C is None:
                continue
            for trans in (False, True):
                for q_s, X in psi.items():
                    r = C.block(qsub(T, q_s), trans)
                    if r is None or r[0] not in rho:
                        continue
                    Phi = X @ r[1].T
                    rho[r[0]] += alpha * (Phi.T @ Phi)
        return rho

    # --------------------------------------------------------------- sweep
    def setup_bond(self, bond: int):
        """Enlarged blocks, operators and H_eff terms at bond (sites bond, bond+1)."""
        L = self.L[bond]
        R = self.R[bond + 2]
        T = self.T
        s_reach = self.reach(0, bond + 1)
        enlR, Eops = self.enlarge_right(R, lambda q: qsub(T, q) in s_reach)
        enlL, Sops = self.enlarge_left(L, lambda q: qsub(T, q) in enlR.dims)
        # drop E sectors without a partner
        enlR.parts = {q: p for q, p in enlR.parts.items() if qsub(T, q) in enlL.dims}
        enlR.dims = {q: d for q, d in enlR.dims.items() if q in enlR.parts}
        terms = self.heff_terms(bond, Sops, Eops)
        return enlL, Sops, enlR, Eops, terms

    def psi_layout(self, enlL: Enlarged, enlR: Enlarged):
        T = self.T
        return {q: (enlL.dims[q], enlR.dims[qsub(T, q)]) for q in enlL.dims
                if qsub(T, q) in enlR.dims}

    def random_psi(self, layout):
        seed = self.opts.seed
        psi = {}
        for q, (ds, de) in layout.items():
            m = np.empty((ds, de))
            for a in range(ds):
                for b in range(de):
                    m[a, b] = 2.0 * hashrand.u01(hashrand.hkey(seed, 3, q[0], q[1], q[2], a, b)) - 1.0
            psi[q] = m
        return psi

    def initialize(self, D: int) -> None:
        """Right blocks R_N .. R_2 by configuration selection (no Davidson)."""
        N, T = self.N, self.T
        self.R = {N: vacuum("R", N)}
        self.L = {0: vacuum("L", 0)}
        for lo in range(N - 1, 1, -1):
            Rn = self.R[lo + 1]
            left_reach = self.reach(0, lo)
            enl, ops = self.enlarge_right(Rn, lambda q: qsub(T, q) in left_reach)
            if self.cideas:
                iso = self.cideas_iso(enl, Rn, D, lo)
            else:
                iso = self.selection_iso(enl.dims, D, 1, lo, mix=not self.opts.select_basis)
            self.R[lo] = self.new_block("R", lo, N, enl, ops, iso, Rn)
        self.psi = None
        self.psi2 = None
        self.psi_bond = 0
        self.psi_fresh = False

    def predict_right(self, bond, psi, enlL: Enlarged, Lnew: Block, enlR: Enlarged, enlL2: Enlarged,
                      enlR2: Enlarged):
        """Guess at bond+1 from psi at bond after S -> L_{bond+1}."""
        T = self.T
        Rold = self.R[bond + 2]
        out = {q: np.zeros((enlL2.dims[q], enlR2.dims[qsub(T, q)])) for q in enlL2.dims
               if qsub(T, q) in enlR2.dims}
        for qS, X in psi.items():
            if qS not in Lnew.iso:
                continue
            Phi = Lnew.iso[qS].T @ X            # (kept) x E(T-qS)
            qE = qsub(T, qS)
            for pe in enlR.parts[qE]:          # pe.sigma = site bond+1, pe.qb = R_{bond+2} sector
                qS2 = qadd(qS, self.delta[bond + 1]) if pe.sigma else qS
                if qS2 not in out:
                    continue
                prow = enlL2.part(qS2, pe.sigma)
                if prow is None or prow.qb != qS:
                    continue
                Y = Phi[:, pe.off:pe.off + pe.dim]          # in R_{bond+2} states of sector pe.qb
                if pe.qb not in Rold.iso:
                    continue
                Vr = Rold.iso[pe.qb]                        # composite(s_{bond+2} * R_{bond+3}) x kept
                comp = Y @ Vr.T
                qE2 = qsub(T, qS2)
                for pc in Rold.iso_parts[pe.qb]:
                    pn = enlR2.part(qE2, pc.sigma)
                    if pn is None or pn.qb != pc.qb:
                        continue
                    out[qS2][prow.off:prow.off + prow.dim, pn.off:pn.off + pn.dim] += \
                        comp[:, pc.off:pc.off + pc.dim]
        return out

    def predict_left(self, bond, psi, enlR: Enlarged, Rnew: Block, enlL: Enlarged, enlL2: Enlarged,
                     enlR2: Enlarged):
        """Guess at bond-1 from psi at bond after E -> R_{bond+1}."""
        T = self.T
        Lold = self.L[bond]
        out = {q: np.zeros((enlL2.dims[q], enlR2.dims[qsub(T, q)])) for q in enlL2.dims
               if qsub(T, q) in enlR2.dims}
        for qS, X in psi.items():
            qE = qsub(T, qS)
            if qE not in Rnew.iso:
                continue
            Phi = X @ Rnew.iso[qE]              # S(qS) x kept
            for ps in enlL.parts[qS]:          # ps.sigma = site bond, ps.qb = L_bond sector
                qE2 = qadd(qE, self.delta[bond]) if ps.sigma else qE
                qS2 = qsub(T, qE2)
                if qS2 not in out:
                    continue
                pcol = enlR2.part(qE2, ps.sigma)
                if pcol is None or pcol.qb != qE:
                    continue
                Y = Phi[ps.off:ps.off + ps.dim, :]
                if ps.qb not in Lold.iso:
                    continue
                Ul = Lold.iso[ps.qb]
                comp = Ul @ Y
                for pc in Lold.iso_parts[ps.qb]:
                    pn = enlL2.part(qS2, pc.sigma)
                    if pn is None or pn.qb != pc.qb:
                        continue
                    out[qS2][pn.off:pn.off + pn.dim, pcol.off:pcol.off + pcol.dim] += \
                        comp[pc.off:pc.off + pc.dim, :]
        return out

    def solve_bond(self, bond, direction, setup):
        enlL, Sops, enlR, Eops, terms = setup
        layout = self.psi_layout(enlL, enlR)
        if self.psi is None:
            guess = self.random_psi(layout)
        else:
            guess = self.psi
        nrm = math.sqrt(self.vdot(guess, guess))
        if nrm < 1e-10:
            guess = self.random_psi(layout)
        diag = self.heff_diag(terms, guess)
        apply = lambda v: self.heff_apply(terms, v)
        theta, x, nprod, conv = self.davidson(apply, diag, guess)
        self.nprod_total += nprod
        if self.opts.n_states == 2:
            # the second state: the lowest eigenpair orthogonal to x, from its
            # own prediction (or the hash-random vector)
            g2 = self.psi2 if self.psi2 is not None else self.random_psi(layout)
            c = self.vdot(x, g2)
            g2 = {q: g2[q] - c * x[q] for q in g2}
            if math.sqrt(self.vdot(g2, g2)) < 1e-10:
                g2 = self.random_psi(layout)
            theta2, x2, nprod2, conv2 = self.davidson(apply, diag, g2, lock=x)
            self.nprod_total += nprod2
            self.psi2, self.theta2 = x2, theta2
            nprod, conv = nprod + nprod2, conv and conv2
        return theta, x, nprod, conv

    def sweep(self, D: int, on_step=None) -> dict:
        """One sweep: left-to-right over bonds 0..N-2, then right-to-left back to 0.

        The first call initialises.  A bond whose state is already the
        converged eigenvector of the same H_eff (the turning points) is not
        solved again.  Returns the sweep energy (minimum step energy) and
        truncation statistics."""
        N = self.N
        if not self.R:
            self.initialize(D)
        thetas, disc_max, nprod0 = [], 0.0, self.nprod_total
        thetas2 = []
        kept_max = 0
        two = self.opts.n_states == 2

        def rho_avg(rho_fn, ops, bond):
            # the two states' density matrices, averaged with equal weights
            rho = rho_fn(self.psi, ops, alpha, bond)
            if two:
                rho2 = rho_fn(self.psi2, ops, alpha, bond)
                rho = {q: 0.5 * (rho[q] + rho2[q]) for q in rho}
            return rho
        alpha = self.opts.noise if self.sweeps_done < self.opts.noise_sweeps else 0.0
        if self.opts.measure:
            self.meas = {k: np.zeros((N, N)) for k in ("pair_ni", "pair_nj", "nn", "hop")}
            self.meas["n1"] = np.zeros(N)
        setup = None
        for bond in range(0, N - 1):
            setup = setup or self.setup_bond(bond)
            if not (self.psi_fresh and self.psi_bond == bond):
                theta, x, nprod, conv = self.solve_bond(bond, "LR", setup)
                self.psi, self.theta, self.psi_bond, self.psi_fresh = x, theta, bond, True
                self.records.append(StepRecord(bond, "LR", theta, nprod, conv, 0.0, 0))
            thetas.append(self.theta)
            thetas2.append(self.theta2)
            if on_step:
                on_step(self, bond, "LR", setup)
            if bond == N - 2:
                break
            enlL, Sops, enlR, Eops, terms = setup
            if self.opts.select_basis:
                iso, disc = self.selection_iso(enlL.dims, D, 2, bond + 1), 0.0
            else:
                iso, disc = self.density_iso(rho_avg(self.rho_left, Sops, bond), D)
            disc_max = max(disc_max, disc)
            kept_max = max(kept_max, sum(U.shape[1] for U in iso.values()))
            Lnew = self.new_block("L", 0, bond + 1, enlL, Sops, iso, self.L[bond])
            self.L[bond + 1] = Lnew
            nsetup = self.setup_bond(bond + 1)
            self.psi = self.predict_right(bond, self.psi, enlL, Lnew, enlR, nsetup[0], nsetup[2])
            if two:
                self.psi2 = self.predict_right(bond, self.psi2, enlL, Lnew, enlR, nsetup[0], nsetup[2])
            self.psi_bond, self.psi_fresh = bond + 1, False
            setup = nsetup
        for bond in range(N - 2, -1, -1):
            setup = setup or self.setup_bond(bond)
            if not (self.psi_fresh and self.psi_bond == bond):
                theta, x, nprod, conv = self.solve_bond(bond, "RL", setup)
                self.psi, self.theta, self.psi_bond, self.psi_fresh = x, theta, bond, True
                self.records.append(StepRecord(bond, "RL", theta, nprod, conv, 0.0, 0))
            thetas.append(self.theta)
            thetas2.append(self.theta2)
            if on_step:
                on_step(self, bond, "RL", setup)
            if self.opts.measure:
                self.measure_bond(bond, setup)
            if bond == 0:
                break
            enlL, Sops, enlR, Eops, terms = setup
            if self.opts.select_basis:
                iso, disc = self.selection_iso(enlR.dims, D, 1, bond + 1), 0.0
            else:
                iso, disc = self.density_iso(rho_avg(self.rho_right, Eops, bond), D)
            disc_max = max(disc_max, disc)
            kept_max = max(kept_max, sum(U.shape[1] for U in iso.values()))
            Rnew = self.new_block("R", bond + 1, N, enlR, Eops, iso, self.R[bond + 2])
            self.R[bond + 1] = Rnew
            nsetup = self.setup_bond(bond - 1)
            self.psi = self.predict_left(bond, self.psi, enlR, Rnew, enlL, nsetup[0], nsetup[2])
            if two:
                self.psi2 = self.predict_left(bond, self.psi2, enlR, Rnew, enlL, nsetup[0], nsetup[2])
            self.psi_bond, self.psi_fresh = bond - 1, False
            setup = nsetup
        self.sweeps_done += 1
        out = dict(energy=min(thetas), last=self.theta, discarded_max=disc_max,
                   nprod=self.nprod_total - nprod0, kept_max=kept_max)
        if two:
            out["energy_excited"] = min(thetas2)
        if self.opts.measure:
            out["s1"], out["mutual"], _ = self.entropies()
        return out

    # ---------------------------------------------------- orbital correlations
    def measure_bond(self, bond: int, setup) -> None:
        """Correlations between the E site j = bond + 1 and every S site i <= bond
        in the state psi at this bond (the entropy paragraph's rho_i and rho_ij
        need <n_i>, <n_j>, <n_i n_j> and <c+_i c_j>; see oracle.entropy).

        With S before E in the Jordan-Wigner order and the E site first in E,
        c_j |s, (r, 1)> = (-1)^N(s) |s, (r, 0)>, so
        <c+_i c_j> = sum_q (-1)^N(q) <psi_q', C_i psi_q restricted to
        (r, 1) -> (r, 0)> with q' = q + dq_i, nonzero only when dq_i = dq_j."""
        enlL, Sops, enlR, Eops, terms = setup
        psi, T, j, m = self.psi, self.T, bond + 1, self.meas

        def occ_cols(q_s):
            # E columns of psi block q_s where the E site is occupied, and the
            # (offset, dim, base sector) of that part
            p = enlR.part(qsub(T, q_s), 1)
            return None if p is None else (p.off, p.dim, p.qb)

        nj = 0.0
        for q, X in psi.items():
            oc = occ_cols(q)
            if oc is not None:
                Y = X[:, oc[0]:oc[0] + oc[1]]
                nj += float(np.sum(Y * Y))
        m["pair_nj"][:bond + 1, j] = nj
        m["n1"][j] = nj
        for i in range(bond + 1):
            Nop = Sops.get(("N", i))
            ni = nn = 0.0
            for q, X in psi.items():
                r = None if Nop is None else Nop.block(q, False)
                if r is None:
                    continue
                Z = r[1] @ X
                ni += float(np.sum(X * Z))
                oc = occ_cols(q)
                if oc is not None:
                    a, d = oc[0], oc[1]
                    nn += float(np.sum(X[:, a:a + d] * Z[:, a:a + d]))
            m["pair_ni"][i, j] = ni
            m["nn"][i, j] = nn
            if bond == 0:
                m["n1"][0] = ni
            if self.delta[i] != self.delta[j]:
                continue
            C = Sops.get(("C", i))
            h = 0.0
            for q, X in psi.items():
                r = None if C is None else C.block(q, False)
                if r is None or r[0] not in psi:
                    continue
                oc = occ_cols(q)
                if oc is None:
                    continue
                q2 = r[0]
                p0 = enlR.part(qsub(T, q2), 0)
                if p0 is None or p0.qb != oc[2]:
                    continue
                Z = r[1] @ X[:, oc[0]:oc[0] + oc[1]]
                W = psi[q2][:, p0.off:p0.off + p0.dim]
                sign = -1.0 if nparticles(q) & 1 else 1.0
                h += sign * float(np.sum(W * Z))
            m["hop"][i, j] = h

    def entropies(self):
        """(s1, I, raw) from the last measured half sweep, in site indices (the
        natural order): s1[site], I[site, site'].  raw holds the correlations in
        chain positions (Jordan-Wigner order = chain order)."""
        from .entropy import entropies
        m = self.meas
        s1c, Ic = entropies(m["n1"], m["pair_ni"], m["pair_nj"], m["nn"], m["hop"])
        order = self.order
        s1 = np.empty(self.N)
        s1[order] = s1c
        I = np.empty((self.N, self.N))
        I[np.ix_(order, order)] = Ic
        return s1, I, m

    # ------------------------------------------------------------ helpers
    def psi_configs(self, enlL: Enlarged, enlR: Enlarged):
        """Determinant (bit mask over chain sites) of every superblock basis
        state, when both blocks are selections of determinants."""
        T = self.T
        Lb = self.L[enlL.site]
        Rb = self.R[enlR.site + 1]
        if Lb.configs is None or Rb.configs is None:
            return None
        out = {}
        for q, (ds, de) in self.psi_layout(enlL, enlR).items():
            sc = []
            for p in enlL.parts[q]:
                bit = (1 << enlL.site) if p.sigma else 0
                sc += [c | bit for c in Lb.configs[p.qb]]
            ec = []
            for p in enlR.parts[qsub(T, q)]:
                bit = (1 << enlR.site) if p.sigma else 0
                ec += [c | bit for c in Rb.configs[p.qb]]
            out[q] = np.array([[a | b for b in ec] for a in sc], dtype=np.uint64)
        return out
