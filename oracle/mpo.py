"""Matrix product operators for H0 and V (oracle; test infrastructure only).

An operator is a sum of terms, each a coefficient times a product of spin-
orbital ladder operators.  Written in the site-product basis (Eq. mpo of the
paper) each term becomes a product of 4x4 site matrices:

* ladder operators are sorted by site (stable), the permutation sign taken
  from the anticommutation of operators on different sites;
* the Jordan-Wigner string of every operator is a parity matrix P on each
  site to its left, so a site carries (product of its own ladder matrices)
  times P^(number of ladder operators on sites to its right).

Terms are merged into an MPO bond by bond: at bond b a term sits in a channel
keyed either by its left operator string (when fewer operators lie on the
left, or equally many and b < b_star) or by its right operator string.  A
channel keyed on the left carries coefficient 1 and the term's coefficient is
applied on the one site where the term switches from a left key to a right
key, so sums over right-keyed channels are the complementary operators.
"""
from __future__ import annotations

import numpy as np

CDAG_A = np.zeros((4, 4)); CDAG_A[1, 0] = 1.0; CDAG_A[3, 2] = 1.0
CDAG_B = np.zeros((4, 4)); CDAG_B[2, 0] = 1.0; CDAG_B[3, 1] = -1.0
PARITY = np.diag([1.0, -1.0, -1.0, 1.0])
IDENT = np.eye(4)
SITE_DN = ((0, 0), (1, 1), (1, -1), (2, 0))


def ladder_matrix(so: int, dag: bool) -> np.ndarray:
    m = CDAG_A if so % 2 == 0 else CDAG_B
    return m if dag else m.T


def operator_terms(h1, eri, annihilators_in=None):
    """Terms of sum_pq h1_pq E_pq + 1/2 sum (pq|rs) a+_p a+_r a_s a_q (spin summed).

    annihilators_in: optional set of orbitals; terms whose annihilators are not
    all in it are dropped (used for the part of V that acts on Psi0).
    Returns dict: ordered op tuple ((so, dag), ...) -> coefficient.
    """
    k = h1.shape[0]
    out = {}

    def add(c, ops):
        if c != 0.0:
            out[ops] = out.get(ops, 0.0) + c

    ok = (lambda *orbs: all(o in annihilators_in for o in orbs)) if annihilators_in is not None \
        else (lambda *orbs: True)
    for p in range(k):
        for q in range(k):
            if h1[p, q] == 0.0 or not ok(q):
                continue
            for s in (0, 1):
                add(h1[p, q], ((2 * p + s, True), (2 * q + s, False)))
    nz = np.argwhere(eri != 0.0)
    for p, q, r, s in nz:
        if not ok(q, s):
            continue
        c = 0.5 * eri[p, q, r, s]
        for sg in (0, 1):
            for tu in (0, 1):
                a, b = 2 * p + sg, 2 * r + tu
                cc, d = 2 * s + tu, 2 * q + sg
                if a == b or cc == d:
                    continue
                add(c, ((a, True), (b, True), (cc, False), (d, False)))
    return out


def canonical(ops):
    """Stable sort by site; returns (sign, sorted ops)."""
    ops = list(ops)
    sign = 1
    for i in range(1, len(ops)):       # insertion sort, counting cross-site swaps
        j = i
        while j > 0 and (ops[j - 1][0] >> 1) > (ops[j][0] >> 1):
            ops[j - 1], ops[j] = ops[j], ops[j - 1]
            sign = -sign
            j -= 1
    return sign, tuple(ops)


def qn_change(ops):
    dn = dsz = 0
    for so, dag in ops:
        sgn = 1 if dag else -1
        dn += sgn
        dsz += sgn * (1 if so % 2 == 0 else -1)
    return dn, dsz


class MPO:
    """W[i]: dict (channel_in, channel_out) -> 4x4 matrix <s|W|s'>.
    dq[b][c]: (dN, d2Sz) that channel c's left part applies to the left block."""

    def __init__(self, terms: dict, n_sites: int, b_star=None):
        canon = {}
        for ops, c in terms.items():
            sg, so = canonical(ops)
            canon[so] = canon.get(so, 0.0) + sg * c
        canon = {k: v for k, v in canon.items() if v != 0.0}
        self.n = n_sites
        sites = {ops: [o[0] >> 1 for o in ops] for ops in canon}
        if b_star is None:
            b_star = n_sites
            for b in range(n_sites + 1):
                left, right = set(), set()
                for ops, st in sites.items():
                    nl = sum(1 for x in st if x < b)
                    if 2 * nl == len(ops):
                        left.add(ops[:nl]); right.add(ops[nl:])
                if len(left) > len(right):
                    b_star = b
                    break
        self.b_star = b_star

        def key(ops, st, b):
            nl = sum(1 for x in st if x < b)
            nr = len(ops) - nl
            if nl < nr or (nl == nr and b < b_star):
                return ('L', ops[:nl])
            return ('R', ops[nl:])

        chans = [dict() for _ in range(n_sites + 1)]
        W = [dict() for _ in range(n_sites)]
        for ops, c in canon.items():
            st = sites[ops]
            keys = [key(ops, st, b) for b in range(n_sites + 1)]
            ids = [chans[b].setdefault(keys[b], len(chans[b])) for b in range(n_sites + 1)]
            for i in range(n_sites):
                m = IDENT.copy()
                for o, x in zip(ops, st):
                    if x == i:
                        m = m @ ladder_matrix(*o)
                n_right = sum(1 for x in st if x > i)
                if n_right % 2:
                    m = m @ PARITY
                e = (ids[i], ids[i + 1])
                if keys[i][0] == 'L' and keys[i + 1][0] == 'R':
                    W[i][e] = W[i].get(e, 0.0) + c * m
                elif e in W[i]:
                    assert np.array_equal(W[i][e], m)
                else:
                    W[i][e] = m
        self.W = W
        self.dims = [len(c) for c in chans]
        self.dq = []
        for b in range(n_sites + 1):
            dq = [None] * len(chans[b])
            for (side, ops), idx in chans[b].items():
                dn, dsz = qn_change(ops)
                dq[idx] = (dn, dsz) if side == 'L' else (-dn, -dsz)
            self.dq.append(dq)

    def dense(self):
        """Contract to a dense 4^n x 4^n matrix (small n only)."""
        T = {0: np.ones((1, 1))}
        for i in range(self.n):
            nt = {}
            for (a, b), m in self.W[i].items():
                if a in T:
                    v = np.kron(T[a], m)
                    nt[b] = nt[b] + v if b in nt else v
            T = nt
        assert list(T.keys()) == [0]
        return T[0]


def build_operators(h, eri, k_a, eps_virt):
    """MPOs of the Dyall H0, of the part of V acting on Psi0 (its annihilators
    all active) and of the full V, over k_a + k_v sites."""
    k = h.shape[0]
    act = np.zeros(k, dtype=bool); act[:k_a] = True
    m4 = act[:, None, None, None] & act[None, :, None, None] & act[None, None, :, None] & act[None, None, None, :]
    eri_act = np.where(m4, eri, 0.0)
    h0 = np.where(np.outer(act, act), h, 0.0)
    h0[k_a:, k_a:] = np.diag(eps_virt)
    hv, gv = h - h0, eri - eri_act
    return {
        "H0": lambda: MPO(operator_terms(h0, eri_act), k),
        "V_psi0": lambda: MPO(operator_terms(hv, gv, annihilators_in=set(range(k_a))), k),
        "V": lambda: MPO(operator_terms(hv, gv), k),
    }
