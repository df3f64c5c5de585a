"""Determinant-space second quantization (oracle; test infrastructure only).

Conventions (shared by every oracle module):

* spatial orbitals p = 0..k-1, active orbitals first, then virtual ones;
* spin orbital j = 2p + sigma with sigma = 0 (alpha) or 1 (beta);
* a determinant is a bit mask over spin orbitals and stands for the ordered
  product of creators in ascending j acting on the vacuum, so
  a^dag_j |n> = (-1)^(number of occupied i < j) |n + e_j>.

The spin-free Hamiltonian is written out from its definition,
H = sum_pq h_pq E_pq + 1/2 sum_pqrs (pq|rs) (E_pq E_rs - delta_qr E_ps),
with E_pq = sum_sigma a^dag_{p sigma} a_{q sigma}.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.sparse as sp


def popcount(x):
    return np.bitwise_count(np.asarray(x, dtype=np.uint64)).astype(np.int64)


def sector_basis(k: int, n_elec: int | None = None, two_sz: int | None = None) -> np.ndarray:
    """Sorted bit masks of all determinants on k spatial orbitals with the given
    electron number and 2Sz (None = no restriction)."""
    nso = 2 * k
    if n_elec is None:
        states = np.arange(1 << nso, dtype=np.int64)
    else:
        states = np.array(sorted(sum(1 << j for j in c) for c in combinations(range(nso), n_elec)),
                          dtype=np.int64)
    if two_sz is not None and len(states):
        amask = sum(1 << (2 * p) for p in range(k))
        na = popcount(states & amask)
        nb = popcount(states) - na
        states = states[(na - nb) == two_sz]
    return states


def _lookup(basis: np.ndarray, states: np.ndarray) -> np.ndarray:
    idx = np.searchsorted(basis, states)
    idx = np.minimum(idx, len(basis) - 1)
    assert np.all(basis[idx] == states), "state outside the target basis"
    return idx


def ladder(j: int, dagger: bool, src: np.ndarray, dst: np.ndarray) -> sp.csr_matrix:
    """Matrix of a^dag_j (dagger) or a_j mapping basis ``src`` to basis ``dst``."""
    bit = np.int64(1) << j
    occ = (src & bit) != 0
    sel = ~occ if dagger else occ
    cols = np.nonzero(sel)[0]
    s = src[cols]
    sign = 1.0 - 2.0 * (popcount(s & (bit - 1)) & 1)
    new = (s | bit) if dagger else (s & ~bit)
    keep = np.isin(new, dst)
    rows = _lookup(dst, new[keep]) if keep.any() else np.zeros(0, dtype=np.int64)
    return sp.csr_matrix((sign[keep], (rows, cols[keep])), shape=(len(dst), len(src)))


def excitation(p: int, q: int, basis: np.ndarray) -> sp.csr_matrix:
    """E_pq = sum_sigma a^dag_{p sigma} a_{q sigma} on an N- and Sz-conserving basis."""
    out = None
    for sig in (0, 1):
        jq, jp = 2 * q + sig, 2 * p + sig
        bq, bp = np.int64(1) << jq, np.int64(1) << jp
        s = basis
        sel = (s & bq) != 0
        idx = np.nonzero(sel)[0]
        s1 = s[idx]
        sign1 = 1.0 - 2.0 * (popcount(s1 & (bq - 1)) & 1)
        s1 = s1 & ~bq
        ok = (s1 & bp) == 0
        idx, s1, sign1 = idx[ok], s1[ok], sign1[ok]
        sign2 = 1.0 - 2.0 * (popcount(s1 & (bp - 1)) & 1)
        s2 = s1 | bp
        m = sp.csr_matrix((sign1 * sign2, (_lookup(basis, s2), idx)), shape=(len(basis),) * 2)
        out = m if out is None else out + m
    return out


def hamiltonian(h: np.ndarray, eri: np.ndarray, basis: np.ndarray) -> sp.csr_matrix:
    """Spin-free Hamiltonian with one-electron matrix h and chemists' integrals
    eri[p,q,r,s] = (pq|rs), on an N- and Sz-conserving determinant basis."""
    k = h.shape[0]
    E = {(p, q): excitation(p, q, basis) for p in range(k) for q in range(k)}
    n = len(basis)
    H = sp.csr_matrix((n, n))
    for p in range(k):
        for q in range(k):
            if h[p, q] != 0.0:
                H = H + h[p, q] * E[p, q]
    for p in range(k):
        for q in range(k):
            F = sp.csr_matrix((n, n))
            for r in range(k):
                for s in range(k):
                    if eri[p, q, r, s] != 0.0:
                        F = F + eri[p, q, r, s] * E[r, s]
            if F.nnz:
                H = H + 0.5 * (E[p, q] @ F)
    contr = np.einsum('pqqs->ps', eri)
    for p in range(k):
        for s in range(k):
            if contr[p, s] != 0.0:
                H = H - 0.5 * contr[p, s] * E[p, s]
    return H.tocsr()


def eri_from_cholesky(B: np.ndarray) -> np.ndarray:
    """(pq|rs) = sum_L B^L_pq B^L_rs."""
    return np.einsum('lpq,lrs->pqrs', B, B)


def n_virtual(basis: np.ndarray, k_a: int) -> np.ndarray:
    """Number of electrons in virtual orbitals (spin orbitals >= 2 k_a)."""
    return popcount(basis >> (2 * k_a))


def site_index(basis: np.ndarray, k: int) -> np.ndarray:
    """Index of each determinant in the site-product basis |s_0 s_1 ... s_{k-1}>,
    s_p = n_{p alpha} + 2 n_{p beta}, site 0 most significant."""
    idx = np.zeros(len(basis), dtype=np.int64)
    for p in range(k):
        s = ((basis >> (2 * p)) & 1) + 2 * ((basis >> (2 * p + 1)) & 1)
        idx = idx * 4 + s
    return idx
