"""Seeded synthetic inputs for MPS perturbation theory (MPS-PT).

This module only draws random numbers and lays out quantum-number structure.
It performs none of the method's arithmetic: no Hamiltonian is applied, no
energy is formed, nothing is solved or decomposed.  Both the HIP library and
the CPU oracle consume what it returns.

Model Hamiltonian (a stand-in for the paper's N2 / cc-pVXZ integrals, which
are not available): k_a active then k_v virtual spatial orbitals,

* orbital energies: active ~ U(-0.5, 0.5), virtual ~ U(1, 3), placed on the
  diagonal of the one-electron matrix h;
* off-diagonal h_pq = h_qp ~ N(0, 0.05) (standard deviation) for every p != q;
* two-electron integrals in Cholesky form (pq|rs) = sum_L B^L_pq B^L_rs with
  each B^L symmetric, entries ~ N(0, 0.1 / sqrt(rank));
* the zeroth-order (Dyall) partition uses the drawn virtual orbital energies
  as the diagonal virtual Fock elements.

Orbital / site order is active orbitals first, then virtual orbitals.  A site
is one spatial orbital with local basis {|0>, |up>, |dn>, |up dn>} carrying
(N, 2Sz) = (0,0), (1,1), (1,-1), (2,0).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SITE_DN = ((0, 0), (1, 1), (1, -1), (2, 0))  # (dN, d2Sz) of the four site states


@dataclass
class Integrals:
    k_a: int
    k_v: int
    h: np.ndarray          # (k, k) symmetric one-electron matrix
    B: np.ndarray          # (rank, k, k) symmetric Cholesky vectors
    eps_virt: np.ndarray   # (k_v,) diagonal virtual energies used by H0

    @property
    def k(self) -> int:
        return self.k_a + self.k_v


def integrals(k_a: int, k_v: int, rank: int, seed: int) -> Integrals:
    """Draw the model Hamiltonian for one seed (draw order is part of the recipe)."""
    rng = np.random.default_rng(seed)
    k = k_a + k_v
    eps_act = rng.uniform(-0.5, 0.5, size=k_a)
    eps_virt = rng.uniform(1.0, 3.0, size=k_v)
    xh = rng.normal(0.0, 0.05, size=(k, k))
    up = np.triu(xh, 1)
    h = np.diag(np.concatenate([eps_act, eps_virt])) + up + up.T
    xb = rng.normal(0.0, 0.1 / np.sqrt(rank), size=(rank, k, k))
    B = np.triu(xb) + np.transpose(np.triu(xb, 1), (0, 2, 1))
    return Integrals(k_a=k_a, k_v=k_v, h=np.ascontiguousarray(h),
                     B=np.ascontiguousarray(B), eps_virt=eps_virt.copy())


# --------------------------------------------------------------------------
# Quantum-number structure of a random starting MPS
# --------------------------------------------------------------------------

def _site_counts(n_sites, virtual_from):
    """Per site: is it a virtual orbital?"""
    return [i >= virtual_from for i in range(n_sites)]


def _site_ok(i, k_a, dn, virt_occ):
    return virt_occ is None or i < k_a or dn in virt_occ[i - k_a]


def bond_sectors(n_sites: int, k_a: int, n_elec: int, two_sz: int, nv_allowed, virt_occ=None):
    """Sectors (N_left, 2Sz_left) that some admissible configuration passes
    through at every bond, with rough left/right configuration counts.

    A configuration is admissible if it has n_elec electrons, total 2Sz, a
    number of electrons in virtual orbitals (sites >= k_a) that lies in
    nv_allowed, and (if virt_occ is given) an electron count on the j-th
    virtual site that lies in virt_occ[j].  Returns a list over bonds
    0..n_sites of dicts {(N, 2Sz): (count_left, count_right)}.
    """
    virt = _site_counts(n_sites, k_a)
    # left DP over (N, 2Sz, nv) -> number of configurations
    left = [dict() for _ in range(n_sites + 1)]
    left[0][(0, 0, 0)] = 1
    for i in range(n_sites):
        for (n, sz, nv), c in left[i].items():
            for dn, dsz in SITE_DN:
                if not _site_ok(i, k_a, dn, virt_occ):
                    continue
                key = (n + dn, sz + dsz, nv + (dn if virt[i] else 0))
                left[i + 1][key] = left[i + 1].get(key, 0) + c
    right = [dict() for _ in range(n_sites + 1)]
    right[n_sites][(0, 0, 0)] = 1
    for i in range(n_sites - 1, -1, -1):
        for (n, sz, nv), c in right[i + 1].items():
            for dn, dsz in SITE_DN:
                if not _site_ok(i, k_a, dn, virt_occ):
                    continue
                key = (n + dn, sz + dsz, nv + (dn if virt[i] else 0))
                right[i][key] = right[i].get(key, 0) + c
    out = []
    for b in range(n_sites + 1):
        cl, cr = {}, {}
        for (nl, szl, nvl), c in left[b].items():
            q = (nl, szl)
            nvr_ok = [nvr for nvr in range(0, 2 * n_sites + 1)
                      if nvl + nvr in nv_allowed and right[b].get((n_elec - nl, two_sz - szl, nvr))]
            if nvr_ok:
                cl[q] = cl.get(q, 0) + c
                for nvr in nvr_ok:
                    key = (q, nvr)
                    if key not in cr:
                        cr[key] = right[b][(n_elec - nl, two_sz - szl, nvr)]
        sec = {}
        for q in cl:
            sec[q] = (cl[q], sum(v for (qq, _), v in cr.items() if qq == q))
        out.append(dict(sorted(sec.items())))
    return out


def _dims(sectors: dict, M: int):
    q = list(sectors.keys())
    d = [min(cl, cr) for cl, cr in sectors.values()]
    while sum(d) > M:
        j = int(np.argmax(d))
        d[j] -= 1
    return [(qq, dd) for qq, dd in zip(q, d) if dd > 0]


@dataclass
class MPSData:
    """MPS as dense site tensors [D_l][4][D_{l+1}] plus per-bond sector lists.

    bonds[l] is a list of ((N, 2Sz), dim) in ascending sector order; the basis
    states of bond l are laid out sector after sector.  Entries of a site
    tensor outside the blocks allowed by particle number / spin are zero.
    """
    bonds: list
    sites: list

    def bond_dims(self):
        return [sum(d for _, d in b) for b in self.bonds]

    def bond_qn(self):
        """Flattened (N, 2Sz) label per basis state, bond after bond."""
        lab = []
        for b in self.bonds:
            for (n, sz), d in b:
                lab.extend([(n, sz)] * d)
        return np.asarray(lab, dtype=np.int32).reshape(-1, 2)


def random_mps(n_sites: int, k_a: int, n_elec: int, two_sz: int, nv_allowed,
               M: int, seed: int, virt_occ=None) -> MPSData:
    """Seeded random block-sparse MPS over the admissible sectors.

    Bond sector dimensions are min(left count, right count), then the largest
    are decremented until the bond dimension is at most M.  Every allowed
    block entry is drawn from N(0, 1).
    """
    rng = np.random.default_rng(seed)
    secs = bond_sectors(n_sites, k_a, n_elec, two_sz, set(nv_allowed), virt_occ)
    bonds = [_dims(s, M) for s in secs]
    sites = []
    for i in range(n_sites):
        bl, br = bonds[i], bonds[i + 1]
        Dl, Dr = sum(d for _, d in bl), sum(d for _, d in br)
        A = np.zeros((Dl, 4, Dr))
        offl = np.cumsum([0] + [d for _, d in bl])
        offr = {q: (o, d) for (q, d), o in zip(br, np.cumsum([0] + [d for _, d in br]))}
        for j, ((n, sz), dl) in enumerate(bl):
            for s, (dn, dsz) in enumerate(SITE_DN):
                tgt = offr.get((n + dn, sz + dsz))
                if tgt is None:
                    continue
                o, dr = tgt
                A[offl[j]:offl[j] + dl, s, o:o + dr] = rng.standard_normal((dl, dr))
        sites.append(A)
    return MPSData(bonds=bonds, sites=sites)


def psi1_guess(k_a: int, k_v: int, n_elec: int, two_sz: int, M1: int, seed: int) -> MPSData:
    """Random first-order MPS restricted to one or two virtual electrons."""
    return random_mps(k_a + k_v, k_a, n_elec, two_sz, (1, 2), M1, seed)


def psi0_guess(k_a: int, n_elec: int, two_sz: int, M0: int, seed: int) -> MPSData:
    """Random active-space MPS (start of a ground-state sweep for Psi0)."""
    return random_mps(k_a, k_a, n_elec, two_sz, (0,), M0, seed)


# Named workloads: (k_a, k_v, n_elec, cholesky rank, M0, M1, sweeps)
WORKLOADS = {
    "c1_4a4v": dict(k_a=4, k_v=4, n_elec=4, rank=16, M0=None, M1=16, sweeps=None),
    "c2_8a16v": dict(k_a=8, k_v=16, n_elec=8, rank=32, M0=64, M1=128, sweeps=4),
}


def mlp_init(seed: int, n_in: int = 8, n_hidden: int = 64) -> np.ndarray:
    """Seeded initial parameters of the preconditioner network, flat float32 in the
    layout W1[h][f], b1[h], W2[h][h], b2[h], w3[h], b3: weights N(0, 1/fan_in),
    biases 0, output bias 0.5413 (softplus(0.5413) = 1, the Jacobi scale)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0.0, 1.0 / np.sqrt(n_in), (n_hidden, n_in))
    W2 = rng.normal(0.0, 1.0 / np.sqrt(n_hidden), (n_hidden, n_hidden))
    w3 = rng.normal(0.0, 0.1 / np.sqrt(n_hidden), n_hidden)
    parts = [W1.ravel(), np.zeros(n_hidden), W2.ravel(), np.zeros(n_hidden), w3, [0.5413248546129181]]
    return np.concatenate(parts).astype(np.float32)
