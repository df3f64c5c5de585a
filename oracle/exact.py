"""Exact (uncontracted) MPS-PT energies in determinant space — oracle only.

Follows the paper's definitions directly:

* Dyall zeroth-order Hamiltonian: the full Hamiltonian restricted to the
  active orbitals plus diagonal virtual orbital energies (the paper's H0 for
  NEVPT; no core orbitals here).  V = H - H0.
* Hylleraas functional (Eq. hyll)
  H[Psi1] = <Psi1|H0 - E0|Psi1> + 2 <Psi1|Q V|Psi0>,
  minimised by the first-order equation (Eq. pt2) (H0 - E0)|Psi1> = -Q V|Psi0>.
* Third-order energy by Wigner's 2n+1 rule (Eq. 3rd)
  E3 = <Psi1|V|Psi1> - E1 <Psi1|Psi1>.

Reading used throughout (paper silent): with no core orbitals every term of V
carries a virtual index, so V|Psi0> only populates determinants with one or
two virtual electrons; Psi1 is sought in that first-order space, where Q acts
as the identity and H0 - E0 is positive definite.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import fock


# --------------------------------------------------------------------------
# Operator integrals for H, H_act, H0, V
# --------------------------------------------------------------------------

def split_integrals(h, eri, k_a, eps_virt):
    """One- and two-electron integrals of H_act (all-active), H0 and V = H - H0.

    Returns dict name -> (h1, eri) such that the operator is
    sum h1_pq E_pq + 1/2 sum eri_pqrs (E_pq E_rs - delta_qr E_ps), plus for H0
    the extra one-body diagonal eps_virt on the virtual orbitals.
    """
    k = h.shape[0]
    act = np.zeros(k, dtype=bool)
    act[:k_a] = True
    h_act = np.where(np.outer(act, act), h, 0.0)
    m4 = act[:, None, None, None] & act[None, :, None, None] & act[None, None, :, None] & act[None, None, None, :]
    eri_act = np.where(m4, eri, 0.0)
    h0 = h_act.copy()
    h0[k_a:, k_a:] = np.diag(eps_virt)
    return {
        "H": (h, eri),
        "H_act": (h_act, eri_act),
        "H0": (h0, eri_act),
        "V": (h - h0, eri - eri_act),
    }


def operator(name, h, eri, k_a, eps_virt, basis):
    h1, g = split_integrals(h, eri, k_a, eps_virt)[name]
    return fock.hamiltonian(h1, g, basis)


# --------------------------------------------------------------------------
# Active-space reference Psi0
# --------------------------------------------------------------------------

def active_ground_state(h, eri, k_a, n_elec, two_sz=0):
    """Lowest eigenpair of H_act in the (n_elec, 2Sz) sector of the active
    orbitals.  Sign fixed so the largest-magnitude amplitude is positive."""
    basis = fock.sector_basis(k_a, n_elec, two_sz)
    H = fock.hamiltonian(h[:k_a, :k_a], eri[:k_a, :k_a, :k_a, :k_a], basis).toarray()
    w, v = np.linalg.eigh(H)
    c = v[:, 0]
    if c[np.argmax(np.abs(c))] < 0:
        c = -c
    return w[0], c, basis


# --------------------------------------------------------------------------
# Brute force in the full determinant space (small systems)
# --------------------------------------------------------------------------

@dataclass
class ExactPT:
    E0: float
    E1: float
    E2: float
    E3: float
    psi1: np.ndarray      # first-order vector on ``fo_basis``
    fo_basis: np.ndarray  # determinants with 1 or 2 virtual electrons
    vpsi0: np.ndarray     # V|Psi0> on fo_basis


def brute_force(h, eri, k_a, eps_virt, n_elec, two_sz, psi0_act, act_basis) -> ExactPT:
    """Exact E0..E3 by a dense solve of Eq. pt2 in the first-order space.

    psi0_act: Psi0 as a vector over ``act_basis`` (active determinants, which
    are also full-space determinants with empty virtual orbitals).
    """
    k = h.shape[0]
    basis = fock.sector_basis(k, n_elec, two_sz)
    H0 = operator("H0", h, eri, k_a, eps_virt, basis)
    V = operator("V", h, eri, k_a, eps_virt, basis)
    psi0 = np.zeros(len(basis))
    psi0[np.searchsorted(basis, act_basis)] = psi0_act
    psi0 /= np.linalg.norm(psi0)
    E0 = psi0 @ (H0 @ psi0)
    vpsi0 = V @ psi0
    E1 = psi0 @ vpsi0
    nv = fock.n_virtual(basis, k_a)
    fo = np.nonzero((nv == 1) | (nv == 2))[0]
    # the rest of V|Psi0> must vanish (every V term carries a virtual index)
    assert np.max(np.abs(np.delete(vpsi0, fo)), initial=0.0) < 1e-12
    A = (H0[fo][:, fo]).toarray() - E0 * np.eye(len(fo))
    b = vpsi0[fo]
    psi1 = np.linalg.solve(A, -b)
    E2 = psi1 @ b
    Vff = V[fo][:, fo]
    E3 = psi1 @ (Vff @ psi1) - E1 * (psi1 @ psi1)
    return ExactPT(E0=E0, E1=E1, E2=E2, E3=E3, psi1=psi1, fo_basis=basis[fo], vpsi0=b)


def hylleraas(x, h, eri, k_a, eps_virt, E0, fo_basis, vpsi0):
    """Eq. hyll evaluated for an arbitrary first-order vector x on fo_basis."""
    n_elec = int(fock.popcount(fo_basis[:1])[0])
    amask = sum(1 << (2 * p) for p in range(h.shape[0]))
    na = int(fock.popcount(fo_basis[:1] & amask)[0])
    basis = fock.sector_basis(h.shape[0], n_elec, 2 * na - n_elec)
    fo = np.searchsorted(basis, fo_basis)
    H0 = operator("H0", h, eri, k_a, eps_virt, basis)[fo][:, fo]
    return x @ (H0 @ x) - E0 * (x @ x) + 2.0 * (x @ vpsi0)


def lambda_energy(h, eri, k_a, eps_virt, n_elec, two_sz, lam):
    """Lowest eigenvalue of H0 + lam V in the full (n_elec, 2Sz) sector."""
    basis = fock.sector_basis(h.shape[0], n_elec, two_sz)
    H0 = operator("H0", h, eri, k_a, eps_virt, basis)
    V = operator("V", h, eri, k_a, eps_virt, basis)
    return np.linalg.eigvalsh((H0 + lam * V).toarray())[0]


# --------------------------------------------------------------------------
# Factorised sum over states (larger active spaces)
# --------------------------------------------------------------------------

def factorised_e2(h, eri, k_a, eps_virt, n_elec, two_sz, psi0_act, act_basis):
    """Exact E2 without building the full determinant space.

    Dyall H0 keeps the virtual occupation pattern P, so the first-order space
    splits into blocks |J, P> (J an active determinant) on which
    H0 - E0 = H_act + eps_P - E0.  With b_P = <., P|V|Psi0> the minimiser of
    Eq. hyll gives E2 = -sum_P b_P^T (H_act + eps_P - E0)^{-1} b_P.

    The pattern determinant |J, P> = a^dag_J a^dag_P |vac> lists virtual
    creators after active ones, in ascending spin-orbital order.  Only terms of
    V that create virtual electrons from the active space survive on Psi0:
      one virtual:  sum_q [h_aq + sum_ts (aq|ts) E_ts] a_{q sig}, moved past
                    N-1 active creators (sign (-1)^(N-1));
      two virtual:  sum_qs (aq|bs) a_{s tau} a_{q sig} for a sig < b tau.
    Returns (E2, dict P -> contribution, E0).
    """
    k = h.shape[0]
    k_v = k - k_a
    ha, ga = h[:k_a, :k_a], eri[:k_a, :k_a, :k_a, :k_a]
    psi = psi0_act / np.linalg.norm(psi0_act)
    H_N = fock.hamiltonian(ha, ga, act_basis)
    E0 = psi @ (H_N @ psi)

    sectors = {}

    def sector(n, sz):
        if (n, sz) not in sectors:
            b = fock.sector_basis(k_a, n, sz)
            Hs = fock.hamiltonian(ha, ga, b).toarray() if len(b) else np.zeros((0, 0))
            w, v = np.linalg.eigh(Hs) if len(b) else (np.zeros(0), np.zeros((0, 0)))
            sectors[(n, sz)] = (b, w, v)
        return sectors[(n, sz)]

    def solve(n, sz, vec, eps_p):
        b, w, v = sector(n, sz)
        c = v.T @ vec
        return -np.sum(c * c / (w + eps_p - E0))

    contrib = {}
    # one virtual electron: pattern (a, sig)
    for sig in (0, 1):
        dsz = 1 if sig == 0 else -1
        n1, sz1 = n_elec - 1, two_sz - dsz
        b1 = sector(n1, sz1)[0]
        u = [fock.ladder(2 * q + sig, False, act_basis, b1) @ psi for q in range(k_a)]
        E1s = {(t, s): fock.excitation(t, s, b1) for t in range(k_a) for s in range(k_a)}
        for a in range(k_v):
            pa = k_a + a
            vec = np.zeros(len(b1))
            for q in range(k_a):
                G = sum(eri[pa, q, t, s] * E1s[t, s] for t in range(k_a) for s in range(k_a))
                vec += h[pa, q] * u[q] + G @ u[q]
            vec *= (-1) ** (n_elec - 1)
            contrib[((a, sig),)] = solve(n1, sz1, vec, eps_virt[a])
    # two virtual electrons: pattern (a sig) < (b tau)
    for sig in (0, 1):
        for tau in (0, 1):
            dsz = (1 if sig == 0 else -1) + (1 if tau == 0 else -1)
            n2, sz2 = n_elec - 2, two_sz - dsz
            b1 = fock.sector_basis(k_a, n_elec - 1, two_sz - (1 if sig == 0 else -1))
            b2 = sector(n2, sz2)[0]
            if len(b2) == 0:
                continue
            # w[q, s] = a_{s tau} a_{q sig} Psi0
            w = {}
            for q in range(k_a):
                uq = fock.ladder(2 * q + sig, False, act_basis, b1) @ psi
                for s in range(k_a):
                    w[q, s] = fock.ladder(2 * s + tau, False, b1, b2) @ uq
            for a in range(k_v):
                for b in range(a, k_v):
                    if 2 * (k_a + a) + sig >= 2 * (k_a + b) + tau:
                        continue
                    vec = sum(eri[k_a + a, q, k_a + b, s] * w[q, s]
                              for q in range(k_a) for s in range(k_a))
                    contrib[((a, sig), (b, tau))] = solve(n2, sz2, vec, eps_virt[a] + eps_virt[b])
    return sum(contrib.values()), contrib, E0


# --------------------------------------------------------------------------
# Psi0 as a matrix product state
# --------------------------------------------------------------------------

SITE_DN = ((0, 0), (1, 1), (1, -1), (2, 0))


def keep_count(eigs, M, rel_floor=1e-14, gap=1e-4):
    """Truncation rule: keep the M largest density-matrix eigenvalues (over all
    sectors), drop those <= rel_floor * trace, and never cut inside a cluster
    of eigenvalues closer than a relative ``gap`` (so spin multiplets stay
    whole).  eigs: list of (lambda, sector, index).  Returns the kept prefix
    length of the list sorted by (-lambda, sector, index).  A vanishing
    density matrix (the local solution is exactly zero, which happens when
    V|Psi0> has no component in the window's space) keeps min(M, dim) states
    in (sector, index) order: every basis is then equally significant."""
    s = sorted(eigs, key=lambda t: (-t[0], t[1], t[2]))
    lam = np.array([t[0] for t in s])
    tr = lam.sum()
    n_sig = int(np.sum(lam > rel_floor * tr)) if tr > 0 else len(lam)
    K0 = min(M, n_sig)
    K = K0
    while 0 < K < len(lam) and lam[K - 1] <= (1.0 + gap) * lam[K]:
        K -= 1
    if K == 0:
        K = K0
    return s, K


def psi0_mps(psi0_act, act_basis, k_a, M0=None):
    """Left-to-right compression of an active-space vector into an MPS
    (density-matrix truncation per (N, 2Sz) sector with ``keep_count``).

    Returns (bonds, sites) in the layout of ``paper_1408_5092_amd.inputs.MPSData``.
    """
    psi = np.zeros(4 ** k_a)
    psi[fock.site_index(act_basis, k_a)] = psi0_act / np.linalg.norm(psi0_act)
    T = psi.reshape(1, -1)
    labels = [(0, 0)]
    bonds = [[((0, 0), 1)]]
    sites = []
    for i in range(k_a):
        D = T.shape[0]
        rest = T.shape[1] // 4
        X = T.reshape(D, 4, rest).reshape(D * 4, rest)
        rlab = [(labels[a][0] + SITE_DN[s][0], labels[a][1] + SITE_DN[s][1])
                for a in range(D) for s in range(4)]
        if i == k_a - 1:
            qs = sorted(set(rlab[r] for r in range(len(rlab)) if np.any(X[r] != 0)))
            assert len(qs) == 1
            A = X.reshape(D, 4, 1)
            sites.append(A)
            bonds.append([(qs[0], 1)])
            break
        groups = {}
        for r, q in enumerate(rlab):
            groups.setdefault(q, []).append(r)
        eigs, vecs = [], {}
        for q in sorted(groups):
            rows = groups[q]
            rho = X[rows] @ X[rows].T
            w, v = np.linalg.eigh(rho)
            w, v = w[::-1], v[:, ::-1]
            vecs[q] = (rows, v)
            eigs += [(w[j], q, j) for j in range(len(w))]
        s, K = keep_count(eigs, M0 if M0 is not None else 10 ** 9)
        kept = {}
        for lam, q, j in s[:K]:
            kept[q] = kept.get(q, 0) + 1
        new_bond = [(q, kept[q]) for q in sorted(kept)]
        Dn = sum(d for _, d in new_bond)
        U = np.zeros((D * 4, Dn))
        off = 0
        new_labels = []
        for q, d in new_bond:
            rows, v = vecs[q]
            U[rows, off:off + d] = v[:, :d]
            off += d
            new_labels += [q] * d
        sites.append(U.reshape(D, 4, Dn))
        bonds.append(new_bond)
        T = U.T @ X
        labels = new_labels
    return bonds, sites


def mps_to_vector(sites, k):
    """Contract a (single-block-row) MPS into a dense vector over 4^k."""
    T = sites[0]
    for A in sites[1:]:
        T = np.tensordot(T, A, axes=([-1], [0]))
    return T.reshape(-1)
