"""Same-algorithm CPU MPS-PT sweep with dense numpy tensors (oracle only).

The first-order wavefunction |Psi1> is an MPS (Eq. mps1); the sweep optimises
two neighbouring site tensors at a time (the two-site variant the paper
uses), keeping the rest fixed.  At window (i, i+1) the partial derivative of
the Hylleraas functional (Eq. hyll) with respect to the two-site tensor x is
set to zero, which gives the local linear equation
    (H0_eff - E0) x = -b,   b = <local basis| V |Psi0>,
solved by Jacobi-preconditioned conjugate gradient.  The local value
x.(A x) + 2 x.b is the running second-order energy.  The solved tensor is
split by the reduced density matrix of the half being renormalised (the
4M -> M mapping of the paper's discussion of discarded weight), keeping the
M1 most significant states.

Dense tensors: a site tensor is [D_left, 4, D_right]; every bond carries an
(N, 2Sz) label per basis state.  Environments are dense [channels, D_bra,
D_ket].  Quantum numbers only enter through the admissibility mask of the
two-site tensor and the sector blocks of the density matrices.
"""
from __future__ import annotations

import numpy as np

from . import mpo as mpomod
from .exact import keep_count

SITE_DN = np.array([[0, 0], [1, 1], [1, -1], [2, 0]])


def site_allowed(i, k_a, dn, virt_occ):
    """May site i hold dn electrons?  virt_occ[j] is the set of electron
    counts allowed on virtual site k_a + j (None: no restriction)."""
    return virt_occ is None or i < k_a or dn in virt_occ[i - k_a]


def admissible(n, k_a, n_elec, two_sz, nv_allowed, virt_occ=None):
    """Per bond: set of (N_left, 2Sz_left) through which a configuration with
    n_elec electrons, total 2Sz, a virtual-electron count in nv_allowed and
    (if given) per-virtual-site counts in virt_occ can pass (sites >= k_a are
    virtual)."""
    left = [set() for _ in range(n + 1)]
    left[0].add((0, 0, 0))
    for i in range(n):
        for (a, s, v) in left[i]:
            for dn, ds in SITE_DN:
                if site_allowed(i, k_a, dn, virt_occ):
                    left[i + 1].add((a + dn, s + ds, v + (dn if i >= k_a else 0)))
    right = [set() for _ in range(n + 1)]
    right[n].add((0, 0, 0))
    for i in range(n - 1, -1, -1):
        for (a, s, v) in right[i + 1]:
            for dn, ds in SITE_DN:
                if site_allowed(i, k_a, dn, virt_occ):
                    right[i].add((a + dn, s + ds, v + (dn if i >= k_a else 0)))
    out = []
    for b in range(n + 1):
        ok = set()
        for (a, s, v) in left[b]:
            for (a2, s2, v2) in right[b]:
                if a + a2 == n_elec and s + s2 == two_sz and v + v2 in nv_allowed:
                    ok.add((a, s))
        out.append(ok)
    return out


def labels_from_bonds(bonds):
    out = []
    for b in bonds:
        lab = []
        for (q, d) in b:
            lab += [q] * d
        out.append(np.array(lab, dtype=np.int64).reshape(-1, 2))
    return out


def left_update(L, W, Abra, Aket, w_out):
    T = np.einsum('wab,bsc->wasc', L, Aket)
    out = np.zeros((w_out, Abra.shape[2], Aket.shape[2]))
    for (c, c2), m in W.items():
        for s, t in np.argwhere(m != 0.0):
            out[c2] += m[s, t] * (Abra[:, s, :].T @ T[c, :, t, :])
    return out


def right_update(R, W, Abra, Aket, w_out):
    T = np.einsum('cxy,bty->cxtb', R, Aket)
    out = np.zeros((w_out, Abra.shape[0], Aket.shape[0]))
    for (c, c2), m in W.items():
        for s, t in np.argwhere(m != 0.0):
            out[c] += m[s, t] * (Abra[:, s, :] @ T[c2, :, t, :])
    return out


def apply_two_site(L, R, W1, W2, x, w_mid):
    """sum over channels of L[w] (x) W1[w,m] (x) W2[m,u] (x) R[u] applied to x."""
    T1 = np.einsum('wab,bstc->wastc', L, x)
    T2 = {}
    for (w, m), op in W1.items():
        v = np.einsum('Ss,astc->aStc', op, T1[w])
        T2[m] = T2[m] + v if m in T2 else v
    T3 = {}
    for (m, u), op in W2.items():
        if m not in T2:
            continue
        v = np.einsum('Tt,aStc->aSTc', op, T2[m])
        T3[u] = T3[u] + v if u in T3 else v
    out = np.zeros((L.shape[1], 4, 4, R.shape[1]))
    for u, v in T3.items():
        out += np.einsum('aSTc,Cc->aSTC', v, R[u])
    return out


def diag_two_site(L, R, W1, W2):
    Ld = np.einsum('waa->wa', L)
    Rd = np.einsum('waa->wa', R)
    D2 = {}
    for (w, m), op in W1.items():
        v = np.einsum('a,S->aS', Ld[w], np.diag(op))
        D2[m] = D2[m] + v if m in D2 else v
    out = np.zeros((L.shape[1], 4, 4, R.shape[1]))
    for (m, u), op in W2.items():
        if m in D2:
            out += np.einsum('aS,T,c->aSTc', D2[m], np.diag(op), Rd[u])
    return out


def pcg(apply_A, rhs, diag, x0, tol, maxit, restarts=3):
    """Jacobi-preconditioned CG for A x = rhs (A positive definite).

    The start vector is first scaled to the best multiple of itself
    (alpha = x0.rhs / x0.A x0), and convergence is always confirmed on the
    true residual rhs - A x; if the recursively updated residual drifted, CG
    restarts from the current x.  Returns (x, iterations, converged, A x)."""
    nb = np.linalg.norm(rhs)
    if nb == 0.0:
        return np.zeros_like(x0), 0, True, np.zeros_like(x0)
    x = x0.copy()
    q = apply_A(x)
    xq = np.vdot(x, q)
    if xq > 0.0:
        a = np.vdot(x, rhs) / xq
        x *= a
        q *= a
    it = 0
    for _ in range(restarts + 1):
        r = rhs - q
        if np.linalg.norm(r) <= tol * nb:
            return x, it, True, q
        z = r / diag
        p = z.copy()
        rz = np.vdot(r, z)
        while it < maxit:
            w = apply_A(p)
            pw = np.vdot(p, w)
            if pw <= 0.0:
                raise FloatingPointError("H0 - E0 is not positive definite on the local space")
            alpha = rz / pw
            x += alpha * p
            r -= alpha * w
            it += 1
            if np.linalg.norm(r) <= tol * nb:
                break
            z = r / diag
            rz_new = np.vdot(r, z)
            p = z + (rz_new / rz) * p
            rz = rz_new
        q = apply_A(x)
        if it >= maxit:
            break
    return x, it, np.linalg.norm(rhs - q) <= tol * nb, q


class Sweeper:
    """Two-site MPS-PT sweep, dense numpy (the oracle's O-B)."""

    def __init__(self, h, eri, k_a, eps_virt, n_elec, two_sz, psi0, psi1, M1,
                 cg_tol=1e-10, cg_maxit=500, virt_occ=None):
        self.k_a = k_a
        self.n = n = h.shape[0]
        self.N, self.tsz, self.M = n_elec, two_sz, M1
        self.cg_tol, self.cg_maxit = cg_tol, cg_maxit
        ops = mpomod.build_operators(h, eri, k_a, eps_virt)
        self.mpo_h0 = ops["H0"]()
        self.mpo_v = ops["V_psi0"]()
        self._mpo_vfull = ops["V"]
        # virt_occ restricts Psi1 to the configurations with allowed electron
        # counts on each virtual site (one virtual pair of the decomposition)
        self.virt_occ = virt_occ
        self.adm = admissible(n, k_a, n_elec, two_sz, (1, 2), virt_occ)
        self.site_ok = np.array([[site_allowed(i, k_a, dn, virt_occ) for dn, _ in SITE_DN] for i in range(n)])
        # Psi0 on active sites, extended by empty virtual sites
        b0, s0 = psi0
        P0 = [np.array(a, dtype=float) for a in s0]
        for _ in range(n - k_a):
            v = np.zeros((1, 4, 1)); v[0, 0, 0] = 1.0
            P0.append(v)
        self.P0 = P0
        one = np.ones((1, 1, 1))
        ov = one
        for a in P0:
            ov = left_update(ov, {(0, 0): np.eye(4)}, a, a, 1)
        self.P0[0] = self.P0[0] / np.sqrt(ov[0, 0, 0])
        E = one
        for i, a in enumerate(self.P0):
            E = left_update(E, self.mpo_h0.W[i], a, a, self.mpo_h0.dims[i + 1])
        self.E0 = float(E[0, 0, 0])
        self.P0x = [np.einsum('asb,btc->astc', self.P0[i], self.P0[i + 1]) for i in range(n - 1)]
        # Psi1 guess
        b1, s1 = psi1
        self.A = [np.array(a, dtype=float) for a in s1]
        self.lab = labels_from_bonds(b1)
        self.LH = [None] * (n + 1); self.RH = [None] * (n + 1)
        self.LV = [None] * (n + 1); self.RV = [None] * (n + 1)
        self.LH[0] = self.LV[0] = one
        self.RH[n] = self.RV[n] = one
        self.trace = []

    # ---------------------------------------------------------------- masks
    def mask(self, i):
        l, r = self.lab[i], self.lab[i + 2]
        ql = l[:, None, None, None, :] + SITE_DN[None, :, None, None, :]
        qr = ql + SITE_DN[None, None, :, None, :]
        ok = np.all(qr == r[None, None, None, :, :], axis=-1)
        mid = np.array([[tuple(q) in self.adm[i + 1] for q in row] for row in ql[:, :, 0, 0, :]])
        occ = self.site_ok[i][:, None] & self.site_ok[i + 1][None, :]
        return ok & mid[:, :, None, None] & occ[None, :, :, None]

    # ---------------------------------------------------------- truncation
    def _select(self, groups, rho_of):
        eigs, vecs = [], {}
        for q in sorted(groups):
            rho = rho_of(groups[q])
            w, v = np.linalg.eigh(rho)
            w, v = w[::-1], v[:, ::-1]
            vecs[q] = v
            eigs += [(w[j], q, j) for j in range(len(w))]
        s, K = keep_count(eigs, self.M)
        tr = sum(t[0] for t in s)
        kept = {}
        for lam, q, j in s[:K]:
            kept[q] = kept.get(q, 0) + 1
        disc = 1.0 - sum(t[0] for t in s[:K]) / tr if tr > 0 else 0.0
        return [(q, kept[q]) for q in sorted(kept)], vecs, disc

    def truncate_forward(self, x, i):
        Dl, _, _, Dr = x.shape
        X = x.reshape(Dl * 4, 4 * Dr)
        rl = (self.lab[i][:, None, :] + SITE_DN[None, :, :]).reshape(-1, 2)
        groups = {}
        for r, q in enumerate(map(tuple, rl)):
            if q in self.adm[i + 1]:
                groups.setdefault(q, []).append(r)
        bond, vecs, disc = self._select(groups, lambda rows: X[rows] @ X[rows].T)
        Dn = sum(d for _, d in bond)
        U = np.zeros((Dl * 4, Dn))
        off, lab = 0, []
        for q, d in bond:
            U[groups[q], off:off + d] = vecs[q][:, :d]
            off += d; lab += [q] * d
        self.A[i] = U.reshape(Dl, 4, Dn)
        self.lab[i + 1] = np.array(lab, dtype=np.int64).reshape(-1, 2)
        return (U.T @ X).reshape(Dn, 4, Dr), bond, disc

    def truncate_backward(self, x, i):
        Dl, _, _, Dr = x.shape
        X = x.reshape(Dl * 4, 4 * Dr)
        cl = (self.lab[i + 2][None, :, :] - SITE_DN[:, None, :]).reshape(-1, 2)
        groups = {}
        for c, q in enumerate(map(tuple, cl)):
            if q in self.adm[i + 1]:
                groups.setdefault(q, []).append(c)
        bond, vecs, disc = self._select(groups, lambda cols: X[:, cols].T @ X[:, cols])
        Dn = sum(d for _, d in bond)
        V = np.zeros((4 * Dr, Dn))
        off, lab = 0, []
        for q, d in bond:
            V[groups[q], off:off + d] = vecs[q][:, :d]
            off += d; lab += [q] * d
        self.A[i + 1] = V.T.reshape(Dn, 4, Dr)
        self.lab[i + 1] = np.array(lab, dtype=np.int64).reshape(-1, 2)
        return (X @ V).reshape(Dl, 4, Dn), bond, disc

    # ---------------------------------------------------------- env updates
    def _upd_left(self, i):
        m0, mv = self.mpo_h0, self.mpo_v
        self.LH[i + 1] = left_update(self.LH[i], m0.W[i], self.A[i], self.A[i], m0.dims[i + 1])
        self.LV[i + 1] = left_update(self.LV[i], mv.W[i], self.A[i], self.P0[i], mv.dims[i + 1])

    def _upd_right(self, i):
        m0, mv = self.mpo_h0, self.mpo_v
        self.RH[i] = right_update(self.RH[i + 1], m0.W[i], self.A[i], self.A[i], m0.dims[i])
        self.RV[i] = right_update(self.RV[i + 1], mv.W[i], self.A[i], self.P0[i], mv.dims[i])

    # ---------------------------------------------------------- local solve
    def solve(self, i, x0):
        m0, mv = self.mpo_h0, self.mpo_v
        mask = self.mask(i)
        L, R = self.LH[i], self.RH[i + 2]
        b = apply_two_site(self.LV[i], self.RV[i + 2], mv.W[i], mv.W[i + 1], self.P0x[i],
                           mv.dims[i + 1]) * mask
        d = diag_two_site(L, R, m0.W[i], m0.W[i + 1]) - self.E0
        d = np.where(mask, d, 1.0)

        def A(v):
            return (apply_two_site(L, R, m0.W[i], m0.W[i + 1], v, m0.dims[i + 1]) - self.E0 * v) * mask

        x, it, conv, ax = pcg(A, -b, d, x0 * mask, self.cg_tol, self.cg_maxit)
        e = float(np.vdot(x, ax) + 2.0 * np.vdot(x, b))
        return x, e, it, conv

    # ---------------------------------------------------------------- sweep
    def right_canonicalize(self):
        n = self.n
        for i in range(n - 2, -1, -1):
            x = np.einsum('asb,btc->astc', self.A[i], self.A[i + 1])
            C, _, _ = self.truncate_backward(x, i)
            self.A[i] = C
            self._upd_right(i + 1)

    def run(self, n_sweeps=None, e_tol=1e-9, max_sweeps=10, on_step=None):
        n = self.n
        self.right_canonicalize()
        x0 = np.einsum('asb,btc->astc', self.A[0], self.A[1])
        e_sweep = []
        sweep = 0
        while True:
            for direction, windows in (("f", range(0, n - 1)), ("b", range(n - 2, -1, -1))):
                for i in windows:
                    x, e, it, conv = self.solve(i, x0)
                    if direction == "f":
                        C, bond, disc = self.truncate_forward(x, i)
                        self._upd_left(i)
                        if i < n - 2:
                            x0 = np.einsum('asc,ctd->astd', C, self.A[i + 2])
                        else:
                            self.A[i + 1] = C
                            x0 = np.einsum('asb,btc->astc', self.A[i], C)
                    else:
                        C, bond, disc = self.truncate_backward(x, i)
                        self._upd_right(i + 1)
                        if i > 0:
                            x0 = np.einsum('asb,btc->astc', self.A[i - 1], C)
                        else:
                            self.A[0] = C
                            x0 = np.einsum('asc,ctd->astd', C, self.A[1])
                    self.trace.append(dict(sweep=sweep, dir=direction, window=i, e2=e,
                                           cg_iters=it, converged=conv, discarded=disc,
                                           bond=bond))
                    self.x_last = x
                    if on_step is not None:
                        on_step(self.trace[-1])
            e_sweep.append(self.trace[-1]["e2"])
            sweep += 1
            if n_sweeps is not None:
                if sweep >= n_sweeps:
                    break
            elif (len(e_sweep) > 1 and abs(e_sweep[-1] - e_sweep[-2]) < e_tol) or sweep >= max_sweeps:
                break
        self.e_sweep = e_sweep
        return e_sweep

    def e3(self):
        """<Psi1|V|Psi1> on the final (untruncated) two-site state at window 0
        (E1 = <Psi0|V|Psi0> = 0 here, so the 2n+1 formula reduces to this)."""
        n = self.n
        mf = self._mpo_vfull()
        R = np.ones((1, 1, 1))
        for i in range(n - 1, 1, -1):
            R = right_update(R, mf.W[i], self.A[i], self.A[i], mf.dims[i])
        x = self.x_last
        y = apply_two_site(np.ones((1, 1, 1)), R, mf.W[0], mf.W[1], x, mf.dims[1])
        return float(np.vdot(x, y))

    def bonds(self):
        out = []
        for lab in self.lab:
            d = {}
            for q in map(tuple, lab):
                d[q] = d.get(q, 0) + 1
            out.append(sorted(d.items()))
        return out
