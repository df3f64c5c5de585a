"""Bond-dimension scans of the first-order state.

The paper's results section judges convergence in M1 the way DMRG does: once
the energy has relaxed from its first, rapid changes, the error of E2 falls
linearly with the weight discarded in the renormalisation steps, so a line
through (discarded weight, E2) points extrapolates to zero weight; and it
reports the bond dimension needed for an E2 within 1 mEh of the exact,
uncontracted value as the virtual space grows.  This module does both on the
library's sweeps:

* ``scan``: one converged sweep sequence per M1 (each from the same guess),
  recording E2 and the largest discarded weight of the last sweep;
* ``fit_line`` / ``extrapolate``: the least-squares line E2 = e0 + s w through
  the points of the largest M1, and its value at w = 0;
* ``m_required``: the smallest M1 of a scan whose E2 is within a tolerance of
  a reference;
* ``main``: the M1-against-k_v study on the seeded model Hamiltonians, with
  the exact uncontracted E2 of each Psi0 from the virtual-pair form at a
  per-pair bond dimension that represents every pair exactly.

Everything but the line fit (a 2 x 2 least-squares problem on the host) is
argument marshalling around the library's entry points.
"""
from __future__ import annotations

import json
import time

import numpy as np

from . import inputs, mpspt, pairs


def scan(ctx: "mpspt.Context", M1s, guess, **sweep_kw):
    """Sweeps to convergence at each M1 in ``M1s`` (ascending), each from
    ``guess`` = (bonds, sites) of the Psi1 start.  The context must hold the
    integrals, the H0 partition and Psi0.  Returns a list of dicts with M1,
    e2, discarded (largest discarded weight of the last sweep), sweeps, cg_iters
    and flags."""
    sweep_kw.setdefault("n_sweeps", 0)
    sweep_kw.setdefault("max_sweeps", 16)
    sweep_kw.setdefault("e_tol", 1e-9)
    sweep_kw.setdefault("compute_e3", False)
    out = []
    for M1 in sorted(int(m) for m in M1s):
        ctx.load_psi1_guess(*guess)
        r = ctx.sweep(M1, **sweep_kw)
        out.append({"M1": M1, "e2": r["e2"], "discarded": r["max_discarded"], "sweeps": r["n_sweeps_done"],
                    "cg_iters": r["cg_iters"], "flags": r["flags"]})
    return out


def fit_line(w, e):
    """Least-squares line e = e0 + s w through the points (w_i, e_i); returns
    (e0, s).  One point gives a horizontal line through it."""
    w = np.asarray(w, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    if w.size == 0:
        raise ValueError("no points")
    if w.size == 1 or np.all(w == w[0]):
        return float(e.mean()), 0.0
    wm, em = w.mean(), e.mean()
    s = float(((w - wm) * (e - em)).sum() / ((w - wm) ** 2).sum())
    return float(em - s * wm), s


def extrapolate(points, n_fit: int = 2, zero_weight: float = 1e-12):
    """Zero-discarded-weight estimate of E2 from a scan: the line through the
    points of the n_fit largest M1 (past the initial relaxation, where the
    discarded weight of the last sweep is not yet a smooth function of M1).
    When the largest M1 discarded nothing (a weight at rounding level,
    below ``zero_weight``) its E2 is already the converged value and is
    returned as is.  Returns (e2_extrapolated, slope, points used)."""
    if not points:
        raise ValueError("no points")
    pts = sorted(points, key=lambda p: -p["M1"])
    if pts[0]["discarded"] <= zero_weight:
        return pts[0]["e2"], 0.0, [pts[0]]
    use = pts[:max(1, n_fit)]
    e0, s = fit_line([p["discarded"] for p in use], [p["e2"] for p in use])
    return e0, s, use


def m_required(points, e_ref: float, tol: float):
    """Smallest M1 of the scan whose E2 is within tol of e_ref, or None."""
    for p in sorted(points, key=lambda p: p["M1"]):
        if abs(p["e2"] - e_ref) <= tol:
            return p["M1"]
    return None


def exact_e2_pairs(h, B, k_a, eps_virt, n_elec, psi0, M1_pair=256, contexts=8, seed=0, precision=0):
    """Uncontracted E2 of Psi0: the virtual-pair form at a per-pair bond
    dimension no bond of an active-space-plus-two-site chain exceeds (for
    up to 8 active orbitals 256 suffices), summed over the pairs."""
    kv = len(eps_virt)
    gs = {}
    for (a, b) in pairs.pair_list(kv):
        mk = pairs.pair_masks(a, b)
        g = inputs.random_mps(k_a + len(mk), k_a, n_elec, 0, (1, 2), M1_pair, seed + 1000 + 100 * a + b,
                              pairs.mask_sets(mk))
        gs[(a, b)] = (g.bonds, g.sites)
    ctxs = pairs.make_contexts(contexts)
    e2, res, _ = pairs.solve_pairs_concurrent(ctxs, h, B, k_a, eps_virt, n_elec, 0, psi0, lambda a, b: gs[(a, b)],
                                              M1_pair, n_sweeps=0, max_sweeps=16, e_tol=1e-10, precision=precision)
    return e2, sum(1 for r in res.values() if r["flags"])


def main(argv=None):
    """M1 against k_v: ``python -m paper_1408_5092_amd.mscan``.

    For each k_v: seeded integrals, Psi0 by the library's DMRG, the exact
    uncontracted E2 from the pair form, then a monolithic M1 scan; prints one
    JSON line per k_v with the scan, the zero-weight extrapolation and the M1
    needed for each tolerance.
    """
    import argparse

    import torch
    ap = argparse.ArgumentParser(description=main.__doc__.splitlines()[0])
    ap.add_argument("--k-a", type=int, default=8)
    ap.add_argument("--k-v", default="4,8,12,16")
    ap.add_argument("--n-elec", type=int, default=None, help="default: k_a")
    ap.add_argument("--rank", type=int, default=32)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--m0", type=int, default=64)
    ap.add_argument("--m1", default="16,32,48,64,96,128,192,256")
    ap.add_argument("--tol", default="1e-3,1e-4")
    ap.add_argument("--n-fit", type=int, default=2)
    a = ap.parse_args(argv)
    if a.k_a > 8:
        ap.error("the pair-form reference is exact only up to 8 active orbitals at per-pair M1 = 256")
    ne = a.k_a if a.n_elec is None else a.n_elec
    torch.cuda.set_device(0)
    tols = [float(t) for t in a.tol.split(",")]
    M1s = [int(m) for m in a.m1.split(",")]
    for kv in (int(k) for k in a.k_v.split(",")):
        t0 = time.perf_counter()
        ints = inputs.integrals(a.k_a, kv, a.rank, a.seed)
        ctx = mpspt.Context(0)
        ctx.load_integrals(a.k_a, kv, ints.h, ints.B)
        ctx.load_h0_partition(ints.eps_virt)
        g0 = inputs.psi0_guess(a.k_a, ne, 0, a.m0, a.seed + 2000)
        e_gs = ctx.ground_state(ne, 0, g0.bonds, g0.sites, a.m0)
        psi0 = ([ctx.get_bond(1, i) for i in range(a.k_a + 1)], [ctx.get_site(1, i) for i in range(a.k_a)])
        e_exact, nc_pairs = exact_e2_pairs(ints.h, ints.B, a.k_a, ints.eps_virt, ne, psi0, seed=a.seed)
        g1 = inputs.psi1_guess(a.k_a, kv, ne, 0, max(M1s), a.seed + 1000)
        pts = scan(ctx, M1s, (g1.bonds, g1.sites))
        e_x, slope, used = extrapolate(pts, a.n_fit)
        print(json.dumps({
            "k_a": a.k_a, "k_v": kv, "n_elec": ne, "rank": a.rank, "seed": a.seed, "M0": a.m0, "psi0_energy": e_gs,
            "e2_exact": e_exact, "pairs_not_converged": nc_pairs, "scan": pts,
            "e2_extrapolated": e_x, "slope": slope, "fit_M1": [p["M1"] for p in used],
            "extrapolation_error": e_x - e_exact, "best_scan_error": pts[-1]["e2"] - e_exact,
            "m1_required": {str(t): m_required(pts, e_exact, t) for t in tols},
            "seconds": time.perf_counter() - t0,
        }), flush=True)


if __name__ == "__main__":
    main()
