"""Bond-dimension scans on the GPU (paper_1408_5092_amd.mscan) against the oracle.

The paper's results section gauges convergence in M1 by the linear relation
between the error of E2 and the discarded weight once the energy has
relaxed, and by the M1 needed for an E2 within 1 mEh of the exact,
uncontracted value.  Checked here:

* 4 active + 4 virtual orbitals: at M1 = 64 (no cut of the 8-site chain has
  a larger Schmidt rank) the scan's E2 is the brute-force E2 to 1e-9 Eh and
  nothing is discarded, so the extrapolation returns it; M1 = 8 and 16 give
  upper bounds.
* 8 active + 16 virtual orbitals (Psi0 compressed to M0 = 64; the stored
  oracle exact E2): E2 at M1 = 64, 128, 192 and 256 are upper bounds of the
  exact E2 (1e-10 Eh) and do not increase with M1 (1e-9 Eh); the pair form
  at per-pair M1 = 256 reproduces the exact E2 (1e-9 Eh); the line through
  the two largest M1 lands closer to the exact E2 than the best scan point;
  1 mEh needs M1 = 128 on this workload.
"""
import json
import os

import pytest

from oracle import exact, fock
from paper_1408_5092_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_8a16v_seed0.json")


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1408_5092_amd import mpspt
    mpspt.load_library()  # fails loudly when the HIP library is missing
    return mpspt


@pytest.fixture(scope="module")
def ms():
    from paper_1408_5092_amd import mscan
    return mscan


def _context(mp, ka, kv, ne, ints, psi0):
    ctx = mp.Context(0)
    ctx.load_integrals(ka, kv, ints.h, ints.B)
    ctx.load_h0_partition(ints.eps_virt)
    ctx.load_psi0(ne, 0, *psi0)
    return ctx


def test_small_system_full_rank(mp, ms):
    print("case: mscan 4a+4v M1 = 8, 16, 64", flush=True)
    ka, kv, ne = 4, 4, 4
    ints = inputs.integrals(ka, kv, 16, 0)
    eri = fock.eri_from_cholesky(ints.B)
    _, c, ab = exact.active_ground_state(ints.h, eri, ka, ne, 0)
    full = exact.brute_force(ints.h, eri, ka, ints.eps_virt, ne, 0, c, ab)
    ctx = _context(mp, ka, kv, ne, ints, exact.psi0_mps(c, ab, ka))
    g = inputs.psi1_guess(ka, kv, ne, 0, 64, 1000)
    pts = ms.scan(ctx, [64, 8, 16], (g.bonds, g.sites))
    assert [p["M1"] for p in pts] == [8, 16, 64]
    for p in pts:
        print(json.dumps(p), "error", p["e2"] - full.E2, flush=True)
        assert p["e2"] >= full.E2 - 1e-10 and p["flags"] == 0
    assert pts[-1]["e2"] == pytest.approx(full.E2, abs=1e-9)
    assert pts[-1]["discarded"] < 1e-12  # rounding only
    e, s, used = ms.extrapolate(pts)
    assert (e, s, used) == (pts[-1]["e2"], 0.0, [pts[-1]])


def test_extrapolation_and_required_m1(mp, ms):
    with open(GOLDEN) as f:
        gold = json.load(f)
    ka, kv, ne = gold["k_a"], gold["k_v"], gold["n_elec"]
    print("case: mscan 8a+16v M1 = 64, 128, 192, 256 and the pair-form exact E2", flush=True)
    ints = inputs.integrals(ka, kv, gold["rank"], gold["seed"])
    eri = fock.eri_from_cholesky(ints.B)
    _, c, ab = exact.active_ground_state(ints.h, eri, ka, ne, 0)
    psi0 = exact.psi0_mps(c, ab, ka, gold["M0"])
    ctx = _context(mp, ka, kv, ne, ints, psi0)
    g = inputs.psi1_guess(ka, kv, ne, 0, 256, gold["psi1_seed"])
    pts = ms.scan(ctx, [64, 128, 192, 256], (g.bonds, g.sites))
    exact_e2 = gold["e2_exact"]
    for p in pts:
        print(json.dumps(p), "error", p["e2"] - exact_e2, flush=True)
        assert p["e2"] >= exact_e2 - 1e-10 and p["flags"] == 0
        assert p["discarded"] > 0.0
    for a, b in zip(pts, pts[1:]):
        assert b["e2"] <= a["e2"] + 1e-9
    e_pairs, not_conv = ms.exact_e2_pairs(ints.h, ints.B, ka, ints.eps_virt, ne, psi0)
    print(f"pair-form E2 {e_pairs:.12f}, oracle exact {exact_e2:.12f}", flush=True)
    assert not_conv == 0
    assert e_pairs == pytest.approx(exact_e2, abs=1e-9)
    e, s, used = ms.extrapolate(pts, 2)
    print(f"extrapolated {e:.9f} (slope {s:.3f}, M1 {[p['M1'] for p in used]}): error {e - exact_e2:.3e}, "
          f"best scan point {pts[-1]['e2'] - exact_e2:.3e}", flush=True)
    assert [p["M1"] for p in used] == [256, 192] and s > 0.0
    assert abs(e - exact_e2) < abs(pts[-1]["e2"] - exact_e2)
    assert ms.m_required(pts, exact_e2, 1e-3) == 128
