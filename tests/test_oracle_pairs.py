"""Pins of the oracle's virtual-pair decomposition (CPU only).

* A dense determinant-space solve on the integrals restricted to the active
  orbitals plus virtuals a, b sees exactly the patterns of pairs (a, a),
  (b, b) and (a, b): its E2 must equal the sum of those three pairs' shares of
  the factorised sum over states of the full problem.  This checks the
  orbital restriction (h, eri and eps indices) and the pattern-to-pair map
  against an independent computation.
* The pairs' shares add up to the full dense-solve E2 (the paper's additivity).
* The same-algorithm sweep restricted to one pair's occupancy reaches that
  pair's exact share at full bond dimension and stays above it when truncated.
"""
import numpy as np
import pytest

from oracle import exact, fock, mps, pairs
from paper_1408_5092_amd import inputs


@pytest.fixture(scope="module")
def small():
    ka, kv, ne = 4, 4, 4
    ints = inputs.integrals(ka, kv, 16, 0)
    eri = fock.eri_from_cholesky(ints.B)
    _, c, ab = exact.active_ground_state(ints.h, eri, ka, ne, 0)
    full = exact.brute_force(ints.h, eri, ka, ints.eps_virt, ne, 0, c, ab)
    _, contrib, _ = exact.factorised_e2(ints.h, eri, ka, ints.eps_virt, ne, 0, c, ab)
    return ka, kv, ne, ints, eri, c, ab, full, pairs.pair_e2(contrib)


def test_every_pattern_has_one_owner(small):
    ka, kv, ne, ints, eri, c, ab, full, pe = small
    assert sorted(pe) == pairs.pairs(kv)
    assert len(pairs.pairs(40)) == 820
    assert sum(pe.values()) == pytest.approx(full.E2, abs=1e-12)


def test_restricted_dense_solve_equals_pair_shares(small):
    ka, kv, ne, ints, eri, c, ab, full, pe = small
    for a in range(kv):
        for b in range(a, kv):
            hp, ep, ev = pairs.restrict(ints.h, eri, ka, ints.eps_virt, a, b)
            r = exact.brute_force(hp, ep, ka, ev, ne, 0, c, ab)
            want = pe[(a, a)] if a == b else pe[(a, a)] + pe[(b, b)] + pe[(a, b)]
            assert r.E2 == pytest.approx(want, abs=1e-12), (a, b)
            assert r.E0 == pytest.approx(full.E0, abs=1e-12)


def test_pair_sweeps_reach_exact_shares_and_add_up(small):
    ka, kv, ne, ints, eri, c, ab, full, pe = small
    psi0 = exact.psi0_mps(c, ab, ka)
    total = 0.0
    for (a, b) in pairs.pairs(kv):
        occ = pairs.occupancy(a, b)
        hp, ep, ev = pairs.restrict(ints.h, eri, ka, ints.eps_virt, a, b)
        g = inputs.random_mps(ka + len(occ), ka, ne, 0, (1, 2), 64, 7 + 10 * a + b, occ)
        sw = mps.Sweeper(hp, ep, ka, ev, ne, 0, psi0, (g.bonds, g.sites), 64, virt_occ=occ)
        e = sw.run()[-1]
        assert e == pytest.approx(pe[(a, b)], abs=1e-9), (a, b)
        total += e
    assert total == pytest.approx(full.E2, abs=1e-8)


def test_truncated_pair_sweep_is_an_upper_bound(small):
    ka, kv, ne, ints, eri, c, ab, full, pe = small
    psi0 = exact.psi0_mps(c, ab, ka)
    for (a, b) in ((0, 0), (1, 3)):
        occ = pairs.occupancy(a, b)
        hp, ep, ev = pairs.restrict(ints.h, eri, ka, ints.eps_virt, a, b)
        g = inputs.random_mps(ka + len(occ), ka, ne, 0, (1, 2), 3, 11, occ)
        sw = mps.Sweeper(hp, ep, ka, ev, ne, 0, psi0, (g.bonds, g.sites), 3, virt_occ=occ)
        e = sw.run()[-1]
        assert e >= pe[(a, b)] - 1e-12
        # restricted configurations only: every kept bond label is admissible
        adm = mps.admissible(ka + len(occ), ka, ne, 0, (1, 2), occ)
        for bnd, labels in zip(sw.bonds(), adm):
            assert all(q in labels for q, _ in bnd)


def test_unrestricted_masks_change_nothing(small):
    """All counts allowed on every virtual site is the plain first-order space."""
    ka, kv, ne, ints, eri, c, ab, full, pe = small
    a0 = mps.admissible(ka + kv, ka, ne, 0, (1, 2))
    a1 = mps.admissible(ka + kv, ka, ne, 0, (1, 2), [{0, 1, 2}] * kv)
    assert a0 == a1
