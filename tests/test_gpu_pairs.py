"""Parity of the virtual-pair form of the HIP path with the oracle.

* 4 active + 4 virtual orbitals: every one of the 10 pairs at a bond
  dimension above the pair's Schmidt ranks reaches its exact share of E2
  (oracle pattern-to-pair assignment of the factorised sum over states), and
  the shares add up to the dense-solve E2; at truncated bond dimensions the
  running E2 and the bond sector tables match the oracle's restricted
  same-algorithm sweep.
* 8 active + 16 virtual orbitals (Psi0 compressed to M0 = 64): sampled pairs
  at M1 = 256 (exact for a pair: no bond of 8 active + 2 virtual sites needs
  more) against the stored exact shares, and two pairs at M1 = 24 against
  the stored same-algorithm traces and bond tables (written by
  tests/golden/make_pairs_golden.py from the oracle).
* Restriction edge cases: masks of the wrong length or outside [1, 7] are
  refused, masks that bond labels cannot express are refused once Psi0 is
  known, and clearing the masks restores the unrestricted sweep.
Tolerances: 1e-9 Eh on the small system, 1e-8 Eh on the large one (both
sides FP64; CG to 1e-10 relative residual).
"""
import json
import os

import numpy as np
import pytest

from oracle import exact, fock, mps, pairs
from paper_1408_5092_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "pairs_8a16v_seed0.json")


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1408_5092_amd import mpspt
    mpspt.load_library()  # fails loudly when the HIP library is missing
    return mpspt


@pytest.fixture(scope="module")
def pp():
    from paper_1408_5092_amd import pairs as product_pairs
    return product_pairs


@pytest.fixture(scope="module")
def small():
    ka, kv, ne = 4, 4, 4
    ints = inputs.integrals(ka, kv, 16, 0)
    eri = fock.eri_from_cholesky(ints.B)
    _, c, ab = exact.active_ground_state(ints.h, eri, ka, ne, 0)
    full = exact.brute_force(ints.h, eri, ka, ints.eps_virt, ne, 0, c, ab)
    _, contrib, _ = exact.factorised_e2(ints.h, eri, ka, ints.eps_virt, ne, 0, c, ab)
    return ka, kv, ne, ints, eri, exact.psi0_mps(c, ab, ka), full, pairs.pair_e2(contrib)


def guess(ka, ne, a, b, M, seed):
    occ = pairs.occupancy(a, b)
    g = inputs.random_mps(ka + len(occ), ka, ne, 0, (1, 2), M, seed, occ)
    return g.bonds, g.sites


def test_small_all_pairs_exact(mp, pp, small):
    ka, kv, ne, ints, eri, psi0, full, share = small
    print("case: 4a+4v all pairs M1=64", flush=True)
    ctx = mp.Context(0)
    total, res, _ = pp.solve_pairs(ctx, ints.h, ints.B, ka, ints.eps_virt, ne, 0, psi0,
                                   lambda a, b: guess(ka, ne, a, b, 64, 7 + 10 * a + b), 64)
    assert sorted(res) == pairs.pairs(kv)
    for p, r in res.items():
        assert r["e0"] == pytest.approx(full.E0, abs=1e-12)
        assert r["e2"] == pytest.approx(share[p], abs=1e-9), p
    assert total == pytest.approx(full.E2, abs=1e-9)


@pytest.mark.parametrize("pair,M1", [((0, 0), 3), ((1, 3), 3), ((2, 2), 4), ((0, 1), 2)])
def test_small_same_algorithm(mp, pp, small, pair, M1):
    ka, kv, ne, ints, eri, psi0, full, share = small
    a, b = pair
    print(f"case: 4a+4v pair {pair} M1={M1}", flush=True)
    g = guess(ka, ne, a, b, M1, 7 + 10 * a + b)
    ctx = mp.Context(0)
    r = pp.solve_pair(ctx, ints.h, ints.B, ka, ints.eps_virt, ne, 0, psi0, a, b, g, M1)
    hp, ep, ev = pairs.restrict(ints.h, eri, ka, ints.eps_virt, a, b)
    sw = mps.Sweeper(hp, ep, ka, ev, ne, 0, psi0, g, M1, virt_occ=pairs.occupancy(a, b))
    sw.run()
    tr = ctx.get_trace()
    np.testing.assert_allclose(tr["e2"], [t["e2"] for t in sw.trace], rtol=0, atol=1e-9)
    assert r["e2"] >= share[pair] - 1e-12
    for i, ob in enumerate(sw.bonds()):
        assert ctx.get_bond(0, i) == [(tuple(q), d) for q, d in ob], f"bond {i}"


@pytest.fixture(scope="module")
def large():
    with open(GOLDEN) as f:
        gold = json.load(f)
    ints = inputs.integrals(gold["k_a"], gold["k_v"], gold["rank"], gold["seed"])
    eri = fock.eri_from_cholesky(ints.B)
    _, c, ab = exact.active_ground_state(ints.h, eri, gold["k_a"], gold["n_elec"], 0)
    psi0 = exact.psi0_mps(c, ab, gold["k_a"], gold["M0"])
    return gold, ints, psi0


@pytest.mark.parametrize("pair", [(0, 0), (0, 1), (3, 11), (7, 7), (14, 15), (15, 15)])
def test_large_sampled_pairs_exact(mp, pp, large, pair):
    gold, ints, psi0 = large
    ka, ne = gold["k_a"], gold["n_elec"]
    a, b = pair
    share = {(x, y): e for x, y, e in gold["share"]}
    print(f"case: 8a+16v pair {pair} M1=256", flush=True)
    ctx = mp.Context(0)
    r = pp.solve_pair(ctx, ints.h, ints.B, ka, ints.eps_virt, ne, 0, psi0, a, b,
                      guess(ka, ne, a, b, 256, 1000 + 100 * a + b), 256)
    assert r["e0"] == pytest.approx(gold["e0"], abs=1e-10)
    assert r["e2"] == pytest.approx(share[pair], abs=1e-8)


def test_large_same_algorithm(mp, pp, large):
    gold, ints, psi0 = large
    ka, ne = gold["k_a"], gold["n_elec"]
    for s in gold["sweeps"]:
        a, b = s["pair"]
        print(f"case: 8a+16v pair ({a},{b}) M1={s['M1']} {s['sweeps']} sweeps", flush=True)
        ctx = mp.Context(0)
        pp.solve_pair(ctx, ints.h, ints.B, ka, ints.eps_virt, ne, 0, psi0, a, b,
                      guess(ka, ne, a, b, s["M1"], s["guess_seed"]), s["M1"], n_sweeps=s["sweeps"])
        tr = ctx.get_trace()
        np.testing.assert_allclose(tr["e2"], s["trace"], rtol=0, atol=1e-8)
        for i, ob in enumerate(s["bonds"]):
            assert ctx.get_bond(0, i) == [((q0, q1), d) for q0, q1, d in ob], f"bond {i}"


def test_restriction_edge_cases(mp, pp, small):
    ka, kv, ne, ints, eri, psi0, full, share = small
    print("case: 4a+4v restriction errors", flush=True)
    ctx = mp.Context(0)
    ctx.load_integrals(ka, kv, ints.h, ints.B)
    ctx.load_h0_partition(ints.eps_virt)
    with pytest.raises(mp.MPSPTError):
        ctx.restrict_virtual([7, 7, 8, 7])
    with pytest.raises(mp.MPSPTError):
        ctx.restrict_virtual([7, 0, 7, 7])
    ctx.load_psi0(ne, 0, *psi0)
    # one or no electron on two neighbouring sites: labels allow a doubly
    # occupied first site followed by an empty second one
    with pytest.raises(mp.MPSPTError):
        ctx.restrict_virtual([3, 3, 1, 1])
    # a refused mask leaves the previous restriction (none) in force
    g = inputs.psi1_guess(ka, kv, ne, 0, 64, 1000)
    ctx.load_psi1_guess(g.bonds, g.sites)
    # a restriction drops the loaded guess; clearing it brings back the plain sweep
    ctx.restrict_virtual(pp.pair_masks(0, 1) + [1, 1])
    with pytest.raises(mp.MPSPTError):
        ctx.sweep(8)
    with pytest.raises(mp.MPSPTError):
        ctx.load_psi1_guess(g.bonds, g.sites)   # sectors outside the restriction
    ctx.restrict_virtual(None)
    ctx.load_psi1_guess(g.bonds, g.sites)
    r = ctx.sweep(64)
    assert r["e2"] == pytest.approx(full.E2, abs=1e-9)


def test_concurrent_contexts_match_sequential(mp, pp, large):
    """Pairs spread over four contexts (own streams, own host threads) give
    bit-identical energies to the same pairs run one after another."""
    gold, ints, psi0 = large
    ka, ne = gold["k_a"], gold["n_elec"]
    share = {(x, y): e for x, y, e in gold["share"]}
    sample = [(0, 0), (0, 5), (1, 1), (2, 9), (4, 12), (6, 6), (7, 15), (10, 13), (15, 15)]
    print(f"case: 8a+16v {len(sample)} pairs M1=48, sequential then 4 contexts", flush=True)

    def guess_of(a, b):
        return guess(ka, ne, a, b, 48, 1000 + 100 * a + b)

    ctx = mp.Context(0)
    e_seq, r_seq, _ = pp.solve_pairs(ctx, ints.h, ints.B, ka, ints.eps_virt, ne, 0, psi0, guess_of, 48,
                                     pairs=sample, n_sweeps=2)
    ctxs = pp.make_contexts(4)
    e_con, r_con, _ = pp.solve_pairs_concurrent(ctxs, ints.h, ints.B, ka, ints.eps_virt, ne, 0, psi0, guess_of, 48,
                                                pairs=sample, n_sweeps=2)
    assert sorted(r_con) == sorted(sample)
    for p in sample:
        assert r_con[p]["e2"] == r_seq[p]["e2"], p
        assert r_con[p]["e2_sweep"] == r_seq[p]["e2_sweep"], p
        assert r_seq[p]["e2"] >= share[p] - 1e-10, p
    assert e_con == e_seq


def test_pairs_at_the_12a40v_shape(mp, pp):
    """The 12-active / 40-virtual pair problems (Psi0 by the library's DMRG at
    M0 = 256), too large for the oracle's solves: properties that hold at any
    size.  For three pairs (one diagonal): E2 < 0, the Hylleraas value does not
    rise when M1 grows from 64 to 256 (both start from guesses at their own
    bond dimension and are swept to convergence), and concurrent contexts give
    the sequential energies bit for bit."""
    k_a, k_v, ne, rank, M0 = 12, 40, 12, 48, 256
    print("case: 12a+40v pairs (0,0) (3,17) (21,39) at M1 = 64 and 256", flush=True)
    ints = inputs.integrals(k_a, k_v, rank, 0)
    ctx = mp.Context(0)
    hp, Bp, ep = pp.pair_integrals(ints.h, ints.B, k_a, ints.eps_virt, 0, 0)
    ctx.load_integrals(k_a, 1, hp, Bp)
    ctx.load_h0_partition(ep)
    g0 = inputs.psi0_guess(k_a, ne, 0, M0, 2000)
    ctx.ground_state(ne, 0, g0.bonds, g0.sites, M0)
    psi0 = ([ctx.get_bond(1, i) for i in range(k_a + 1)], [ctx.get_site(1, i) for i in range(k_a)])
    sample = [(0, 0), (3, 17), (21, 39)]
    e2 = {}
    for M1 in (64, 256):
        def guess_of(a, b, M1=M1):
            return guess(k_a, ne, a, b, M1, 1000 + 100 * a + b)
        _, res, _ = pp.solve_pairs(ctx, ints.h, ints.B, k_a, ints.eps_virt, ne, 0, psi0, guess_of, M1,
                                   pairs=sample)
        for p, r in res.items():
            assert r["flags"] == 0, p
            e2[(p, M1)] = r["e2"]
        if M1 == 256:
            ctxs = pp.make_contexts(3)
            _, rc, _ = pp.solve_pairs_concurrent(ctxs, ints.h, ints.B, k_a, ints.eps_virt, ne, 0, psi0, guess_of,
                                                 M1, pairs=sample)
            for p in sample:
                assert rc[p]["e2"] == res[p]["e2"], p
    for p in sample:
        assert e2[(p, 256)] < 0.0
        assert e2[(p, 256)] <= e2[(p, 64)] + 1e-10, p
