"""Write expected per-pair values for the virtual-pair form of the
8-active / 16-virtual workload (same integrals and Psi0 as the monolithic
golden file: seed 0, Cholesky rank 32, Psi0 compressed to M0 = 64).

Calls only the oracle (and the seeded input generator):
  * every pair's exact share of E2 (the factorised sum over states, with each
    virtual pattern assigned to the pair that owns it), 136 pairs;
  * the same-algorithm dense sweep restricted to a few sampled pairs at a
    truncated bond dimension: running E2 per local solve and the final bond
    sector tables.

Usage:  python tests/golden/make_pairs_golden.py [out.json]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact, fock, mps, pairs  # noqa: E402
from paper_1408_5092_amd import inputs  # noqa: E402

K_A, K_V, N_ELEC, RANK, M0, SEED = 8, 16, 8, 32, 64, 0
SWEEP_PAIRS, SWEEP_M1, SWEEPS = ((0, 0), (2, 9)), 24, 2


def guess_seed(a, b):
    return SEED + 1000 + 100 * a + b


def main(out):
    t0 = time.time()
    ints = inputs.integrals(K_A, K_V, RANK, SEED)
    eri = fock.eri_from_cholesky(ints.B)
    _, c, ab = exact.active_ground_state(ints.h, eri, K_A, N_ELEC, 0)
    psi0 = exact.psi0_mps(c, ab, K_A, M0)
    v0 = exact.mps_to_vector(psi0[1], K_A)
    act = v0[fock.site_index(ab, K_A)]
    e2, contrib, e0 = exact.factorised_e2(ints.h, eri, K_A, ints.eps_virt, N_ELEC, 0, act, ab)
    share = pairs.pair_e2(contrib)
    print(f"[pairs golden] exact E2={e2:.12f} over {len(share)} pairs ({time.time() - t0:.0f}s)", flush=True)
    sweeps = []
    for (a, b) in SWEEP_PAIRS:
        occ = pairs.occupancy(a, b)
        hp, ep, ev = pairs.restrict(ints.h, eri, K_A, ints.eps_virt, a, b)
        g = inputs.random_mps(K_A + len(occ), K_A, N_ELEC, 0, (1, 2), SWEEP_M1, guess_seed(a, b), occ)
        sw = mps.Sweeper(hp, ep, K_A, ev, N_ELEC, 0, psi0, (g.bonds, g.sites), SWEEP_M1, virt_occ=occ)
        sw.run(n_sweeps=SWEEPS)
        print(f"[pairs golden] pair ({a},{b}) M1={SWEEP_M1} e2={sw.e_sweep[-1]:.12f} "
              f"exact share {share[(a, b)]:.12f} ({time.time() - t0:.0f}s)", flush=True)
        sweeps.append(dict(pair=[a, b], M1=SWEEP_M1, sweeps=SWEEPS, guess_seed=guess_seed(a, b),
                           e2_sweep=sw.e_sweep, trace=[t["e2"] for t in sw.trace],
                           bonds=[[[int(q[0]), int(q[1]), int(d)] for q, d in bb] for bb in sw.bonds()]))
    res = dict(workload="pairs_8a16v", k_a=K_A, k_v=K_V, n_elec=N_ELEC, rank=RANK, M0=M0, seed=SEED,
               e0=e0, e2_exact=e2,
               share=[[a, b, share[(a, b)]] for (a, b) in sorted(share)],
               sweeps=sweeps)
    tmp = out + ".tmp"
    with open(tmp, "w") as f:
        json.dump(res, f, indent=1)
    os.replace(tmp, out)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(__file__), "pairs_8a16v_seed0.json"))
