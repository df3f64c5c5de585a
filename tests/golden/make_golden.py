"""Write expected MPS-PT values for the 8-active / 16-virtual workload.

Calls only the oracle (and the seeded input generator):
  * exact uncontracted E2 by the factorised sum over states (upper-bound
    reference for any finite bond dimension);
  * the same-algorithm dense sweep at M1 = 128 with Psi0 compressed to M0 = 64,
    four sweeps: running E2 per local solve, E2 per sweep, E3, final bond
    sector tables.

Usage:  python tests/golden/make_golden.py [out.json]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact, fock, mps  # noqa: E402
from paper_1408_5092_amd import inputs  # noqa: E402

K_A, K_V, N_ELEC, RANK, M0, M1, SWEEPS, SEED = 8, 16, 8, 32, 64, 128, 4, 0


def main(out):
    t0 = time.time()
    ints = inputs.integrals(K_A, K_V, RANK, SEED)
    eri = fock.eri_from_cholesky(ints.B)
    e_fci, c, ab = exact.active_ground_state(ints.h, eri, K_A, N_ELEC, 0)
    psi0 = exact.psi0_mps(c, ab, K_A, M0)
    v0 = exact.mps_to_vector(psi0[1], K_A)
    act = v0[fock.site_index(ab, K_A)]
    e2_exact, _, e0_exact = exact.factorised_e2(ints.h, eri, K_A, ints.eps_virt, N_ELEC, 0, act, ab)
    print(f"[golden] fci E={e_fci:.12f} psi0(M0={M0}) E0={e0_exact:.12f} exact E2={e2_exact:.12f} "
          f"({time.time() - t0:.0f}s)", flush=True)
    g = inputs.psi1_guess(K_A, K_V, N_ELEC, 0, M1, SEED + 1000)
    sw = mps.Sweeper(ints.h, eri, K_A, ints.eps_virt, N_ELEC, 0, psi0, (g.bonds, g.sites), M1)
    print(f"[golden] mpo dims H0 {max(sw.mpo_h0.dims)} V {max(sw.mpo_v.dims)} ({time.time() - t0:.0f}s)",
          flush=True)

    def step(t):
        print(f"[golden] sweep {t['sweep']} {t['dir']} window {t['window']:2d} e2={t['e2']:.12f} "
              f"cg={t['cg_iters']} disc={t['discarded']:.2e} ({time.time() - t0:.0f}s)", flush=True)

    sw.run(n_sweeps=SWEEPS, on_step=step)
    e3 = sw.e3()
    print(f"[golden] e3={e3:.12f} ({time.time() - t0:.0f}s)", flush=True)
    res = dict(workload="c2_8a16v", k_a=K_A, k_v=K_V, n_elec=N_ELEC, rank=RANK, M0=M0, M1=M1,
               sweeps=SWEEPS, seed=SEED, psi1_seed=SEED + 1000,
               e_fci=e_fci, e0=sw.E0, e2_exact=e2_exact, e2_sweep=sw.e_sweep, e3=e3,
               trace=[dict(sweep=t["sweep"], dir=t["dir"], window=t["window"], e2=t["e2"],
                           cg_iters=t["cg_iters"], discarded=t["discarded"]) for t in sw.trace],
               bonds=[[[int(q[0]), int(q[1]), int(d)] for q, d in b] for b in sw.bonds()],
               psi0_bonds=[[[int(q[0]), int(q[1]), int(d)] for q, d in b] for b in psi0[0]])
    tmp = out + ".tmp"
    with open(tmp, "w") as f:
        json.dump(res, f, indent=1)
    os.replace(tmp, out)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(__file__), "c2_8a16v_seed0.json"))
