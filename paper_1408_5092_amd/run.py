"""One MPS-PT solve on synthetic integrals, in several sigma precisions.

    python -m paper_1408_5092_amd.run --k-a 16 --k-v 60 --rank 96 --m0 512 \\
        --m1 512 --guess-m 128 --sweeps 1 --precisions 0,1,2

Builds the seeded integrals, computes Psi0 with the library's DMRG at M0, loads
a seeded random Psi1 guess at bond dimension guess-m (the sweeps grow it to
M1), and runs the same sweeps once per precision (0 FP64, 1 FP32, 2 BF16x3
sigma with FP64 refinement).  Prints one JSON line per precision with E2
(and E3 with --e3), the difference from the first precision listed, CG
counts, host phase times and the grouped-GEMM rate (flops and algorithmic
bytes) from sampled HIP events.
Argument marshalling only: every step runs in the library's kernels.
"""
from __future__ import annotations

import argparse
import json
import time

from . import inputs, mpspt


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--k-a", type=int, default=8)
    ap.add_argument("--k-v", type=int, default=16)
    ap.add_argument("--n-elec", type=int, default=None, help="default: k_a")
    ap.add_argument("--rank", type=int, default=32)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--m0", type=int, default=64)
    ap.add_argument("--m0-sweeps", type=int, default=0, help="DMRG sweeps for Psi0 (0: until converged)")
    ap.add_argument("--m1", type=int, default=128)
    ap.add_argument("--guess-m", type=int, default=None, help="bond dimension of the Psi1 guess (default: M1)")
    ap.add_argument("--sweeps", type=int, default=4)
    ap.add_argument("--precisions", default="0,1,2")
    ap.add_argument("--e3", action="store_true")
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    ne = a.k_a if a.n_elec is None else a.n_elec
    ints = inputs.integrals(a.k_a, a.k_v, a.rank, a.seed)
    ctx = mpspt.Context(0)
    ctx.load_integrals(a.k_a, a.k_v, ints.h, ints.B)
    ctx.load_h0_partition(ints.eps_virt)
    g0 = inputs.psi0_guess(a.k_a, ne, 0, a.m0, a.seed + 2000)
    t = time.perf_counter()
    e_gs = ctx.ground_state(ne, 0, g0.bonds, g0.sites, a.m0, n_sweeps=a.m0_sweeps)
    t_gs = time.perf_counter() - t
    g1 = inputs.psi1_guess(a.k_a, a.k_v, ne, 0, a.guess_m or a.m1, a.seed + 1000)
    ctx.load_psi1_guess(g1.bonds, g1.sites)
    first = None
    for prec in (int(p) for p in a.precisions.split(",")):
        ctx.profile(True, every=8)
        t = time.perf_counter()
        r = ctx.sweep(a.m1, n_sweeps=a.sweeps, precision=prec, compute_e3=a.e3)
        wall = time.perf_counter() - t
        gemm = [ctx.kernel_stats(k) for k in (0, 6)]
        ctx.profile(False)
        sec = sum(s["seconds"] for s in gemm)
        out = {
            "k_a": a.k_a, "k_v": a.k_v, "n_elec": ne, "rank": a.rank, "seed": a.seed, "M0": a.m0, "M1": a.m1,
            "guess_m": a.guess_m or a.m1, "sweeps": a.sweeps, "psi0_energy": e_gs, "psi0_seconds": t_gs,
            "precision": ["fp64", "fp32", "bf16x3"][prec], "wall_s": wall, "e2": r["e2"],
            "e3": r["e3"] if a.e3 else None, "cg_iters": r["cg_iters"], "sigma_lo_calls": r["sigma_lo_calls"],
            "refinements": r["refinements"], "flags": r["flags"], "host_phase_seconds": r["t_phase"],
            "gemm_tflops_sampled": sum(s["flops"] for s in gemm) / sec / 1e12 if sec else None,
            # algorithmic bytes (operand blocks once per term, outputs once) over the recorded time,
            # and that as a fraction of the 8 TB/s HBM peak
            "gemm_gbs_sampled": sum(s["bytes"] for s in gemm) / sec / 1e9 if sec else None,
            "gemm_hbm_frac_sampled": sum(s["bytes"] for s in gemm) / sec / 8e12 if sec else None,
            "gemm_avg_launch_us": 1e6 * sec / max(1, sum(s["launches"] for s in gemm)),
        }
        if first is None:
            first = out
        else:
            out["e2_minus_" + first["precision"]] = r["e2"] - first["e2"]
            if a.e3:
                out["e3_minus_" + first["precision"]] = r["e3"] - first["e3"]
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
