"""Autotuner for the grouped GEMM's launch shapes.

    python -m paper_1408_5092_amd.autotune [--write]

The grouped GEMM sums the same terms whichever way a work list is tiled; four
parameters choose how (see mpspt_set_tuning): the k-chain length at which a
list runs one workgroup per 16 x 16 tile with its k chunks spread over 4, 8
or 16 waves (split_waves) instead of one wave per tile (wide_chunks), and the segment length
above which an output block's k range is split and reduced in order
(kseg_min, kseg_div).  This script runs the 8-active / 16-virtual benchmark
solve (Psi0 by the library's DMRG at M0 = 64, M1 = 128, Jacobi PCG, four
sweeps) once per candidate after a warm-up, times every launch of the GEMM
and block-axpy kinds with HIP events (the split-k reductions are block
axpys), and picks the candidate with the least summed time; ties within 1%
keep the defaults.  With --write the choice and the measured table go to
tuning.json beside the library (or --out), which every new context then
applies when it sits beside the library.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import time

from . import inputs, mpspt

DEFAULT = {"wide_chunks": 8, "kseg_min": 512, "kseg_div": 8192, "split_waves": 4}
GRID = {"wide_chunks": (2, 4, 8, 1 << 20), "kseg_min": (128, 256, 512), "kseg_div": (8192, 16384),
        "split_waves": (4, 8, 16)}


def measure(ctx, M1, sweeps, tune):
    ctx.set_tuning(tune["wide_chunks"], tune["kseg_min"], tune["kseg_div"], tune["split_waves"])
    ctx.profile(True, every=1)
    t = time.perf_counter()
    r = ctx.sweep(M1, n_sweeps=sweeps, compute_e3=False)
    wall = time.perf_counter() - t
    st = [ctx.kernel_stats(k) for k in (0, 1)]  # FP64 GEMM, block axpy
    ctx.profile(False)
    return {"gemm_axpy_s": sum(s["seconds"] for s in st), "gemm_s": st[0]["seconds"], "axpy_s": st[1]["seconds"],
            "wall_s": wall, "e2": r["e2"]}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--write", action="store_true")
    ap.add_argument("--out", default=mpspt.TUNING_PATH, help="where --write puts the table")
    ap.add_argument("--sweeps", type=int, default=4)
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    k_a, k_v, n, rank, M0, M1 = 8, 16, 8, 32, 64, 128
    ints = inputs.integrals(k_a, k_v, rank, 0)
    ctx = mpspt.Context(0)
    ctx.load_integrals(k_a, k_v, ints.h, ints.B)
    ctx.load_h0_partition(ints.eps_virt)
    g0 = inputs.psi0_guess(k_a, n, 0, M0, 2000)
    ctx.ground_state(n, 0, g0.bonds, g0.sites, M0)
    g1 = inputs.psi1_guess(k_a, k_v, n, 0, M1, 1000)
    ctx.load_psi1_guess(g1.bonds, g1.sites)
    measure(ctx, M1, a.sweeps, DEFAULT)  # warm-up
    base = measure(ctx, M1, a.sweeps, DEFAULT)
    rows = []
    for vals in itertools.product(*GRID.values()):
        tune = dict(zip(GRID, vals))
        m = measure(ctx, M1, a.sweeps, tune)
        rows.append({**tune, **m})
        print(json.dumps(rows[-1]), flush=True)
    best = min(rows, key=lambda r: r["gemm_axpy_s"])
    choice = {k: best[k] for k in GRID} if best["gemm_axpy_s"] < 0.99 * base["gemm_axpy_s"] else dict(DEFAULT)
    out = {"workload": "8a+16v, M0=64 (library DMRG), M1=128, FP64, Jacobi PCG, "
                       f"{a.sweeps} sweeps; GEMM + block-axpy event time of every launch",
           "default": {**DEFAULT, **base}, "choice": choice, "candidates": rows}
    print(json.dumps({"default": out["default"], "choice": choice}), flush=True)
    if a.write:
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
