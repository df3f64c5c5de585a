"""Train the learned CG preconditioner on solves the method generates.

  python -m paper_1408_5092_amd.precond_train [--out FILE] [--steps N]
  python -m paper_1408_5092_amd.precond_train --eval-pairs [--params FILE]

Harvests (features, target) samples from Jacobi-preconditioned solves of
the 4-active/4-virtual workload (seeds 0-31) and of the 8-active/16-virtual
workload (seeds 0-3), trains the network with the library's own training
kernels (mini-batch Adam), then compares CG iterations and solve time of
Jacobi and learned preconditioning on held-out seeds (100-103 and 100-101).
Psi0 comes from the library's DMRG, the Psi1 guess from the seeded input
generator.  Everything runs through the C ABI.

--eval-pairs evaluates a trained network (--params, default the file the
training writes) on the virtual-pair form of the 12-active/40-virtual system
instead: integral seeds 100-107, a seeded sample of pairs per seed, Jacobi
against learned scaling on concurrent contexts, CG iterations and wall time.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

from . import inputs, mpspt

CONFIGS = {  # name: (k_a, k_v, n_elec, Cholesky rank, M0, M1)
    "4a4v": (4, 4, 4, 16, 16, 16),
    "8a16v": (8, 16, 8, 32, 64, 128),
}


def problem(name, seed):
    """A context with integrals, partition, Psi0 (DMRG) and the Psi1 guess loaded."""
    _torch_device()
    k_a, k_v, n, rank, M0, M1 = CONFIGS[name]
    ints = inputs.integrals(k_a, k_v, rank, seed)
    ctx = mpspt.Context(0)
    ctx.load_integrals(k_a, k_v, ints.h, ints.B)
    ctx.load_h0_partition(ints.eps_virt)
    g0 = inputs.psi0_guess(k_a, n, 0, M0, seed + 2000)
    ctx.ground_state(n, 0, g0.bonds, g0.sites, M0)
    g1 = inputs.psi1_guess(k_a, k_v, n, 0, M1, seed + 1000)
    ctx.load_psi1_guess(g1.bonds, g1.sites)
    return ctx, M1


def _torch_device():
    import torch  # device selection and memory as for every caller of the library
    if not torch.cuda.is_available():
        raise RuntimeError("needs a GPU")
    torch.cuda.set_device(0)


def harvest(cases, log=print):
    Xs, ts = [], []
    for name, seed in cases:
        ctx, M1 = problem(name, seed)
        ctx.harvest(True)
        ctx.sweep(M1, compute_e3=False)
        X, t = ctx.harvest_get()
        Xs.append(X)
        ts.append(t)
        log(f"[harvest] {name} seed {seed}: {len(t)} samples")
    return np.concatenate(Xs), np.concatenate(ts)


def train(X, t, steps=400, lr=3e-3, batch=4096, seed=0, log=print):
    _torch_device()
    ctx = mpspt.Context(0)
    ctx.precond_set(inputs.mlp_init(seed))
    rng = np.random.default_rng(seed)
    for s in range(steps):
        idx = rng.choice(len(t), min(batch, len(t)), replace=False)
        loss = ctx.mlp_train_step(X[idx], t[idx], lr)
        if s % 50 == 0 or s == steps - 1:
            log(f"[train] step {s} loss {loss:.5f}")
    full, _ = ctx.mlp_grad(X[:min(len(t), 65536)], t[:min(len(t), 65536)])
    return ctx.precond_get(), full


def evaluate(cases, params, log=print):
    out = []
    for name, seed in cases:
        row = {"case": f"{name}/{seed}"}
        for label, pc in (("jacobi", 0), ("learned", 1)):
            ctx, M1 = problem(name, seed)
            if pc:
                ctx.precond_set(params)
            t0 = time.perf_counter()
            r = ctx.sweep(M1, compute_e3=False, precond=pc)
            row[label] = {"cg_iters": r["cg_iters"], "seconds": time.perf_counter() - t0, "e2": r["e2"]}
        log(f"[eval] {row['case']}: CG iterations {row['jacobi']['cg_iters']} -> {row['learned']['cg_iters']}, "
            f"dE2 {row['learned']['e2'] - row['jacobi']['e2']:.1e}")
        out.append(row)
    return out


PAIR_SHAPE = (12, 40, 12, 48, 256, 256)  # k_a, k_v, n_elec, Cholesky rank, M0, M1 per pair


def evaluate_pairs(params, seeds=range(100, 108), n_pairs=8, contexts=8, log=print):
    from . import pairs as pp
    _torch_device()
    k_a, k_v, n, rank, M0, M1 = PAIR_SHAPE
    ctxs = pp.make_contexts(contexts)
    rows = []
    for seed in seeds:
        ints = inputs.integrals(k_a, k_v, rank, seed)
        c0 = mpspt.Context(0)
        hp, Bp, ep = pp.pair_integrals(ints.h, ints.B, k_a, ints.eps_virt, 0, 0)
        c0.load_integrals(k_a, 1, hp, Bp)
        c0.load_h0_partition(ep)
        g0 = inputs.psi0_guess(k_a, n, 0, M0, seed + 2000)
        c0.ground_state(n, 0, g0.bonds, g0.sites, M0)
        psi0 = ([c0.get_bond(1, i) for i in range(k_a + 1)], [c0.get_site(1, i) for i in range(k_a)])
        c0.close()
        allp = pp.pair_list(k_v)
        rng = np.random.default_rng(seed)
        sel = [allp[i] for i in sorted(rng.choice(len(allp), n_pairs, replace=False))]
        guesses = {}
        for (a, b) in sel:
            mk = pp.pair_masks(a, b)
            g = inputs.random_mps(k_a + len(mk), k_a, n, 0, (1, 2), M1, seed + 1000 + 100 * a + b, pp.mask_sets(mk))
            guesses[(a, b)] = (g.bonds, g.sites)
        row = {"case": f"pairs12a40v/{seed}", "pairs": [list(p) for p in sel]}
        for label, pc in (("jacobi", 0), ("learned", 1)):
            if pc:
                for c in ctxs:
                    c.precond_set(params)
            e2, res, dt = pp.solve_pairs_concurrent(ctxs, ints.h, ints.B, k_a, ints.eps_virt, n, 0, psi0,
                                                    lambda a, b: guesses[(a, b)], M1, pairs=sel, precond=pc)
            row[label] = {"cg_iters": sum(r["cg_iters"] for r in res.values()), "seconds": dt, "e2": e2}
        log(f"[eval] {row['case']}: CG iterations {row['jacobi']['cg_iters']} -> {row['learned']['cg_iters']}, "
            f"time {row['jacobi']['seconds']:.2f}s -> {row['learned']['seconds']:.2f}s, "
            f"dE2 {row['learned']['e2'] - row['jacobi']['e2']:.1e}")
        rows.append(row)
    for c in ctxs:
        c.close()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "precond_params.npy"))
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--small-seeds", type=int, default=32)
    ap.add_argument("--large-seeds", type=int, default=4)
    ap.add_argument("--eval-pairs", action="store_true", help="evaluate a trained network on the pair form")
    ap.add_argument("--params", default=None, help="trained network (default: --out)")
    ap.add_argument("--pairs-per-seed", type=int, default=8)
    args = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)  # noqa: E731
    if args.eval_pairs:
        params = np.load(args.params or args.out)
        rows = evaluate_pairs(params, n_pairs=args.pairs_per_seed, log=log)
        tot = {k: sum(r[k]["cg_iters"] for r in rows) for k in ("jacobi", "learned")}
        print(json.dumps({"eval_pairs": rows, "cg_iters_total": tot}))
        return 0
    cases = [("4a4v", s) for s in range(args.small_seeds)] + [("8a16v", s) for s in range(args.large_seeds)]
    X, t = harvest(cases, log)
    log(f"[harvest] {len(t)} samples; target quantiles {np.quantile(t, [0.05, 0.5, 0.95])}")
    params, loss = train(X, t, args.steps, log=log)
    np.save(args.out, params)
    rows = evaluate([("4a4v", s) for s in (100, 101, 102, 103)] + [("8a16v", s) for s in (100, 101)], params, log)
    print(json.dumps({"samples": int(len(t)), "final_loss": loss, "eval": rows}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
