"""Reduced-precision sigma (FP32 MFMA, BF16x3) with FP64 refinement.

The CG iterations apply H0_eff - E0 in FP32 or as three BF16 products of
split FP32 operands; every restart recomputes the residual in FP64, and the
solve ends on the same FP64 residual test as the plain FP64 path.  So:

* 4 active + 4 virtual orbitals, M1 = 16 and 8: running E2, bond tables and
  E3 match the oracle's FP64 same-algorithm sweep to 1e-9 Eh, with the
  reduced-precision kernels doing the CG applications;
* 8 active + 16 virtual orbitals, M1 = 128, four sweeps (the benchmarked
  workload): E2 per sweep and E3 match the stored oracle values to 1e-6 Eh,
  and the FP64 GPU run to 1e-8 Eh (the difference is printed per energy);
* every launch shape of the reduced-precision GEMM (4 or 16 waves per tile,
  heavy split-k) matches the oracle on the small system;
* bad precision arguments are refused.
"""
import json
import os

import numpy as np
import pytest

from oracle import exact, fock, mps
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
def c1():
    ints = inputs.integrals(4, 4, 16, 0)
    eri = fock.eri_from_cholesky(ints.B)
    _, c, ab = exact.active_ground_state(ints.h, eri, 4, 4, 0)
    return ints, eri, exact.psi0_mps(c, ab, 4)


@pytest.mark.parametrize("precision", [1, 2])
@pytest.mark.parametrize("M1", [16, 8])
def test_small_matches_fp64_oracle(mp, c1, precision, M1):
    ints, eri, psi0 = c1
    print(f"case: 4a+4v M1={M1} precision {precision}", flush=True)
    g = inputs.psi1_guess(4, 4, 4, 0, M1, 1000)
    ctx = mp.Context(0)
    ctx.load_integrals(4, 4, ints.h, ints.B)
    ctx.load_h0_partition(ints.eps_virt)
    ctx.load_psi0(4, 0, *psi0)
    ctx.load_psi1_guess(g.bonds, g.sites)
    ctx.profile(True)
    res = ctx.sweep(M1, precision=precision)
    lo = ctx.kernel_stats(6)
    ctx.profile(False)
    sw = mps.Sweeper(ints.h, eri, 4, ints.eps_virt, 4, 0, psi0, (g.bonds, g.sites), M1)
    sw.run()
    tr = ctx.get_trace()
    np.testing.assert_allclose(tr["e2"], [t["e2"] for t in sw.trace], rtol=0, atol=1e-9)
    assert res["e3"] == pytest.approx(sw.e3(), abs=1e-9)
    for b, ob in enumerate(sw.bonds()):
        assert ctx.get_bond(0, b) == [(tuple(q), d) for q, d in ob], f"bond {b}"
    assert res["flags"] == 0
    assert res["sigma_lo_calls"] > 0 and lo["launches"] > 0
    assert res["sigma_lo_calls"] < res["sigma_calls"]  # FP64 residuals remain


@pytest.fixture(scope="module")
def c2(mp):
    with open(GOLDEN) as f:
        gold = json.load(f)
    ints = inputs.integrals(gold["k_a"], gold["k_v"], gold["rank"], gold["seed"])
    eri = fock.eri_from_cholesky(ints.B)
    _, c, ab = exact.active_ground_state(ints.h, eri, gold["k_a"], gold["n_elec"], 0)
    psi0 = exact.psi0_mps(c, ab, gold["k_a"], gold["M0"])
    g = inputs.psi1_guess(gold["k_a"], gold["k_v"], gold["n_elec"], 0, gold["M1"], gold["psi1_seed"])

    def run(precision):
        ctx = mp.Context(0)
        ctx.load_integrals(gold["k_a"], gold["k_v"], ints.h, ints.B)
        ctx.load_h0_partition(ints.eps_virt)
        ctx.load_psi0(gold["n_elec"], 0, *psi0)
        ctx.load_psi1_guess(g.bonds, g.sites)
        return ctx.sweep(gold["M1"], n_sweeps=gold["sweeps"], precision=precision)

    print("case: 8a+16v M1=128 FP64 reference run", flush=True)
    return gold, run, run(0)


@pytest.mark.parametrize("precision", [1, 2])
def test_benchmark_workload(mp, c2, precision):
    gold, run, ref = c2
    print(f"case: 8a+16v M1=128 precision {precision}", flush=True)
    res = run(precision)
    d_sweep = np.abs(np.array(res["e2_sweep"]) - np.array(ref["e2_sweep"])).max()
    print(f"precision {precision}: |dE2| vs FP64 GPU {abs(res['e2'] - ref['e2']):.3e} (max over sweeps "
          f"{d_sweep:.3e}), |dE3| {abs(res['e3'] - ref['e3']):.3e}; vs oracle |dE2| "
          f"{abs(res['e2'] - gold['e2_sweep'][-1]):.3e} |dE3| {abs(res['e3'] - gold['e3']):.3e}; "
          f"cg {res['cg_iters']} (FP64 {ref['cg_iters']}), refinements {res['refinements']}", flush=True)
    np.testing.assert_allclose(res["e2_sweep"], gold["e2_sweep"], rtol=0, atol=1e-6)
    assert res["e3"] == pytest.approx(gold["e3"], abs=1e-6)
    assert d_sweep < 1e-8
    assert abs(res["e3"] - ref["e3"]) < 1e-8
    assert res["flags"] == 0


@pytest.mark.parametrize("waves", [4, 16])
@pytest.mark.parametrize("precision", [1, 2])
def test_reduced_precision_launch_shapes(mp, c1, precision, waves):
    """The FP32 and BF16x3 GEMM instances in every launch shape: all work
    lists on one workgroup of 4 or 16 waves per tile with heavy split-k
    segmenting, same running E2 and bond tables as the oracle's FP64 sweep."""
    ints, eri, psi0 = c1
    print(f"case: 4a+4v M1=16 precision {precision}, {waves} waves per tile, split k", flush=True)
    g = inputs.psi1_guess(4, 4, 4, 0, 16, 1000)
    ctx = mp.Context(0)
    ctx.set_tuning(1, 16, 1, waves)
    ctx.load_integrals(4, 4, ints.h, ints.B)
    ctx.load_h0_partition(ints.eps_virt)
    ctx.load_psi0(4, 0, *psi0)
    ctx.load_psi1_guess(g.bonds, g.sites)
    res = ctx.sweep(16, precision=precision)
    sw = mps.Sweeper(ints.h, eri, 4, ints.eps_virt, 4, 0, psi0, (g.bonds, g.sites), 16)
    sw.run()
    np.testing.assert_allclose(ctx.get_trace()["e2"], [t["e2"] for t in sw.trace], rtol=0, atol=1e-9)
    for b, ob in enumerate(sw.bonds()):
        assert ctx.get_bond(0, b) == [(tuple(q), d) for q, d in ob], f"bond {b}"
    assert res["flags"] == 0 and res["sigma_lo_calls"] > 0


def test_bad_precision_arguments(mp, c1):
    ints, eri, psi0 = c1
    print("case: precision argument errors", flush=True)
    g = inputs.psi1_guess(4, 4, 4, 0, 8, 1000)
    ctx = mp.Context(0)
    ctx.load_integrals(4, 4, ints.h, ints.B)
    ctx.load_h0_partition(ints.eps_virt)
    ctx.load_psi0(4, 0, *psi0)
    ctx.load_psi1_guess(g.bonds, g.sites)
    with pytest.raises(mp.MPSPTError):
        ctx.sweep(8, precision=3)
    with pytest.raises(mp.MPSPTError):
        ctx.sweep(8, precision=1, inner_rel_tol=1.5)
    r = ctx.sweep(8, precision=1, inner_rel_tol=1e-2)
    assert r["flags"] == 0
