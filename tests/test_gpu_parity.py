"""Parity of the HIP MPS-PT path (through the C ABI) with the CPU oracle.

* 4 active + 4 virtual orbitals (exact Psi0): at M1 = 64 the sweep must reach
  the exact uncontracted E2/E3 of the determinant-space solve; at M1 = 16, 8
  and 4 every running E2, every bond sector table, E3 and the final Psi1
  (contracted to a determinant-space vector) must match the oracle's
  same-algorithm sweep.
* 8 active + 16 virtual orbitals (Psi0 compressed to M0 = 64, M1 = 128, four
  sweeps; the benchmarked workload): E2 per sweep and E3 against stored
  values written by tests/golden/make_golden.py from the oracle, the final
  bond tables exactly, and the Hylleraas upper bound against the exact E2.
Tolerances: 1e-9 Eh on the small system (both sides FP64, same algorithm,
CG to 1e-10 relative residual); 1e-6 Eh on the large one.
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
    ref = exact.brute_force(ints.h, eri, 4, ints.eps_virt, 4, 0, c, ab)
    return ints, eri, exact.psi0_mps(c, ab, 4), ref


def run_gpu(mp, ints, n_elec, psi0, guess, M1, **kw):
    ctx = mp.Context(0)
    ctx.load_integrals(ints.k_a, ints.k_v, ints.h, ints.B)
    ctx.load_h0_partition(ints.eps_virt)
    ctx.load_psi0(n_elec, 0, *psi0)
    ctx.load_psi1_guess(guess.bonds, guess.sites)
    res = ctx.sweep(M1, **kw)
    return ctx, res


def state_vector(sites):
    v = sites[0]
    for a in sites[1:]:
        v = np.tensordot(v, a, axes=([-1], [0]))
    return v.reshape(-1)


def test_full_bond_dimension_reaches_exact(mp, c1):
    ints, eri, psi0, ref = c1
    print("case: 4a+4v M1=64 seed 0", flush=True)
    g = inputs.psi1_guess(4, 4, 4, 0, 64, 1000)
    ctx, res = run_gpu(mp, ints, 4, psi0, g, 64)
    assert res["e0"] == pytest.approx(ref.E0, abs=1e-12)
    assert res["e2"] == pytest.approx(ref.E2, abs=1e-9)
    assert res["e3"] == pytest.approx(ref.E3, abs=1e-9)


@pytest.mark.parametrize("M1", [16, 8, 4])
def test_same_algorithm_parity(mp, c1, M1):
    ints, eri, psi0, ref = c1
    print(f"case: 4a+4v M1={M1} seed 0", flush=True)
    g = inputs.psi1_guess(4, 4, 4, 0, M1, 1000)
    ctx, res = run_gpu(mp, ints, 4, psi0, g, M1)
    sw = mps.Sweeper(ints.h, eri, 4, ints.eps_virt, 4, 0, psi0, (g.bonds, g.sites), M1)
    sw.run()
    tr = ctx.get_trace()
    oref = np.array([t["e2"] for t in sw.trace])
    assert len(tr["e2"]) == len(oref)
    np.testing.assert_allclose(tr["e2"], oref, rtol=0, atol=1e-9)
    np.testing.assert_allclose(tr["discarded"], [t["discarded"] for t in sw.trace], rtol=0, atol=1e-9)
    assert res["e2"] >= ref.E2 - 1e-10                 # Hylleraas upper bound
    assert res["e3"] == pytest.approx(sw.e3(), abs=1e-9)
    for b, ob in enumerate(sw.bonds()):
        assert ctx.get_bond(0, b) == [(tuple(q), d) for q, d in ob], f"bond {b}"
    vg = state_vector([ctx.get_site(0, i) for i in range(8)])
    vo = state_vector(sw.A)
    assert np.abs(vg - vo).max() < 1e-8 * np.abs(vo).max()


def test_seeds_and_spin_sectors(mp):
    """Other seeds and an open-shell reference (5 electrons, 2Sz = 1)."""
    for (ka, kv, ne, tsz, seed, M1) in ((4, 4, 4, 0, 3, 12), (4, 3, 5, 1, 4, 10)):
        print(f"case: {ka}a+{kv}v N={ne} 2Sz={tsz} seed {seed} M1={M1}", flush=True)
        ints = inputs.integrals(ka, kv, 12, seed)
        eri = fock.eri_from_cholesky(ints.B)
        _, c, ab = exact.active_ground_state(ints.h, eri, ka, ne, tsz)
        psi0 = exact.psi0_mps(c, ab, ka)
        g = inputs.random_mps(ka + kv, ka, ne, tsz, (1, 2), M1, seed + 1000)
        ctx = mp.Context(0)
        ctx.load_integrals(ka, kv, ints.h, ints.B)
        ctx.load_h0_partition(ints.eps_virt)
        ctx.load_psi0(ne, tsz, *psi0)
        ctx.load_psi1_guess(g.bonds, g.sites)
        res = ctx.sweep(M1)
        sw = mps.Sweeper(ints.h, eri, ka, ints.eps_virt, ne, tsz, psi0, (g.bonds, g.sites), M1)
        sw.run()
        np.testing.assert_allclose(ctx.get_trace()["e2"], [t["e2"] for t in sw.trace], rtol=0, atol=1e-9)
        assert res["e3"] == pytest.approx(sw.e3(), abs=1e-9)


def test_ground_state_reference(mp, c1):
    """The library's own Psi0 (two-site DMRG with Davidson): exact at a bond
    dimension above the Schmidt ranks, variational below (between the FCI
    energy and the energy of the FCI vector compressed to the same M0)."""
    ints, eri, psi0, ref = c1
    print("case: DMRG Psi0 4 active orbitals M0=16", flush=True)
    ctx = mp.Context(0)
    ctx.load_integrals(4, 4, ints.h, ints.B)
    ctx.load_h0_partition(ints.eps_virt)
    g0 = inputs.psi0_guess(4, 4, 0, 16, 2000)
    e = ctx.ground_state(4, 0, g0.bonds, g0.sites, 16)
    assert e == pytest.approx(ref.E0, abs=1e-10)
    g = inputs.psi1_guess(4, 4, 4, 0, 64, 1000)
    ctx.load_psi1_guess(g.bonds, g.sites)
    res = ctx.sweep(64)
    assert res["e0"] == pytest.approx(ref.E0, abs=1e-10)
    assert res["e2"] == pytest.approx(ref.E2, abs=1e-8)
    print("case: DMRG Psi0 8 active orbitals M0=64", flush=True)
    ints8 = inputs.integrals(8, 16, 32, 0)
    eri8 = fock.eri_from_cholesky(ints8.B)
    efci, c, ab = exact.active_ground_state(ints8.h, eri8, 8, 8, 0)
    b0, s0 = exact.psi0_mps(c, ab, 8, 64)
    v = exact.mps_to_vector(s0, 8)[fock.site_index(ab, 8)]
    esvd = v @ (fock.hamiltonian(ints8.h[:8, :8], eri8[:8, :8, :8, :8], ab) @ v) / (v @ v)
    ctx8 = mp.Context(0)
    ctx8.load_integrals(8, 16, ints8.h, ints8.B)
    ctx8.load_h0_partition(ints8.eps_virt)
    g0 = inputs.psi0_guess(8, 8, 0, 64, 2000)
    e8 = ctx8.ground_state(8, 0, g0.bonds, g0.sites, 64)
    assert efci - 1e-10 <= e8 <= esvd + 1e-8


def test_errors_are_reported(mp, c1):
    ints, eri, psi0, ref = c1
    ctx = mp.Context(0)
    with pytest.raises(mp.MPSPTError) as e:
        ctx.sweep(16)
    assert e.value.status == -6  # MPSPT_E_STATE
    ctx.load_integrals(4, 4, ints.h, ints.B)
    ctx.load_h0_partition(ints.eps_virt)
    bonds, sites = psi0
    bad = [s.copy() for s in sites]
    assert tuple(bonds[1][0][0]) == (0, 0) and tuple(bonds[2][0][0]) == (0, 0)
    bad[1][0, 1, 0] = 1.0  # (0,0) + up electron cannot reach the (0,0) state: outside every block
    with pytest.raises(mp.MPSPTError) as e:
        ctx.load_psi0(4, 0, bonds, bad)
    assert e.value.status == -2  # MPSPT_E_QN
    # an indefinite zeroth-order operator is detected by CG (p.Ap <= 0)
    ctx2 = mp.Context(0)
    ctx2.load_integrals(4, 4, ints.h, ints.B)
    ctx2.load_h0_partition(np.full(4, -5.0))
    ctx2.load_psi0(4, 0, *psi0)
    g = inputs.psi1_guess(4, 4, 4, 0, 16, 1000)
    ctx2.load_psi1_guess(g.bonds, g.sites)
    with pytest.raises(mp.MPSPTError) as e:
        ctx2.sweep(16)
    assert e.value.status == -5  # MPSPT_E_INDEFINITE


def test_deterministic(mp, c1):
    ints, eri, psi0, ref = c1
    g = inputs.psi1_guess(4, 4, 4, 0, 16, 1000)
    a = run_gpu(mp, ints, 4, psi0, g, 16)[0].get_trace()["e2"]
    b = run_gpu(mp, ints, 4, psi0, g, 16)[0].get_trace()["e2"]
    assert np.array_equal(a, b)


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden values not generated")
def test_benchmark_workload_against_stored_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1408_5092_amd import mpspt as mp
    gold = json.load(open(GOLDEN))
    ka, kv, ne = gold["k_a"], gold["k_v"], gold["n_elec"]
    print(f"case: {ka}a+{kv}v M0={gold['M0']} M1={gold['M1']} sweeps={gold['sweeps']} seed {gold['seed']}",
          flush=True)
    ints = inputs.integrals(ka, kv, gold["rank"], gold["seed"])
    eri = fock.eri_from_cholesky(ints.B)
    _, c, ab = exact.active_ground_state(ints.h, eri, ka, ne, 0)
    psi0 = exact.psi0_mps(c, ab, ka, gold["M0"])
    g = inputs.psi1_guess(ka, kv, ne, 0, gold["M1"], gold["psi1_seed"])
    ctx, res = run_gpu(mp, ints, ne, psi0, g, gold["M1"], n_sweeps=gold["sweeps"])
    assert res["e0"] == pytest.approx(gold["e0"], abs=1e-10)
    np.testing.assert_allclose(res["e2_sweep"], gold["e2_sweep"], rtol=0, atol=1e-6)
    assert res["e3"] == pytest.approx(gold["e3"], abs=1e-6)
    tr = ctx.get_trace()["e2"]
    np.testing.assert_allclose(tr, [t["e2"] for t in gold["trace"]], rtol=0, atol=1e-6)
    assert res["e2"] >= gold["e2_exact"] - 1e-10
    for b, ob in enumerate(gold["bonds"]):
        assert ctx.get_bond(0, b) == [((n, s), d) for n, s, d in ob], f"bond {b}"


def test_kernel_timing_sampling(mp, c1):
    """Kernel timing records every launch, or a hashed one-in-N sample of each kind."""
    ints, eri, psi0, ref = c1
    print("case: 4a+4v M1=8 kernel timing every 1 / every 4", flush=True)
    g = inputs.psi1_guess(4, 4, 4, 0, 8, 1000)
    ctx = mp.Context(0)
    ctx.load_integrals(4, 4, ints.h, ints.B)
    ctx.load_h0_partition(ints.eps_virt)
    ctx.load_psi0(4, 0, *psi0)
    ctx.load_psi1_guess(g.bonds, g.sites)
    for every in (1, 4):
        ctx.profile(True, every=every)
        ctx.sweep(8)
        st = [ctx.kernel_stats(k) for k in sorted(ctx.KERNELS)]
        ctx.profile(False)
        gemm = st[0]
        assert gemm["launches_all"] > 0 and gemm["seconds"] > 0
        for s in st:
            if every == 1:
                assert s["launches"] == s["launches_all"], s
            else:
                assert s["launches"] <= s["launches_all"], s
                if s["launches_all"] >= 400:
                    assert abs(s["launches"] / s["launches_all"] - 1 / every) < 0.1, s
    with pytest.raises(mp.MPSPTError):
        ctx.profile(True, every=-1)


def test_degenerate_cases(mp, c1):
    """Cases the method degenerates in, against the oracle's dense solve:
    no coupling between active and virtual orbitals (V|Psi0> = 0, so E2 = E3 = 0
    and every local right-hand side vanishes); a single virtual orbital; a
    bond dimension of one (the most severe truncation: still an upper bound);
    one electron."""
    ints, eri, psi0, ref = c1
    print("case: 4a+4v zero coupling", flush=True)
    ka, k = 4, ints.k
    nv = (np.arange(k) >= ka).astype(int)
    cnt = nv[:, None, None, None] + nv[None, :, None, None] + nv[None, None, :, None] + nv[None, None, None, :]
    eri0 = np.where((cnt == 1) | (cnt == 2), 0.0, eri)
    h0 = ints.h.copy()
    h0[:ka, ka:] = 0.0
    h0[ka:, :ka] = 0.0
    _, c, ab = exact.active_ground_state(h0, eri0, ka, 4, 0)
    g = inputs.psi1_guess(4, 4, 4, 0, 16, 1000)
    ctx = mp.Context(0)
    ctx.load_integrals_eri(4, 4, h0, eri0)
    ctx.load_h0_partition(ints.eps_virt)
    ctx.load_psi0(4, 0, *exact.psi0_mps(c, ab, 4))
    ctx.load_psi1_guess(g.bonds, g.sites)
    r = ctx.sweep(16)
    assert abs(r["e2"]) < 1e-14 and abs(r["e3"]) < 1e-14

    print("case: 4a+1v exact, and M1=1 upper bound", flush=True)
    ints1 = inputs.integrals(4, 1, 8, 6)
    eri1 = fock.eri_from_cholesky(ints1.B)
    _, c, ab = exact.active_ground_state(ints1.h, eri1, 4, 4, 0)
    ex = exact.brute_force(ints1.h, eri1, 4, ints1.eps_virt, 4, 0, c, ab)
    p0 = exact.psi0_mps(c, ab, 4)
    for M1 in (64, 1):
        g = inputs.psi1_guess(4, 1, 4, 0, M1, 1001)
        ctx = mp.Context(0)
        ctx.load_integrals(4, 1, ints1.h, ints1.B)
        ctx.load_h0_partition(ints1.eps_virt)
        ctx.load_psi0(4, 0, *p0)
        ctx.load_psi1_guess(g.bonds, g.sites)
        r = ctx.sweep(M1)
        sw = mps.Sweeper(ints1.h, eri1, 4, ints1.eps_virt, 4, 0, p0, (g.bonds, g.sites), M1)
        sw.run()
        np.testing.assert_allclose(ctx.get_trace()["e2"], [t["e2"] for t in sw.trace], rtol=0, atol=1e-9)
        if M1 == 64:
            assert r["e2"] == pytest.approx(ex.E2, abs=1e-9) and r["e3"] == pytest.approx(ex.E3, abs=1e-9)
        else:
            assert r["e2"] >= ex.E2 - 1e-12

    print("case: 3a+2v one electron", flush=True)
    ints2 = inputs.integrals(3, 2, 6, 7)
    eri2 = fock.eri_from_cholesky(ints2.B)
    _, c, ab = exact.active_ground_state(ints2.h, eri2, 3, 1, 1)
    ex = exact.brute_force(ints2.h, eri2, 3, ints2.eps_virt, 1, 1, c, ab)
    g = inputs.random_mps(5, 3, 1, 1, (1, 2), 16, 1002)
    ctx = mp.Context(0)
    ctx.load_integrals(3, 2, ints2.h, ints2.B)
    ctx.load_h0_partition(ints2.eps_virt)
    ctx.load_psi0(1, 1, *exact.psi0_mps(c, ab, 3))
    ctx.load_psi1_guess(g.bonds, g.sites)
    r = ctx.sweep(16)
    assert r["e2"] == pytest.approx(ex.E2, abs=1e-10) and r["e3"] == pytest.approx(ex.E3, abs=1e-10)


def test_size_limits(mp):
    """Orbital counts beyond the library's limit (128) and empty spaces are refused."""
    print("case: size limits", flush=True)
    ctx = mp.Context(0)
    for ka, kv in ((100, 29), (0, 4), (4, 0)):
        k = ka + kv
        h = np.eye(max(k, 1))[:k, :k]
        B = np.zeros((1, k, k))
        with pytest.raises(mp.MPSPTError) as e:
            ctx.load_integrals(ka, kv, h, B)
        assert e.value.status == -1  # MPSPT_E_ARG


def test_launch_shapes_and_split_k(mp, c1):
    """The grouped GEMM's launch shapes and split-k segments change how the
    same sums are tiled and ordered, not what is summed: forcing every list
    to one wave per tile, or to one workgroup of 4, 8 or 16 waves per tile,
    with or without heavy k splitting, gives the same running E2 and bond
    tables as the defaults (and the oracle) to rounding."""
    ints, eri, psi0, ref = c1
    print("case: 4a+4v M1=8 launch shapes x split-k", flush=True)
    g = inputs.psi1_guess(4, 4, 4, 0, 8, 1000)
    sw = mps.Sweeper(ints.h, eri, 4, ints.eps_virt, 4, 0, psi0, (g.bonds, g.sites), 8)
    sw.run()
    oref = [t["e2"] for t in sw.trace]
    for wide, kmin, kdiv, waves in ((8, 512, 8192, 4), (1, 512, 8192, 4), (1 << 20, 512, 8192, 4), (1, 16, 1, 4),
                                    (1 << 20, 16, 1, 4), (1, 512, 8192, 8), (1, 512, 8192, 16), (1, 16, 1, 16)):
        ctx = mp.Context(0)
        ctx.set_tuning(wide, kmin, kdiv, waves)
        assert ctx.get_tuning() == {"wide_chunks": wide, "kseg_min": kmin, "kseg_div": kdiv, "split_waves": waves}
        ctx.load_integrals(4, 4, ints.h, ints.B)
        ctx.load_h0_partition(ints.eps_virt)
        ctx.load_psi0(4, 0, *psi0)
        ctx.load_psi1_guess(g.bonds, g.sites)
        ctx.sweep(8)
        np.testing.assert_allclose(ctx.get_trace()["e2"], oref, rtol=0, atol=1e-9)
        for b, ob in enumerate(sw.bonds()):
            assert ctx.get_bond(0, b) == [(tuple(q), d) for q, d in ob], (wide, kmin, kdiv, waves, b)
    with pytest.raises(mp.MPSPTError):
        ctx.set_tuning(0, 512, 8192)
    with pytest.raises(mp.MPSPTError):
        ctx.set_tuning(4, 512, 8192, 6)
