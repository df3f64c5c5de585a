"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/mpspt.h declares, refuses to run without a gfx950 device, and
its MPO builder (host logic) contracts to the oracle's determinant-space
operators (Eq. mpo)."""
import os
import re

import numpy as np
import pytest

from oracle import exact, fock
from paper_1408_5092_amd import inputs, mpspt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "mpspt.h")).read()
    return sorted(set(re.findall(r"\b(mpspt_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mpspt.LIB_PATH):
        from paper_1408_5092_amd import build
        build.build()
    return mpspt.load_library()


def test_exports_every_declared_symbol(lib):
    decl = declared_symbols()
    assert len(decl) >= 14
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(decl) == sorted(mpspt.EXPORTED)


def test_create_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(mpspt.MPSPTError) as e:
        mpspt.Context(0, stream=None, lib=lib)
    assert e.value.status == -7  # MPSPT_E_NODEV


@pytest.mark.parametrize("ka,kv,seed", [(2, 2, 3), (3, 2, 5), (2, 3, 9)])
def test_library_mpo_matches_determinant_operator(lib, ka, kv, seed):
    ints = inputs.integrals(ka, kv, 8, seed)
    eri = fock.eri_from_cholesky(ints.B)
    k = ka + kv
    basis = fock.sector_basis(k)
    perm = fock.site_index(basis, k)
    parts = exact.split_integrals(ints.h, eri, ka, ints.eps_virt)
    dense = {}
    for which, name in ((0, "H0"), (2, "V")):
        F = fock.hamiltonian(*parts[name], basis).toarray()
        Fs = np.zeros_like(F)
        Fs[np.ix_(perm, perm)] = F
        D = mpspt.mpo_dense(ka, kv, ints.h, eri, ints.eps_virt, which, lib=lib)
        assert np.abs(D - Fs).max() < 1e-13, name
        dense[name] = Fs
    # the part of V used for the right-hand side equals V on states with empty virtuals
    D1 = mpspt.mpo_dense(ka, kv, ints.h, eri, ints.eps_virt, 1, lib=lib)
    empty = np.zeros(4 ** k, dtype=bool)
    empty[perm[fock.n_virtual(basis, ka) == 0]] = True
    assert np.abs(D1[:, empty] - dense["V"][:, empty]).max() < 1e-13
    # the part of V used for E3 equals V between states with one or two virtual electrons
    D3 = mpspt.mpo_dense(ka, kv, ints.h, eri, ints.eps_virt, 3, lib=lib)
    psi1 = np.zeros(4 ** k, dtype=bool)
    nv = fock.n_virtual(basis, ka)
    psi1[perm[(nv == 1) | (nv == 2)]] = True
    assert np.abs(D3[np.ix_(psi1, psi1)] - dense["V"][np.ix_(psi1, psi1)]).max() < 1e-13


def test_mpo_channel_counts_scale_as_paper(lib):
    """The MPO bond dimension of H0 and of the part of V acting on Psi0 is
    O(k_a^2) and does not grow with the number of virtual orbitals."""
    dims = []
    for kv in (2, 4, 8):
        ints = inputs.integrals(3, kv, 8, 1)
        eri = fock.eri_from_cholesky(ints.B)
        d0 = mpspt.mpo_dims(3, kv, ints.h, eri, ints.eps_virt, 0, lib=lib)
        d1 = mpspt.mpo_dims(3, kv, ints.h, eri, ints.eps_virt, 1, lib=lib)
        assert max(d0[3:]) == 2           # virtual region: complete H_act and identity
        dims.append(max(d1))
    assert dims[2] - dims[1] <= 4 * (8 - 4)  # growth at most linear in k_v (single virtual ops)


def test_arguments_are_validated(lib):
    ints = inputs.integrals(2, 2, 8, 3)
    eri = fock.eri_from_cholesky(ints.B)
    bad = ints.h.copy()
    bad[0, 1] += 1.0
    with pytest.raises(mpspt.MPSPTError) as e:
        mpspt.mpo_dense(2, 2, bad, eri, ints.eps_virt, 0, lib=lib)
    assert e.value.status == -1
    nan = ints.h.copy()
    nan[0, 0] = np.nan
    with pytest.raises(mpspt.MPSPTError):
        mpspt.mpo_dims(2, 2, nan, eri, ints.eps_virt, 0, lib=lib)


def test_profile_summaries_name_kernels_with_their_template_arguments(tmp_path):
    """The rocprofv3 summary helper keeps each kernel instance apart (the
    GEMM's launch shapes and precisions are template arguments) and takes
    the window between the library's two k_profile_mark dispatches."""
    from paper_1408_5092_amd import profiling
    assert profiling._short("void mpspt::dev::(anonymous namespace)::k_gemm_grouped_lo_split<1, 8>(mpspt::dev::BasesF)") \
        == "k_gemm_grouped_lo_split<1, 8>"
    assert profiling._short("mpspt::dev::(anonymous namespace)::k_gemm_grouped_split<8>(Bases, ...)") \
        == "k_gemm_grouped_split<8>"
    assert profiling._short("k_eig_reduce<true>(EigJob const*)") == "k_eig_reduce<true>"
    assert profiling._short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"
    rows = [("k_gemm_grouped(Bases)", 0, 5), ("k_profile_mark(int)", 10, 11), ("k_gemm_grouped(Bases)", 20, 32),
            ("k_gemm_grouped_split<8>(Bases)", 40, 44), ("k_profile_mark(int)", 50, 51), ("k_dot(double*)", 60, 70)]
    with open(tmp_path / "run_kernel_trace.csv", "w") as f:
        f.write("Kernel_Name,Start_Timestamp,End_Timestamp\n")
        for n, s, e in rows:
            f.write(f"\"{n}\",{s * 1000},{e * 1000}\n")
    out = profiling.trace(str(tmp_path))
    assert out["window_ms"] == pytest.approx(0.040)
    assert set(out["kernels"]) == {"k_gemm_grouped", "k_gemm_grouped_split<8>"}
    assert out["kernels"]["k_gemm_grouped"]["avg_us"] == pytest.approx(12.0)
