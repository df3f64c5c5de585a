"""Host-side checks of the virtual-pair form (no GPU): the product's pair
bookkeeping against the oracle's, and the stored per-pair values against the
stored monolithic ones."""
import json
import os

import numpy as np
import pytest

from oracle import pairs as opairs
from paper_1408_5092_amd import inputs
from paper_1408_5092_amd import pairs as ppairs

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_pair_lists_and_masks_agree_with_oracle():
    for kv in (1, 4, 16, 40):
        assert ppairs.pair_list(kv) == opairs.pairs(kv)
        for (a, b) in ppairs.pair_list(kv):
            assert ppairs.mask_sets(ppairs.pair_masks(a, b)) == opairs.occupancy(a, b)
    assert len(ppairs.pair_list(40)) == 820


def test_pair_integrals_restrict_cholesky_vectors():
    ints = inputs.integrals(4, 5, 8, 3)
    for (a, b) in ((0, 0), (1, 4), (3, 3)):
        hp, Bp, ep = ppairs.pair_integrals(ints.h, ints.B, 4, ints.eps_virt, a, b)
        eri = np.einsum("lpq,lrs->pqrs", ints.B, ints.B)
        ho, go, eo = opairs.restrict(ints.h, eri, 4, ints.eps_virt, a, b)
        assert np.array_equal(hp, ho) and np.array_equal(ep, eo)
        assert np.allclose(np.einsum("lpq,lrs->pqrs", Bp, Bp), go, atol=1e-15)


def test_stored_pair_shares_add_up_to_stored_e2():
    with open(os.path.join(GOLD, "pairs_8a16v_seed0.json")) as f:
        pg = json.load(f)
    with open(os.path.join(GOLD, "c2_8a16v_seed0.json")) as f:
        mg = json.load(f)
    assert len(pg["share"]) == 136
    assert sum(e for _, _, e in pg["share"]) == pytest.approx(mg["e2_exact"], abs=1e-11)
    assert pg["e0"] == pytest.approx(mg["e0"], abs=1e-11)
    assert all(e < 0 for _, _, e in pg["share"])
    for s in pg["sweeps"]:
        a, b = s["pair"]
        share = {(x, y): e for x, y, e in pg["share"]}[(a, b)]
        assert s["e2_sweep"][-1] >= share  # truncated sweep: Hylleraas upper bound


def test_tuning_file_matches_the_binding():
    """The committed launch-shape table has the keys Context applies, within
    the ranges mpspt_set_tuning accepts."""
    import json
    import os
    from paper_1408_5092_amd import autotune, mpspt
    with open(mpspt.TUNING_PATH) as f:
        t = json.load(f)
    choice = t["choice"]
    assert set(choice) == set(autotune.DEFAULT) == set(autotune.GRID)
    assert choice["wide_chunks"] >= 1 and choice["kseg_min"] >= 16 and choice["kseg_div"] >= 1
    assert choice["split_waves"] in (4, 8, 16)
    assert os.path.dirname(mpspt.TUNING_PATH) == os.path.dirname(os.path.abspath(mpspt.__file__))
