"""Host logic of the bond-dimension scans (paper_1408_5092_amd.mscan): the
least-squares line, the choice of points for the zero-weight extrapolation,
and the smallest bond dimension meeting a tolerance."""
import numpy as np
import pytest

from paper_1408_5092_amd import mscan


def test_fit_line_exact_and_least_squares():
    w = np.array([1e-4, 3e-4, 7e-4])
    e0, s = mscan.fit_line(w, -0.15 + 1.3 * w)
    assert e0 == pytest.approx(-0.15, abs=1e-15) and s == pytest.approx(1.3, rel=1e-12)
    rng = np.random.default_rng(3)
    w = rng.uniform(0, 1e-3, 7)
    e = -0.2 + 0.9 * w + rng.normal(0, 1e-6, 7)
    # normal equations of the two-parameter fit, written out
    A = np.array([[len(w), w.sum()], [w.sum(), (w * w).sum()]])
    rhs = np.array([e.sum(), (w * e).sum()])
    ref = np.linalg.solve(A, rhs)
    e0, s = mscan.fit_line(w, e)
    assert e0 == pytest.approx(ref[0], abs=1e-12) and s == pytest.approx(ref[1], rel=1e-9)
    assert mscan.fit_line([2e-4], [-0.1]) == (-0.1, 0.0)
    assert mscan.fit_line([2e-4, 2e-4], [-0.1, -0.3]) == (pytest.approx(-0.2), 0.0)
    with pytest.raises(ValueError):
        mscan.fit_line([], [])


def _pts(rows):
    return [{"M1": m, "e2": e, "discarded": w} for m, e, w in rows]


def test_extrapolate_uses_the_largest_bond_dimensions():
    # relaxation at small M1 (discarded weight not monotone), linear after
    pts = _pts([(16, -0.10, 2.0e-3), (32, -0.12, 1.0e-3), (64, -0.14, 1.5e-3),
                (128, -0.2 + 1.0 * 4e-4, 4e-4), (256, -0.2 + 1.0 * 1e-4, 1e-4)])
    e, s, used = mscan.extrapolate(pts, 2)
    assert [p["M1"] for p in used] == [256, 128]
    assert e == pytest.approx(-0.2, abs=1e-15) and s == pytest.approx(1.0)
    # a scan whose largest M1 discarded nothing (up to rounding) is already converged
    pts.append({"M1": 512, "e2": -0.2, "discarded": 4e-16})
    assert mscan.extrapolate(pts, 3) == (-0.2, 0.0, [pts[-1]])
    with pytest.raises(ValueError):
        mscan.extrapolate([], 2)


def test_m_required():
    pts = _pts([(64, -0.145, 0), (32, -0.13, 0), (128, -0.1501, 0), (96, -0.1494, 0)])
    assert mscan.m_required(pts, -0.1509, 1e-3) == 128
    assert mscan.m_required(pts, -0.1509, 2e-3) == 96
    assert mscan.m_required(pts, -0.1509, 1e-5) is None
