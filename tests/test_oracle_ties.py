"""The tie scenes (tests/ties.py) do put samples exactly on the kinks: the
oracle's union sum is exactly 1, a difference's operands are exactly equal,
an intersection's sum is exactly N - 1, and linear-sigma arguments are
exactly +-1/2 on some samples; and there the oracle's gradient takes the
rules of its reading (no gradient through a clamp at the tie, the linear
sigma's derivative 0 at its breakpoints), which central differences straddling
the kink cannot decide.  The GPU tests compare the kernels with the oracle on
these same scenes."""
import numpy as np
import pytest

from oracle import primitives as prm
from oracle import scene as S
from tests import ties


def _fills(cfg, comp):
    d = cfg["scene"]
    vals = S.resolve(d, cfg["p"])
    pts = S.plane_points(d, comp)
    return [np.broadcast_to(prm.evaluate(pr, vals[i], pts)[0], (1, 48, 64)) for i, pr in enumerate(d["prims"])]


def _args(cfg, comp, prim, lo_field):
    """The linear-sigma argument t of a box's x-bound at every x sample."""
    from oracle.lattice import component_samples
    d = cfg["scene"]
    vals = S.resolve(d, cfg["p"])
    c, w = component_samples(d, comp)["x"]
    x = vals[prim][lo_field]
    return (c - x) / w if lo_field == 0 else (x - c) / w


def test_union_scene_has_exact_ties():
    cfg = ties.union_ties()
    for comp in ("x", "y", "z"):
        f = _fills(cfg, comp)
        tot = f[0] + f[1] + f[2]
        both = (f[0] > 0) & (f[0] < 1) & (f[1] > 0) & (f[1] < 1)
        assert np.count_nonzero(both & (tot == 1.0)) >= 10
    assert np.any(np.abs(_args(cfg, "z", 2, 0)) == 0.5)
    assert np.any(np.abs(_args(cfg, "x", 2, 1)) == 0.5)


def test_difference_scene_has_exact_ties():
    cfg = ties.difference_ties()
    for comp in ("x", "y", "z"):
        f = _fills(cfg, comp)
        part = (f[0] > 0) & (f[0] < 1)
        assert np.count_nonzero(part & (f[0] == f[1])) >= 5


@pytest.mark.parametrize("case", ["intersection", "meet"])
def test_intersection_scenes_have_exact_ties(case):
    cfg = ties.CASES[case]()
    for comp in ("x", "y", "z"):
        f = _fills(cfg, comp)
        part = (f[0] > 0) & (f[0] < 1) & (f[1] > 0) & (f[1] < 1)
        assert np.count_nonzero(part & (f[0] + f[1] == 1.0)) >= 5


@pytest.mark.parametrize("case", sorted(ties.CASES))
def test_tie_rules_decide_the_gradient(case):
    # the oracle's analytic gradient differs from a central difference that
    # straddles the kinks (each side of a kink has another derivative), so the
    # rules, not the arithmetic, decide these values
    cfg = ties.CASES[case]()
    g = S.sensitivity(cfg["E"], cfg["A"], cfg["omega"])
    ga = S.grad_analytic(cfg["scene"], cfg["p"], g)
    gf = S.grad_fd(cfg["scene"], cfg["p"], g, 1e-9)
    assert np.all(np.isfinite(ga))
    assert np.linalg.norm(ga - gf) / np.linalg.norm(gf) > 1e-3
