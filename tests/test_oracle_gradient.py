"""Pins of the oracle's gradient: central and forward differences of its own
permittivity agree with its reverse-mode gradient (the paper states the
AutoDiff gradient is exact, Sec. "Single-polarization blazed grating
coupler in 2D"), and closed forms fix the contraction of eq:1.

Sensitivity pin (eq:1): with E = exp(i phi) and E_adj = i exp(-i phi)/(2 omega)
the unconjugated product gives g = 2 omega Im(E E_adj) = 1 for every phi; a
conjugated or sign-flipped contraction does not.  With g = 1 and a linear-sigma
box spanning the whole y (and z) extent, sum_j d eps_j / d x1 is the discrete
shape derivative Delta_eps * Ny * Nz / w(edge sample) -- a closed form."""
import numpy as np
import pytest

from oracle import scene as S
from oracle.lattice import axis_samples
from paper_2311_05646_amd import workloads as W


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("name,h,tol", [("c1", 1e-4, 1e-10), ("c2_small", 1e-5, 1e-9),
                                        ("c3_small", 1e-8, 1e-6), ("c4_small", 1e-6, 1e-7)])
def test_central_fd_matches_analytic(name, h, tol):
    cfg = W.CONFIGS[name]()
    g = S.sensitivity(cfg["E"], cfg["A"], cfg["omega"])
    ga = S.grad_analytic(cfg["scene"], cfg["p"], g)
    params = None if cfg["scene"]["n_params"] <= 24 else list(range(0, cfg["scene"]["n_params"], 3))
    gf = S.grad_fd(cfg["scene"], cfg["p"], g, h, params)
    sel = slice(None) if params is None else params
    assert _rel(gf[sel], ga[sel]) < tol


@pytest.mark.parametrize("dim,root", [(2, "union"), (3, "union"), (3, "difference"), (2, "intersection"),
                                      (2, "deep"), (3, "deep")])
def test_zoo_fd_matches_analytic(dim, root):
    cfg = W.make_zoo(dim=dim, root=root)
    g = S.sensitivity(cfg["E"], cfg["A"], cfg["omega"])
    ga = S.grad_analytic(cfg["scene"], cfg["p"], g)
    gf = S.grad_fd(cfg["scene"], cfg["p"], g, 1e-6)
    assert _rel(gf, ga) < 1e-6
    assert np.count_nonzero(ga) >= 8


@pytest.mark.parametrize("dim", [2, 3])
def test_levels_fd_matches_analytic(dim):
    # the non-binary union (Alg. cap) through the whole scene
    cfg = W.make_levels(dim=dim)
    g = S.sensitivity(cfg["E"], cfg["A"], cfg["omega"])
    ga = S.grad_analytic(cfg["scene"], cfg["p"], g)
    gf = S.grad_fd(cfg["scene"], cfg["p"], g, 1e-6)
    assert _rel(gf, ga) < 1e-6
    assert np.count_nonzero(ga) >= 12


@pytest.mark.parametrize("dim", [2, 3])
def test_polar2d_scene_fd_matches_analytic(dim):
    cfg = W.make_polar2d_small(dim=dim)
    g = S.sensitivity(cfg["E"], cfg["A"], cfg["omega"])
    ga = S.grad_analytic(cfg["scene"], cfg["p"], g)
    gf = S.grad_fd(cfg["scene"], cfg["p"], g, 1e-6)
    assert _rel(gf, ga) < 1e-6
    assert np.count_nonzero(ga) == cfg["scene"]["n_params"]


def test_blazed_composition_fd_matches_analytic():
    # three op levels, etch depths and the oxide thickness as parameters
    cfg = W.make_blazed_small()
    g = S.sensitivity(cfg["E"], cfg["A"], cfg["omega"])
    ga = S.grad_analytic(cfg["scene"], cfg["p"], g)
    assert _rel(S.grad_fd(cfg["scene"], cfg["p"], g, 1e-5), ga) < 1e-9
    assert np.count_nonzero(ga) == cfg["scene"]["n_params"]


def test_forward_fd_matches_analytic_c1():
    cfg = W.make_c1()
    g = S.sensitivity(cfg["E"], cfg["A"], cfg["omega"])
    ga = S.grad_analytic(cfg["scene"], cfg["p"], g)
    assert _rel(S.grad_fd_forward(cfg["scene"], cfg["p"], g, cfg["h"]), ga) < 1e-9


def _slab_scene(comp):
    X = W.graded_nodes(W.raised_cosine_widths(40, 10.0, 25.0))
    Y = W.uniform_nodes(13, 0.02)
    box = W.box(x=(W.P(0), W.P(1)))
    return {"name": "slab", "dim": 2, "nodes": [X, Y, np.array([0.0, 1.0])], "components": (comp,),
            "eps_bg": 1.5, "eps_fg": 9.5, "n_params": 2, "prims": [box],
            "tree": {"op": "union", "children": [0]}}, X


@pytest.mark.parametrize("comp", ["x", "y"])
def test_box_sum_rule_with_unit_sensitivity(comp):
    desc, X = _slab_scene(comp)
    p = np.array([X[7] + 0.0037, X[29] + 0.0061])
    rng = np.random.default_rng(1)
    omega = 2 * np.pi / 1.55
    phi = rng.uniform(0, 2 * np.pi, size=(1, 1, 13, 40))
    E = np.exp(1j * phi)
    A = 1j * np.exp(-1j * phi) / (2 * omega)
    g = S.sensitivity(E, A, omega)
    assert np.allclose(g, 1.0, atol=1e-13)
    assert not np.allclose(2 * omega * np.imag(E * np.conj(A)), 1.0)
    grad = S.grad_analytic(desc, p, g)
    c, w = axis_samples(X, cell_centered=(comp == "x"))
    de = desc["eps_fg"] - desc["eps_bg"]
    for k, sign in ((0, -1.0), (1, 1.0)):
        i = np.nonzero(np.abs(c - p[k]) < 0.5 * w)[0]
        assert len(i) == 1
        assert grad[k] == pytest.approx(sign * de * 13 / w[i[0]], rel=1e-12)
