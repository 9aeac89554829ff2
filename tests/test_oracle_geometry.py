"""Pins of the oracle's primitives and permittivity against exact
volumetric averaging (Sec. "Approximating sub-pixel smoothing", Sec.
"Experimental choice of nonlinear function for Prop. 1"):

* cuboids with linear sigma equal the volume average exactly (the paper's
  zero-error claim), on uniform and graded lattices, in 2D and 3D;
* a 45-degree rotated square (Poly2D) with quadratic sigma, k = 1/dx, is exact
  except near its corners;
* a GeneralCartesian2D boundary at 45 degrees with quadratic sigma is exact;
  a flat one reduces to a box;
* an ellipse takes the boundary value 1/2 on its boundary; a circle's
  one-shot error against a 1000-vertex polygon is of the order the paper
  reports (order of magnitude only: the grid extent and the optimal k are in
  figures the text does not carry -- partially pinned);
* culling only drops what is below FP64 resolution, and whole-cell
  translations change nothing."""
import numpy as np
import pytest

from oracle import primitives as prm
from oracle import scene as S
from oracle import volavg as V
from oracle.lattice import axis_samples
from paper_2311_05646_amd import workloads as W


@pytest.mark.parametrize("name", ["c1", "c2_small"])
def test_cuboid_linear_sigma_zero_error(name):
    cfg = W.CONFIGS[name]()
    e = S.eps(cfg["scene"], cfg["p"])
    assert np.max(np.abs(e - V.eps_boxes(cfg["scene"], cfg["p"]))) < 1e-12


def test_cuboid_zero_error_3d_graded():
    rng = np.random.default_rng(5)
    X = W.graded_nodes(W.raised_cosine_widths(23, 12.0, 31.0))
    Y = W.uniform_nodes(17, 0.03)
    Z = W.graded_nodes(W.raised_cosine_widths(9, 10.0, 40.0, coarse_at_ends=True))
    bx = W.box(x=(W.K(X[3] + 0.004), W.P(0)), y=(W.P(1), W.K(Y[14] - 0.011)), z=(W.K(Z[2] + 0.003), W.P(2)))
    hole = W.box(x=(W.P(3), W.K(X[12] + 0.002)), y=(W.K(Y[6] + 0.007), W.K(Y[11] + 0.004)), z=(W.K(Z[3] + 0.004), W.K(Z[6] + 0.002)))
    desc = {"name": "b3", "dim": 3, "nodes": [X, Y, Z], "components": ("x", "y", "z"),
            "eps_bg": 2.0, "eps_fg": 12.0, "n_params": 4, "prims": [bx, hole],
            "tree": {"op": "difference", "children": [0, 1]}}
    p = np.array([X[19] + 0.0051, Y[2] + 0.0041, Z[7] + 0.0033, X[7] + 0.0029])
    assert np.max(np.abs(S.eps(desc, p) - V.eps_boxes(desc, p))) < 1e-12


def _plane2d(nx, dx, x0):
    X = W.uniform_nodes(nx, dx, x0)
    return X, (X[:-1], np.full(nx, dx))


def test_rotated_square_quadratic_zero_error_away_from_corners():
    dx = 0.08
    X, (xc, xw) = _plane2d(30, dx, -1.2)
    R, cx, cy = 0.7, 0.013, -0.021
    verts = [(cx, cy - R), (cx + R, cy), (cx, cy + R), (cx - R, cy)]
    prim = W.poly([W.K(v[0]) for v in verts], [W.K(v[1]) for v in verts], sig=("quadratic", "fixed", 1.0 / dx))
    pts = {"x": (xc[None, :], xw[None, :]), "y": (xc[:, None], xw[:, None]), "z": (0.0, 1.0)}
    s, _ = prm.poly(prim, [v[0] for v in verts] + [v[1] for v in verts] + [0.0, 0.0], pts)
    ref = V.clip_fraction_grid(verts, xc, xw, xc, xw)
    dist = np.min([np.hypot(xc[None, :] - vx, xc[:, None] - vy) for vx, vy in verts], axis=0)
    far = dist > 1.5 * dx
    assert np.max(np.abs(s - ref)[far]) < 1e-12
    assert np.max(np.abs(s - ref)[~far]) > 1e-4     # the corners are where the error lives
    assert np.count_nonzero((ref > 0) & (ref < 1) & far) > 20


def test_gcart_45_degree_boundary_quadratic_zero_error():
    dx = 0.05
    X, (xc, xw) = _plane2d(40, dx, 0.0)
    c = 0.3137
    xv = [0.1, 0.6, 1.1, 1.6, 1.9]
    prim = W.gcart(W.K(-5.0), W.K(5.0), xv, [W.K(x + c) for x in xv], [W.K(-9.0)] * 5,
                   sig_x=("linear", "fixed", 1.0), sig_y=("quadratic", "fixed", 1.0 / (np.sqrt(2.0) * dx)))
    vals = [-5.0, 5.0] + [x + c for x in xv] + [-9.0] * 5 + [0.0, 0.0]
    pts = {"x": (xc[None, :], xw[None, :]), "y": (xc[:, None], xw[:, None]), "z": (0.0, 1.0)}
    s, _ = prm.gcart(prim, vals, pts)
    big = [(-3.0, -3.0 + c), (3.0, 3.0 + c), (3.0, -3.0), (-3.0, -3.0)]   # region below y = x + c, CCW
    big = [(-3.0, -3.0), (3.0, -3.0), (3.0, 3.0 + c), (-3.0, -3.0 + c)]
    ref = V.clip_fraction_grid(big, xc, xw, xc, xw)
    inner = (xc[None, :] > xv[0] + dx) & (xc[None, :] < xv[-1] - dx) & np.ones((40, 1), bool)
    assert np.max(np.abs(s - ref)[inner]) < 1e-12
    assert np.count_nonzero((ref > 0) & (ref < 1) & inner) > 20


def test_gcart_flat_equals_box():
    X = W.graded_nodes(W.raised_cosine_widths(31, 15.0, 35.0))
    sx = axis_samples(X, True)
    sy = axis_samples(X, False)
    pts = {"x": (sx[0][None, :], sx[1][None, :]), "y": (sy[0][:, None], sy[1][:, None]), "z": (0.0, 1.0)}
    y0, y1, x0, x1 = 0.2013, 0.5471, 0.1017, 0.6123
    g = W.gcart(W.K(x0), W.K(x1), [0.0, 0.3, 0.9], [W.K(y1)] * 3, [W.K(y0)] * 3)
    b = W.box(x=(W.K(x0), W.K(x1)), y=(W.K(y0), W.K(y1)))
    sg, _ = prm.gcart(g, [x0, x1, y1, y1, y1, y0, y0, y0, 0, 0], pts)
    sb, _ = prm.box(b, [x0, x1, y0, y1, 0, 0], pts)
    assert np.max(np.abs(sg - sb)) < 1e-13   # (1-t) y + t y rounds


def test_ellipse_boundary_value_half():
    th = np.linspace(0, 2 * np.pi, 97)
    x0, y0, r, ax, ay = 0.31, -0.22, 0.137, 1.15, 1 / 1.15
    e = W.ellipse(W.K(x0), W.K(y0), W.K(r), aspect=(ax, ay), sig=("sigmoid", "fixed", 226.0))
    pts = {"x": (x0 + r * ax * np.cos(th), np.full(97, 0.025)), "y": (y0 + r * ay * np.sin(th), np.full(97, 0.025)),
           "z": (0.0, 1.0)}
    s, _ = prm.ellipse(e, [x0, y0, r, 0, 0], pts)
    assert np.allclose(s, 0.5, atol=1e-12)
    pts_in = {"x": (x0 + 0.5 * r * ax * np.cos(th), np.full(97, 0.025)),
              "y": (y0 + 0.5 * r * ay * np.sin(th), np.full(97, 0.025)), "z": (0.0, 1.0)}
    assert np.all(prm.ellipse(e, [x0, y0, r, 0, 0], pts_in)[0] > 0.5)


def test_circle_one_shot_mse_order_of_magnitude():
    # Circ2D R = 0.5 at (0, -0.5) (Tab. autodiffgeo example) on dx = 0.08
    dx = 0.08
    X, (xc, xw) = _plane2d(30, dx, -1.2)
    xc = xc + 0.5 * dx
    ref = V.clip_fraction_grid(V.ellipse_polygon(0.0, -0.5, 0.5, nvert=1000), xc, xw, xc, xw)
    best = {}
    for kind in ("sin", "linear", "quadratic"):
        mses = []
        for kr in np.linspace(0.5, 2.0, 31):
            e = W.ellipse(W.K(0.0), W.K(-0.5), W.K(0.5), sig=(kind, "fixed", kr / dx))
            pts = {"x": (xc[None, :], xw[None, :]), "y": (xc[:, None], xw[:, None]), "z": (0.0, 1.0)}
            s, _ = prm.ellipse(e, [0.0, -0.5, 0.5, 0, 0], pts)
            mses.append(np.mean((s - ref) ** 2))
        best[kind] = min(mses)
    # the paper reports ~2-4e-5 for the best functions on its (unstated) extent
    for kind, m in best.items():
        assert 1e-7 < m < 1e-4, (kind, m)


def test_culled_equals_brute_force():
    cfg = W.make_c4_small()
    d, p = cfg["scene"], cfg["p"]
    full = S.eps(d, p)
    rng = np.random.default_rng(0)
    for ci in range(3):
        idx = rng.choice(full[ci].size, 500, replace=False)
        assert np.max(np.abs(S.eps_at(d, p, ci, idx, cull=True) - full[ci].ravel()[idx])) < 1e-13
    g = S.sensitivity(cfg["E"], cfg["A"], cfg["omega"])
    ref = S.grad_analytic(d, p, g)
    acc = np.zeros(d["n_params"])
    for ci in range(3):
        sel = np.unique(np.concatenate([S.support_samples(d, p, i, ci) for i in range(1, len(d["prims"]))]))
        S.grad_analytic_region(d, p, lambda f, ci=ci: g[ci].ravel()[f], ci, sel, acc)
    assert np.linalg.norm(acc - ref) / np.linalg.norm(ref) < 1e-13


def test_whole_cell_translation_invariance():
    cfg = W.make_c1()
    d, p = cfg["scene"], cfg["p"]
    g = S.sensitivity(cfg["E"], cfg["A"], cfg["omega"])
    shift = 3 * 0.02
    d2 = dict(d)
    X, Y, Z = d["nodes"]
    d2["nodes"] = [X + shift, Y, Z]
    assert np.allclose(S.eps(d2, p + shift), S.eps(d, p), atol=1e-12)
    assert np.allclose(S.grad_analytic(d2, p + shift, g), S.grad_analytic(d, p, g), rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("name", ["c1", "c2_small", "c3_small", "c4_small"])
def test_eps_within_material_levels(name):
    cfg = W.CONFIGS[name]()
    e = S.eps(cfg["scene"], cfg["p"])
    lo = min(cfg["scene"]["eps_bg"], cfg["scene"]["eps_fg"])
    hi = max(cfg["scene"]["eps_bg"], cfg["scene"]["eps_fg"])
    assert e.min() >= lo - 1e-12 and e.max() <= hi + 1e-12
    assert e.min() < lo + 1e-9 and e.max() > hi - 1e-9
