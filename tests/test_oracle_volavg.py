"""Pins of oracle.volavg.supersample, the S x S midpoint quadrature of a
point-in-shape test used as an independent cross-check of the exact fill
fractions (Sec. "Experimental choice of nonlinear function for Prop. 1",
Fig. quadrature_oneshot: quadrature on a uniform sub-grid of each cell)."""
import numpy as np
import pytest

from oracle.volavg import box_fraction, clip_fraction_grid, supersample


def _lattice(X, Y):
    return 0.5 * (X[1:] + X[:-1]), np.diff(X), 0.5 * (Y[1:] + Y[:-1]), np.diff(Y)


@pytest.mark.parametrize("S", [4, 8])
def test_exact_for_a_box_on_subsample_boundaries(S):
    # non-square cells (dyadic sizes, so every boundary below is exact in
    # binary); the box's edges sit on sub-sample boundaries, so every
    # sub-sample midpoint is strictly inside or outside and the quadrature is
    # the exact covered fraction: the product of interval overlaps
    X = 0.125 * np.arange(7)
    Y = 0.0625 * np.arange(9)
    xs, xw, ys, yw = _lattice(X, Y)
    x0, x1 = 0.125 * 1 + 3 * 0.125 / S, 0.125 * 4 + 1 * 0.125 / S
    y0, y1 = 0.0625 * 2 + 1 * 0.0625 / S, 0.0625 * 6 + (S - 1) * 0.0625 / S

    def inside(x, y):
        return (x >= x0) & (x <= x1) & (y >= y0) & (y <= y1)

    got = supersample(inside, xs, xw, ys, yw, S)
    ref = box_fraction([(x0, x1), (y0, y1), None],
                       {"x": (xs[None, :], xw[None, :]), "y": (ys[:, None], yw[:, None]), "z": (0.0, 1.0)})
    assert got.shape == (len(ys), len(xs))
    assert np.array_equal(got, ref)
    assert got.max() == 1.0 and ((got > 0.0) & (got < 1.0)).sum() >= 10


def _ellipse_gon(nvert=1000):
    th = 2.0 * np.pi * np.arange(nvert) / nvert
    return np.stack([0.41 + 0.31 * np.cos(th), 0.33 + 0.23 * np.sin(th)], axis=1)


def test_converges_to_the_exact_polygon_fraction():
    # a convex 1000-gon (the paper's ground-truth curved shapes are 1000-vertex
    # polygons) against its exact clipped fraction: a cell's quadrature error
    # is at most the share of sub-cells the boundary cuts, which a boundary
    # arc shorter than the cell's perimeter keeps below 1 / S; the mean error
    # falls with S
    poly = _ellipse_gon()
    X = 0.1 * np.arange(9)
    Y = 0.08 * np.arange(9)
    xs, xw, ys, yw = _lattice(X, Y)
    exact = clip_fraction_grid(poly, xs, xw, ys, yw)
    ex, ey = poly[:, 0], poly[:, 1]
    fx, fy = np.roll(ex, -1) - ex, np.roll(ey, -1) - ey

    def inside(x, y):
        x, y = np.broadcast_arrays(x, y)
        ok = np.ones(x.shape, dtype=bool)
        for i in range(len(ex)):      # left of every counter-clockwise edge
            ok &= fx[i] * (y - ey[i]) - fy[i] * (x - ex[i]) >= 0.0
        return ok

    mean = {}
    for S in (8, 16, 32, 64):
        err = np.abs(supersample(inside, xs, xw, ys, yw, S) - exact)
        assert err.max() <= 1.0 / S
        mean[S] = err.mean()
    assert mean[64] < mean[8] / 8.0
    assert ((exact > 1e-9) & (exact < 1.0 - 1e-9)).sum() >= 20
