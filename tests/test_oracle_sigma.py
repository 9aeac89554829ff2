"""Pins of oracle.sigma against what the paper fixes: the [0,1]-bounded,
monotone building block with value 1/2 on boundaries (Sec. "AutoDiffGeo",
Tab. nonlinearfunctions), and the volumetric-averaging identities of
eq:linear / eq:quadratic and eq:dlinear / eq:dquadratic computed here by
exact polygon clipping (an independent computation)."""
import os

import numpy as np
import pytest

from oracle.sigma import KINDS, dsigma, sigma
from oracle.volavg import clip_fraction

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


T = np.linspace(-8.0, 8.0, 4001)


@pytest.mark.parametrize("kind", KINDS)
def test_boundary_value_and_symmetry(kind):
    g = _gold("paper_constants.txt")
    assert sigma(kind, 0.0) == pytest.approx(g["boundary_value"], abs=1e-15)
    assert np.allclose(sigma(kind, T) + sigma(kind, -T), 1.0, atol=1e-15)


@pytest.mark.parametrize("kind", KINDS)
def test_bounded_monotone_limits(kind):
    s = sigma(kind, T)
    assert s.min() >= 0.0 and s.max() <= 1.0
    assert np.all(np.diff(s) >= 0.0)
    assert sigma(kind, -60.0) < 1e-20 and sigma(kind, 60.0) > 1.0 - 1e-15


@pytest.mark.parametrize("kind", ["sin", "linear", "quadratic"])
def test_compact_breakpoints(kind):
    g = _gold("paper_constants.txt")
    b = g[f"{kind}_break"]
    assert sigma(kind, b + 1e-12) == 1.0 and sigma(kind, -b - 1e-12) == 0.0
    assert sigma(kind, b - 1e-3) < 1.0 and sigma(kind, -b + 1e-3) > 0.0


@pytest.mark.parametrize("kind", KINDS)
def test_derivative_matches_difference_quotient(kind):
    t = np.linspace(-3.0, 3.0, 601) + 1.234e-3      # avoids every breakpoint
    h = 1e-6
    fd = (sigma(kind, t + h) - sigma(kind, t - h)) / (2 * h)
    assert np.allclose(dsigma(kind, t), fd, atol=1e-8)


def _half_plane_fraction(x, angle_deg, dx):
    """Covered fraction of the cell [-dx/2, dx/2]^2 by the half-plane whose
    boundary has unit normal n (pointing into the shape) at the given angle,
    with the cell center at signed distance x inside the shape."""
    th = np.radians(angle_deg)
    n = np.array([np.cos(th), np.sin(th)])
    tvec = np.array([-n[1], n[0]])
    p0 = -x * n                                   # a point on the boundary
    L = 100.0 * dx
    poly = [p0 - L * tvec, p0 - L * tvec + L * n, p0 + L * tvec + L * n, p0 + L * tvec]  # counter-clockwise
    return clip_fraction([tuple(v) for v in poly], 0.0, dx, 0.0, dx)


@pytest.mark.parametrize("dx", [0.08, 0.025])
def test_linear_is_grid_parallel_volume_average(dx):
    # eq:linear: a_o(x) = x/dx + 1/2 on |x| <= dx/2 equals linear sigma with k = 1/dx
    for x in np.linspace(-0.7 * dx, 0.7 * dx, 57):
        assert sigma("linear", x / dx) == pytest.approx(_half_plane_fraction(x, 0.0, dx), abs=1e-12)


@pytest.mark.parametrize("dx", [0.08, 0.025])
def test_quadratic_is_45_degree_volume_average(dx):
    # eq:quadratic equals quadratic sigma with k = 1/dx
    for x in np.linspace(-0.8 * dx, 0.8 * dx, 57):
        assert sigma("quadratic", x / dx) == pytest.approx(_half_plane_fraction(x, 45.0, dx), abs=1e-12)


def test_volume_average_derivatives():
    # eq:dlinear / eq:dquadratic: d a_o / dx = k * sigma'(k x) with k = 1/dx,
    # against difference quotients of the clipped areas
    dx, h = 0.05, 1e-7
    for x in np.linspace(-0.3 * dx, 0.3 * dx, 13) + 1e-5:
        for ang, kind in ((0.0, "linear"), (45.0, "quadratic")):
            fd = (_half_plane_fraction(x + h, ang, dx) - _half_plane_fraction(x - h, ang, dx)) / (2 * h)
            assert dsigma(kind, x / dx) / dx == pytest.approx(fd, rel=1e-6)


def test_paper_printed_inverse_length_scale():
    g = _gold("paper_constants.txt")
    assert g["psgc_k_r"] == pytest.approx(4 * np.sqrt(2), rel=1e-15)
    assert round(g["psgc_k_r"] / g["psgc_dx_um"], 1) == g["psgc_k_printed"]
