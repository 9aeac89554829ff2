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


def test_grating_coupler_workload_uses_the_printed_inverse_length_scale():
    # the paper prints k = 4 sqrt(2) / dx = 188.6 / um at dx = 30 nm (Fig.
    # psgc_full_jac_smh caption); the grating-coupler workloads keep k_r and
    # scale it to their 25 nm spacing
    from paper_2311_05646_amd import workloads as W
    g = _gold("paper_constants.txt")
    assert round(g["psgc_k_r"] / g["psgc_dx_um"], 1) == g["psgc_k_printed"]
    for mk in (W.make_c4, W.make_psgc):
        d = mk(with_fields=False, nside=2, nz=8)["scene"]
        dx = float(d["nodes"][0][1] - d["nodes"][0][0])
        for pr in d["prims"][1:]:
            assert pr["sigma"][0][:2] == ("sigmoid", "fixed")
            assert pr["sigma"][0][2] == pytest.approx(g["psgc_k_r"] / dx, rel=1e-15)


# ---- values of each kind that its definition in Tab. nonlinearfunctions fixes,
# chosen so that a wrong scale of the argument (e.g. sigmoid(2t), or the erf
# kind read as the normal CDF (1 + erf(t / sqrt 2)) / 2) fails

def test_sigmoid_closed_form_values():
    # (1 + e^-t)^-1 at t = +-ln 3 is 3/4 and 1/4; at ln 9, 9/10
    assert sigma("sigmoid", np.log(3.0)) == pytest.approx(0.75, abs=1e-15)
    assert sigma("sigmoid", -np.log(3.0)) == pytest.approx(0.25, abs=1e-15)
    assert sigma("sigmoid", np.log(9.0)) == pytest.approx(0.9, abs=1e-15)


def _erf_maclaurin(t, terms=60):
    # erf(t) = 2/sqrt(pi) sum_n (-1)^n t^(2n+1) / (n! (2n+1)), summed here
    # independently of any library error function
    s, term = 0.0, t
    for n in range(terms):
        s += term / (2 * n + 1)
        term *= -t * t / (n + 1)
    return 2.0 / np.sqrt(np.pi) * s


def test_erf_kind_against_published_table_and_series():
    g = _gold("erf_table.txt")
    for t in (0.5, 1.0, 2.0):
        ref = 0.5 * (1.0 + g[f"erf_{t}"])
        assert sigma("erf", t) == pytest.approx(ref, abs=1e-10)
        assert sigma("erf", t) == pytest.approx(0.5 * (1.0 + _erf_maclaurin(t)), abs=1e-14)
        assert sigma("erf", -t) == pytest.approx(0.5 * (1.0 - g[f"erf_{t}"]), abs=1e-10)


def test_piecewise_closed_form_values():
    # sin: (1 + sin t) / 2 -> 3/4 at pi/6; linear: t + 1/2 -> 3/4 at 1/4;
    # quadratic: (1/sqrt2 + t)^2 -> 1/8 at t = -1/(2 sqrt2), 7/8 at +1/(2 sqrt2)
    assert sigma("sin", np.pi / 6) == pytest.approx(0.75, abs=1e-15)
    assert sigma("sin", -np.pi / 6) == pytest.approx(0.25, abs=1e-15)
    assert sigma("linear", 0.25) == pytest.approx(0.75, abs=1e-15)
    assert sigma("linear", -0.4) == pytest.approx(0.1, abs=1e-15)
    q = 1.0 / (2.0 * np.sqrt(2.0))
    assert sigma("quadratic", -q) == pytest.approx(0.125, abs=1e-15)
    assert sigma("quadratic", q) == pytest.approx(0.875, abs=1e-15)


# the slope at the boundary, from difference quotients of sigma itself:
# sigmoid 1/4, erf 1/sqrt(pi), sin 1/2, linear 1, quadratic sqrt 2
SLOPE0 = {"sigmoid": 0.25, "erf": 1.0 / np.sqrt(np.pi), "sin": 0.5, "linear": 1.0, "quadratic": np.sqrt(2.0)}
# sigma is a cumulative distribution whose density is sigma'; its variance
# int t^2 sigma'(t) dt: logistic pi^2/3, normal with variance 1/2, the
# half-cosine density pi^2/4 - 2, uniform on [-1/2, 1/2] 1/12, the triangle of
# half-width 1/sqrt 2 1/12
VARIANCE = {"sigmoid": np.pi ** 2 / 3.0, "erf": 0.5, "sin": np.pi ** 2 / 4.0 - 2.0, "linear": 1.0 / 12.0,
            "quadratic": 1.0 / 12.0}


@pytest.mark.parametrize("kind", KINDS)
def test_slope_at_the_boundary(kind):
    h = 1e-6
    # the piecewise kinds are kinked only away from 0 (quadratic: its two
    # pieces meet at 0 with equal slope)
    fd = (sigma(kind, h) - sigma(kind, -h)) / (2 * h)
    assert fd == pytest.approx(SLOPE0[kind], rel=1e-5)


@pytest.mark.parametrize("kind", KINDS)
def test_second_moment_of_the_derivative(kind):
    # int t^2 d sigma(t), by the midpoint rule over the increments of sigma
    t = np.linspace(-60.0, 60.0, 1_200_001)
    ds = np.diff(sigma(kind, t))
    tm = 0.5 * (t[1:] + t[:-1])
    assert float(np.sum(ds)) == pytest.approx(1.0, abs=1e-12)
    assert float(np.sum(tm * tm * ds)) == pytest.approx(VARIANCE[kind], rel=1e-6)
