"""Pins of the oracle's Fourier polar primitive (GeneralPolar2D with the
radius of eq:PSGCboundary):

* with every Fourier coefficient zero it is Circ2D (the oracle's ellipse with
  unit aspect), value and partials;
* on the rays theta = 0 and theta = pi/2 the boundary sits where the radius
  formula, evaluated by hand, puts it (sigma = 1/2 there);
* rotating the sample about the center by phi and the coefficients by n phi
  (R'(theta) = R(theta - phi)) leaves the value unchanged, in every quadrant;
* every analytic partial matches central differences of the value."""
import numpy as np
import pytest

from oracle import primitives as prm
from paper_2311_05646_amd import workloads as W

SIG = ("sigmoid", "fixed", 60.0)


def _pts(x, y, w=0.02):
    x, y = np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64)
    return {"x": (x, np.full_like(x, w)), "y": (y, np.full_like(y, w)), "z": (np.zeros_like(x), np.ones_like(x))}


def _vals(pr):
    return [f[0] for f in pr["fields"]]


def test_zero_coefficients_is_circ2d():
    rng = np.random.default_rng(1)
    x, y = rng.uniform(-0.4, 0.4, 500), rng.uniform(-0.4, 0.4, 500)
    pol = W.polar(W.K(0.03), W.K(-0.02), W.K(0.21), [W.K(0.0)] * 4, [W.K(0.0)] * 4, sig=SIG)
    ell = W.ellipse(W.K(0.03), W.K(-0.02), W.K(0.21), sig=SIG)
    fp, pp = prm.polar(pol, _vals(pol), _pts(x, y))
    fe, pe = prm.ellipse(ell, _vals(ell), _pts(x, y))
    assert np.max(np.abs(fp - fe)) < 1e-14
    dp, de = dict((i, d) for i, d in pp), dict((i, d) for i, d in pe)
    for i in range(3):            # x0, y0, R0 <-> x0, y0, r
        assert np.max(np.abs(dp[i] - de[i])) < 1e-10 * max(1.0, np.max(np.abs(de[i])))


@pytest.mark.parametrize("kind", ["sigmoid", "linear"])
def test_boundary_on_axes(kind):
    # N = 3, c_2 = a, s_3 = b: R(0) = R0 - a, R(pi/2) = R0 + a + b
    R0, a, b = 0.2, 0.03, 0.017
    x0, y0 = 0.1, -0.05
    cs = [W.K(0.0), W.K(a), W.K(0.0)]
    ss = [W.K(0.0), W.K(0.0), W.K(b)]
    pr = W.polar(W.K(x0), W.K(y0), W.K(R0), cs, ss, sig=(kind, "fixed", 60.0))
    f, _ = prm.polar(pr, _vals(pr), _pts([x0 + R0 - a, x0], [y0, y0 + R0 + a + b]))
    assert np.max(np.abs(f - 0.5)) < 1e-12


def test_rotation_covariance():
    rng = np.random.default_rng(2)
    N = 5
    c = rng.normal(0, 0.01, N)
    s = rng.normal(0, 0.01, N)
    x0, y0, R0 = 0.02, 0.01, 0.18
    x = x0 + rng.uniform(-0.25, 0.25, 400)
    y = y0 + rng.uniform(-0.25, 0.25, 400)
    pr = W.polar(W.K(x0), W.K(y0), W.K(R0), [W.K(v) for v in c], [W.K(v) for v in s], sig=SIG)
    f0, _ = prm.polar(pr, _vals(pr), _pts(x, y))
    for phi in (0.7, 2.1, -2.6, np.pi):
        n = np.arange(1, N + 1)
        c2 = c * np.cos(n * phi) - s * np.sin(n * phi)
        s2 = c * np.sin(n * phi) + s * np.cos(n * phi)
        xr = x0 + np.cos(phi) * (x - x0) - np.sin(phi) * (y - y0)
        yr = y0 + np.sin(phi) * (x - x0) + np.cos(phi) * (y - y0)
        pr2 = W.polar(W.K(x0), W.K(y0), W.K(R0), [W.K(v) for v in c2], [W.K(v) for v in s2], sig=SIG)
        f1, _ = prm.polar(pr2, _vals(pr2), _pts(xr, yr))
        assert np.max(np.abs(f1 - f0)) < 1e-12, phi


@pytest.mark.parametrize("kind", ["sigmoid", "erf", "sin", "quadratic"])
def test_partials_match_central_differences(kind):
    rng = np.random.default_rng(3)
    N = 4
    vals0 = [0.01, -0.02, 0.2] + list(rng.normal(0, 0.008, 2 * N)) + [0.0, 0.0]
    pr = W.polar(W.K(0), W.K(0), W.K(0), [W.K(0)] * N, [W.K(0)] * N, sig=(kind, "fixed", 25.0))
    # samples near the boundary, away from the center
    th = rng.uniform(-np.pi, np.pi, 300)
    rr = 0.2 + rng.uniform(-0.04, 0.04, 300)
    pts = _pts(0.01 + rr * np.cos(th), -0.02 + rr * np.sin(th))
    _, parts = prm.polar(pr, vals0, pts)
    h = 1e-6
    for fi, d in parts[:3 + 2 * N]:
        vp, vm = list(vals0), list(vals0)
        vp[fi] += h
        vm[fi] -= h
        fd = (prm.polar(pr, vp, pts)[0] - prm.polar(pr, vm, pts)[0]) / (2 * h)
        assert np.max(np.abs(fd - d)) < 1e-5 * max(1.0, np.max(np.abs(d))), fi
