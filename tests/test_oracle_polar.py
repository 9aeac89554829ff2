"""Pins of the oracle's Fourier polar primitive (GeneralPolar2D with the
radius of eq:PSGCboundary):

* with every Fourier coefficient zero it is Circ2D (the oracle's ellipse with
  unit aspect), value and partials;
* on the rays theta = 0 and theta = pi/2 the boundary sits where the radius
  formula, evaluated by hand, puts it (sigma = 1/2 there);
* rotating the sample about the center by phi and the coefficients by n phi
  (R'(theta) = R(theta - phi)) leaves the value unchanged, in every quadrant;
* every analytic partial matches central differences of the value;
of Polar2D (Tab. autodiffgeo, sigma_k(R (1 + delta cos(alpha theta)) - r)):
with delta = 0 it is Circ2D, value and the x0, y0, R partials; on the rays
theta = 0 and theta = pi / alpha the boundary sits at R (1 + delta) and
R (1 - delta); it is the Fourier primitive with R0 = R and c_alpha = -R delta,
in value; its partials match central differences;
and of the taper's sine-series boundary (eq:taper_boundary): with no sine
terms and equal end widths it is a box; at mid-length (envelope 1) the
boundary sits where the series, evaluated by hand, puts it; its partials
match central differences."""
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


# ---- Polar2D (Tab. autodiffgeo)
def test_polar2d_zero_delta_is_circ2d():
    rng = np.random.default_rng(11)
    x, y = rng.uniform(-0.5, 0.5, 500), rng.uniform(-0.5, 0.5, 500)
    p2 = W.polar2d(W.K(0.03), W.K(-0.02), W.K(0.31), W.K(0.0), 4, sig=SIG)
    ell = W.ellipse(W.K(0.03), W.K(-0.02), W.K(0.31), sig=SIG)
    f2, q2 = prm.polar2d(p2, _vals(p2), _pts(x, y))
    fe, qe = prm.ellipse(ell, _vals(ell), _pts(x, y))
    assert np.max(np.abs(f2 - fe)) < 1e-14
    d2, de = dict(q2), dict(qe)
    for i in range(3):            # x0, y0, R <-> x0, y0, r
        assert np.max(np.abs(d2[i] - de[i])) < 1e-10 * max(1.0, np.max(np.abs(de[i])))


@pytest.mark.parametrize("kind", ["sigmoid", "linear"])
@pytest.mark.parametrize("alpha", [3, 4])
def test_polar2d_boundary_on_rays(kind, alpha):
    # theta = 0: R (1 + delta); theta = pi / alpha: R (1 - delta); the paper's example R = 0.5, delta = 0.2
    R, d, x0, y0 = 0.5, 0.2, 0.07, -0.04
    pr = W.polar2d(W.K(x0), W.K(y0), W.K(R), W.K(d), alpha, sig=(kind, "fixed", 60.0))
    th = np.pi / alpha
    xs = [x0 + R * (1 + d), x0 + R * (1 - d) * np.cos(th)]
    ys = [y0, y0 + R * (1 - d) * np.sin(th)]
    f, _ = prm.polar2d(pr, _vals(pr), _pts(xs, ys))
    assert np.max(np.abs(f - 0.5)) < 1e-12


def test_polar2d_is_the_fourier_radius_with_one_product_coefficient():
    rng = np.random.default_rng(12)
    R, d, a = 0.27, -0.13, 5
    x, y = 0.01 + rng.uniform(-0.4, 0.4, 600), -0.02 + rng.uniform(-0.4, 0.4, 600)
    p2 = W.polar2d(W.K(0.01), W.K(-0.02), W.K(R), W.K(d), a, sig=SIG)
    cs = [W.K(0.0)] * a
    cs[a - 1] = W.K(-R * d)           # R(theta) = R0 - c_a cos(a theta) (the pi shift)
    pf = W.polar(W.K(0.01), W.K(-0.02), W.K(R), cs, [W.K(0.0)] * a, sig=SIG)
    f2, _ = prm.polar2d(p2, _vals(p2), _pts(x, y))
    ff, _ = prm.polar(pf, _vals(pf), _pts(x, y))
    assert np.max(np.abs(f2 - ff)) < 1e-13


@pytest.mark.parametrize("kind", ["sigmoid", "erf", "sin", "quadratic"])
def test_polar2d_partials_match_central_differences(kind):
    rng = np.random.default_rng(13)
    vals0 = [0.01, -0.02, 0.3, 0.18, 0.0, 0.0]
    pr = W.polar2d(W.K(0), W.K(0), W.K(0), W.K(0), 4, sig=(kind, "fixed", 25.0))
    th = rng.uniform(-np.pi, np.pi, 300)
    rr = 0.3 * (1 + 0.18 * np.cos(4 * th)) + rng.uniform(-0.05, 0.05, 300)
    pts = _pts(0.01 + rr * np.cos(th), -0.02 + rr * np.sin(th))
    _, parts = prm.polar2d(pr, vals0, pts)
    h = 1e-6
    for fi, dd in parts[:4]:
        vp, vm = list(vals0), list(vals0)
        vp[fi] += h
        vm[fi] -= h
        fd = (prm.polar2d(pr, vp, pts)[0] - prm.polar2d(pr, vm, pts)[0]) / (2 * h)
        assert np.max(np.abs(fd - dd)) < 1e-5 * max(1.0, np.max(np.abs(dd))), fi


# ---- the taper's sine-series boundary (eq:taper_boundary, eq:taper_eps)
def _series(vs, w_in=0.5, w_out=0.5, kind="linear"):
    return W.series(W.K(-1.0), W.K(5.0), [W.K(v) for v in vs], x0=0.3, L=2.0, w_in=w_in, w_out=w_out, yc=0.4,
                    sig_x=(kind, "local", 1.0), sig_y=(kind, "local", 1.0))


def test_series_straight_guide_is_a_box():
    # no sine terms and equal widths: a box yc +- w/2 over [xs, xe]
    rng = np.random.default_rng(4)
    x, y = rng.uniform(-1.5, 5.5, 600), rng.uniform(-0.2, 1.0, 600)
    pr = _series([0.0, 0.0, 0.0], w_in=0.5, w_out=0.5)
    bx = W.box(x=(W.K(-1.0), W.K(5.0)), y=(W.K(0.4 - 0.25), W.K(0.4 + 0.25)))
    pts = _pts(x, y, 0.03)
    fs, _ = prm.series(pr, _vals(pr), pts)
    fb, _ = prm.box(bx, _vals(bx), pts)
    assert np.max(np.abs(fs - fb)) < 1e-14


@pytest.mark.parametrize("kind", ["linear", "sigmoid"])
def test_series_boundary_at_mid_length(kind):
    # x = x0 + L/2: envelope 1, sin(i pi / 2) = 1, 0, -1, 0, 1: f = ramp + v1 - v3 + v5
    vs = [0.03, 0.02, -0.011, 0.05, 0.007]
    w_in, w_out = 0.5, 1.3
    f = w_in / 2 + (w_out - w_in) / 4 + vs[0] - vs[2] + vs[4]
    pr = _series(vs, w_in, w_out, kind)
    val, _ = prm.series(pr, _vals(pr), _pts([1.3, 1.3], [0.4 + f, 0.4 - f], 0.03))
    assert np.max(np.abs(val - 0.5)) < 1e-12


def test_series_partials_match_central_differences():
    rng = np.random.default_rng(6)
    K = 7
    vals0 = [0.0, 4.0] + list(rng.normal(0, 0.02, K)) + [0.0, 0.0]
    pr = _series([0.0] * K, 0.5, 1.1, "sigmoid")
    x = rng.uniform(0.0, 4.2, 400)
    y = 0.4 + rng.choice([-1.0, 1.0], 400) * (0.25 + 0.3 * (x - 0.3) / 2.0) + rng.uniform(-0.08, 0.08, 400)
    pts = _pts(x, y, 0.03)
    _, parts = prm.series(pr, vals0, pts)
    h = 1e-6
    for fi, d in parts[:2 + K]:
        vp, vm = list(vals0), list(vals0)
        vp[fi] += h
        vm[fi] -= h
        fd = (prm.series(pr, vp, pts)[0] - prm.series(pr, vm, pts)[0]) / (2 * h)
        assert np.max(np.abs(fd - d)) < 1e-5 * max(1.0, np.max(np.abs(d))), fi


def test_fourier_fraction_derivative_matches_clipped_differences():
    # the boundary-integral derivative of each cell's covered fraction equals
    # central differences of the exact polygon clip (fine polygon, small h)
    from oracle import volavg as V
    xn = np.linspace(-0.3, 0.3, 13)
    yn = np.linspace(-0.3, 0.3, 13)
    xs, ys = 0.5 * (xn[1:] + xn[:-1]), 0.5 * (yn[1:] + yn[:-1])
    xw, yw = np.diff(xn), np.diff(yn)
    cs, ss = [0.01, -0.006, 0.004], [0.003, 0.005, -0.002]
    h = 1e-4
    for which, idx in ((("c", 1), 0), (("s", 2), 1), (("R0", 0), None)):
        def frac(dv):
            c2, s2, r0 = list(cs), list(ss), 0.17
            if which[0] == "c":
                c2[idx] += dv
            elif which[0] == "s":
                s2[idx] += dv
            else:
                r0 += dv
            return V.clip_fraction_grid(V.fourier_polygon(0.01, -0.02, r0, c2, s2, 3000), xs, xw, ys, yw)
        fd = (frac(h) - frac(-h)) / (2 * h)
        an = V.fourier_fraction_derivative(0.01, -0.02, 0.17, cs, ss, which, xn, yn, 400000)
        assert np.max(np.abs(fd - an)) < 2e-3 * np.max(np.abs(fd)), which
