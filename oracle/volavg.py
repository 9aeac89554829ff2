"""The "Standard" permittivity of Sec. "Approximating sub-pixel smoothing":
eps = eps_bg + (eps_fg - eps_bg) * a_o, with a_o the fraction of a sample's
averaging box covered by the shape (scalar arithmetic average, as the paper
compares against).

* box_fraction   -- exact: product of interval overlaps.
* clip_fraction  -- exact for polygons: Sutherland-Hodgman clip of the
                    polygon against the averaging rectangle, shoelace area.
* supersample    -- S x S midpoint sub-samples of a point-in-shape test.
* eps_boxes      -- exact set algebra for box-only scenes whose unions have
                    pairwise disjoint members and whose differences have the
                    subtrahend inside the minuend (what the generators build).
* fourier_polygon, fourier_fraction_derivative -- the star-shaped region
                    r < R(theta) of eq:PSGCboundary: its polygon, and the
                    derivative of each cell's covered fraction with respect to
                    one Fourier coefficient (the h -> 0 limit of the exact
                    volume-averaged finite difference; parity unpinned beyond
                    the test against clip_fraction differences).
"""
import numpy as np

from .lattice import AXES, component_samples
from .scene import check_scene, resolve


def interval_fraction(lo, hi, c, w):
    return np.maximum(0.0, np.minimum(hi, c + 0.5 * w) - np.maximum(lo, c - 0.5 * w)) / w


def box_fraction(bounds, pts):
    """bounds: [(lo, hi) or None per axis]; pts: {axis: (center, width)}."""
    f = 1.0
    for ai, a in enumerate(AXES):
        if bounds[ai] is not None:
            f = f * interval_fraction(bounds[ai][0], bounds[ai][1], pts[a][0], pts[a][1])
    return f


def _box_bounds(prim, vals):
    return [(vals[2 * i], vals[2 * i + 1]) if prim["bounded"][i] else None for i in range(3)]


def _overlap(b1, b2):
    for i in range(3):
        if b1[i] is None or b2[i] is None:
            continue
        if min(b1[i][1], b2[i][1]) <= max(b1[i][0], b2[i][0]):
            return False
    return True


def _inside(inner, outer):
    for i in range(3):
        if outer[i] is None:
            continue
        if inner[i] is None or inner[i][0] < outer[i][0] or inner[i][1] > outer[i][1]:
            return False
    return True


def _node_boxes(node, desc, vals):
    if isinstance(node, (int, np.integer)):
        pr = desc["prims"][int(node)]
        if pr["type"] != "box":
            raise ValueError("eps_boxes handles box primitives only")
        return [_box_bounds(pr, vals[int(node)])]
    out = []
    for ch in node["children"]:
        out += _node_boxes(ch, desc, vals)
    return out


def _fraction(node, desc, vals, pts):
    if isinstance(node, (int, np.integer)):
        return box_fraction(_box_bounds(desc["prims"][int(node)], vals[int(node)]), pts)
    op = node["op"]
    if op == "union":
        groups = [_node_boxes(ch, desc, vals) for ch in node["children"]]
        for i in range(len(groups)):
            for j in range(i + 1, len(groups)):
                if any(_overlap(a, b) for a in groups[i] for b in groups[j]):
                    raise ValueError("union members overlap; exact set algebra needs disjoint members")
        return sum(_fraction(ch, desc, vals, pts) for ch in node["children"])
    if op == "difference":
        a, b = node["children"]
        outer = _node_boxes(a, desc, vals)
        if len(outer) != 1:
            raise ValueError("difference minuend must be a single box")
        for bb in _node_boxes(b, desc, vals):
            if not _inside(bb, outer[0]):
                raise ValueError("difference subtrahend must lie inside the minuend")
        return _fraction(a, desc, vals, pts) - _fraction(b, desc, vals, pts)
    # intersection of boxes is a box
    bl = [_node_boxes(ch, desc, vals) for ch in node["children"]]
    if any(len(b) != 1 for b in bl):
        raise ValueError("intersection of single boxes only")
    inter = []
    for i in range(3):
        iv = [b[0][i] for b in bl if b[0][i] is not None]
        inter.append(None if not iv else (max(v[0] for v in iv), min(v[1] for v in iv)))
    inter = [None if v is None else (v[0], max(v[0], v[1])) for v in inter]
    return box_fraction(inter, pts)


def eps_boxes(desc, p):
    """Exact volumetric average of a box-only scene, (C, Nz, Ny, Nx)."""
    check_scene(desc)
    vals = resolve(desc, p)
    de = desc["eps_fg"] - desc["eps_bg"]
    out = []
    shp = {"x": (1, 1, -1), "y": (1, -1, 1), "z": (-1, 1, 1)}
    for comp in desc["components"]:
        smp = component_samples(desc, comp)
        pts = {a: (smp[a][0].reshape(shp[a]), smp[a][1].reshape(shp[a])) for a in AXES}
        X, Y, Z = desc["nodes"]
        f = np.broadcast_to(_fraction(desc["tree"], desc, vals, pts),
                            (len(Z) - 1, len(Y) - 1, len(X) - 1))
        out.append(desc["eps_bg"] + de * f)
    return np.stack(out)


# ----------------------------------------------------------------- polygons
def _clip(poly, axis, bound, keep_greater):
    """Clip polygon (list of (x, y)) by the half-plane coord[axis] >= bound
    (or <= bound)."""
    out = []
    n = len(poly)
    for i in range(n):
        cur, nxt = poly[i], poly[(i + 1) % n]
        ci = (cur[axis] >= bound) if keep_greater else (cur[axis] <= bound)
        ni = (nxt[axis] >= bound) if keep_greater else (nxt[axis] <= bound)
        if ci:
            out.append(cur)
        if ci != ni:
            t = (bound - cur[axis]) / (nxt[axis] - cur[axis])
            out.append((cur[0] + t * (nxt[0] - cur[0]), cur[1] + t * (nxt[1] - cur[1])))
    return out


def shoelace(poly):
    if len(poly) < 3:
        return 0.0
    a = 0.0
    for i in range(len(poly)):
        x0, y0 = poly[i]
        x1, y1 = poly[(i + 1) % len(poly)]
        a += x0 * y1 - x1 * y0
    return 0.5 * a


def clip_fraction(poly, xc, xw, yc, yw):
    """Area of (polygon, CCW) inside the rectangle centered at (xc, yc) with
    sides xw, yw, over the rectangle area (convex or concave polygon)."""
    q = [tuple(v) for v in poly]
    q = _clip(q, 0, xc - 0.5 * xw, True)
    if q:
        q = _clip(q, 0, xc + 0.5 * xw, False)
    if q:
        q = _clip(q, 1, yc - 0.5 * yw, True)
    if q:
        q = _clip(q, 1, yc + 0.5 * yw, False)
    return shoelace(q) / (xw * yw) if q else 0.0


def clip_fraction_grid(poly, xs, xw, ys, yw):
    """clip_fraction for every (y, x) sample of a 2D lattice -> (Ny, Nx)."""
    poly = np.asarray(poly, dtype=np.float64)
    bx0, bx1 = poly[:, 0].min(), poly[:, 0].max()
    by0, by1 = poly[:, 1].min(), poly[:, 1].max()
    out = np.zeros((len(ys), len(xs)))
    pl = [tuple(v) for v in poly]
    for j in range(len(ys)):
        if ys[j] + 0.5 * yw[j] < by0 or ys[j] - 0.5 * yw[j] > by1:
            continue
        for i in range(len(xs)):
            if xs[i] + 0.5 * xw[i] < bx0 or xs[i] - 0.5 * xw[i] > bx1:
                continue
            out[j, i] = clip_fraction(pl, xs[i], xw[i], ys[j], yw[j])
    return out


def ellipse_polygon(x0, y0, r, ax=1.0, ay=1.0, nvert=1000):
    """Vertices (CCW) on the ellipse ((x-x0)/(r ax))^2 + ((y-y0)/(r ay))^2 = 1;
    the paper's ground-truth curved shapes are 1000-vertex polygons."""
    th = 2.0 * np.pi * np.arange(nvert) / nvert
    return np.stack([x0 + r * ax * np.cos(th), y0 + r * ay * np.sin(th)], axis=1)


def supersample(inside, xs, xw, ys, yw, S):
    """Fraction of S x S midpoint sub-samples of each cell for which
    inside(x, y) holds -> (Ny, Nx)."""
    u = (np.arange(S) + 0.5) / S - 0.5
    X = xs[None, :, None, None] + xw[None, :, None, None] * u[None, None, None, :]
    Y = ys[:, None, None, None] + yw[:, None, None, None] * u[None, None, :, None]
    return inside(X, Y).mean(axis=(2, 3))


def fourier_radius(R0, cs, ss, th):
    """R(theta) = R0 + sum_n c_n cos(n theta + pi) + s_n sin(n theta + pi)."""
    R = R0 + 0.0 * th
    for n in range(1, len(cs) + 1):
        R = R + cs[n - 1] * np.cos(n * th + np.pi) + ss[n - 1] * np.sin(n * th + np.pi)
    return R


def fourier_polygon(x0, y0, R0, cs, ss, nvert=1000):
    """Vertices (CCW) of r = R(theta) about (x0, y0) at nvert equal angles."""
    th = 2.0 * np.pi * np.arange(nvert) / nvert
    R = fourier_radius(R0, cs, ss, th)
    return np.stack([x0 + R * np.cos(th), y0 + R * np.sin(th)], axis=1)


def fourier_fraction_derivative(x0, y0, R0, cs, ss, which, xnodes, ynodes, nsamp=200000):
    """d (covered fraction of each cell) / d coefficient for the region
    r < R(theta): the area inside a cell changes at the boundary points that
    lie in it, by R(theta) dR/dcoef dtheta (area = 1/2 int R^2 dtheta), summed
    with the midpoint rule over nsamp angles and divided by the cell area.
    which = ("c", n) or ("s", n) or ("R0", 0).  -> (Ny, Nx) on the cell lattice
    given by the node arrays."""
    th = 2.0 * np.pi * (np.arange(nsamp) + 0.5) / nsamp
    R = fourier_radius(R0, cs, ss, th)
    kind, n = which
    if kind == "R0":
        dR = np.ones_like(th)
    elif kind == "c":
        dR = np.cos(n * th + np.pi)
    else:
        dR = np.sin(n * th + np.pi)
    x, y = x0 + R * np.cos(th), y0 + R * np.sin(th)
    ix = np.searchsorted(xnodes, x, side="right") - 1
    iy = np.searchsorted(ynodes, y, side="right") - 1
    nx, ny = len(xnodes) - 1, len(ynodes) - 1
    ok = (ix >= 0) & (ix < nx) & (iy >= 0) & (iy < ny)
    out = np.zeros((ny, nx))
    np.add.at(out, (iy[ok], ix[ok]), (R * dR)[ok] * (2.0 * np.pi / nsamp))
    area = np.diff(ynodes)[:, None] * np.diff(xnodes)[None, :]
    return out / area
