"""AutoDiffGeo primitives (Tab. autodiffgeo, Sec. "AutoDiffGeo") with their
analytic partial derivatives, in FP64, sampled once per sample at its center
("one-shot sampling", Sec. "Experimental choice of nonlinear function for
Prop. 1").

Every function takes broadcastable sample arrays ``pts`` =
{"x": (center, width), "y": ..., "z": ...} and the resolved field values of
one primitive, and returns (s, partials) where ``partials`` is a list of
(field_index, d s / d field) pairs; field_index is an int, or an int array
of the shape of s when the field a sample depends on varies from sample to
sample (the vertices of a piecewise boundary).

k modes (a reading: the paper only uses k = k_r / dx on uniform grids):
"local" gives k = k_r / width of the sample along the argument's axis,
"fixed" uses k as given.  Radial and oblique arguments must be "fixed".
"""
import numpy as np

from .sigma import dsigma, sigma


def kval(sig, width):
    kind, kmode, k = sig
    if kmode == "local":
        return k / width
    if kmode == "fixed":
        return k * np.ones_like(width)
    raise ValueError(kmode)


def rect1d(sig, c, w, lo, hi):
    """Rect1D(x, x0, x1) = sigma_k(x - x0) * sigma_k(x1 - x) and its partials
    with respect to x0 and x1."""
    kind = sig[0]
    k = kval(sig, w)
    ta = k * (c - lo)
    tb = k * (hi - c)
    sa, sb = sigma(kind, ta), sigma(kind, tb)
    return sa * sb, -k * dsigma(kind, ta) * sb, k * sa * dsigma(kind, tb)


def _z_factor(prim, vals, pts, zf0):
    """Extrusion along z (a Rect1D in z, the 'planarity transformation'),
    or 1 when the primitive is unbounded along z."""
    if not prim["bounded"][2]:
        return 1.0, []
    zc, zw = pts["z"]
    v, dlo, dhi = rect1d(prim["sigma"][2], zc, zw, vals[zf0], vals[zf0 + 1])
    return v, [(zf0, dlo), (zf0 + 1, dhi)]


def box(prim, vals, pts):
    """RectdD: product of Rect1D over the bounded axes; fields x0 x1 y0 y1 z0 z1."""
    facs, parts = [], []
    for ai, a in enumerate("xyz"):
        if prim["bounded"][ai]:
            c, w = pts[a]
            v, dlo, dhi = rect1d(prim["sigma"][ai], c, w, vals[2 * ai], vals[2 * ai + 1])
            facs.append(v)
            parts.append((2 * ai, dlo, ai))
            parts.append((2 * ai + 1, dhi, ai))
        else:
            facs.append(1.0)
    s = facs[0] * facs[1] * facs[2]
    out = []
    for fi, d, ai in parts:
        other = 1.0
        for aj in range(3):
            if aj != ai:
                other = other * facs[aj]
        out.append((fi, d * other))
    return s, out


def ellipse(prim, vals, pts):
    """Circ2D with an aspect-ratio transform: sigma_k(r - rho_e), rho_e =
    sqrt(((x-x0)/ax)^2 + ((y-y0)/ay)^2); fields x0 y0 r z0 z1."""
    x0, y0, r = vals[0], vals[1], vals[2]
    ax, ay = prim["consts"][0], prim["consts"][1]
    (xc, xw), (yc, _) = pts["x"], pts["y"]
    dx, dy = xc - x0, yc - y0
    rho = np.sqrt((dx / ax) ** 2 + (dy / ay) ** 2)
    k = kval(prim["sigma"][0], xw)
    t = k * (r - rho)
    f = sigma(prim["sigma"][0][0], t)
    df = k * dsigma(prim["sigma"][0][0], t)          # d f / d (r - rho)
    safe = np.where(rho > 0.0, rho, 1.0)
    drho_dx0 = np.where(rho > 0.0, -dx / (ax * ax * safe), 0.0)
    drho_dy0 = np.where(rho > 0.0, -dy / (ay * ay * safe), 0.0)
    zv, zparts = _z_factor(prim, vals, pts, 3)
    out = [(0, -df * drho_dx0 * zv), (1, -df * drho_dy0 * zv), (2, df * zv)]
    out += [(fi, f * d) for fi, d in zparts]
    return f * zv, out


def poly(prim, vals, pts):
    """Poly2D (convex, vertices counter-clockwise): product over edges of
    Step2D = sigma_k(n . (r - r_i)) with n the inward (left) unit normal of
    edge i -> i+1; fields x_1..x_N y_1..y_N z0 z1."""
    N = prim["nvert"]
    xs, ys = vals[:N], vals[N:2 * N]
    (xc, xw), (yc, _) = pts["x"], pts["y"]
    kind = prim["sigma"][0][0]
    k = kval(prim["sigma"][0], xw)
    sig_i, dsig_i, dd = [], [], []
    for i in range(N):
        j = (i + 1) % N
        ex, ey = xs[j] - xs[i], ys[j] - ys[i]
        L = np.hypot(ex, ey)
        wx, wy = xc - xs[i], yc - ys[i]
        d = (ex * wy - ey * wx) / L
        t = k * d
        sig_i.append(sigma(kind, t))
        dsig_i.append(k * dsigma(kind, t))
        # d(d)/d(vertex coords): d = c / L with c = e x w
        dd.append({
            i: (((ey - wy) / L) + d * ex / (L * L), ((wx - ex) / L) + d * ey / (L * L)),
            j: ((wy / L) - d * ex / (L * L), (-wx / L) - d * ey / (L * L)),
        })
    f = np.ones(np.broadcast(xc, yc, xw).shape)
    for s in sig_i:
        f = f * s
    zv, zparts = _z_factor(prim, vals, pts, 2 * N)
    acc_x = [0.0] * N
    acc_y = [0.0] * N
    for i in range(N):
        other = 1.0
        for j in range(N):
            if j != i:
                other = other * sig_i[j]
        g = dsig_i[i] * other * zv
        for v, (ddx, ddy) in dd[i].items():
            acc_x[v] = acc_x[v] + g * ddx
            acc_y[v] = acc_y[v] + g * ddy
    out = [(v, acc_x[v]) for v in range(N)] + [(N + v, acc_y[v]) for v in range(N)]
    out += [(fi, f * d) for fi, d in zparts]
    return f * zv, out


def gcart(prim, vals, pts):
    """Two-sided GeneralCartesian2D: sigma_k(f+(x) - y) * sigma_k(y - f-(x))
    times Rect1D(x; xs, xe), with f+- piecewise linear through the vertices
    (x_j, y+-_j) and held constant beyond the end vertices.
    Fields xs xe y+_1..y+_M y-_1..y-_M z0 z1; consts x_1..x_M."""
    M = prim["nvert"]
    xv = np.asarray(prim["consts"], dtype=np.float64)
    yp = np.asarray(vals[2:2 + M], dtype=np.float64)
    ym = np.asarray(vals[2 + M:2 + 2 * M], dtype=np.float64)
    (xc, xw), (yc, yw) = pts["x"], pts["y"]
    xc_b = np.broadcast_to(xc, np.broadcast(xc, yc).shape)
    j = np.clip(np.searchsorted(xv, xc_b, side="right") - 1, 0, M - 2)
    t = np.clip((xc_b - xv[j]) / (xv[j + 1] - xv[j]), 0.0, 1.0)
    fp = (1.0 - t) * yp[j] + t * yp[j + 1]
    fm = (1.0 - t) * ym[j] + t * ym[j + 1]
    sy = prim["sigma"][1]
    ky = kval(sy, yw)
    up, um = ky * (fp - yc), ky * (yc - fm)
    sp, sm = sigma(sy[0], up), sigma(sy[0], um)
    dsp, dsm = ky * dsigma(sy[0], up), ky * dsigma(sy[0], um)
    rx, drx0, drx1 = rect1d(prim["sigma"][0], xc, xw, vals[0], vals[1])
    zv, zparts = _z_factor(prim, vals, pts, 2 + 2 * M)
    fy = sp * sm
    f = rx * fy
    gp = rx * dsp * sm * zv          # d s / d f+
    gm = -rx * sp * dsm * zv         # d s / d f-
    out = [(0, drx0 * fy * zv), (1, drx1 * fy * zv),
           (2 + j, gp * (1.0 - t)), (3 + j, gp * t),
           (2 + M + j, gm * (1.0 - t)), (3 + M + j, gm * t)]
    out += [(fi, f * d) for fi, d in zparts]
    return f * zv, out


def polar(prim, vals, pts):
    """GeneralPolar2D with the Fourier radius of eq:PSGCboundary (Tab.
    autodiffgeo; Sec. "Experimental choice of nonlinear function for Prop. 2"):
    sigma_k(R(theta) - r) with r, theta the polar coordinates of the sample
    about (x0, y0) and R(theta) = R0 + sum_n c_n cos(n theta + pi) + s_n
    sin(n theta + pi), n = 1..N.  theta = atan2(y - y0, x - x0) (the paper's
    arctan of the ratio, over the full turn).  Fields x0 y0 R0 c_1..c_N
    s_1..s_N z0 z1; nvert = N.  At the center (r = 0) theta is taken as 0 and
    the center partials as 0."""
    N = prim["nvert"]
    x0, y0, R0 = vals[0], vals[1], vals[2]
    cs = [vals[3 + n] for n in range(N)]
    ss = [vals[3 + N + n] for n in range(N)]
    (xc, xw), (yc, _) = pts["x"], pts["y"]
    dx, dy = xc - x0, yc - y0
    r = np.hypot(dx, dy)
    th = np.arctan2(dy, dx)
    R = R0 * np.ones(np.broadcast(xc, yc).shape)
    dR = np.zeros_like(R)            # d R / d theta
    basis_c, basis_s = [], []
    for n in range(1, N + 1):
        bc, bs = np.cos(n * th + np.pi), np.sin(n * th + np.pi)
        basis_c.append(bc)
        basis_s.append(bs)
        R = R + cs[n - 1] * bc + ss[n - 1] * bs
        dR = dR + n * (-cs[n - 1] * bs + ss[n - 1] * bc)
    kind = prim["sigma"][0][0]
    k = kval(prim["sigma"][0], xw)
    t = k * (R - r)
    f = sigma(kind, t)
    df = k * dsigma(kind, t)           # d f / d (R - r)
    safe = np.where(r > 0.0, r, 1.0)
    # d r / d x0 = -dx / r, d theta / d x0 = dy / r^2 (and the y0 pair)
    d_x0 = np.where(r > 0.0, dR * dy / (safe * safe) + dx / safe, 0.0)
    d_y0 = np.where(r > 0.0, -dR * dx / (safe * safe) + dy / safe, 0.0)
    zv, zparts = _z_factor(prim, vals, pts, 3 + 2 * N)
    g = df * zv
    out = [(0, g * d_x0), (1, g * d_y0), (2, g)]
    out += [(3 + n, g * basis_c[n]) for n in range(N)]
    out += [(3 + N + n, g * basis_s[n]) for n in range(N)]
    out += [(fi, f * d) for fi, d in zparts]
    return f * zv, out


def polar2d(prim, vals, pts):
    """Polar2D (Tab. autodiffgeo): sigma_k(R (1 + delta cos(alpha theta)) - r)
    with r, theta the polar coordinates of the sample about (x0, y0) (note 5
    and 6 of the table; theta = atan2(y - y0, x - x0), the arctan of the ratio
    over the full turn) and alpha a positive integer (the lobes of a
    star-convex shape; nvert = alpha).  Fields x0 y0 R delta z0 z1.  At the
    center (r = 0) theta is taken as 0 and the center partials as 0."""
    alpha = int(prim["nvert"])
    x0, y0, R, delta = vals[0], vals[1], vals[2], vals[3]
    (xc, xw), (yc, _) = pts["x"], pts["y"]
    dx, dy = xc - x0, yc - y0
    r = np.hypot(dx, dy)
    th = np.arctan2(dy, dx)
    ca, sa = np.cos(alpha * th), np.sin(alpha * th)
    Rth = R * (1.0 + delta * ca)
    dR = -R * delta * alpha * sa               # d R(theta) / d theta
    kind = prim["sigma"][0][0]
    k = kval(prim["sigma"][0], xw)
    t = k * (Rth - r)
    f = sigma(kind, t)
    df = k * dsigma(kind, t)                  # d f / d (R(theta) - r)
    safe = np.where(r > 0.0, r, 1.0)
    # d r / d x0 = -dx / r, d theta / d x0 = dy / r^2 (and the y0 pair)
    d_x0 = np.where(r > 0.0, dR * dy / (safe * safe) + dx / safe, 0.0)
    d_y0 = np.where(r > 0.0, -dR * dx / (safe * safe) + dy / safe, 0.0)
    zv, zparts = _z_factor(prim, vals, pts, 4)
    g = df * zv
    out = [(0, g * d_x0), (1, g * d_y0), (2, g * (1.0 + delta * ca)), (3, g * R * ca)]
    out += [(fi, f * d) for fi, d in zparts]
    return f * zv, out


def series(prim, vals, pts):
    """Two-sided GeneralCartesian2D whose boundary is the taper's sine series
    (eq:taper_boundary): Rect1D(x; xs, xe) sigma_k(f(x) - (y - yc))
    sigma_k(f(x) + (y - yc)), f(x) = w_in / 2 + (w_out - w_in) / 2 (x - x0) / L
    + envelope(x) sum_i v_i sin(i pi (x - x0) / L), envelope(x) = 0.1 + 0.45
    (1 - cos(2 pi (x - x0) / L)).  Fields xs xe v_1..v_K z0 z1; consts x0 L
    w_in w_out yc; nvert = K."""
    K = prim["nvert"]
    x0, L, w_in, w_out, yc = [float(c) for c in prim["consts"]]
    v = vals[2:2 + K]
    (xc, xw), (yc_s, yw) = pts["x"], pts["y"]
    shape = np.broadcast(xc, yc_s).shape
    xb = np.broadcast_to(xc, shape)
    u = (xb - x0) / L
    env = 0.1 + 0.45 * (1.0 - np.cos(2.0 * np.pi * u))
    basis = [env * np.sin(i * np.pi * u) for i in range(1, K + 1)]
    f = w_in / 2.0 + (w_out - w_in) / 2.0 * u
    for i in range(K):
        f = f + v[i] * basis[i]
    yr = yc_s - yc
    sy = prim["sigma"][1]
    ky = kval(sy, yw)
    tp, tm = ky * (f - yr), ky * (f + yr)
    sp, sm = sigma(sy[0], tp), sigma(sy[0], tm)
    dsp, dsm = ky * dsigma(sy[0], tp), ky * dsigma(sy[0], tm)
    rx, drx0, drx1 = rect1d(prim["sigma"][0], xc, xw, vals[0], vals[1])
    zv, zparts = _z_factor(prim, vals, pts, 2 + K)
    fy = sp * sm
    gf = rx * (dsp * sm + sp * dsm) * zv        # d s / d f
    out = [(0, drx0 * fy * zv), (1, drx1 * fy * zv)]
    out += [(2 + i, gf * basis[i]) for i in range(K)]
    out += [(fi, rx * fy * d) for fi, d in zparts]
    return rx * fy * zv, out


EVAL = {"box": box, "ellipse": ellipse, "poly": poly, "gcart": gcart, "polar": polar, "polar2d": polar2d,
        "series": series}


def evaluate(prim, vals, pts):
    return EVAL[prim["type"]](prim, vals, pts)


def bbox(prim, vals, wmax):
    """Conservative axis-aligned box outside which the primitive is 0 to
    below FP64 resolution (compact sigma: exactly).  wmax: largest sample
    width per axis (for local k)."""
    from .sigma import support

    def reach(sig, ai):
        kind, kmode, k = sig
        kk = k / wmax[ai] if kmode == "local" else k
        return support(kind) / kk

    t = prim["type"]
    inf = np.inf
    lo, hi = [-inf] * 3, [inf] * 3
    if t == "box":
        for ai in range(3):
            if prim["bounded"][ai]:
                r = reach(prim["sigma"][ai], ai)
                lo[ai], hi[ai] = vals[2 * ai] - r, vals[2 * ai + 1] + r
        return lo, hi
    if t == "ellipse":
        x0, y0, r = vals[0], vals[1], vals[2]
        ax, ay = prim["consts"]
        rr = max(r, 0.0) + reach(prim["sigma"][0], 0)
        lo[0], hi[0] = x0 - rr * ax, x0 + rr * ax
        lo[1], hi[1] = y0 - rr * ay, y0 + rr * ay
        zf = 3
    elif t == "polar":
        # R(theta) <= R0 + sum |c_n| + |s_n|
        N = prim["nvert"]
        rmax = max(vals[2] + sum(abs(v) for v in vals[3:3 + 2 * N]), 0.0) + reach(prim["sigma"][0], 0)
        lo[0], hi[0] = vals[0] - rmax, vals[0] + rmax
        lo[1], hi[1] = vals[1] - rmax, vals[1] + rmax
        zf = 3 + 2 * N
    elif t == "polar2d":
        # R (1 + delta cos) <= R (1 + |delta|) for R >= 0, and <= |R| (1 + |delta|) always
        rmax = max(abs(vals[2]) * (1.0 + abs(vals[3])), 0.0) + reach(prim["sigma"][0], 0)
        lo[0], hi[0] = vals[0] - rmax, vals[0] + rmax
        lo[1], hi[1] = vals[1] - rmax, vals[1] + rmax
        zf = 4
    elif t == "series":
        # |f| <= the larger end of the linear ramp over [xs, xe] + sum |v_i| (envelope <= 1)
        K = prim["nvert"]
        x0, L, w_in, w_out, yc = [float(c) for c in prim["consts"]]
        ramp = [abs(w_in / 2.0 + (w_out - w_in) / 2.0 * (x - x0) / L) for x in (vals[0], vals[1])]
        R = max(ramp) + sum(abs(x) for x in vals[2:2 + K]) + reach(prim["sigma"][1], 1)
        rx = reach(prim["sigma"][0], 0)
        lo[0], hi[0] = vals[0] - rx, vals[1] + rx
        lo[1], hi[1] = yc - R, yc + R
        zf = 2 + K
    elif t == "poly":
        N = prim["nvert"]
        rr = reach(prim["sigma"][0], 0)
        lo[0], hi[0] = min(vals[:N]) - rr, max(vals[:N]) + rr
        lo[1], hi[1] = min(vals[N:2 * N]) - rr, max(vals[N:2 * N]) + rr
        zf = 2 * N
    else:
        M = prim["nvert"]
        rx = reach(prim["sigma"][0], 0)
        ry = reach(prim["sigma"][1], 1)
        lo[0], hi[0] = vals[0] - rx, vals[1] + rx
        lo[1] = min(vals[2 + M:2 + 2 * M]) - ry
        hi[1] = max(vals[2:2 + M]) + ry
        zf = 2 + 2 * M
    if prim["bounded"][2]:
        r = reach(prim["sigma"][2], 2)
        lo[2], hi[2] = vals[zf] - r, vals[zf + 1] + r
    return lo, hi
