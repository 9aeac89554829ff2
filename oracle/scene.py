"""Scene-level oracle: permittivity, adjoint sensitivity, reverse-mode and
finite-difference gradients, all FP64 and brute force.

* eps (eq:eps, Sec. "AutoDiffGeo"): every primitive is evaluated at every
  sample, composed by the op tree and scaled to the two material levels:
  eps = eps_bg + (eps_fg - eps_bg) * s_root.
* composition: union = min{1, sum s_i} (eq:union); intersection =
  max{N-1, sum s_i} - (N-1) (eq:intersection); difference, which the paper
  uses as "subtract the unified scattering object from the waveguide"
  without a formula, is read as max{0, a - b} (equal to eq:intersection of
  a and 1-b).  Derivative rules at the clamps: union passes the gradient iff
  sum < 1, intersection iff sum > N-1, difference iff a - b > 0.
* sensitivity (eq:1, mu term dropped): g = 2*omega*Im(E * E_adj), no
  conjugation, i.e. Re(c E E_adj) with c = -2i*omega.
* grad_analytic (eq:AD / eq:jaceps): grad_k = sum_c sum_j g_cj d eps_cj / d p_k
  by the chain rule through the tree and the primitives; never forms the
  Jacobian.
* grad_fd: central differences of eps(p) contracted with g (the paper's
  finite-difference baseline of Sec. "Automatic differentiation based
  acceleration", in its central form).

Points can be the whole grid of a component or a subset (flattened indices);
for subsets of large grids primitives are culled by their support boxes,
which drops only sigma tails below FP64 resolution.
"""
import numpy as np

from . import primitives as prm
from .lattice import AXES, component_samples


# ----------------------------------------------------------------- parsing
def check_scene(desc):
    """Validate a scene description; returns the list of primitive indices
    that appear in the tree."""
    seen = []

    def walk(node):
        if isinstance(node, (int, np.integer)):
            seen.append(int(node))
            return
        op = node["op"]
        if op not in ("union", "intersection", "difference", "levels"):
            raise ValueError(f"unknown op {op!r}")
        if op == "levels":
            if node is not desc["tree"]:
                raise ValueError("a levels node must be the root")
            lv = [float(x) for x in node["levels"]]
            if len(lv) != len(node["children"]) or len(lv) < 2:
                raise ValueError("levels: one level per child, at least two")
            if any(not (b >= a > 0.0) for a, b in zip(lv, lv[1:])) or lv[0] <= 0.0:
                raise ValueError("levels must be positive and ascending")
            if abs(lv[-1] - (desc["eps_fg"] - desc["eps_bg"])) > 1e-12 * max(1.0, abs(lv[-1])):
                raise ValueError("the top level must equal eps_fg - eps_bg")
        if op == "difference" and len(node["children"]) != 2:
            raise ValueError("difference takes exactly two operands")
        if len(node["children"]) == 0:
            raise ValueError("empty op node")
        for ch in node["children"]:
            walk(ch)

    walk(desc["tree"])
    if len(seen) != len(set(seen)):
        raise ValueError("a primitive appears twice in the tree")
    for i in seen:
        pr = desc["prims"][i]
        if pr["type"] in ("ellipse", "poly", "polar", "polar2d") and pr["sigma"][0][1] != "fixed":
            raise ValueError("radial / oblique sigma arguments need a fixed k")
        for a, b, idx in pr["fields"]:
            if idx >= desc["n_params"]:
                raise ValueError("parameter index out of range")
    return seen


def resolve(desc, p):
    """Field values a + b * p[idx] of every primitive."""
    p = np.asarray(p, dtype=np.float64)
    out = []
    for pr in desc["prims"]:
        out.append([a + b * p[idx] if idx >= 0 else a for (a, b, idx) in pr["fields"]])
    return out


def sensitivity(E, A, omega):
    """g = 2 omega Im(E * E_adj) in FP64 (eq:1, epsilon term)."""
    E = np.asarray(E).astype(np.complex128)
    A = np.asarray(A).astype(np.complex128)
    return 2.0 * omega * np.imag(E * A)


# ----------------------------------------------------------------- points
def plane_points(desc, comp):
    """Broadcastable sample arrays covering a whole (Nz, Ny, Nx) plane."""
    smp = component_samples(desc, comp)
    shp = {"x": (1, 1, -1), "y": (1, -1, 1), "z": (-1, 1, 1)}
    return {a: (smp[a][0].reshape(shp[a]), smp[a][1].reshape(shp[a])) for a in AXES}


def subset_points(desc, comp, flat_idx):
    """Sample arrays for the flattened (z, y, x) indices of a plane."""
    X, Y, Z = desc["nodes"]
    nx, ny = len(X) - 1, len(Y) - 1
    flat_idx = np.asarray(flat_idx, dtype=np.int64)
    iz, rem = np.divmod(flat_idx, nx * ny)
    iy, ix = np.divmod(rem, nx)
    smp = component_samples(desc, comp)
    return {"x": (smp["x"][0][ix], smp["x"][1][ix]), "y": (smp["y"][0][iy], smp["y"][1][iy]),
            "z": (smp["z"][0][iz], smp["z"][1][iz])}


def _max_widths(desc):
    wm = []
    for nodes in desc["nodes"]:
        w = np.diff(np.asarray(nodes, dtype=np.float64))
        wm.append(float(w.max()))
    return wm


# ----------------------------------------------------------------- tree
def _compose(node, svals, shape):
    """Forward value of a tree node and, for each primitive under it, the
    derivative of the node value with respect to that primitive's value."""
    if isinstance(node, (int, np.integer)):
        return svals[int(node)], [(int(node), np.ones(shape))]
    vals, lists = [], []
    for ch in node["children"]:
        v, l = _compose(ch, svals, shape)
        vals.append(np.broadcast_to(v, shape))
        lists.append(l)
    op = node["op"]
    if op == "levels":
        # Alg. cap (non-binary union): s = v_1; s = min{1, (eps^{k-1} / eps^k) s
        # + v_k} for k = 2..K; the node value is s (eps = eps_bg + eps^K s)
        lv = [float(x) for x in node["levels"]]
        s = vals[0]
        passes, qs = [None], [None]
        for k in range(1, len(vals)):
            q = lv[k - 1] / lv[k]
            x = q * s + vals[k]
            passes.append((x < 1.0).astype(np.float64))
            qs.append(q)
            s = np.minimum(1.0, x)
        # d s / d v_k = pass_k prod_{j > k} pass_j q_j (k >= 2), prod_{j >= 2} pass_j q_j (k = 1)
        coef = [None] * len(vals)
        acc = np.ones(shape)
        for k in range(len(vals) - 1, 0, -1):
            coef[k] = acc * passes[k]
            acc = acc * passes[k] * qs[k]
        coef[0] = acc
        return s, [(i, c * coef[k]) for k, l in enumerate(lists) for (i, c) in l]
    if op == "union":
        S = np.sum(vals, axis=0)
        out = np.minimum(1.0, S)
        m = (S < 1.0).astype(np.float64)
        return out, [(i, c * m) for l in lists for (i, c) in l]
    if op == "intersection":
        N = len(vals)
        S = np.sum(vals, axis=0)
        out = np.maximum(N - 1.0, S) - (N - 1.0)
        m = (S > N - 1.0).astype(np.float64)
        return out, [(i, c * m) for l in lists for (i, c) in l]
    a, b = vals
    d = a - b
    out = np.maximum(0.0, d)
    m = (d > 0.0).astype(np.float64)
    return out, [(i, c * m) for (i, c) in lists[0]] + [(i, -c * m) for (i, c) in lists[1]]


def _eval_points(desc, vals, pts, want_parts, cull):
    shape = np.broadcast(*[pts[a][0] for a in AXES]).shape
    svals, parts = {}, {}
    wmax = _max_widths(desc) if cull else None
    for i in check_scene(desc):
        pr = desc["prims"][i]
        if cull:
            lo, hi = prm.bbox(pr, vals[i], wmax)
            inside = np.ones(shape, dtype=bool)
            for ai, a in enumerate(AXES):
                c = np.broadcast_to(pts[a][0], shape)
                inside &= (c >= lo[ai]) & (c <= hi[ai])
            if not inside.any():
                svals[i] = np.zeros(shape)
                parts[i] = []
                continue
        s, pl = prm.evaluate(pr, vals[i], pts)
        svals[i] = np.broadcast_to(s, shape)
        parts[i] = pl if want_parts else None
    root, coefs = _compose(desc["tree"], svals, shape)
    return root, coefs, parts, shape


# ----------------------------------------------------------------- API
def eps(desc, p, comps=None):
    """eps as (C, Nz, Ny, Nx) FP64, every primitive at every sample."""
    vals = resolve(desc, p)
    de = desc["eps_fg"] - desc["eps_bg"]
    out = []
    for comp in (comps or desc["components"]):
        pts = plane_points(desc, comp)
        s, _, _, _ = _eval_points(desc, vals, pts, False, False)
        out.append(desc["eps_bg"] + de * s)
    return np.stack(out)


def eps_at(desc, p, comp_index, flat_idx, cull=True):
    """eps at selected samples of one component plane (FP64)."""
    vals = resolve(desc, p)
    pts = subset_points(desc, desc["components"][comp_index], flat_idx)
    s, _, _, _ = _eval_points(desc, vals, pts, False, cull)
    return desc["eps_bg"] + (desc["eps_fg"] - desc["eps_bg"]) * s


def _accumulate(desc, vals, pts, g, grad, cull):
    de = desc["eps_fg"] - desc["eps_bg"]
    _, coefs, parts, shape = _eval_points(desc, vals, pts, True, cull)
    g = np.broadcast_to(g, shape)
    for i, coef in coefs:
        w = g * de * coef
        fields = desc["prims"][i]["fields"]
        for fi, d in parts[i]:
            contrib = w * d
            if isinstance(fi, (int, np.integer)):
                a, b, idx = fields[fi]
                if idx >= 0:
                    grad[idx] += b * contrib.sum()
            else:
                fi_b = np.broadcast_to(fi, shape).ravel()
                per_field = np.bincount(fi_b, weights=contrib.ravel(), minlength=len(fields))
                for f in np.nonzero(per_field)[0]:
                    a, b, idx = fields[f]
                    if idx >= 0:
                        grad[idx] += b * per_field[f]


def grad_analytic(desc, p, g):
    """grad_k = sum over components and samples of g * d eps / d p_k by the
    chain rule (reverse mode, eq:AD).  g: (C, Nz, Ny, Nx)."""
    vals = resolve(desc, p)
    grad = np.zeros(desc["n_params"])
    for ci, comp in enumerate(desc["components"]):
        pts = plane_points(desc, comp)
        _accumulate(desc, vals, pts, np.asarray(g[ci], dtype=np.float64), grad, False)
    return grad


def grad_analytic_region(desc, p, g_fn, comp_index, flat_idx, grad=None):
    """Analytic gradient restricted to the listed samples of one component;
    g_fn(flat_idx) returns g at those samples.  Summing over every sample
    that any parameter's derivative touches gives the full gradient."""
    vals = resolve(desc, p)
    if grad is None:
        grad = np.zeros(desc["n_params"])
    pts = subset_points(desc, desc["components"][comp_index], flat_idx)
    _accumulate(desc, vals, pts, g_fn(flat_idx), grad, True)
    return grad


def grad_fd(desc, p, g, h, params=None):
    """Central differences (eps(p + h e_k) - eps(p - h e_k)) / (2h)
    contracted with g, for every k (or the listed ones)."""
    p = np.asarray(p, dtype=np.float64)
    ks = range(desc["n_params"]) if params is None else params
    out = np.zeros(desc["n_params"])
    for k in ks:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        d = (eps(desc, pp) - eps(desc, pm)) / (2.0 * h)
        out[k] = np.sum(np.asarray(g, dtype=np.float64) * d)
    return out


def grad_fd_forward(desc, p, g, h):
    """The paper's n+1 form: (eps(p + h e_k) - eps(p)) / h."""
    p = np.asarray(p, dtype=np.float64)
    base = eps(desc, p)
    out = np.zeros(desc["n_params"])
    for k in range(desc["n_params"]):
        pp = p.copy()
        pp[k] += h
        out[k] = np.sum(np.asarray(g, dtype=np.float64) * (eps(desc, pp) - base) / h)
    return out


def support_samples(desc, p, prim_index, comp_index):
    """Flattened sample indices of one component plane inside the support box
    of one primitive (every sample where it or its derivative is non-zero)."""
    vals = resolve(desc, p)
    lo, hi = prm.bbox(desc["prims"][prim_index], vals[prim_index], _max_widths(desc))
    smp = component_samples(desc, desc["components"][comp_index])
    sel = []
    for ai, a in enumerate(AXES):
        c = smp[a][0]
        sel.append(np.nonzero((c >= lo[ai]) & (c <= hi[ai]))[0])
    X, Y, _ = desc["nodes"]
    nx, ny = len(X) - 1, len(Y) - 1
    iz, iy, ix = np.meshgrid(sel[2], sel[1], sel[0], indexing="ij")
    return ((iz * ny + iy) * nx + ix).ravel()
