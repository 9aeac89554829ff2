"""The oracle's whole-grid gradient of a large workload, computed tile by tile
(test infrastructure: it calls only oracle functions, on sub-scenes).

The gradient of eq:1 is a sum over samples, and each sample's term depends
only on p and that sample's own fields, so the sum over the whole grid is the
sum over any partition of it.  A tile is a block of in-plane samples (all of
the column axis that any primitive reaches); its sub-scene keeps the grid
nodes of the tile and the primitives whose support box (oracle
primitives.bbox: the sigma support, beyond which a primitive is 0 to below
FP64 resolution) meets the tile's samples, with the op tree pruned to them.

Exactness conditions, checked here:
* the in-plane lattices are uniform, so a node-centered sample at a tile's
  first node has the same width as in the whole grid (the first node of a
  lattice takes w_{-1} := w_0);
* along z the kept layers start and end below / above every primitive's
  support box, so the one layer whose node-centered width can differ (the
  first kept node) has a zero extrusion factor either way.
Dropping a primitive from a union changes the sum by less than FP64
resolution; a pruned difference b - 0 = b and an intersection with an empty
member is 0 (eq:union, eq:intersection and the difference reading)."""
import multiprocessing as mp

import numpy as np

from oracle import primitives as prm
from oracle import scene as S
from oracle.lattice import component_samples

_G = {}


def _uniform(a):
    d = np.diff(np.asarray(a, dtype=np.float64))
    return bool(np.allclose(d, d[0], rtol=0.0, atol=1e-12 * max(1.0, abs(d[0]))))


def _prune(node, keep):
    """The tree restricted to the primitives in `keep` (old index -> new),
    or None when nothing of it remains."""
    if isinstance(node, (int, np.integer)):
        return keep.get(int(node))
    ch = [_prune(c, keep) for c in node["children"]]
    op = node["op"]
    if op == "difference":
        a, b = ch
        if a is None:
            return None
        return a if b is None else {"op": "difference", "children": [a, b]}
    if op == "intersection":
        if any(c is None for c in ch):
            return None
        return {"op": "intersection", "children": ch}
    if op == "levels":
        raise ValueError("tiling of a levels root is not supported")
    ch = [c for c in ch if c is not None]
    return {"op": op, "children": ch} if ch else None


def _task(args):
    ci, (x0, x1), (y0, y1) = args
    d, p, vals, boxes, zr = _G["d"], _G["p"], _G["vals"], _G["boxes"], _G["zr"]
    X, Y, Z = d["nodes"]
    comp = d["components"][ci]
    smp = component_samples(d, comp)
    xs, ys = smp["x"][0][x0:x1], smp["y"][0][y0:y1]
    iz0, iz1 = zr
    keep = {}
    prims = []
    for i in S.check_scene(d):
        lo, hi = boxes[i]
        if lo[0] <= xs[-1] and hi[0] >= xs[0] and lo[1] <= ys[-1] and hi[1] >= ys[0]:
            keep[i] = len(prims)
            prims.append(d["prims"][i])
    tree = _prune(d["tree"], keep)
    if tree is None:
        return np.zeros(d["n_params"])
    if isinstance(tree, int):
        tree = {"op": "union", "children": [tree]}
    sub = dict(d)
    sub.update(nodes=[X[x0:x1 + 1], Y[y0:y1 + 1], Z[iz0:iz1 + 1]], components=(comp,), prims=prims, tree=tree)
    E = _G["E"][ci, iz0:iz1, y0:y1, x0:x1]
    A = _G["A"][ci, iz0:iz1, y0:y1, x0:x1]
    g = S.sensitivity(E, A, _G["omega"])[None]
    return S.grad_analytic(sub, p, g)


def tiled_grad(desc, p, E, A, omega, tile=(40, 40), workers=8):
    """The oracle's gradient over the whole grid of `desc` (FP64), summed over
    in-plane tiles of tile = (x samples, y samples)."""
    X, Y, Z = desc["nodes"]
    if not (_uniform(X) and _uniform(Y)):
        raise ValueError("tiled_grad needs uniform x and y lattices")
    vals = S.resolve(desc, p)
    wmax = [float(np.diff(np.asarray(a)).max()) for a in (X, Y, Z)]
    used = S.check_scene(desc)
    boxes = {i: prm.bbox(desc["prims"][i], vals[i], wmax) for i in used}
    nz = len(Z) - 1
    zlo = min(boxes[i][0][2] for i in used)
    zhi = max(boxes[i][1][2] for i in used)
    if desc["dim"] == 3 and np.isfinite(zlo) and np.isfinite(zhi) and not _uniform(Z):
        # first kept layer wholly below every support (both of its sample
        # positions), last kept layer above
        below = np.nonzero(Z < zlo)[0]
        iz0 = max(0, int(below[-1]) - 1) if below.size else 0
        above = np.nonzero(Z > zhi)[0]
        iz1 = min(nz, int(above[0]) + 1) if above.size else nz
    elif desc["dim"] == 3 and np.isfinite(zlo) and np.isfinite(zhi):
        iz0 = max(0, int(np.searchsorted(Z, zlo)) - 2)
        iz1 = min(nz, int(np.searchsorted(Z, zhi)) + 2)
    else:
        iz0, iz1 = 0, nz
    tasks = []
    nx, ny = len(X) - 1, len(Y) - 1
    for ci in range(len(desc["components"])):
        for x0 in range(0, nx, tile[0]):
            for y0 in range(0, ny, tile[1]):
                tasks.append((ci, (x0, min(nx, x0 + tile[0])), (y0, min(ny, y0 + tile[1]))))
    _G.update(d=desc, p=np.asarray(p, dtype=np.float64), vals=vals, boxes=boxes, zr=(iz0, iz1), E=E, A=A,
              omega=omega)
    try:
        if workers <= 1:
            parts = [_task(t) for t in tasks]
        else:
            with mp.get_context("fork").Pool(workers) as pool:
                parts = pool.map(_task, tasks, chunksize=1)
    finally:
        _G.clear()
    return np.sum(parts, axis=0)
