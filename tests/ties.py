"""Scenes whose samples sit exactly on the kinks of the method (input
generators only: no arithmetic of the method here).

Every coordinate is a multiple of 2^-8 um on a 2^-6 um uniform grid, so each
linear-sigma argument t = (c - x0) / w and each fill value is exact in
binary, and the oracle and the GPU reach the same exact values:
* union: two abutting boxes share an edge position inside a sample's
  averaging interval, so their fills there are 0.75 and 0.25 and the union's
  sum is exactly 1 (eq:union passes the gradient only below 1);
* a box edge on an averaging-interval face, where the linear sigma's
  argument is exactly +-1/2 (Tab. nonlinearfunctions: the kink);
* difference: minuend and subtrahend with the same edge position, so a - b
  is exactly 0 on the samples that straddle it;
* intersection: two boxes whose edges meet inside a sample, so the sum of
  their fills is exactly N - 1 there (eq:intersection passes only above)."""
import numpy as np

from paper_2311_05646_amd import workloads as W

D = 2.0 ** -6      # grid spacing (um)
Q = 2.0 ** -8      # a quarter of it


def _grid(nx=64, ny=48):
    return W.uniform_nodes(nx, D), W.uniform_nodes(ny, D)


def _scene(name, prims, tree, n_params):
    X, Y = _grid()
    return {"name": name, "dim": 2, "nodes": [X, Y, np.array([0.0, 1.0])], "components": ("x", "y", "z"),
            "eps_bg": 2.0, "eps_fg": 10.0, "n_params": n_params, "prims": prims, "tree": tree}


def _fields(scene, seed):
    return W.make_fields(scene, seed)


def union_ties():
    X, Y = _grid()
    ye = (W.K(Y[10] + 3 * Q), W.K(Y[30] + Q))
    shared = X[20] + Q                   # inside the averaging intervals of x-sample 20
    p = [X[6] + 2 * Q, shared, shared, X[33] - 3 * Q,
         X[40] - 2 * Q,                  # on the lower face of node-centered sample 40
         X[52]]                          # on a cell face: cell-centered t = -1/2 / +1/2
    prims = [W.box(x=(W.P(0), W.P(1)), y=ye), W.box(x=(W.P(2), W.P(3)), y=ye),
             W.box(x=(W.P(4), W.P(5)), y=ye)]
    sc = _scene("ties_union", prims, {"op": "union", "children": [0, 1, 2]}, 6)
    E, A = _fields(sc, 901)
    return {"scene": sc, "p": np.array(p), "E": E, "A": A, "omega": 2 * np.pi / 1.55}


def difference_ties():
    X, Y = _grid()
    p = [X[12] + Q, X[12] + Q, X[30] + 3 * Q, X[45] - Q]
    slab = W.box(x=(W.P(0), W.K(X[60] + Q)), y=(W.K(Y[8] + Q), W.K(Y[40] - 3 * Q)))
    # the etch starts at the slab's own edge (a - b = 0 across it) and its top
    # face coincides with the slab's
    etch = W.box(x=(W.P(1), W.P(2)), y=(W.K(Y[20] + 2 * Q), W.K(Y[40] - 3 * Q)))
    etch2 = W.box(x=(W.P(3), W.K(X[50] + 2 * Q)), y=(W.K(Y[8] + Q), W.K(Y[16] - 2 * Q)))
    tree = {"op": "difference", "children": [0, {"op": "union", "children": [1, 2]}]}
    sc = _scene("ties_difference", [slab, etch, etch2], tree, 4)
    E, A = _fields(sc, 902)
    return {"scene": sc, "p": np.array(p), "E": E, "A": A, "omega": 2 * np.pi / 1.55}


def intersection_ties():
    """An intersection of two boxes whose x-extents meet inside a sample (the
    sum of their fills is exactly N - 1 = 1 there), unioned with a third box
    whose edge lies on an averaging-interval face (two groups under a union
    root)."""
    X, Y = _grid()
    meet = X[26] + Q
    p = [X[8] + 3 * Q, meet, meet, X[40] - Q, X[44] + 2 * Q]
    a = W.box(x=(W.P(0), W.P(1)), y=(W.K(Y[4] + Q), W.K(Y[36] + 2 * Q)))
    b = W.box(x=(W.P(2), W.P(3)), y=(W.K(Y[6] - Q), W.K(Y[30] + Q)))
    c = W.box(x=(W.P(4), W.K(X[58] + Q)), y=(W.K(Y[20] + 2 * Q), W.K(Y[44])))
    tree = {"op": "union", "children": [{"op": "intersection", "children": [0, 1]}, 2]}
    sc = _scene("ties_intersection", [a, b, c], tree, 5)
    E, A = _fields(sc, 903)
    return {"scene": sc, "p": np.array(p), "E": E, "A": A, "omega": 2 * np.pi / 1.55}


def meeting_intersection():
    """Two boxes whose x-extents meet inside a sample, intersected: the sum of
    their fills is exactly 1 = N - 1 there."""
    X, Y = _grid()
    meet = X[26] + Q
    p = [X[8] + 3 * Q, meet, meet, X[50] - Q]
    ye = (W.K(Y[10] + Q), W.K(Y[30] + 2 * Q))
    a = W.box(x=(W.P(0), W.P(1)), y=ye)
    b = W.box(x=(W.P(2), W.P(3)), y=ye)
    sc = _scene("ties_meet", [a, b], {"op": "intersection", "children": [0, 1]}, 4)
    E, A = _fields(sc, 904)
    return {"scene": sc, "p": np.array(p), "E": E, "A": A, "omega": 2 * np.pi / 1.55}


CASES = {"union": union_ties, "difference": difference_ties, "intersection": intersection_ties,
         "meet": meeting_intersection}
