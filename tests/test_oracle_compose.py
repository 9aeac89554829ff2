"""Pins of the oracle's composition (eq:union, eq:intersection, the
difference reading) against the paper's truth table (Tab. truthtable), its
stated boundary behaviour and the [0,1] bound of every node."""
import os

import numpy as np
import pytest

from oracle.scene import _compose

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _op(op, *vals):
    vals = [np.asarray(v, dtype=np.float64) for v in vals]
    shape = np.broadcast(*vals).shape
    node = {"op": op, "children": list(range(len(vals)))}
    out, _ = _compose(node, {i: np.broadcast_to(v, shape) for i, v in enumerate(vals)}, shape)
    return out


def test_union_truth_table():
    for line in open(os.path.join(GOLD, "union_truth_table.txt")):
        if line.strip() and not line.startswith("#"):
            b1, b2, o = (float(v) for v in line.split())
            assert _op("union", b1, b2) == o


def test_intersection_binary_corners():
    for bits in np.ndindex(2, 2, 2):
        assert _op("intersection", *bits) == float(all(bits))


def test_overlapping_boundaries_union_to_one():
    assert _op("union", 0.5, 0.5) == 1.0
    assert _op("intersection", 0.5, 0.5) == 0.0


def test_difference_reading_equals_intersection_with_complement():
    a, b = np.meshgrid(np.linspace(0, 1, 41), np.linspace(0, 1, 41))
    assert np.allclose(_op("difference", a, b), _op("intersection", a, 1.0 - b), atol=1e-15)


def test_nodes_stay_in_unit_interval():
    rng = np.random.default_rng(3)
    for n in range(1, 7):
        v = rng.uniform(0, 1, size=(n, 2000))
        for op in ("union", "intersection"):
            o = _op(op, *v)
            assert o.min() >= 0.0 and o.max() <= 1.0
    o = _op("difference", rng.uniform(0, 1, 2000), rng.uniform(0, 1, 2000))
    assert o.min() >= 0.0 and o.max() <= 1.0


def test_clamp_derivative_rules():
    node = {"op": "union", "children": [0, 1]}
    s = {0: np.array([0.3, 0.6, 0.5]), 1: np.array([0.2, 0.6, 0.5])}
    _, coefs = _compose(node, s, (3,))
    assert [list(c) for _, c in coefs] == [[1.0, 0.0, 0.0]] * 2      # passes iff sum < 1
    node = {"op": "difference", "children": [0, 1]}
    s = {0: np.array([0.7, 0.4]), 1: np.array([0.2, 0.4])}
    _, coefs = _compose(node, s, (2,))
    assert [list(c) for _, c in coefs] == [[1.0, 0.0], [-1.0, -0.0]]


# ---- non-binary union (Alg. cap, Sec. "Non-binary material systems")
def _levels(levels, *vals):
    vals = [np.asarray(v, dtype=np.float64) for v in vals]
    shape = np.broadcast(*vals).shape
    node = {"op": "levels", "levels": list(levels), "children": list(range(len(vals)))}
    return _compose(node, {i: np.broadcast_to(v, shape) for i, v in enumerate(vals)}, shape)


def test_levels_single_set_gives_its_own_level():
    # where only set k is present (fill v), eps - eps_bg = eps^k v
    lv = (0.1, 0.34, 0.62, 1.0)
    v = np.linspace(0.0, 1.0, 11)
    z = np.zeros_like(v)
    for k in range(4):
        vals = [z] * 4
        vals[k] = v
        s, _ = _levels(lv, *vals)
        assert np.max(np.abs(lv[-1] * s - lv[k] * v)) < 1e-15


def test_levels_priority_to_the_largest_level():
    # where sets overlap fully, the largest present level wins
    lv = (0.1, 0.34, 0.62, 1.0)
    for present in np.ndindex(2, 2, 2, 2):
        if sum(present) == 0:
            continue
        s, _ = _levels(lv, *[np.array(float(b)) for b in present])
        top = max(lv[k] for k in range(4) if present[k])
        assert abs(lv[-1] * float(s) - top) < 1e-15, present


def test_levels_with_equal_levels_is_the_union():
    rng = np.random.default_rng(3)
    vals = [rng.uniform(0, 1, 200) * rng.integers(0, 2, 200) for _ in range(3)]
    s, _ = _levels((1.0, 1.0, 1.0), *vals)
    assert np.max(np.abs(s - _op("union", *vals))) < 1e-15


def test_levels_chain_rule_matches_differences():
    rng = np.random.default_rng(4)
    lv = (0.2, 0.5, 1.3)
    vals = [rng.uniform(0, 0.6, 500) for _ in range(3)]
    _, parts = _levels(lv, *vals)
    h = 1e-7
    for i, d in parts:
        vp = [v.copy() for v in vals]
        vm = [v.copy() for v in vals]
        vp[i] += h
        vm[i] -= h
        fd = (_levels(lv, *vp)[0] - _levels(lv, *vm)[0]) / (2 * h)
        # away from the clamp kinks the chain rule is the derivative
        x_far = np.ones(500, dtype=bool)
        s = vals[0]
        for k in (1, 2):
            x = lv[k - 1] / lv[k] * s + vals[k]
            x_far &= np.abs(x - 1.0) > 1e-5
            s = np.minimum(1.0, x)
        assert np.max(np.abs(fd - d)[x_far]) < 1e-6, i
