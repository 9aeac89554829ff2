"""The allocation-free entry point eps_grad_vjp_noalloc (for callers that
cannot allocate device memory) against eps_grad_vjp on the same inputs,
through the C-ABI: two calls in a row on the shared per-device scratch array,
the second with a smaller input (so it must not depend on what the first left
there), in atomic mode (equal up to the order of the FP64 atomic additions)
and in deterministic mode (bitwise equal); both also against the oracle; and
a scene whose staging does not fit the scratch is refused before any launch."""
import numpy as np
import pytest
import torch

from oracle import scene as S
from tests.gpu_util import api, config, fields_c64, rel, to_dev
from paper_2311_05646_amd import workloads as W

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4


def _pair(name, det):
    A_ = api()
    cfg = config(name)
    sc = A_.Scene(cfg["scene"])
    sc.set_deterministic(det)
    E, A = fields_c64(cfg)
    Ed, Ad = to_dev(E), to_dev(A)
    return cfg, sc, E, A, Ed, Ad


# the first input of each sequence is larger than the second; zoo3_union has
# p-dependent extrusion tables and the spread accumulation, psgc3_small shares
# its shape coefficients among scatterers, psgc3_small_mixed interleaves three
# coefficient sets, taper3_sine_small37 reduces 37 sine terms in groups of 16
@pytest.mark.parametrize("det", [False, True])
@pytest.mark.parametrize("seq", [("zoo3_union", "c3_small"), ("c4_small", "psgc3_small"),
                                 ("psgc3_small_mixed", "taper3_sine_small37")])
def test_noalloc_equals_vjp_on_two_calls(seq, det):
    A_ = api()
    print(f"[noalloc] {seq} deterministic={det}", flush=True)
    first = _pair(seq[0], det)
    second = _pair(seq[1], det)
    assert np.prod(first[1].shape) > np.prod(second[1].shape)
    for cfg, sc, E, A, Ed, Ad in (first, second):
        ref = A_.eps_grad_vjp(sc, cfg["p"], Ed, Ad, cfg["omega"])
        got = A_.eps_grad_vjp_noalloc(sc, cfg["p"], Ed, Ad, cfg["omega"])
        # device p and grad as well
        pd = torch.tensor(cfg["p"], dtype=torch.float64, device="cuda")
        gd = A_.eps_grad_vjp_noalloc(sc, pd, Ed, Ad, cfg["omega"]).cpu().numpy()
        if det:
            assert np.array_equal(got, ref) and np.array_equal(gd, ref)
        else:
            assert rel(got, ref) <= 1e-12 and rel(gd, ref) <= 1e-12
        oracle = S.grad_analytic(cfg["scene"], cfg["p"], S.sensitivity(E, A, cfg["omega"]))
        assert rel(got, oracle) <= GRAD_TOL


def test_noalloc_refuses_a_scene_beyond_the_scratch():
    from paper_2311_05646_amd._lib import SGError
    A_ = api()
    # 15000 boxes: their records alone exceed the 4 MiB scratch
    X = W.uniform_nodes(60, 0.02)
    Y = W.uniform_nodes(40, 0.02)
    prims = [W.box(x=(W.K(0.01 + 1e-4 * i), W.K(0.5 + 1e-4 * i)), y=(W.K(0.2), W.K(0.6))) for i in range(14999)]
    prims.append(W.box(x=(W.P(0), W.K(0.9)), y=(W.K(0.1), W.K(0.7))))
    desc = {"name": "big", "dim": 2, "nodes": [X, Y, np.array([0.0, 1.0])], "components": ("z",),
            "eps_bg": 1.0, "eps_fg": 2.0, "n_params": 1, "prims": prims,
            "tree": {"op": "union", "children": list(range(len(prims)))}}
    sc = A_.Scene(desc)
    E = torch.ones(sc.shape, dtype=torch.complex64, device="cuda")
    with pytest.raises(SGError) as e:
        A_.eps_grad_vjp_noalloc(sc, np.array([0.3]), E, E, 1.0)
    assert e.value.code == -3
    # the regular entry point serves the same scene
    g = A_.eps_grad_vjp(sc, np.array([0.3]), E, E, 1.0)
    assert np.isfinite(g).all()
