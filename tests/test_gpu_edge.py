"""Degenerate inputs through the C-ABI against the oracle: shapes that miss
the grid (no candidate in any tile), a scene without parameters, a one-cell
grid, a one-step column, an inverted (empty) box and a zero-radius circle;
and the boundary counts of the gradient kernel's grouped reductions (sine
series of 1, 16 and 17 terms, shared Fourier coefficients of order 1, 6, 7)."""
import numpy as np
import pytest

from oracle import scene as S
from tests.gpu_util import api, fields_c64, rel, to_dev
from paper_2311_05646_amd import workloads as W

pytestmark = pytest.mark.gpu


def _scene(prims, nx, ny, nz, n_params, tree=None, dim=3, comps=("x", "y", "z")):
    Z = W.uniform_nodes(nz, 0.03) if dim == 3 else np.array([0.0, 1.0])
    return {"name": "edge", "dim": dim, "nodes": [W.uniform_nodes(nx, 0.025), W.uniform_nodes(ny, 0.025), Z],
            "components": comps, "eps_bg": 2.1, "eps_fg": 11.7, "n_params": n_params, "prims": prims,
            "tree": tree or {"op": "union", "children": list(range(len(prims)))}}


def _check(desc, p, expect_zero_grad=False):
    sc = api().Scene(desc)
    E, A = W.make_fields(desc, 5)
    E, A = E.astype(np.complex64), A.astype(np.complex64)
    eps = api().eps_build(sc, p).cpu().numpy()
    assert np.max(np.abs(eps - S.eps(desc, p))) <= 1e-6
    g = api().eps_grad_vjp(sc, p, to_dev(E), to_dev(A), 1.3)
    gs = api().eps_grad_vjp_sparse(sc, p, to_dev(E), to_dev(A), 1.3)
    assert g.shape == (desc["n_params"],) and gs.shape == (desc["n_params"],)
    if desc["n_params"]:
        ref = S.grad_analytic(desc, p, S.sensitivity(E, A, 1.3))
        if expect_zero_grad:
            # the GPU takes sigmoid tails beyond k|t| = 24 as exactly 0 / 1; the
            # oracle keeps them (here below 1e-60)
            assert np.all(g == 0.0) and np.all(gs == 0.0) and np.max(np.abs(ref)) < 1e-30
        else:
            assert rel(g, ref) <= 1e-4 and rel(gs, ref) <= 1e-4
    return sc


def test_shapes_outside_the_grid():
    prims = [W.box(x=(W.P(0), W.P(1)), y=(W.K(5.0), W.K(6.0)), z=(W.K(0.0), W.K(0.1))),
             W.ellipse(W.P(2), W.K(-3.0), W.K(0.1), z=(W.K(0.0), W.K(0.1)))]
    desc = _scene(prims, 20, 12, 6, 3)
    p = np.array([0.1, 0.3, 0.2])
    sc = _check(desc, p, expect_zero_grad=True)
    eps = api().eps_build(sc, p).cpu().numpy()
    assert np.all(eps == np.float32(2.1))


def test_scene_without_parameters():
    prims = [W.box(x=(W.K(0.11), W.K(0.33)), y=(W.K(0.05), W.K(0.2)), z=(W.K(0.02), W.K(0.11)))]
    _check(_scene(prims, 20, 12, 6, 0), np.zeros(0))


def test_one_cell_grid():
    prims = [W.box(x=(W.P(0), W.P(1)), y=(W.P(2), W.K(0.5)), z=(W.K(-1.0), W.K(1.0)))]
    _check(_scene(prims, 1, 1, 1, 3), np.array([0.007, 0.019, 0.011]))


def test_one_step_column_and_one_sample_rows():
    prims = [W.ellipse(W.P(0), W.P(1), W.P(2), z=(W.K(-1.0), W.K(1.0)), sig=("sigmoid", "fixed", 60.0)),
             W.box(x=(W.P(3), W.K(0.4)), y=None, z=(W.K(-1.0), W.K(1.0)))]
    _check(_scene(prims, 17, 1, 1, 4), np.array([0.2, 0.012, 0.11, 0.31]))


def test_empty_box_and_zero_radius():
    # x0 > x1: the box is empty; r = 0 with a compact sigma: only the support
    # ring around the center can be nonzero
    prims = [W.box(x=(W.P(0), W.P(1)), y=(W.K(0.05), W.K(0.2)), z=(W.K(0.0), W.K(0.15))),
             W.ellipse(W.P(2), W.P(3), W.P(4), z=(W.K(0.0), W.K(0.15)), sig=("linear", "fixed", 40.0)),
             W.box(x=(W.K(0.02), W.K(0.1)), y=(W.K(0.13), W.P(5)), z=(W.K(0.0), W.K(0.15)))]
    _check(_scene(prims, 20, 12, 6, 6), np.array([0.3, 0.12, 0.21, 0.14, 0.0, 0.23]))


@pytest.mark.parametrize("nterm", [1, 16, 17])
def test_series_term_counts(nterm):
    """Sine-series boundaries whose term count is one, exactly one, or just
    over one group of the gradient kernel's 16-term reduction."""
    rng = np.random.Generator(np.random.PCG64(300 + nterm))
    desc, p = W.taper_sine_scene(rng, nx=60, ny=28, nz=6, nterm=nterm, w_in=0.2, w_out=0.6, x_a=0.213,
                                 x_b=1.313, y_m=0.357, amp=0.03)
    _check(desc, p)


@pytest.mark.parametrize("order", [1, 6, 7])
def test_fourier_orders_with_shared_coefficients(order):
    """Fourier scatterers sharing their coefficients at orders 1 and 6 (the
    gradient kernel's per-wavefront running sums, up to order 6) and 7 (the
    per-candidate path of the same kernel)."""
    rng = np.random.Generator(np.random.PCG64(400 + order))
    desc, p = W.psgc_scene(rng, nside=6, nx=60, ny=60, nz=6, order=order)
    _check(desc, p)
