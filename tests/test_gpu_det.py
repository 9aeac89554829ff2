"""Deterministic reduction mode: the wavefront sums of eq. (1) are added as
exact fixed-point numbers (integer limbs), so the gradient does not depend on
the order in which the additions land and is bitwise repeatable.  It holds
the oracle within the gradient tolerance, and the atomic mode within the
bound a change of tiling is held to: the gcart vertex sums go through
wavefront reductions instead of the LDS buckets (whose FP32 additions land in
hardware order), which groups their FP32 sums differently."""
import numpy as np
import pytest

from oracle import scene as S
from tests.gpu_util import api, config, fields_c64, rel, to_dev
from paper_2311_05646_amd import workloads as W

pytestmark = pytest.mark.gpu

# gcart bucket flushes (zoo, c4), polar coefficient slots (psgc3), dense
# series partials (taper), the levels chain, crowded tiles
CASES = ["c2_small", "c3_small", "c4_small", "zoo2_union", "zoo3_union", "zoo2_difference", "crowd3",
         "psgc3_small", "psgc3_small_local", "psgc3_small_mixed", "taper3_sine_small", "taper3_sine_small37", "levels3"]
GRAD_TOL = 1e-4
ORDER_TOL = 1e-6


def _scene(cfg, det):
    sc = api().Scene(cfg["scene"])
    sc.set_deterministic(det)
    return sc


@pytest.mark.parametrize("name", CASES)
def test_vjp_deterministic(name):
    cfg = config(name)
    print(f"[det-vjp] {name}", flush=True)
    E, A = fields_c64(cfg)
    Ed, Ad = to_dev(E), to_dev(A)
    det = _scene(cfg, True)
    g1 = api().eps_grad_vjp(det, cfg["p"], Ed, Ad, cfg["omega"])
    g2 = api().eps_grad_vjp(det, cfg["p"], Ed, Ad, cfg["omega"])
    atom = api().eps_grad_vjp(_scene(cfg, False), cfg["p"], Ed, Ad, cfg["omega"])
    ref = S.grad_analytic(cfg["scene"], cfg["p"], S.sensitivity(E, A, cfg["omega"]))
    assert np.array_equal(g1, g2)
    assert rel(g1, ref) <= GRAD_TOL
    assert rel(g1, atom) <= ORDER_TOL


@pytest.mark.parametrize("name", CASES)
def test_sparse_and_geps_deterministic(name):
    cfg = config(name)
    print(f"[det-sparse-geps] {name}", flush=True)
    E, A = fields_c64(cfg)
    Ed, Ad = to_dev(E), to_dev(A)
    det = _scene(cfg, True)
    s1 = api().eps_grad_vjp_sparse(det, cfg["p"], Ed, Ad, cfg["omega"])
    s2 = api().eps_grad_vjp_sparse(det, cfg["p"], Ed, Ad, cfg["omega"])
    ge = to_dev(W.make_geps(cfg["scene"], 5))
    q1 = api().eps_grad_vjp_geps(det, cfg["p"], ge)
    q2 = api().eps_grad_vjp_geps(det, cfg["p"], ge)
    atom = _scene(cfg, False)
    s_atom = api().eps_grad_vjp_sparse(atom, cfg["p"], Ed, Ad, cfg["omega"])
    q_atom = api().eps_grad_vjp_geps(atom, cfg["p"], ge)
    assert np.array_equal(s1, s2)
    assert np.array_equal(q1, q2)
    assert rel(s1, s_atom) <= ORDER_TOL
    assert rel(q1, q_atom) <= ORDER_TOL


def test_deterministic_toggle_and_growth():
    """Switching the mode on a live scene, and between tilings, keeps the
    results."""
    cfg = config("c4_small")
    print("[det-toggle] c4_small", flush=True)
    E, A = fields_c64(cfg)
    Ed, Ad = to_dev(E), to_dev(A)
    sc = _scene(cfg, False)
    atom = api().eps_grad_vjp(sc, cfg["p"], Ed, Ad, cfg["omega"])
    sc.set_deterministic(True)
    sc.set_launch(64, 1)                      # one segment per column: fewer blocks
    d1 = api().eps_grad_vjp(sc, cfg["p"], Ed, Ad, cfg["omega"])
    sc.set_launch(0, 0)
    d2 = api().eps_grad_vjp(sc, cfg["p"], Ed, Ad, cfg["omega"])
    d3 = api().eps_grad_vjp(sc, cfg["p"], Ed, Ad, cfg["omega"])
    sc.set_deterministic(False)
    a2 = api().eps_grad_vjp(sc, cfg["p"], Ed, Ad, cfg["omega"])
    assert np.array_equal(d2, d3)
    assert rel(d1, atom) <= 1e-6             # another tiling regroups the FP32 sums
    assert rel(d1, d2) <= 1e-6
    assert rel(d2, atom) <= ORDER_TOL
    assert np.array_equal(a2, atom) or rel(a2, atom) <= 1e-12   # atomics: FP64 order only


def test_out_of_range_contribution_gives_nan():
    """A wavefront contribution beyond the fixed-point range (|.| >= 2^31)
    turns the whole gradient into NaN instead of wrapping silently; the atomic
    mode adds it as FP64."""
    cfg = config("c2_small")
    print("[det-range] c2_small", flush=True)
    ge = to_dev(W.make_geps(cfg["scene"], 5) * 1e15)
    det = _scene(cfg, True)
    g = api().eps_grad_vjp_geps(det, cfg["p"], ge)
    atom = api().eps_grad_vjp_geps(_scene(cfg, False), cfg["p"], ge)
    assert np.all(np.isnan(g))
    assert np.all(np.isfinite(atom)) and np.max(np.abs(atom)) >= 2.0 ** 31
    det.set_deterministic(True)
    ok = api().eps_grad_vjp_geps(det, cfg["p"], to_dev(W.make_geps(cfg["scene"], 5)))
    assert np.all(np.isfinite(ok))            # the range flag is cleared per call


@pytest.mark.parametrize("name", ["c2_small", "c4_small", "zoo3_union", "psgc3_small"])
def test_atomic_run_to_run_spread(name):
    """Atomic mode: repeated calls differ only by the order of the FP64
    atomic additions (spread far below 1e-6 relative)."""
    cfg = config(name)
    print(f"[atomic-spread] {name}", flush=True)
    E, A = fields_c64(cfg)
    Ed, Ad = to_dev(E), to_dev(A)
    sc = _scene(cfg, False)
    runs = [api().eps_grad_vjp(sc, cfg["p"], Ed, Ad, cfg["omega"]) for _ in range(5)]
    spread = max(rel(r, runs[0]) for r in runs[1:])
    print(f"[atomic-spread] {name}: {spread:.2e}", flush=True)
    assert spread <= 1e-12
