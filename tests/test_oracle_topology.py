"""Pin of the oracle's adjoint sensitivity and sigmoid through the paper's
closed-form topology-optimization gradient (eq:top_AD, Sec. "Automatic
differentiation based acceleration"): for the per-pixel map
eps(v) = B (Delta_eps sigma(v) + eps_l 1) with a broadcasting matrix B,
grad_v f = 2 omega Delta_eps sigma(v) (1 - sigma(v)) B^T Im(E E_adj).

The left side is computed from the oracle's pieces (oracle.scene.sensitivity
contracted with central differences of the map built on oracle.sigma); the
right side is the printed formula.  A conjugated product, a dropped factor 2
or omega, or a mis-scaled sigmoid fails it."""
import numpy as np
import pytest

from oracle import scene as S
from oracle.sigma import sigma


@pytest.mark.parametrize("nz", [1, 4])
def test_per_pixel_map_gradient_matches_eq_top_ad(nz):
    rng = np.random.default_rng(11)
    ny, nx = 5, 7
    n = ny * nx
    v = rng.normal(0.0, 1.5, size=n)
    eps_l, deps = 2.085, 9.996
    omega = 2.0 * np.pi / 1.55
    # B enforces planarity: every pixel is repeated along z (m = nz * n)
    B = np.kron(np.ones((nz, 1)), np.eye(n))
    shape = (1, nz, ny, nx)
    E = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    A = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    g = S.sensitivity(E, A, omega).reshape(-1)

    def eps(vv):
        return B @ (deps * sigma("sigmoid", vv) + eps_l)

    h = 1e-6
    lhs = np.empty(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        lhs[i] = g @ (eps(v + e) - eps(v - e)) / (2.0 * h)
    s = 1.0 / (1.0 + np.exp(-v))
    rhs = 2.0 * omega * deps * s * (1.0 - s) * (B.T @ np.imag(E * A).reshape(-1))
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs) < 1e-8
    # unconstrained pixels (sigma dropped, B = I) reduce to 2 omega Delta_eps Im(E E_adj)
    if nz == 1:
        lin = np.array([g @ (deps * np.eye(n)[i]) for i in range(n)])
        assert np.allclose(lin, 2.0 * omega * deps * np.imag(E * A).reshape(-1), rtol=1e-13, atol=0)
