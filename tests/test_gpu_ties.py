"""The kernels' tie and kink rules against the oracle's, element by element,
on scenes whose samples sit exactly on the kinks (tests/ties.py): union sums
of exactly 1, difference operands exactly equal, intersection sums of exactly
N - 1 and linear-sigma arguments of exactly +-1/2 (eq:union,
eq:intersection, the difference reading, Tab. nonlinearfunctions).  Every
value involved is exact in binary, so both sides take the same branch; a
kernel that took the other branch would be off by a whole sample's term."""
import numpy as np
import pytest

from oracle import scene as S
from tests import ties
from tests.gpu_util import api, rel, to_dev
from paper_2311_05646_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", sorted(ties.CASES))
def test_ties_eps_and_gradients(case):
    A_ = api()
    cfg = ties.CASES[case]()
    print(f"[ties] {case}", flush=True)
    sc = A_.Scene(cfg["scene"])
    eps = A_.eps_build(sc, cfg["p"]).cpu().numpy()
    ref_eps = S.eps(cfg["scene"], cfg["p"])
    assert np.max(np.abs(eps - ref_eps)) <= 1e-6
    E, A = cfg["E"].astype(np.complex64), cfg["A"].astype(np.complex64)
    Ed, Ad = to_dev(E), to_dev(A)
    ref = S.grad_analytic(cfg["scene"], cfg["p"], S.sensitivity(E, A, cfg["omega"]))
    ge = W.make_geps(cfg["scene"], 11)
    ref_g = S.grad_analytic(cfg["scene"], cfg["p"], ge.astype(np.float64))
    outs = [(name, fn(sc, cfg["p"], Ed, Ad, cfg["omega"]), ref)
            for name, fn in (("vjp", A_.eps_grad_vjp), ("sparse", A_.eps_grad_vjp_sparse))]
    outs.append(("geps", A_.eps_grad_vjp_geps(sc, cfg["p"], to_dev(ge)), ref_g))
    for name, got, r in outs:
        print(f"[ties] {case} {name}: gpu {np.array2string(got, precision=6)} oracle "
              f"{np.array2string(r, precision=6)}", flush=True)
        scale = np.max(np.abs(r))
        if scale == 0.0:
            # two boxes that only touch: their intersection and its gradient
            # are exactly zero everywhere, the tie samples included
            assert np.all(got == 0.0)
        else:
            assert np.max(np.abs(got - r)) <= 1e-5 * scale
