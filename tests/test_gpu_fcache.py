"""The F cache (eps_build, eps_grad_vjp and eps_grad_vjp_geps keep the
in-plane sums F_c of every sample, and a later call whose fields are all
unchanged loads them instead of evaluating them) against kernels that always
evaluate F (scenes created with SG_F_CACHE=1 and =0).  In deterministic mode every
eps and gradient must be bitwise equal, over sequences of calls that repeat
p, change one field, interleave calls that overwrite the scene's staging
(finite differences, the allocation-free entry point, the geps backward) and
change the launch split."""
import os

import numpy as np
import pytest
import torch

from tests.gpu_util import api, config, to_dev

pytestmark = pytest.mark.gpu

NAMES = ["c3_small", "c4_small", "psgc3_small", "psgc3_small_mixed", "taper3_sine_small", "zoo3_union", "zoo2_deep", "blazed_small",
         "levels2", "crowd3", "many2", "polar2d_small"]


def _pair(cfg):
    old = os.environ.get("SG_F_CACHE")
    try:
        os.environ["SG_F_CACHE"] = "1"
        cached = api().Scene(cfg["scene"])
        os.environ["SG_F_CACHE"] = "0"
        plain = api().Scene(cfg["scene"])
    finally:
        if old is None:
            del os.environ["SG_F_CACHE"]
        else:
            os.environ["SG_F_CACHE"] = old
    for sc in (cached, plain):
        sc.set_deterministic(True)
    return cached, plain


def _fields(cfg):
    E = to_dev(cfg["E"].astype(np.complex64))
    A = to_dev(cfg["A"].astype(np.complex64))
    return E, A


def _one_field_changed(cfg, p):
    """p with one parameter moved by a small step (one primitive's field)."""
    q = p.copy()
    q[len(q) // 2] += 1e-4 * max(1e-3, abs(q[len(q) // 2]))
    return q


@pytest.mark.parametrize("name", NAMES)
def test_cached_equals_evaluated_over_call_sequences(name):
    cfg = config(name)
    cached, plain = _pair(cfg)
    E, A = _fields(cfg)
    om = cfg["omega"]
    p0 = cfg["p"]
    p1 = _one_field_changed(cfg, p0)
    rng = np.random.default_rng(3)
    p2 = p0 + 1e-4 * rng.standard_normal(p0.shape) * (np.abs(p0) + 1e-3)
    geps = torch.randn(cached.shape, dtype=torch.float32, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    print(f"[fcache] {name}: n={cached.n_params}", flush=True)

    def both(kind, p):
        if kind == "eps":
            a, b = api().eps_build(cached, p), api().eps_build(plain, p)
            return a.cpu().numpy(), b.cpu().numpy()
        if kind == "vjp":
            return api().eps_grad_vjp(cached, p, E, A, om), api().eps_grad_vjp(plain, p, E, A, om)
        if kind == "geps":
            return api().eps_grad_vjp_geps(cached, p, geps), api().eps_grad_vjp_geps(plain, p, geps)
        raise ValueError(kind)

    seq = [("eps", p0), ("vjp", p0), ("vjp", p0), ("eps", p1), ("vjp", p1), ("geps", p1), ("vjp", p0),
           ("fd", p2), ("vjp", p0), ("noalloc", p2), ("vjp", p0), ("eps", p2), ("launch", None), ("vjp", p2),
           ("eps", p2), ("launch0", None), ("vjp", p1)]
    for i, (kind, p) in enumerate(seq):
        if kind == "fd":
            # overwrites the scene's staging with p +- h
            api().eps_grad_fd(cached, p, E, A, om, cfg.get("h", 1e-6))
            continue
        if kind == "noalloc":
            api().eps_grad_vjp_noalloc(cached, p, E, A, om)
            continue
        if kind == "launch":
            cached.set_launch(32 if cached.shape[-1] >= 32 else 16, 0)
            plain.set_launch(32 if plain.shape[-1] >= 32 else 16, 0)
            continue
        if kind == "launch0":
            cached.set_launch(0, 0)
            plain.set_launch(0, 0)
            continue
        a, b = both(kind, p)
        assert np.array_equal(a, b), (name, i, kind, float(np.max(np.abs(np.asarray(a) - np.asarray(b)))))
