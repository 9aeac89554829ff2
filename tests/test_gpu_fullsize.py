"""Parity at the full workload sizes (the launch configuration bench.py
times): eps on randomly sampled samples of every component; the fused
gradient of every parameter against the oracle's whole-grid gradient (summed
over in-plane tiles, tests/oracle_tiles.py) on the 3D workloads, and on
sampled parameters of the 2D blazed grating, each computed by the oracle over
every sample where that parameter's derivative can be non-zero; plus the GPU
finite-difference Jacobian against the fused gradient at full size."""
import os

import numpy as np
import pytest
import torch

from oracle import primitives as prm
from oracle import scene as S
from oracle.lattice import component_samples
from tests.gpu_util import api, rel, to_dev
from tests.oracle_tiles import tiled_grad
from paper_2311_05646_amd import workloads as W

pytestmark = pytest.mark.gpu

_CACHE = {}


def _setup(name):
    # every full-size workload stays resident once generated (a few GB of
    # host and device memory for all of them), so that the tests of one
    # workload need not follow each other
    if name not in _CACHE:
        print(f"[fullsize] generating {name}", flush=True)
        cfg = W.CONFIGS[name]()
        sc = api().Scene(cfg["scene"])
        E, A = np.asarray(cfg["E"], dtype=np.complex64), np.asarray(cfg["A"], dtype=np.complex64)
        _CACHE[name] = (cfg, sc, E, A, to_dev(E), to_dev(A))
    return _CACHE[name]


def _param_region(desc, p, k, ci):
    """Flat indices (component ci) of every sample where d eps / d p_k can be
    non-zero: the support boxes of the primitives that reference p_k; for a
    vertex of a piecewise-linear boundary, cut to the vertex's hat support in x
    and to the boundary's reach in y."""
    vals = S.resolve(desc, p)
    X, Y, Z = desc["nodes"]
    wmax = [float(np.diff(np.asarray(a)).max()) for a in (X, Y, Z)]
    smp = component_samples(desc, desc["components"][ci])
    nx, ny = len(X) - 1, len(Y) - 1
    out = []
    for i, pr in enumerate(desc["prims"]):
        hits = [fi for fi, f in enumerate(pr["fields"]) if f[2] == k]
        if not hits:
            continue
        lo, hi = prm.bbox(pr, vals[i], wmax)
        lo, hi = list(lo), list(hi)
        if pr["type"] == "gcart":
            M = pr["nvert"]
            xv = pr["consts"]
            for fi in hits:
                if 2 <= fi < 2 + 2 * M:
                    j = (fi - 2) % M
                    side = vals[i][2:2 + M] if fi < 2 + M else vals[i][2 + M:2 + 2 * M]
                    lo[0] = max(lo[0], xv[max(j - 1, 0)] - (1e9 if j == 0 else 0.0))
                    hi[0] = min(hi[0], xv[min(j + 1, M - 1)] + (1e9 if j == M - 1 else 0.0))
                    reach = 0.5 * wmax[1]
                    ys = side[max(j - 1, 0):min(j + 2, M)]
                    lo[1], hi[1] = min(ys) - reach, max(ys) + reach
        sel = [np.nonzero((smp[a][0] >= lo[ai]) & (smp[a][0] <= hi[ai]))[0] for ai, a in enumerate("xyz")]
        iz, iy, ix = np.meshgrid(sel[2], sel[1], sel[0], indexing="ij")
        out.append(((iz * ny + iy) * nx + ix).ravel())
    return np.unique(np.concatenate(out)) if out else np.zeros(0, dtype=np.int64)


def _workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


@pytest.mark.parametrize("name", ["c2", "c3", "c4", "psgc3", "taper3_sine"])
def test_eps_sampled(name):
    cfg, sc, E, A, Ed, Ad = _setup(name)
    eps = api().eps_build(sc, cfg["p"]).cpu().numpy()
    rng = np.random.default_rng(7)
    for ci in range(sc.ncomp):
        flat = eps[ci].ravel()
        # random samples plus samples near every primitive boundary (where eps varies)
        idx = rng.choice(flat.size, 3000, replace=False)
        mid = np.nonzero((flat > cfg["scene"]["eps_bg"] + 1e-3) & (flat < cfg["scene"]["eps_fg"] - 1e-3))[0]
        if mid.size:
            idx = np.concatenate([idx, rng.choice(mid, min(3000, mid.size), replace=False)])
        ref = S.eps_at(cfg["scene"], cfg["p"], ci, idx)
        print(f"[fullsize] {name} comp {ci}: {idx.size} samples", flush=True)
        assert np.max(np.abs(flat[idx] - ref)) <= 1e-6


@pytest.mark.parametrize("name", ["c3", "c4", "psgc3", "taper3_sine"])
def test_vjp_whole_grid_oracle(name):
    """Every parameter of the 3D workloads against the oracle's gradient over
    the whole grid: the taper's 192 sidewall vertices, the grating coupler's
    4800 hole parameters, the Fourier-scatterer grating's 1600 radii and its
    12 shape coefficients that every scatterer shares (they take the spread
    accumulation and the LDS coefficient slots), and the sine-series taper's
    100 terms (each reaches the whole boundary)."""
    cfg, sc, E, A, Ed, Ad = _setup(name)
    got = api().eps_grad_vjp(sc, cfg["p"], Ed, Ad, cfg["omega"])
    print(f"[fullsize] {name}: oracle over the whole grid", flush=True)
    ref = tiled_grad(cfg["scene"], cfg["p"], E, A, cfg["omega"], tile=(40, 40), workers=_workers())
    r = rel(got, ref)
    print(f"[fullsize] {name}: whole-gradient rel L2 {r:.3e}", flush=True)
    assert np.count_nonzero(ref) == ref.size
    assert r <= 1e-4
    if name == "psgc3":
        rg = rel(got[:12], ref[:12])
        print(f"[fullsize] psgc3 shared coefficients rel L2 {rg:.3e}", flush=True)
        assert rg <= 1e-4
    if name == "taper3_sine":
        # every term on its own, not only in the norm of the whole vector
        assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-3


@pytest.mark.parametrize("name,nk", [("c2", 16), ("c3", 10), ("c4", 12)])
def test_vjp_sampled_params(name, nk):
    cfg, sc, E, A, Ed, Ad = _setup(name)
    got = api().eps_grad_vjp(sc, cfg["p"], Ed, Ad, cfg["omega"])
    rng = np.random.default_rng(3)
    ks = np.sort(rng.choice(sc.n_params, nk, replace=False))
    ref = np.zeros(nk)
    d = cfg["scene"]
    for j, k in enumerate(ks):
        acc = np.zeros(d["n_params"])
        for ci in range(sc.ncomp):
            region = _param_region(d, cfg["p"], int(k), ci)
            g_fn = lambda f, ci=ci: S.sensitivity(E[ci].ravel()[f], A[ci].ravel()[f], cfg["omega"])
            S.grad_analytic_region(d, cfg["p"], g_fn, ci, region, acc)
        ref[j] = acc[k]
        print(f"[fullsize] {name} param {k}: gpu {got[k]:.6e} oracle {ref[j]:.6e}", flush=True)
    assert rel(got[ks], ref) <= 1e-4


@pytest.mark.parametrize("name", ["c2", "c3", "c4"])
def test_vjp_sparse_full_size(name):
    """The sparse VJP equals the dense one (pinned to the oracle above) up to
    the order of its sums, at full size and in the launch configuration the
    benchmark times."""
    cfg, sc, E, A, Ed, Ad = _setup(name)
    g_dense = api().eps_grad_vjp(sc, cfg["p"], Ed, Ad, cfg["omega"])
    g_sparse = api().eps_grad_vjp_sparse(sc, cfg["p"], Ed, Ad, cfg["omega"])
    reads = sc.sparse_reads()
    total = int(np.prod(sc.shape))
    print(f"[fullsize] {name} sparse vs dense rel {rel(g_sparse, g_dense):.3e}, "
          f"read {reads} of {total} samples", flush=True)
    assert rel(g_sparse, g_dense) <= 1e-6
    assert 0 < reads <= total


def test_vjp_psgc_full_size():
    """Fourier-radius scatterers at full size: sampled per-scatterer radii
    against the oracle over their regions, and the 12 global shape
    coefficients (every scatterer's boundary feeds them) also against the GPU
    finite-difference Jacobian (the oracle check of every parameter is
    test_vjp_whole_grid_oracle)."""
    cfg, sc, E, A, Ed, Ad = _setup("psgc3")
    got = api().eps_grad_vjp(sc, cfg["p"], Ed, Ad, cfg["omega"])
    rng = np.random.default_rng(4)
    ks = np.sort(rng.choice(np.arange(12, sc.n_params), 8, replace=False))
    d = cfg["scene"]
    ref = np.zeros(len(ks))
    for j, k in enumerate(ks):
        acc = np.zeros(d["n_params"])
        for ci in range(sc.ncomp):
            region = _param_region(d, cfg["p"], int(k), ci)
            g_fn = lambda f, ci=ci: S.sensitivity(E[ci].ravel()[f], A[ci].ravel()[f], cfg["omega"])
            S.grad_analytic_region(d, cfg["p"], g_fn, ci, region, acc)
        ref[j] = acc[k]
        print(f"[fullsize] psgc3 param {k}: gpu {got[k]:.6e} oracle {ref[j]:.6e}", flush=True)
    assert rel(got[ks], ref) <= 1e-4
    fd = api().eps_grad_fd(sc, cfg["p"], Ed, Ad, cfg["omega"], cfg["h"])
    print(f"[fullsize] psgc3 global coefficients fd vs vjp rel {rel(fd[:12], got[:12]):.3e}", flush=True)
    assert rel(fd[:12], got[:12]) <= 1e-4
    assert rel(fd, got) <= 1e-4


def test_vjp_taper_sine_full_size():
    """The taper's 100 sine-series coefficients at full size: the fused
    gradient also against the GPU finite-difference Jacobian, and the sparse
    VJP against the dense one (the oracle check is
    test_vjp_whole_grid_oracle)."""
    cfg, sc, E, A, Ed, Ad = _setup("taper3_sine")
    got = api().eps_grad_vjp(sc, cfg["p"], Ed, Ad, cfg["omega"])
    fd = api().eps_grad_fd(sc, cfg["p"], Ed, Ad, cfg["omega"], cfg["h"])
    sparse = api().eps_grad_vjp_sparse(sc, cfg["p"], Ed, Ad, cfg["omega"])
    print(f"[fullsize] taper3_sine fd vs vjp rel {rel(fd, got):.3e}, sparse vs dense {rel(sparse, got):.3e}",
          flush=True)
    assert rel(fd, got) <= 1e-4
    assert rel(sparse, got) <= 1e-6


@pytest.mark.parametrize("name", ["c2", "c3", "c4"])
def test_fd_matches_vjp_full_size(name):
    cfg, sc, E, A, Ed, Ad = _setup(name)
    g_vjp = api().eps_grad_vjp(sc, cfg["p"], Ed, Ad, cfg["omega"])
    g_fd = api().eps_grad_fd(sc, cfg["p"], Ed, Ad, cfg["omega"], cfg["h"])
    g_fs = api().eps_grad_fd_sparse(sc, cfg["p"], Ed, Ad, cfg["omega"], cfg["h"])
    print(f"[fullsize] {name} fd vs vjp rel {rel(g_fd, g_vjp):.3e}, sparse fd vs fd {rel(g_fs, g_fd):.3e}",
          flush=True)
    assert rel(g_fd, g_vjp) <= 1e-4
    # the plain FD's dot accumulates in FP32 within a block, the fused one in FP64
    assert rel(g_fs, g_fd) <= 1e-6
