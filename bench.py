#!/usr/bin/env python3
"""Shape-gradient throughput on one MI355X.

A step is one pass of the whole gradient path on the 2D multi-etch blazed
grating workload (4000 x 600 rectilinear grid, dx graded 10-25 nm, dy 10 nm,
3 complex64 field components, 101 primitives, n = 200 edge parameters):
staging of p, eps_build (step 2 of the adjoint loop) and the fused adjoint
gradient eps_grad_vjp (step 5, eq:1 / eq:AD), with p, fields and outputs
resident in HBM.  Four field sets are rotated so the 115 MB per set cannot
be served from the 256 MB Infinity Cache.

Printed JSON line: value = gradient evaluations per second; roofline of the
dominant kernel (the fused VJP column kernel, timed with HIP events on its
own stream inside the library, on every 7th launch of the timed loop); the
GPU finite-difference Jacobian baseline
at matched accuracy; the 3D workloads' kernel bandwidth; and the CPU oracle
timed on a bounded slice of the same workload on this host's cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
import argparse
import ctypes as C
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TIMING_EVERY = 7
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_2311_05646_amd/csrc/sg_kernels.hip", "paper_2311_05646_amd/csrc/sg_column.h",
                  "paper_2311_05646_amd/csrc/sg_device.h", "paper_2311_05646_amd/csrc/sg_internal.h"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_src_sha():
    """Hash of the kernel sources with comments and blank space removed (a
    comment edit leaves the profiled code, and so its counters, valid)."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, f)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def read_traffic(name):
    """HBM bytes per launch of the named kernel from the committed rocprofv3
    counter summary, or None if absent or taken on other kernel sources."""
    path = os.path.join(PROFILE_DIR, f"pmc_{name}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_src_sha") != kernel_src_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


class Fast:
    """Pre-marshalled C-ABI calls for the timed loop (no per-call Python
    argument checks; the checked wrappers in api are used everywhere else)."""

    def __init__(self, api, scene, p_dev, eps_out, grad_out, sets, omega, stream):
        from paper_2311_05646_amd._lib import lib
        self.L = lib()
        self.ctx, self.sc = scene.ctx, scene.handle
        self.p = C.c_void_p(p_dev.data_ptr())
        self.eps = C.c_void_p(eps_out.data_ptr())
        self.grad = C.c_void_p(grad_out.data_ptr())
        self.sets = [(api._plane_ptrs(scene, E), api._plane_ptrs(scene, A)) for E, A in sets]
        self.omega = float(omega)
        self.st = C.c_void_p(stream.cuda_stream)

    def step(self, i):
        fe, fa = self.sets[i % len(self.sets)]
        r1 = self.L.eps_build(self.ctx, self.sc, self.p, 1, self.eps, self.st)
        r2 = self.L.eps_grad_vjp(self.ctx, self.sc, self.p, 1, fe, fa, self.omega, self.grad, 1, self.st)
        if r1 or r2:
            raise RuntimeError(self.L.sg_last_error().decode())


def cpu_baseline(W, cfg, fields0, seconds_budget):
    """The oracle (FP64 NumPy, single thread) on a contiguous x-slice of the
    same workload: eps + reverse-mode gradient; scaled to a whole evaluation."""
    import numpy as np
    from oracle import scene as S
    d, p = cfg["scene"], cfg["p"]
    X, Y, Z = d["nodes"]
    i0, w = 1000, 600
    d2 = dict(d)
    d2["nodes"] = [X[i0:i0 + w + 1], Y, Z]
    E, A = fields0
    E2 = np.ascontiguousarray(E[:, :, :, i0:i0 + w])
    A2 = np.ascontiguousarray(A[:, :, :, i0:i0 + w])
    t = time.perf_counter()
    S.eps(d2, p)
    S.grad_analytic(d2, p, S.sensitivity(E2, A2, cfg["omega"]))
    dt = time.perf_counter() - t
    n_slice = E2.size
    n_full = W.n_samples(d)
    sec_per_eval = dt * n_full / n_slice
    return {"value": 1.0 / sec_per_eval, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"x-slice [{i0}, {i0 + w}) of 4000 columns ({n_slice} of {n_full} samples, all 101 "
                      f"primitives, eps + reverse-mode gradient), {dt:.1f} s, scaled by {n_full / n_slice:.2f}",
            "seconds_per_eval": sec_per_eval}


def time_kernels(api, scene, p_dev, E, A, omega, reps):
    """Column-kernel times of eps_build, eps_grad_vjp and eps_grad_vjp_sparse,
    each call repeated back to back (interleaving them adds the write-back of
    eps to the VJP's HBM traffic).  The sparse VJP reads the fields only where
    d eps / d p can be nonzero: its share of the samples and its rate over the
    bytes it needs are reported apart from the dense kernel's bandwidth."""
    import torch
    g = torch.empty(scene.n_params, dtype=torch.float64, device="cuda")
    gs = torch.empty(scene.n_params, dtype=torch.float64, device="cuda")
    e = torch.empty(scene.shape, dtype=torch.float32, device="cuda")
    for _ in range(3):
        api.eps_build(scene, p_dev, out=e)
        api.eps_grad_vjp(scene, p_dev, E, A, omega, grad=g)
        api.eps_grad_vjp_sparse(scene, p_dev, E, A, omega, grad=gs)
    torch.cuda.synchronize()
    reads = scene.sparse_reads()
    sparse_rel = float(torch.linalg.norm(gs - g) / torch.linalg.norm(g))
    scene.set_timing(True)
    for _ in range(reps):
        api.eps_build(scene, p_dev, out=e)
    torch.cuda.synchronize()
    for _ in range(reps):
        api.eps_grad_vjp(scene, p_dev, E, A, omega, grad=g)
    torch.cuda.synchronize()
    for _ in range(reps):
        api.eps_grad_vjp_sparse(scene, p_dev, E, A, omega, grad=gs)
    torch.cuda.synchronize()
    ve, ne = scene.kernel_time("eps")
    vv, nv = scene.kernel_time("vjp")
    vs, ns = scene.kernel_time("sparse")
    scene.set_timing(False)
    m = scene.shape[0] * scene.shape[1] * scene.shape[2] * scene.shape[3]
    return {"vjp_us": 1e3 * vv / nv, "vjp_GBps": 16.0 * m / (vv / nv * 1e-3) / 1e9,
            "eps_us": 1e3 * ve / ne, "eps_GBps": 4.0 * m / (ve / ne * 1e-3) / 1e9, "samples": m,
            "sparse": {"us": 1e3 * vs / ns, "speedup_vs_dense_vjp": vv / nv / (vs / ns),
                       "samples_read": reads, "read_fraction": reads / m,
                       "GBps_of_bytes_read": 16.0 * reads / (vs / ns * 1e-3) / 1e9,
                       "rel_l2_vs_dense": sparse_rel}}


def time_deterministic(api, scene, p_dev, E, A, omega, reps):
    """Whole-call time of eps_grad_vjp with atomic and with deterministic
    (per-wavefront rows + ordered second pass) reduction, and the two
    gradients' distance."""
    import torch
    res, grads = {}, {}
    for name, det in (("atomic", False), ("deterministic", True)):
        scene.set_deterministic(det)
        g = torch.empty(scene.n_params, dtype=torch.float64, device="cuda")
        for _ in range(3):
            api.eps_grad_vjp(scene, p_dev, E, A, omega, grad=g)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            api.eps_grad_vjp(scene, p_dev, E, A, omega, grad=g)
        torch.cuda.synchronize()
        res[name + "_call_us"] = 1e6 * (time.perf_counter() - t) / reps
        grads[name] = g
    scene.set_deterministic(False)
    res["rel_l2"] = float(torch.linalg.norm(grads["deterministic"] - grads["atomic"]) /
                          torch.linalg.norm(grads["atomic"]))
    return res


def kernels_3d(api, W, gen, reps):
    """Column-kernel bandwidth of eps_build and eps_grad_vjp on the 3D taper
    (600x240x100), the 3D polarization-splitting grating with elliptical holes
    (400x400x80), the same grating with Fourier-radius scatterers whose 12
    shape coefficients are global parameters, and the taper with its
    100-term sine-series boundary."""
    import torch
    dev = torch.device("cuda", 0)
    also = {}
    for name, mk in (("c3", W.make_c3), ("c4", W.make_c4), ("psgc3", W.make_psgc), ("taper3_sine", W.make_taper_sine)):
        log(f"[bench] {name} kernels")
        c = mk(with_fields=False)
        sc = api.Scene(c["scene"])
        E = torch.complex(torch.randn(sc.shape, device=dev, generator=gen), torch.randn(sc.shape, device=dev, generator=gen))
        A = torch.complex(torch.randn(sc.shape, device=dev, generator=gen), torch.randn(sc.shape, device=dev, generator=gen))
        pd = torch.tensor(c["p"], dtype=torch.float64, device=dev)
        r = time_kernels(api, sc, pd, E, A, c["omega"], reps)
        r["vjp_frac_of_peak"] = r["vjp_GBps"] / HBM_PEAK_GBS
        r["n_params"] = sc.n_params
        also[name] = r
        del E, A, sc
        torch.cuda.empty_cache()
    return also


def bench_serving(api, W, seconds=3.0, think_us=200.0):
    """64 closed-loop sessions (the serving mix) against the serving loop:
    each session submits, waits for its gradient, thinks Exp(think_us) and
    submits again with fresh p and a fresh field seed.  The same requests are
    then replayed one at a time through the single-request entry points."""
    import numpy as np
    import torch
    mix = W.make_serving_mix()
    scenes = [api.Scene(c["scene"]) for c in mix]
    srv = api.Server(hbm_budget_bytes=24 << 30, max_slots=64, max_batch=16, n_streams=2)
    sids = [srv.open_session(sc) for sc in scenes]
    rng = np.random.default_rng(5)
    seed_ctr = [1]

    def new_req(i):
        c = mix[i]
        p = c["p"] + c["jitter"] * rng.standard_normal(c["p"].shape)
        seed_ctr[0] += 1
        return p, (W.BASE_SEED << 16) + seed_ctr[0]

    # warm-up: one request per session (allocates each session's buffers)
    warm = [(i, srv.submit(sids[i], *new_req(i), mix[i]["omega"])) for i in range(len(mix))]
    for i, t in warm:
        srv.poll(t, scenes[i].n_params)
    # timed closed loop
    lat, done_reqs = [], []
    outstanding = {}
    next_at = {i: 0.0 for i in range(len(mix))}
    t0 = time.perf_counter()
    while True:
        now = time.perf_counter() - t0
        if now >= seconds and not outstanding:
            break
        for i in range(len(mix)):
            if i not in outstanding and now < seconds and now >= next_at[i]:
                p, sd = new_req(i)
                outstanding[i] = (srv.submit(sids[i], p, sd, mix[i]["omega"]), p, sd)
        for i in list(outstanding):
            t, p, sd = outstanding[i]
            st, g, stt = srv.poll(t, scenes[i].n_params, timeout_us=0)
            if st == "ok":
                del outstanding[i]
                lat.append((stt["done_ns"] - stt["submit_ns"]) * 1e-6)
                done_reqs.append((i, p, sd))
                next_at[i] = (time.perf_counter() - t0) + rng.exponential(think_us * 1e-6)
    wall = time.perf_counter() - t0
    cnt = srv.counters()
    srv.close()
    # the same requests, one at a time
    t1 = time.perf_counter()
    seq_lat = []
    for i, p, sd in done_reqs:
        ts = time.perf_counter()
        E, A = api.fieldgen(scenes[i], sd)
        api.eps_grad_vjp(scenes[i], p, E, A, mix[i]["omega"])      # host grad: waits for the result
        seq_lat.append((time.perf_counter() - ts) * 1e3)
    seq_wall = time.perf_counter() - t1
    kinds = {k: sum(1 for c in mix if c["kind"] == k) for k in ("c1", "c2s", "c3")}
    lat = np.array(lat)
    return {"sessions": len(mix), "session_kinds": kinds, "requests": len(done_reqs), "seconds": wall,
            "grads_per_s": len(done_reqs) / wall, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "batches": cnt["batches"], "max_batch": cnt["max_batch"],
            "sequential": {"grads_per_s": len(done_reqs) / seq_wall,
                           "p50_ms": float(np.percentile(seq_lat, 50)), "p99_ms": float(np.percentile(seq_lat, 99))},
            "speedup_vs_sequential": (len(done_reqs) / wall) / (len(done_reqs) / seq_wall),
            "think_us": think_us}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--quick", action="store_true", help="timed loop only (for profiler runs)")
    ap.add_argument("--calib-copy", action="store_true", help="also run the reference copy kernel (1 GiB)")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--kernels-3d", action="store_true",
                    help="only the 3D workloads' column-kernel loops (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the path shards by grid slab "
              "with one n-vector all-reduce; that multi-GPU path is not built here)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2311_05646_amd import _lib, workloads as W
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2311_05646_amd import build
        build.build()
    from paper_2311_05646_amd import api

    if args.kernels_3d:
        gen = torch.Generator(device=torch.device("cuda", 0))
        gen.manual_seed(W.BASE_SEED)
        print(json.dumps({"3d": kernels_3d(api, W, gen, max(1, args.steps))}), flush=True)
        return

    log("[bench] generating c2 inputs")
    cfg = W.make_c2()
    scene = api.Scene(cfg["scene"])
    dev = torch.device("cuda", 0)
    E0 = torch.from_numpy(cfg["E"]).to(dev)
    A0 = torch.from_numpy(cfg["A"]).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(W.BASE_SEED)
    sets = [(E0, A0)]
    for _ in range(3):
        sets.append(tuple(torch.complex(torch.randn(scene.shape, device=dev, generator=gen),
                                        torch.randn(scene.shape, device=dev, generator=gen)) for _ in range(2)))
    p_dev = torch.tensor(cfg["p"], dtype=torch.float64, device=dev)
    eps_out = torch.empty(scene.shape, dtype=torch.float32, device=dev)
    grad_out = torch.empty(scene.n_params, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    fast = Fast(api, scene, p_dev, eps_out, grad_out, sets, cfg["omega"], stream)

    if args.calib_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        api.util_copy(dst, src)
        torch.cuda.synchronize()
        log("[bench] reference copy of 1 GiB done")

    log(f"[bench] warmup {args.warmup}")
    scene.set_timing(True)          # also fills the event pool the timed loop reuses
    for i in range(max(args.warmup, args.steps)):
        fast.step(i)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    # every TIMING_EVERY-th column launch of each kind is bracketed by HIP
    # events: an event pair adds device time to its launch, and 7 (odd) walks
    # the timed launches over all four field sets
    scene.set_timing(True, every=TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        fast.step(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    vjp_ms, nv = scene.kernel_time("vjp")
    eps_ms, ne = scene.kernel_time("eps")
    scene.set_timing(False)
    sec = t1 - t0
    m = W.n_samples(cfg["scene"])
    vjp_avg_s = vjp_ms / nv * 1e-3
    alg_bytes = 16.0 * m + 16.0 * scene.n_params
    achieved = alg_bytes / vjp_avg_s / 1e9
    traffic = read_traffic("vjp_c2")
    out = {
        "metric": "shape-gradient evals/s (eps_build + fused VJP); HBM GB/s of the VJP kernel vs the GPU "
                  "FD-Jacobian; serve p50/p99",
        "value": args.steps / sec,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 geometry + f32 fields",
        "data": "synthetic (seeded; fields i.i.d. N(0,1) complex64, 4 rotated sets)",
        "config": {"workload": "c2 2D multi-etch blazed grating: 4000x600 rectilinear (dx 10-25 nm graded, "
                               "dy 10 nm), Ex/Ey/Ez complex64, slab minus union of 50 full + 50 shallow etches, "
                               "n=200, linear sigma", "samples": m, "n_params": scene.n_params},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_column<MODE_VJP_FIELDS> (eps_grad_vjp)",
                     "kernel_us": vjp_avg_s * 1e6, "algorithmic_bytes_per_launch": alg_bytes,
                     "timed_launches": nv, "timing_every": TIMING_EVERY},
        "eps_build_kernel": {"us": eps_ms / ne * 1e3, "GBps": 4.0 * m / (eps_ms / ne * 1e-3) / 1e9},
    }
    if args.quick:
        print(json.dumps(out), flush=True)
        return

    # ---- GPU finite-difference Jacobian baseline at matched accuracy
    log("[bench] FD baseline")
    gfd = torch.empty(scene.n_params, dtype=torch.float64, device=dev)
    gvjp = api.eps_grad_vjp(scene, p_dev, E0, A0, cfg["omega"])
    api.eps_grad_fd(scene, p_dev, E0, A0, cfg["omega"], cfg["h"], grad=gfd)
    torch.cuda.synchronize()
    reps = 3
    t = time.perf_counter()
    for _ in range(reps):
        api.eps_grad_fd(scene, p_dev, E0, A0, cfg["omega"], cfg["h"], grad=gfd)
    torch.cuda.synchronize()
    fd_s = (time.perf_counter() - t) / reps
    rel = float(torch.linalg.norm(gfd - gvjp) / torch.linalg.norm(gvjp))
    # the tile-skipping FD (re-rasterizes only where each parameter acts)
    gfs = torch.empty(scene.n_params, dtype=torch.float64, device=dev)
    api.eps_grad_fd_sparse(scene, p_dev, E0, A0, cfg["omega"], cfg["h"], grad=gfs)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        api.eps_grad_fd_sparse(scene, p_dev, E0, A0, cfg["omega"], cfg["h"], grad=gfs)
    torch.cuda.synchronize()
    fds_s = (time.perf_counter() - t) / reps
    vjp_only = time_kernels(api, scene, p_dev, E0, A0, cfg["omega"], 50)
    out["sparse_vjp"] = vjp_only["sparse"]
    out["deterministic_vjp"] = time_deterministic(api, scene, p_dev, E0, A0, cfg["omega"], 50)
    out["fd"] = {"evals_per_s": 1.0 / fd_s, "seconds_per_eval": fd_s, "scheme": "central", "h_um": cfg["h"],
                 "rel_l2_vs_vjp": rel,
                 "vjp_kernel_speedup": fd_s / (vjp_only["vjp_us"] * 1e-6),
                 "step_speedup": fd_s / (sec / args.steps),
                 "fd_alg_GBps": (20.0 * m + scene.n_params * 12.0 * m) / fd_s / 1e9,
                 "sparse": {"evals_per_s": 1.0 / fds_s, "seconds_per_eval": fds_s,
                            "speedup_vs_fd": fd_s / fds_s,
                            "vjp_kernel_speedup": fds_s / (vjp_only["vjp_us"] * 1e-6),
                            "rel_l2_vs_fd": float(torch.linalg.norm(gfs - gfd) / torch.linalg.norm(gfd))}}

    # ---- 3D workloads: kernel bandwidth (not the bench line's workload)
    out["3d"] = kernels_3d(api, W, gen, 20)

    # ---- serving: continuous batching vs one-at-a-time launches
    log("[bench] serving")
    out["serve"] = bench_serving(api, W, seconds=args.serve_seconds)

    # ---- CPU oracle on this host
    log("[bench] cpu baseline (oracle)")
    out["cpu_baseline"] = cpu_baseline(W, cfg, (cfg["E"], cfg["A"]), 20)
    out["cpu_baseline"]["gpu_over_cpu"] = out["value"] / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
