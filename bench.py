#!/usr/bin/env python3
"""Shape-gradient throughput on one MI355X.

A step is one pass of the whole gradient path on the 3D non-adiabatic taper
(600 x 240 x 100 rectilinear grid, 40 nm in plane, dz graded 10-40 nm,
Ex/Ey/Ez complex64 planes, input waveguide + 96-vertex two-sided taper +
output waveguide extruded over a 220 nm slab, n = 192 sidewall parameters):
staging of p, eps_build (step 2 of the adjoint loop) and the fused adjoint
gradient eps_grad_vjp (step 5, eq:1 / eq:AD), with p, fields and outputs
resident in HBM.  The 691 MB of field planes per gradient exceed the 256 MB
Infinity Cache, so one field set is read from HBM on every step.

Printed JSON line: value = gradient evaluations per second on the taper;
roofline of the dominant kernel (the fused VJP column kernel, timed with HIP
events attached to the launch itself inside the library, so they take the
kernel's own start and end, on every 7th launch of the timed loop; traffic
from the committed rocprofv3 counter summary); the 3D
grating coupler (400 x 400 x 80, 1601 primitives, n = 4800) and the 2D
blazed grating with the same structure; the GPU finite-difference Jacobian
baseline on all three at matched accuracy; the paper's own 3D
parameterizations (Fourier scatterers, sine-series taper); serving; and the
CPU oracle on this host's cores, which also checks the whole taper gradient.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
import argparse
import ctypes as C
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TIMING_EVERY = 7
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_2311_05646_amd/csrc/sg_kernels.hip", "paper_2311_05646_amd/csrc/sg_column.h",
                  "paper_2311_05646_amd/csrc/sg_device.h", "paper_2311_05646_amd/csrc/sg_internal.h"]
CPU_WORKERS_MAX = 16       # the host CPU share of one GPU


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


def host_info():
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_allowed": affinity}


class Fast:
    """Pre-marshalled C-ABI calls for the timed loop (no per-call Python
    argument checks; the checked wrappers in api are used everywhere else)."""

    def __init__(self, api, scene, p_devs, eps_out, grad_out, sets, omega, stream):
        from paper_2311_05646_amd._lib import lib
        self.L = lib()
        self.ctx, self.sc = scene.ctx, scene.handle
        self.ps = [C.c_void_p(p.data_ptr()) for p in p_devs]
        self.eps = C.c_void_p(eps_out.data_ptr())
        self.grad = C.c_void_p(grad_out.data_ptr())
        self.sets = [(api._plane_ptrs(scene, E), api._plane_ptrs(scene, A)) for E, A in sets]
        self.omega = float(omega)
        self.st = C.c_void_p(stream.cuda_stream)

    def step(self, i):
        # an optimizer's step: a new p (the library then re-evaluates the
        # in-plane sums in eps_build and reuses them in the gradient at the
        # same p), eps at p, the gradient at p on the step's fields
        fe, fa = self.sets[i % len(self.sets)]
        p = self.ps[i % len(self.ps)]
        r1 = self.L.eps_build(self.ctx, self.sc, p, 1, self.eps, self.st)
        r2 = self.L.eps_grad_vjp(self.ctx, self.sc, p, 1, fe, fa, self.omega, self.grad, 1, self.st)
        if r1 or r2:
            raise RuntimeError(self.L.sg_last_error().decode())


def run_steps(api, W, cfg, sets, steps, warmup, traffic_name=None):
    """The timed step loop of one workload: eps_build + eps_grad_vjp per step
    with p and the fields resident in HBM, the field sets rotated.  Returns
    throughput, the step time and the VJP column kernel's roofline."""
    import torch
    dev = torch.device("cuda", 0)
    scene = api.Scene(cfg["scene"])
    p_dev = torch.tensor(cfg["p"], dtype=torch.float64, device=dev)
    # a new p every step, as in an optimization (4 points 0.1 pm apart, cycled)
    p_devs = [p_dev + 1e-7 * k for k in range(4)]
    eps_out = torch.empty(scene.shape, dtype=torch.float32, device=dev)
    grad_out = torch.empty(scene.n_params, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    fast = Fast(api, scene, p_devs, eps_out, grad_out, sets, cfg["omega"], stream)
    scene.set_timing(True)          # also fills the event pool the timed loop reuses
    for i in range(max(warmup, 2 * TIMING_EVERY)):
        fast.step(i)
    torch.cuda.synchronize()
    # every TIMING_EVERY-th column launch of each kind carries a pair of HIP
    # events that take the kernel's start and end; 7 is odd, so with several
    # field sets the timed launches cycle through all of them
    scene.set_timing(True, every=TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        fast.step(i)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    vjp_ms, nv = scene.kernel_time("vjp")
    eps_ms, ne = scene.kernel_time("eps")
    scene.set_timing(False)
    m = W.n_samples(cfg["scene"])
    vjp_s = vjp_ms / nv * 1e-3
    alg = 16.0 * m + 16.0 * scene.n_params
    achieved = alg / vjp_s / 1e9
    out = {"value": steps / sec, "ms_per_step": 1e3 * sec / steps,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS,
                        "traffic": read_traffic(traffic_name) if traffic_name else None,
                        "kernel": "k_column<MODE_VJP_FIELDS> (eps_grad_vjp)", "kernel_us": vjp_s * 1e6,
                        "algorithmic_bytes_per_launch": alg, "timed_launches": nv, "timing_every": TIMING_EVERY},
           "eps_build_kernel": {"us": eps_ms / ne * 1e3, "GBps": 4.0 * m / (eps_ms / ne * 1e-3) / 1e9,
                                "frac": 4.0 * m / (eps_ms / ne * 1e-3) / 1e9 / HBM_PEAK_GBS},
           "step_GBps": (20.0 * m + 16.0 * scene.n_params) / (sec / steps) / 1e9,
           "samples": m, "n_params": scene.n_params}
    return out, scene, p_dev, grad_out


def fd_baseline(api, scene, p_dev, E, A, cfg, vjp_us, step_ms, reps=2):
    """GPU finite-difference Jacobian (central, every parameter re-rasterized
    over the whole grid, difference plane reduced against g) and its
    tile-skipping form, against the fused VJP on the same inputs."""
    import torch
    dev = torch.device("cuda", 0)
    m = scene.shape[0] * scene.shape[1] * scene.shape[2] * scene.shape[3]
    gvjp = api.eps_grad_vjp(scene, p_dev, E, A, cfg["omega"])
    out = {"scheme": "central", "h_um": cfg["h"], "n_params": scene.n_params}
    for name, fn in (("plain", api.eps_grad_fd), ("tile_skipping", api.eps_grad_fd_sparse)):
        g = torch.empty(scene.n_params, dtype=torch.float64, device=dev)
        fn(scene, p_dev, E, A, cfg["omega"], cfg["h"], grad=g)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn(scene, p_dev, E, A, cfg["omega"], cfg["h"], grad=g)
        torch.cuda.synchronize()
        s = (time.perf_counter() - t) / reps
        out[name] = {"evals_per_s": 1.0 / s, "seconds_per_eval": s,
                     "rel_l2_vs_vjp": float(torch.linalg.norm(g - gvjp) / torch.linalg.norm(gvjp)),
                     "vjp_kernel_speedup": s / (vjp_us * 1e-6), "step_speedup": s / (step_ms * 1e-3)}
    out["plain"]["fd_alg_GBps"] = (20.0 * m + scene.n_params * 12.0 * m) / out["plain"]["seconds_per_eval"] / 1e9
    return out


def time_kernels(api, scene, p_dev, E, A, omega, reps):
    """Column-kernel times of eps_build, eps_grad_vjp, eps_grad_vjp_sparse and
    eps_grad_vjp_geps, each call repeated back to back (interleaving them adds the write-back of
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
    # eps_build at alternating p: every call evaluates the in-plane sums (and
    # keeps them); each gradient at the p of an eps_build before it, as in an
    # optimization step (the in-plane sums come from the cache)
    p_alt = (p_dev + 1e-7, p_dev)
    for i in range(reps):
        api.eps_build(scene, p_alt[i % 2], out=e)
    torch.cuda.synchronize()
    for _ in range(reps):
        api.eps_grad_vjp(scene, p_dev, E, A, omega, grad=g)
    torch.cuda.synchronize()
    for _ in range(reps):
        api.eps_grad_vjp_sparse(scene, p_dev, E, A, omega, grad=gs)
    torch.cuda.synchronize()
    # the eps-upstream gradient (the autograd op's backward) on dF/deps =
    # 2 omega Im(E Eadj): the same gradient from a 4-byte plane
    geps = ((2.0 * omega) * (E * A).imag).float().contiguous()
    gg = torch.empty_like(g)
    for _ in range(reps):
        api.eps_grad_vjp_geps(scene, p_dev, geps, grad=gg)
    torch.cuda.synchronize()
    ve, ne = scene.kernel_time("eps")
    vv, nv = scene.kernel_time("vjp")
    vs, ns = scene.kernel_time("sparse")
    vg, ng = scene.kernel_time("geps")
    scene.set_timing(False)
    geps_rel = float(torch.linalg.norm(gg - g) / torch.linalg.norm(g))
    del geps
    m = scene.shape[0] * scene.shape[1] * scene.shape[2] * scene.shape[3]
    return {"vjp_us": 1e3 * vv / nv, "vjp_GBps": 16.0 * m / (vv / nv * 1e-3) / 1e9,
            "vjp_frac_of_peak": 16.0 * m / (vv / nv * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "eps_us": 1e3 * ve / ne, "eps_GBps": 4.0 * m / (ve / ne * 1e-3) / 1e9, "samples": m,
            "sparse": {"us": 1e3 * vs / ns, "speedup_vs_dense_vjp": vv / nv / (vs / ns),
                       "samples_read": reads, "read_fraction": reads / m,
                       "GBps_of_bytes_read": 16.0 * reads / (vs / ns * 1e-3) / 1e9,
                       "rel_l2_vs_dense": sparse_rel},
            "geps": {"us": 1e3 * vg / ng, "GBps": 4.0 * m / (vg / ng * 1e-3) / 1e9,
                     "frac_of_peak": 4.0 * m / (vg / ng * 1e-3) / 1e9 / HBM_PEAK_GBS, "rel_l2_vs_vjp": geps_rel}}


def time_deterministic(api, scene, p_dev, E, A, omega, reps):
    """Whole-call time of eps_grad_vjp with atomic and with deterministic
    (exact fixed-point) reduction, and the two gradients' distance."""
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


def kernels_3d(api, W, gen, reps, names=("c3", "c4", "psgc3", "taper3_sine")):
    """Column-kernel bandwidth of eps_build, eps_grad_vjp and the sparse VJP,
    each back to back, on the 3D taper, the grating coupler with elliptical
    holes, the same grating with Fourier-radius scatterers whose 12 shape
    coefficients are global parameters, and the taper with its 100-term
    sine-series boundary."""
    import torch
    dev = torch.device("cuda", 0)
    makers = {"c3": W.make_c3, "c4": W.make_c4, "psgc3": W.make_psgc, "taper3_sine": W.make_taper_sine}
    also = {}
    for name in names:
        log(f"[bench] {name} kernels")
        c = makers[name](with_fields=False)
        sc = api.Scene(c["scene"])
        E = torch.complex(torch.randn(sc.shape, device=dev, generator=gen), torch.randn(sc.shape, device=dev, generator=gen))
        A = torch.complex(torch.randn(sc.shape, device=dev, generator=gen), torch.randn(sc.shape, device=dev, generator=gen))
        pd = torch.tensor(c["p"], dtype=torch.float64, device=dev)
        r = time_kernels(api, sc, pd, E, A, c["omega"], reps)
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


def serve_open_loop(api, W, loads=(0.1, 0.3, 0.5, 0.7, 0.9), seconds=1.0, max_launch_us=200, n_streams=2,
                    budget=24 << 30, n_burst=3000):
    """Open-loop Poisson arrivals from the serving mix's 64 sessions, each
    request for a session drawn uniformly.  The capacity these loads are
    fractions of is measured for that same draw: a burst of n_burst requests
    submitted at once, completions per second until the last is done (the
    same burst replayed one request at a time gives the sequential capacity).
    At each load the requests are submitted at their arrival times whatever
    is in flight, latency = completion - submission (both stamped by the
    server).  The same arrival trace is then replayed one request at a time on
    one stream (field generation + eps_grad_vjp, a request starting when it
    has arrived and the previous one is done), its latency counted from the
    arrival."""
    import numpy as np
    mix = W.make_serving_mix()
    scenes = [api.Scene(c["scene"]) for c in mix]
    rng = np.random.default_rng(23)
    srv = api.Server(hbm_budget_bytes=budget, max_slots=64, max_batch=16, n_streams=n_streams,
                     max_launch_us=max_launch_us)
    sids = [srv.open_session(sc) for sc in scenes]
    warm = [(i, srv.submit(sids[i], mix[i]["p"], 1000 + i, mix[i]["omega"])) for i in range(len(mix))]
    for i, t in warm:
        srv.poll(t, scenes[i].n_params)
    seed = [(W.BASE_SEED << 20)]

    def draw():
        i = int(rng.integers(len(mix)))
        seed[0] += 1
        return i, mix[i]["p"] + mix[i]["jitter"] * rng.standard_normal(mix[i]["p"].shape), seed[0]

    def sequential(i, p, sd):
        E, A = api.fieldgen(scenes[i], sd)
        api.eps_grad_vjp(scenes[i], p, E, A, mix[i]["omega"])     # host grad: waits for the result

    burst = [draw() for _ in range(n_burst)]
    t0 = time.perf_counter()
    tickets = [(i, srv.submit(sids[i], p, sd, mix[i]["omega"])) for i, p, sd in burst]
    for i, t in tickets:
        srv.poll(t, scenes[i].n_params)
    capacity = n_burst / (time.perf_counter() - t0)
    t0 = time.perf_counter()
    for i, p, sd in burst:
        sequential(i, p, sd)
    seq_capacity = n_burst / (time.perf_counter() - t0)
    log(f"[bench] open-loop capacity: served {capacity:.0f}/s, one at a time {seq_capacity:.0f}/s")
    out = {"max_launch_us": max_launch_us, "n_streams": n_streams, "hbm_budget_bytes": budget,
           "seconds_per_load": seconds, "capacity_grads_per_s": capacity,
           "sequential_capacity_grads_per_s": seq_capacity, "capacity_burst": n_burst, "loads": []}
    for f in loads:
        lam = f * capacity
        arr = np.cumsum(rng.exponential(1.0 / lam, size=int(lam * seconds * 1.5) + 10))
        arr = arr[arr < seconds]
        trace = [(a,) + draw() for a in arr]
        log(f"[bench] open loop at {f:.0%} of capacity: {len(trace)} requests")
        tickets = []
        t0 = time.perf_counter()
        lag = 0.0
        for a, i, p, sd in trace:
            while time.perf_counter() - t0 < a:
                pass
            lag = max(lag, time.perf_counter() - t0 - a)
            tickets.append((i, srv.submit(sids[i], p, sd, mix[i]["omega"])))
        lat = []
        for i, t in tickets:
            st, g, stt = srv.poll(t, scenes[i].n_params)
            lat.append((stt["done_ns"] - stt["submit_ns"]) * 1e-6)
        # the same trace, one request at a time
        t0 = time.perf_counter()
        seq = []
        for a, i, p, sd in trace:
            while time.perf_counter() - t0 < a:
                pass
            sequential(i, p, sd)
            seq.append((time.perf_counter() - t0 - a) * 1e3)
        lat, seq = np.array(lat), np.array(seq)
        out["loads"].append({"load": f, "rate_per_s": lam, "requests": len(trace),
                             "max_submit_lag_ms": lag * 1e3,
                             "server": {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99))},
                             "sequential": {"p50_ms": float(np.percentile(seq, 50)),
                                            "p99_ms": float(np.percentile(seq, 99))}})
    c = srv.counters()
    out["bytes_held_end"] = c["bytes_held"]
    srv.close()
    return out


# ---------------------------------------------------------------- CPU oracle
_CPU = {}


def _oracle_slice(i0_i1):
    """Oracle eps + reverse-mode gradient over the x-columns [i0, i1) of the
    workload held in _CPU (a whole number of columns: every sample's
    contribution to the gradient depends only on its own fields)."""
    import numpy as np
    from oracle import scene as S
    i0, i1 = i0_i1
    d, p, E, A, omega = _CPU["d"], _CPU["p"], _CPU["E"], _CPU["A"], _CPU["omega"]
    X, Y, Z = d["nodes"]
    d2 = dict(d)
    d2["nodes"] = [X[i0:i1 + 1], Y, Z]
    E2 = np.ascontiguousarray(E[:, :, :, i0:i1])
    A2 = np.ascontiguousarray(A[:, :, :, i0:i1])
    t = time.perf_counter()
    S.eps(d2, p)
    g = S.grad_analytic(d2, p, S.sensitivity(E2, A2, omega))
    return g, time.perf_counter() - t, E2.size


def hbm_reference(api, torch, nbytes, reps=10):
    """A plain streaming copy (the library's sg_util_copy: 16-byte loads and
    stores, grid-stride) of nbytes, timed with events: what one pass of
    reads and writes of that size reaches on this GPU, beside the 8 TB/s
    of the datasheet."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        api.util_copy(dst, src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        api.util_copy(dst, src)
    e1.record()
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    del src, dst
    return {"copy_bytes": nbytes, "copy_us": us, "copy_GBps": 2 * nbytes / (us * 1e-6) / 1e9,
            "kernel": "sg_util_copy (k_copy, 4096 x 256 threads, uint4 grid-stride)"}


def cpu_baseline(cfg, cols=25, single_chunks=24, reps=3):
    """The oracle (FP64 NumPy, not tuned) on this host: the taper split into
    x-slabs of `cols` columns (a uniform x lattice, so a slab's samples and
    their widths are exactly those of the whole grid).  One core runs
    `single_chunks` slabs; then a process pool on all allowed cores (at most
    the 16 of one GPU's share) computes the whole gradient `reps` times (about
    25 s of CPU work in all), and the last is compared with the GPU's."""
    import multiprocessing as mp
    import numpy as np
    nx = len(cfg["scene"]["nodes"][0]) - 1
    dx = np.diff(cfg["scene"]["nodes"][0])
    assert np.allclose(dx, dx[0], rtol=0, atol=1e-12), "slabs need a uniform x lattice"
    _CPU.update(d=cfg["scene"], p=cfg["p"], E=cfg["E"], A=cfg["A"], omega=cfg["omega"])
    chunks = [(i, min(nx, i + cols)) for i in range(0, nx, cols)]
    total = cfg["E"].size
    t = time.perf_counter()
    done = 0
    for ch in chunks[:single_chunks]:
        done += _oracle_slice(ch)[2]
    t1 = time.perf_counter() - t
    host = host_info()
    workers = max(1, min(CPU_WORKERS_MAX, host["cpus_allowed"] or 1))
    with mp.get_context("fork").Pool(workers) as pool:
        t = time.perf_counter()
        for _ in range(reps):
            parts = pool.map(_oracle_slice, chunks, chunksize=1)
        tall = (time.perf_counter() - t) / reps
    grad = np.sum([g for g, _, _ in parts], axis=0)
    _CPU.clear()
    return {"value": 1.0 / tall, "unit": "evals/s", "cores": workers, "kind": "oracle",
            "sample": f"the whole taper gradient (eps + reverse mode, {total} samples) in {len(chunks)} x-slabs of "
                      f"{cols} columns over a {workers}-process pool, {reps} times, {tall:.2f} s wall each",
            "seconds_per_eval": tall,
            "single_core": {"value": 1.0 / (t1 * total / done), "cores": 1,
                            "sample": f"{single_chunks} x-slabs ({done} of {total} samples), {t1:.1f} s, scaled by "
                                      f"{total / done:.2f}"},
            "host": host}, grad


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--quick", action="store_true", help="the headline loop only (for profiler runs)")
    ap.add_argument("--calib-copy", action="store_true", help="also run the reference copy kernel (1 GiB)")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--kernels-3d", action="store_true",
                    help="only the 3D workloads' column-kernel loops (for profiler runs)")
    ap.add_argument("--workload", default="c3", choices=["c3", "c4", "c2"],
                    help="with --quick: the workload of the step loop")
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

    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(W.BASE_SEED)
    if args.calib_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        api.util_copy(dst, src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] reference copy of 1 GiB done")

    if args.kernels_3d:
        print(json.dumps({"3d": kernels_3d(api, W, gen, max(1, args.steps))}), flush=True)
        return

    def randset(shape):
        return tuple(torch.complex(torch.randn(shape, device=dev, generator=gen),
                                   torch.randn(shape, device=dev, generator=gen)) for _ in range(2))

    names = {"c3": ("3D non-adiabatic taper: 600x240x100 rectilinear (40 nm in plane, dz 10-40 nm graded), "
                    "Ex/Ey/Ez complex64, input WG + 96-vertex two-sided taper + output WG extruded 220 nm, "
                    "n=192, linear sigma"),
             "c4": ("3D polarization-splitting grating: 400x400x80 at 25 nm, Ex/Ey/Ez complex64, slab minus "
                    "40x40 elliptical holes (x, y, r each), n=4800, sigmoid k=4sqrt2/dx in plane, linear z"),
             "c2": ("2D multi-etch blazed grating: 4000x600 rectilinear (dx 10-25 nm graded, dy 10 nm), "
                    "Ex/Ey/Ez complex64, slab minus union of 50 full + 50 shallow etches, n=200, linear sigma")}
    makers = {"c3": W.make_c3, "c4": W.make_c4, "c2": W.make_c2}

    def workload(name, steps, warmup):
        log(f"[bench] {name}: inputs")
        cfg = makers[name]()
        shape = (len(cfg["scene"]["components"]),) + tuple(len(a) - 1 for a in cfg["scene"]["nodes"][::-1])
        E0 = torch.from_numpy(cfg["E"]).to(dev)
        A0 = torch.from_numpy(cfg["A"]).to(dev)
        sets = [(E0, A0)]
        if name == "c2":     # 115 MB per set fits the Infinity Cache: rotate four
            sets += [randset(shape) for _ in range(3)]
        log(f"[bench] {name}: {steps} steps")
        res, scene, p_dev, g = run_steps(api, W, cfg, sets, steps, warmup, traffic_name=f"vjp_{name}")
        res["config"] = {"workload": names[name], "samples": res.pop("samples"), "n_params": res.pop("n_params"),
                         "field_sets": len(sets)}
        return res, cfg, scene, p_dev, g, (E0, A0)

    head = args.workload if args.quick else "c3"
    res3, cfg3, sc3, p3, g3, (E3, A3) = workload(head, args.steps, args.warmup)
    out = {
        "metric": "shape-gradient evals/s (eps_build + fused VJP); HBM GB/s of the VJP kernel vs the GPU "
                  "FD-Jacobian; serve p50/p99",
        "value": res3["value"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res3["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 geometry + f32 fields",
        "data": "synthetic (seeded; fields i.i.d. N(0,1) complex64)",
        "config": res3["config"],
        "roofline": res3["roofline"],
        "eps_build_kernel": res3["eps_build_kernel"],
        "step_GBps": res3["step_GBps"],
    }
    if args.quick:
        print(json.dumps(out), flush=True)
        return

    gpu_grad3 = g3.cpu().numpy()
    out["fd"] = {head: fd_baseline(api, sc3, p3, E3, A3, cfg3, res3["roofline"]["kernel_us"],
                                   res3["ms_per_step"])}
    del E3, A3, sc3
    torch.cuda.empty_cache()

    # ---- a plain copy of the VJP's byte count, as a measured reference
    ref = hbm_reference(api, torch, int(res3["roofline"]["algorithmic_bytes_per_launch"]) // 2 // 16 * 16)
    ref["vjp_over_copy"] = res3["roofline"]["achieved"] / ref["copy_GBps"]
    out["hbm_reference"] = ref

    # ---- the grating coupler and the blazed grating, same structure
    for name in ("c4", "c2"):
        r, cfg, sc, pd, g, (E, A) = workload(name, args.steps, args.warmup)
        log(f"[bench] {name}: FD baseline")
        r["fd"] = fd_baseline(api, sc, pd, E, A, cfg, r["roofline"]["kernel_us"], r["ms_per_step"],
                              reps=1 if name == "c4" else 2)
        out["fd"][name] = r.pop("fd")
        if name == "c2":
            out["deterministic_vjp"] = time_deterministic(api, sc, pd, E, A, cfg["omega"], 50)
        out[name] = r
        del E, A, sc, cfg
        torch.cuda.empty_cache()

    # ---- the paper's own 3D parameterizations and the sparse VJP, back to back
    out["3d_kernels"] = kernels_3d(api, W, gen, 20)

    # ---- serving: continuous batching vs one-at-a-time launches
    log("[bench] serving")
    out["serve"] = bench_serving(api, W, seconds=args.serve_seconds)
    out["serve"]["open_loop"] = serve_open_loop(api, W)

    # ---- CPU oracle on this host (and the whole taper gradient checked)
    log("[bench] cpu baseline (oracle)")
    cb, ograd = cpu_baseline(cfg3)
    cb["gpu_over_cpu"] = out["value"] / cb["value"]
    cb["gpu_grad_rel_l2_vs_oracle"] = float(np.linalg.norm(gpu_grad3 - ograd) / np.linalg.norm(ograd))
    out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
