"""Serving loop on the GPU: every request's gradient is the same served in a
mixed, continuously batched stream as computed alone (within the reordering
of FP64 atomic additions; bitwise for sessions in deterministic mode), and
matches the oracle on fields drawn by the oracle's own Philox generator."""
import numpy as np
import pytest
import torch

from oracle import philox
from oracle import scene as S
from tests.gpu_util import api, config, rel

pytestmark = pytest.mark.gpu

NAMES = ["c1", "c2_small", "c3_small", "c4_small", "zoo3_union", "zoo2_difference"]


def test_fieldgen_matches_oracle_philox():
    shape = (3, 5, 7, 11)
    E, A = api().fieldgen(shape, 987654321012345)
    Eo, Ao = philox.fields(shape, 987654321012345)
    assert np.max(np.abs(E.cpu().numpy() - Eo)) < 2e-5
    assert np.max(np.abs(A.cpu().numpy() - Ao)) < 2e-5


def _requests(rng, cfgs, per=5):
    reqs = []
    for name, cfg in cfgs.items():
        for i in range(per):
            p = cfg["p"] + 1e-4 * rng.standard_normal(cfg["p"].shape)
            reqs.append((name, p, int(rng.integers(1, 2 ** 62)), cfg["omega"]))
    order = rng.permutation(len(reqs))
    return [reqs[i] for i in order]


@pytest.mark.parametrize("det", [False, True], ids=["atomic", "deterministic"])
def test_alone_equals_mix(det):
    rng = np.random.default_rng(11)
    cfgs = {n: config(n) for n in NAMES}
    scenes = {n: api().Scene(c["scene"]) for n, c in cfgs.items()}
    for sc in scenes.values():
        sc.set_deterministic(det)
    srv = api().Server(hbm_budget_bytes=1 << 30, max_slots=16, max_batch=8, n_streams=2)
    sids = {n: srv.open_session(sc) for n, sc in scenes.items()}
    reqs = _requests(rng, cfgs)
    print(f"[serve] {len(reqs)} requests", flush=True)
    tickets = [srv.submit(sids[n], p, seed, om) for n, p, seed, om in reqs]
    mixed = []
    for t, (n, p, seed, om) in zip(tickets, reqs):
        st, g, stats = srv.poll(t, scenes[n].n_params)
        assert st == "ok"
        mixed.append((g, stats))
    c = srv.counters()
    assert c["completed"] == len(reqs) and c["max_batch"] > 1
    for (n, p, seed, om), (g, _) in zip(reqs, mixed):
        # alone through the server
        t = srv.submit(sids[n], p, seed, om)
        st, g1, s1 = srv.poll(t, scenes[n].n_params)
        assert s1["batch_size"] == 1
        # alone through the single-request entry point, same fields
        E, A = api().fieldgen(scenes[n], seed)
        g2 = api().eps_grad_vjp(scenes[n], p, E, A, om)
        if det:
            assert np.array_equal(g, g1) and np.array_equal(g, g2), n
        else:
            assert rel(g, g1) <= 1e-10 and rel(g, g2) <= 1e-10, n
    srv.close()


@pytest.mark.parametrize("name", ["c3_small", "c4_small", "zoo2_difference"])
def test_served_gradient_matches_oracle(name):
    cfg = config(name)
    sc = api().Scene(cfg["scene"])
    srv = api().Server(hbm_budget_bytes=1 << 30, max_slots=4, max_batch=4, n_streams=2)
    sid = srv.open_session(sc)
    seed = 4242 + len(name)
    t = srv.submit(sid, cfg["p"], seed, cfg["omega"])
    st, g, _ = srv.poll(t, sc.n_params)
    E, A = philox.fields(sc.shape, seed)
    ref = S.grad_analytic(cfg["scene"], cfg["p"], S.sensitivity(E, A, cfg["omega"]))
    assert rel(g, ref) <= 1e-4
    srv.close()


@pytest.mark.parametrize("det", [False, True], ids=["atomic", "deterministic"])
def test_caller_fields_equal_vjp(det):
    """Requests on the caller's field planes (serve_submit_fields): each result
    equals eps_grad_vjp on the same planes, batched with seeded requests."""
    rng = np.random.default_rng(13)
    names = ["c2_small", "c3_small", "c4_small", "zoo3_union"]
    cfgs = {n: config(n) for n in names}
    scenes = {n: api().Scene(c["scene"]) for n, c in cfgs.items()}
    for sc in scenes.values():
        sc.set_deterministic(det)
    planes = {n: (torch.from_numpy(c["E"].astype(np.complex64)).cuda(),
                  torch.from_numpy(c["A"].astype(np.complex64)).cuda()) for n, c in cfgs.items()}
    srv = api().Server(hbm_budget_bytes=1 << 30, max_slots=16, max_batch=8, n_streams=2)
    sids = {n: srv.open_session(sc) for n, sc in scenes.items()}
    sent = []
    for i in range(12):
        n = names[i % len(names)]
        p = cfgs[n]["p"] + 1e-4 * rng.standard_normal(cfgs[n]["p"].shape)
        if i % 3 == 2:      # a seeded request among them
            seed = int(rng.integers(1, 2 ** 62))
            sent.append((n, p, seed, srv.submit(sids[n], p, seed, cfgs[n]["omega"])))
        else:
            E, A = planes[n]
            sent.append((n, p, None, srv.submit_fields(sids[n], p, E, A, cfgs[n]["omega"])))
    print(f"[serve] {len(sent)} caller-field / seeded requests", flush=True)
    for n, p, seed, t in sent:
        st, g, _ = srv.poll(t, scenes[n].n_params)
        assert st == "ok"
        E, A = planes[n] if seed is None else api().fieldgen(scenes[n], seed)
        ref = api().eps_grad_vjp(scenes[n], p, E, A, cfgs[n]["omega"])
        if det:
            assert np.array_equal(g, ref), n
        else:
            assert rel(g, ref) <= 1e-10, n
    srv.close()


@pytest.mark.parametrize("det", [False, True], ids=["atomic", "deterministic"])
def test_sliced_requests_equal_whole(det):
    """max_launch_us slices the 3D taper's requests (about 300 us of estimated
    work each: field generation, then column blocks) over several batches of
    one stream, beside whole small requests; every result equals the whole
    computation."""
    from paper_2311_05646_amd import workloads as W
    rng = np.random.default_rng(17)
    cfgs = {"c3": W.make_c3(with_fields=False), "c4_small": config("c4_small"), "c1": config("c1")}
    names = list(cfgs)
    scenes = {n: api().Scene(c["scene"]) for n, c in cfgs.items()}
    for sc in scenes.values():
        sc.set_deterministic(det)
    srv = api().Server(hbm_budget_bytes=8 << 30, max_slots=16, max_batch=8, n_streams=2, max_launch_us=50)
    sids = {n: srv.open_session(sc) for n, sc in scenes.items()}
    sent = []
    for i in range(9):
        n = names[i % len(names)]
        p = cfgs[n]["p"] + 1e-4 * rng.standard_normal(cfgs[n]["p"].shape)
        seed = int(rng.integers(1, 2 ** 62))
        sent.append((n, p, seed, srv.submit(sids[n], p, seed, cfgs[n]["omega"])))
    for n, p, seed, t in sent:
        st, g, _ = srv.poll(t, scenes[n].n_params)
        assert st == "ok"
        E, A = api().fieldgen(scenes[n], seed)
        ref = api().eps_grad_vjp(scenes[n], p, E, A, cfgs[n]["omega"])
        if det:
            assert np.array_equal(g, ref), n
        else:
            assert rel(g, ref) <= 1e-10, n
        del E, A
    c = srv.counters()
    print(f"[serve] sliced: {c}", flush=True)
    assert c["batches"] >= 3 * sum(1 for n, *_ in sent if n == "c3")     # the taper requests were sliced
    srv.close()
