"""Scheduling logic of the serving loop, on the CPU: the C++ scheduler runs
with its fake executor (no device work; a request's result is
grad_k = 2 p_k + (seed mod 1000) after a fixed delay).  Covers routing of
results to tickets, HBM-budget admission in arrival order, slot limits,
batching of requests that arrive while others run, cancellation, polling
time-outs, invalid requests, an injected launch failure and the budget taken
from SG_HBM_BUDGET."""
import os
import subprocess
import sys
import time

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _server(**kw):
    from paper_2311_05646_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2311_05646_amd import build
        build.build()
    from paper_2311_05646_amd.api import Server
    kw.setdefault("fake_executor", True)
    return Server(**kw)


def _expect(p, seed):
    return 2.0 * np.asarray(p) + (seed % 1000)


def test_results_reach_their_tickets():
    srv = _server(hbm_budget_bytes=1 << 20, max_slots=8, max_batch=4, n_streams=2, fake_us=2000)
    sids = [srv.open_fake_session(n, 1000) for n in (3, 7, 1)]
    rng = np.random.default_rng(0)
    sent = []
    for i in range(30):
        sid = sids[i % 3]
        p = rng.standard_normal(srv.n_params[sid])
        sent.append((srv.submit(sid, p, 1000 + i, 1.0), sid, p, 1000 + i))
    for t, sid, p, seed in sent:
        st, g, stats = srv.poll(t, srv.n_params[sid])
        assert st == "ok"
        assert np.array_equal(g, _expect(p, seed))
        assert stats["submit_ns"] <= stats["admit_ns"] <= stats["launch_ns"] <= stats["done_ns"]
    c = srv.counters()
    assert c["completed"] == 30 and c["bytes_in_use"] == 0
    assert 1 < c["max_batch"] <= 4
    srv.close()


def test_budget_admits_in_arrival_order():
    # budget fits 2 requests of 400 bytes at a time
    srv = _server(hbm_budget_bytes=1000, max_slots=16, max_batch=16, n_streams=1, fake_us=20000)
    sid = srv.open_fake_session(2, 400)
    tickets = [srv.submit(sid, [i, i], i, 1.0) for i in range(6)]
    time.sleep(0.005)
    assert srv.counters()["bytes_in_use"] <= 1000
    admits = []
    for i, t in enumerate(tickets):
        st, g, stats = srv.poll(t, 2)
        assert st == "ok" and np.array_equal(g, _expect([i, i], i))
        admits.append(stats["admit_ns"])
    assert admits == sorted(admits)
    # at most two batches' worth of requests ran at once: 3 rounds of 20 ms
    srv.close()


def test_too_large_is_rejected_immediately():
    from paper_2311_05646_amd._lib import SGError
    srv = _server(hbm_budget_bytes=1000, max_slots=4, max_batch=4, n_streams=1, fake_us=0)
    sid = srv.open_fake_session(1, 5000)
    with pytest.raises(SGError) as e:
        srv.submit(sid, [0.0], 1, 1.0)
    assert e.value.code == -3
    srv.close()


def test_slot_limit():
    srv = _server(hbm_budget_bytes=1 << 30, max_slots=2, max_batch=8, n_streams=4, fake_us=30000)
    sid = srv.open_fake_session(1, 10)
    ts = [srv.submit(sid, [float(i)], i, 1.0) for i in range(5)]
    time.sleep(0.01)
    c = srv.counters()
    assert c["bytes_in_use"] == 20          # two admitted, three waiting
    for t in ts:
        assert srv.poll(t, 1)[0] == "ok"
    assert srv.counters()["max_batch"] <= 2
    srv.close()


def test_continuous_batching_of_late_arrivals():
    srv = _server(hbm_budget_bytes=1 << 30, max_slots=64, max_batch=64, n_streams=2, fake_us=30000)
    sid = srv.open_fake_session(1, 10)
    first = srv.submit(sid, [1.0], 1, 1.0)
    time.sleep(0.005)                         # the first batch is running
    late = [srv.submit(sid, [float(i)], i, 1.0) for i in range(10)]
    st, g, s_first = srv.poll(first, 1)
    stats = [srv.poll(t, 1)[2] for t in late]
    # late arrivals were admitted and launched on the free stream while the
    # first request was still running, several per launch
    assert min(s["launch_ns"] for s in stats) < s_first["done_ns"]
    assert len({s["launch_ns"] for s in stats}) <= 3
    assert max(s["batch_size"] for s in stats) > 1
    srv.close()


def test_cancel_and_timeout():
    from paper_2311_05646_amd._lib import SGError
    srv = _server(hbm_budget_bytes=1 << 30, max_slots=1, max_batch=1, n_streams=1, fake_us=50000)
    sid = srv.open_fake_session(1, 10)
    t1 = srv.submit(sid, [1.0], 1, 1.0)
    t2 = srv.submit(sid, [2.0], 2, 1.0)      # waits behind t1 (one slot)
    assert srv.poll(t1, 1, timeout_us=1000)[0] == "pending"
    srv.cancel(t2)
    with pytest.raises(SGError) as e:
        srv.poll(t2, 1)
    assert e.value.code == -5
    assert srv.poll(t1, 1)[0] == "ok"
    with pytest.raises(SGError):
        srv.poll(t1, 1)                       # retired
    srv.close()


def test_invalid_requests():
    from paper_2311_05646_amd._lib import SGError
    srv = _server(hbm_budget_bytes=1 << 20, max_slots=4, max_batch=4, n_streams=1, fake_us=0)
    sid = srv.open_fake_session(2, 10)
    with pytest.raises(SGError):
        srv.submit(sid, [np.nan, 0.0], 1, 1.0)
    with pytest.raises(SGError):
        srv.submit(sid + 5, [0.0, 0.0], 1, 1.0)
    with pytest.raises(ValueError):
        srv.submit(sid, [0.0], 1, 1.0)
    srv.close()


def test_injected_launch_failure_fails_only_that_batch():
    code = r'''
import sys, numpy as np
sys.path.insert(0, sys.argv[1])
from paper_2311_05646_amd.api import Server
from paper_2311_05646_amd._lib import SGError
srv = Server(hbm_budget_bytes=1 << 20, max_slots=1, max_batch=1, n_streams=1, fake_executor=True, fake_us=1000)
sid = srv.open_fake_session(1, 10)
ts = [srv.submit(sid, [float(i)], i, 1.0) for i in range(4)]
out = []
for t in ts:
    try:
        out.append(srv.poll(t, 1)[0])
    except SGError as e:
        out.append(e.code)
print(out)
srv.close()
'''
    env = dict(os.environ, SG_FAULT_INJECT="launch:1")
    r = subprocess.run([sys.executable, "-c", code, ROOT], capture_output=True, text=True, env=env, timeout=60)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "['ok', -4, 'ok', 'ok']"


@pytest.mark.parametrize("value,expect", [("4K", "-3"), ("8k", "ok"), ("1G", "ok"), ("abc", "create -1"),
                                          ("0", "create -1"), ("12X", "create -1")])
def test_budget_from_environment(value, expect):
    """hbm_budget_bytes = 0 takes SG_HBM_BUDGET (bytes with an optional binary
    K / M / G suffix); a malformed value fails server creation."""
    code = r'''
import sys
sys.path.insert(0, sys.argv[1])
from paper_2311_05646_amd.api import Server
from paper_2311_05646_amd._lib import SGError
try:
    srv = Server(hbm_budget_bytes=0, max_slots=2, max_batch=2, n_streams=1, fake_executor=True, fake_us=0)
except SGError as e:
    print("create", e.code)
    sys.exit(0)
sid = srv.open_fake_session(1, 5000)
try:
    print(srv.poll(srv.submit(sid, [1.0], 3, 1.0), 1)[0])
except SGError as e:
    print(e.code)
srv.close()
'''
    _server(hbm_budget_bytes=1 << 20).close()          # builds the library if needed
    env = dict(os.environ, SG_HBM_BUDGET=value)
    r = subprocess.run([sys.executable, "-c", code, ROOT], capture_output=True, text=True, env=env, timeout=60)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == expect


def test_idle_buffers_count_against_the_budget():
    # a session keeps its buffers for its next requests, but the budget bounds
    # every buffer that exists: another session's request frees the least
    # recently released idle buffer instead of waiting for it forever
    srv = _server(hbm_budget_bytes=1000, max_slots=8, max_batch=8, n_streams=1, fake_us=2000)
    a = srv.open_fake_session(1, 400)
    b = srv.open_fake_session(1, 400)
    ta = [srv.submit(a, [float(i)], i, 1.0) for i in range(2)]
    for t in ta:
        assert srv.poll(t, 1)[0] == "ok"
    c = srv.counters()
    assert c["bytes_in_use"] == 0 and c["bytes_held"] == 800
    st, g, _ = srv.poll(srv.submit(b, [5.0], 7, 1.0), 1, timeout_us=5_000_000)
    assert st == "ok" and np.array_equal(g, _expect([5.0], 7))
    c = srv.counters()
    assert c["bytes_held"] == 800 and c["bytes_in_use"] == 0
    # both sessions keep serving within the budget
    ts = [srv.submit(s, [1.0], 3, 1.0) for s in (a, b, a, b)]
    for t in ts:
        assert srv.poll(t, 1, timeout_us=5_000_000)[0] == "ok"
        assert srv.counters()["bytes_held"] <= 1000
    srv.close()


def test_deep_queue_waits_for_its_own_buffers():
    # a session with a request in flight takes another buffer only from
    # unused budget: its queued requests then wait for its own buffers instead
    # of freeing the idle buffer of another session (every free waits for the
    # device), and that other session's request passes them
    srv = _server(hbm_budget_bytes=1000, max_slots=8, max_batch=8, n_streams=1, fake_us=20000)
    a = srv.open_fake_session(1, 400)
    b = srv.open_fake_session(1, 400)
    assert srv.poll(srv.submit(b, [1.0], 1, 1.0), 1)[0] == "ok"
    assert srv.counters()["bytes_held"] == 400
    ta = [srv.submit(a, [float(i)], 10 + i, 1.0) for i in range(6)]
    time.sleep(0.005)
    tb = srv.submit(b, [2.0], 2, 1.0)
    st, g, sb = srv.poll(tb, 1, timeout_us=5_000_000)
    assert st == "ok" and np.array_equal(g, _expect([2.0], 2))
    done = []
    for i, t in enumerate(ta):
        st, g, sa = srv.poll(t, 1, timeout_us=5_000_000)
        assert st == "ok" and np.array_equal(g, _expect([float(i)], 10 + i))
        assert srv.counters()["bytes_held"] == 800
        done.append(sa["done_ns"])
    # b's request did not wait for a's queue (a's requests run one or two at a time)
    assert sb["done_ns"] < done[2]
    srv.close()


def test_allocation_failure_with_nothing_running_is_retired():
    # every buffer allocation after the first fails: a request that needs a
    # new buffer while nothing runs (so nothing can free memory) comes back
    # SG_E_NOMEM instead of waiting forever
    code = r'''
import sys
sys.path.insert(0, sys.argv[1])
from paper_2311_05646_amd.api import Server
from paper_2311_05646_amd._lib import SGError
srv = Server(hbm_budget_bytes=1 << 20, max_slots=4, max_batch=4, n_streams=1, fake_executor=True, fake_us=1000)
a = srv.open_fake_session(1, 100)
b = srv.open_fake_session(1, 100)
out = []
for s in (a, b, a):
    try:
        out.append(srv.poll(srv.submit(s, [1.0], 1, 1.0), 1, timeout_us=10_000_000)[0])
    except SGError as e:
        out.append(e.code)
print(out, srv.counters()["bytes_held"])
srv.close()
'''
    _server(hbm_budget_bytes=1 << 20).close()
    env = dict(os.environ, SG_FAULT_INJECT="alloc:1")
    r = subprocess.run([sys.executable, "-c", code, ROOT], capture_output=True, text=True, env=env, timeout=60)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "['ok', -2, -2] 0"


def _latency(stats):
    return (stats["done_ns"] - stats["submit_ns"]) * 1e-6


@pytest.mark.parametrize("sliced", [True, False])
def test_large_request_does_not_hold_small_ones(sliced):
    # one stream; a request estimated at 20 ms (bytes at 4.5 TB/s) and a small
    # one right behind it: with max_launch_us the large one is sliced and the
    # small one runs after at most one slice, else it waits for all of it
    srv = _server(hbm_budget_bytes=1 << 40, max_slots=8, max_batch=8, n_streams=1, fake_us=0,
                  max_launch_us=1000 if sliced else 0)
    big = srv.open_fake_session(2, int(4.5e6 * 20000))
    small = srv.open_fake_session(1, 1000)
    tb = srv.submit(big, [1.0, 2.0], 5, 1.0)
    time.sleep(0.002)
    ts = srv.submit(small, [3.0], 6, 1.0)
    st, gs, ss = srv.poll(ts, 1)
    st2, gb, sb = srv.poll(tb, 2)
    assert st == st2 == "ok"
    assert np.array_equal(gb, _expect([1.0, 2.0], 5)) and np.array_equal(gs, _expect([3.0], 6))
    if sliced:
        assert _latency(ss) < 5.0 and _latency(sb) > 15.0
        assert srv.counters()["batches"] >= 20
    else:
        assert ss["done_ns"] >= sb["done_ns"] - 1_000_000
    srv.close()


def test_cancel_a_sliced_request():
    srv = _server(hbm_budget_bytes=1 << 40, max_slots=8, max_batch=8, n_streams=1, fake_us=0, max_launch_us=1000)
    big = srv.open_fake_session(1, int(4.5e6 * 30000))
    small = srv.open_fake_session(1, 1000)
    tb = srv.submit(big, [1.0], 1, 1.0)
    time.sleep(0.004)
    srv.cancel(tb)
    from paper_2311_05646_amd._lib import SGError
    with pytest.raises(SGError) as e:
        srv.poll(tb, 1, timeout_us=5_000_000)
    assert e.value.code == -5
    # the stream is free again and the budget released
    st, g, _ = srv.poll(srv.submit(small, [2.0], 3, 1.0), 1, timeout_us=5_000_000)
    assert st == "ok" and np.array_equal(g, _expect([2.0], 3))
    c = srv.counters()
    assert c["bytes_in_use"] == 0 and c["batches"] < 15
    srv.close()
