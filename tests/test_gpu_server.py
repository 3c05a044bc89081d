"""Served form on the GPU: every request's result equals the partition it
gets alone, whatever else shares its run; runs respect the slot and memory
budgets; the footprint estimate bounds the memory partitions really hold."""
import sys
import threading

import numpy as np
import pytest

import oracle
from paper_2012_13618_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_13618_amd as mod
    mod.lib()
    return mod


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _requests():
    out = []
    for i in range(10):
        h = I.random_small(300 + 250 * i, 360 + 300 * i, 2, 4 + 6 * (i % 4), 70 + i,
                           weighted_nodes=i % 3 == 0, weighted_hedges=i % 2 == 1)
        out.append((h, (2, 4, 16, 3, 2)[i % 5], (0.05, 0.03, 0.1)[i % 3]))
    out.append((I.random_small(50, 40, 1, 1, 90), 2, 0.05))   # no hyperedge survives
    out.append((I.random_small(400, 500, 2, 8, 91), 1, 0.05))  # k = 1
    return out


def test_server_results_match_oracle(bp):
    reqs = _requests()
    say("server", len(reqs), "requests")
    with bp.Server(hbm_budget_bytes=32 << 30, max_slots=64) as s:
        tickets = [s.submit(h, k, e) for h, k, e in reqs]
        for t, (h, k, e) in zip(tickets, reqs):
            part, cut, st, stats = s.wait(t)
            ref = oracle.partition(h.num_nodes, h.offsets, h.pins, k, e, h.node_w, h.hedge_w)
            assert np.array_equal(part, ref[0]) and cut == ref[1], (h.name, k, e)
            assert stats.cut == cut and stats.batch_size >= 1
            assert stats.latency_ms >= stats.run_ms >= 0 and stats.queue_ms >= 0


def test_server_from_threads_with_tight_budget(bp):
    """Four submitting threads; a budget that admits only a few requests per
    run and at most three slots: results still equal the plain path."""
    reqs = [(I.serve_request(r), None, None) for r in range(12)]
    reqs = [(h, h.meta["k"], h.meta["eps"]) for h, _, _ in reqs]
    big = max(bp.request_footprint(h.num_nodes, h.num_hedges, h.num_pins, k) for h, k, _ in reqs)
    say("server threads, budget", big * 2)
    results = {}
    with bp.Server(hbm_budget_bytes=2 * big, max_slots=3) as s:
        def client(idx):
            for i in idx:
                h, k, e = reqs[i]
                t = s.submit(h, k, e)
                results[i] = s.wait(t)
        th = [threading.Thread(target=client, args=(list(range(j, 12, 4)),)) for j in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=300)
    assert len(results) == 12
    for i, (h, k, e) in enumerate(reqs):
        part, cut, st, stats = results[i]
        alone, cut_alone, st_alone, _ = bp.partition(h.num_nodes, h.offsets, h.pins, k, e)
        assert np.array_equal(part, alone) and cut == cut_alone and st == st_alone, i
        assert 1 <= stats.batch_size <= 3


def test_queued_requests_share_a_run(bp):
    """One worker: a large request followed at once by small ones; the small
    ones queued behind it are served together by one run, each with its own
    plain result."""
    big = I.serve_request(3)
    small = [I.random_small(500, 600, 2, 10, 200 + i) for i in range(6)]
    with bp.Server(hbm_budget_bytes=64 << 30, workers=1, max_run_pins=big.num_pins) as s:
        tb = s.submit(big, 16, 0.05)
        ts = [s.submit(h, 2, 0.05) for h in small]
        pb, cb, _, sb = s.wait(tb)
        got = [s.wait(t) for t in ts]
    say("batch sizes", sb.batch_size, [g[3].batch_size for g in got])
    assert max(g[3].batch_size for g in got) >= 2
    alone = bp.partition(big.num_nodes, big.offsets, big.pins, 16, 0.05)
    assert np.array_equal(pb, alone[0]) and cb == alone[1]
    for h, g in zip(small, got):
        ref = bp.partition(h.num_nodes, h.offsets, h.pins, 2, 0.05)
        assert np.array_equal(g[0], ref[0]) and g[1] == ref[1]


def test_small_request_does_not_wait_for_a_running_large_one(bp):
    """Continuous admission: a small request submitted while a large k=16
    request is on the device starts on another worker and completes first,
    with its plain result; the large one keeps its plain result too."""
    import time
    big = I.vlsi(seed=31, n=400_000)      # 2.2M pins, k = 16: tens of milliseconds
    small = I.random_small(2000, 2400, 2, 8, 301)
    done = {}
    with bp.Server(hbm_budget_bytes=64 << 30, workers=4) as s:
        tb = s.submit(big, 16, 0.05)
        time.sleep(0.005)                 # the large run is under way
        ts = s.submit(small, 2, 0.05)

        def waiter(name, t):
            r = s.wait(t)
            done[name] = (time.perf_counter(), r)

        th = [threading.Thread(target=waiter, args=a) for a in (("big", tb), ("small", ts))]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=300)
    say("small latency", done["small"][1][3].latency_ms, "ms; big latency", done["big"][1][3].latency_ms, "ms")
    assert done["small"][0] < done["big"][0]
    assert done["small"][1][3].batch_size == 1 and done["big"][1][3].batch_size == 1
    ref = bp.partition(small.num_nodes, small.offsets, small.pins, 2, 0.05)
    assert np.array_equal(done["small"][1][0], ref[0]) and done["small"][1][1] == ref[1]
    alone = bp.partition(big.num_nodes, big.offsets, big.pins, 16, 0.05)
    assert np.array_equal(done["big"][1][0], alone[0]) and done["big"][1][1] == alone[1]


def test_overlapping_runs_keep_every_result(bp):
    """Many requests of mixed sizes from several threads, four workers whose
    runs overlap on the device: every result equals the plain path."""
    reqs = [I.serve_request(r) for r in range(16)]
    results = {}
    with bp.Server(hbm_budget_bytes=64 << 30, workers=4, max_run_pins=1 << 20) as s:
        def client(idx):
            for i in idx:
                h = reqs[i]
                results[i] = s.wait(s.submit(h, h.meta["k"], h.meta["eps"]))
        th = [threading.Thread(target=client, args=(list(range(j, 16, 4)),)) for j in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=300)
    assert len(results) == 16
    for i, h in enumerate(reqs):
        part, cut, st, stats = results[i]
        alone = bp.partition(h.num_nodes, h.offsets, h.pins, h.meta["k"], h.meta["eps"])
        assert np.array_equal(part, alone[0]) and cut == alone[1] and st == alone[2], i


def test_footprint_estimate_bounds_device_memory(bp):
    cases = [(I.vlsi(), 2, 0.05), (I.vlsi(), 16, 0.05), (I.column_net(), 8, 0.03),
             (I.column_net(dmin=2), 8, 0.03), (I.serve_request(7), 16, 0.05), (I.tiny(), 2, 0.05),
             (I.batch_member(255), 4, 0.05),
             (I.random_small(20000, 15000, 1, 400, 5, weighted_hedges=True), 64, 0.03)]
    for h, k, e in cases:
        dh = bp.DeviceHypergraph.from_host(h)
        _, _, _, rep = bp.partition_device(dh, k, e)
        est = bp.request_footprint(h.num_nodes, h.num_hedges, h.num_pins, k)
        say(h.name, "k", k, "held", rep.device_bytes, "estimate", est, f"{rep.device_bytes / est:.3f}")
        assert rep.device_bytes <= est, h.name
