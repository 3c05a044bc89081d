"""Served form, host side: configuration and submission errors, unknown
tickets and shutdown with requests still queued.  None of these needs a GPU:
the checks happen before any device work, and a queued request that never
runs completes with BP_ERR_SHUTDOWN."""
import threading
import time

import pytest

import paper_2012_13618_amd as bp
from paper_2012_13618_amd import inputs as I


def _status(fn):
    with pytest.raises(bp.BipartError) as ei:
        fn()
    return ei.value.status


def test_bad_config_is_rejected():
    assert _status(lambda: bp.Server(hbm_budget_bytes=0)) == -1
    assert _status(lambda: bp.Server(max_slots=0)) == -1
    assert _status(lambda: bp.Server(max_batch_delay_us=-1)) == -1
    assert _status(lambda: bp.Server(prm=bp.params(policy=7))) == -1
    assert _status(lambda: bp.Server(workers=0)) == -1
    assert _status(lambda: bp.Server(workers=17)) == -1
    assert _status(lambda: bp.Server(max_run_pins=0)) == -1


def test_footprint_estimate_grows_with_size_and_k():
    a = bp.request_footprint(1000, 1200, 5000, 2)
    assert a > 0
    assert bp.request_footprint(2000, 2400, 10000, 2) > a
    assert bp.request_footprint(1000, 1200, 5000, 16) > a
    assert _status(lambda: bp.request_footprint(-1, 0, 0, 2)) == -1


def test_submission_errors_and_unknown_tickets():
    h = I.random_small(200, 150, 2, 6, 1)
    with bp.Server(hbm_budget_bytes=1 << 40, max_batch_delay_us=10_000_000) as s:
        bad = I.Hypergraph(h.num_nodes, h.offsets, h.pins.copy(), h.node_w, h.hedge_w)
        bad.pins[0] = h.num_nodes
        assert _status(lambda: s.submit(bad, 2, 0.05)) == -2
        assert _status(lambda: s.submit(h, 0, 0.05)) == -1
        assert _status(lambda: s.submit(h, 2, -1.0)) == -1
        assert _status(lambda: s.wait(12345)) == -8
    # a request above the budget is refused at submission
    need = bp.request_footprint(h.num_nodes, h.num_hedges, h.num_pins, 2)
    with bp.Server(hbm_budget_bytes=need - 1) as s:
        assert _status(lambda: s.submit(h, 2, 0.05)) == -6


def test_destroy_completes_queued_requests_with_shutdown():
    h = I.random_small(300, 200, 2, 6, 2)
    s = bp.Server(hbm_budget_bytes=1 << 40, max_batch_delay_us=60_000_000)
    tickets = [s.submit(h, 2, 0.05) for _ in range(3)]
    got = {}

    def waiter(t):
        try:
            s.wait(t)
            got[t] = 0
        except bp.BipartError as e:
            got[t] = e.status

    th = [threading.Thread(target=waiter, args=(t,)) for t in tickets]
    for t in th:
        t.start()
    time.sleep(0.3)  # the waiters are blocked inside the library
    s.close()
    for t in th:
        t.join(timeout=30)
    assert got == {t: -7 for t in tickets}
