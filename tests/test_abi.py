"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and rejects bad input on the host before touching a GPU."""
import os
import re

import numpy as np
import pytest

import paper_2012_13618_amd as bp
from paper_2012_13618_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "bipart.h")).read()
    return sorted(set(re.findall(r"\b(bp_[a-z_]+)\s*\(", text)))


def test_header_declarations_are_exported():
    lib = bp.lib()
    names = _declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(bp.EXPORTS) == names


def test_default_params_and_status_strings():
    p = bp.default_params()
    assert (p.policy, p.max_levels, p.refine_iters, p.min_coarse_nodes) == (bp.LDH, 25, 2, 100)
    for code, name in bp.STATUS.items():
        assert bp.lib().bp_status_string(code).decode() == name


def _expect(status, fn):
    with pytest.raises(bp.BipartError) as ei:
        fn()
    assert ei.value.status == status, str(ei.value)


def test_host_validation_errors():
    h = I.random_small(20, 15, 2, 4, 0)
    n, off, pins = h.num_nodes, h.offsets, h.pins
    bad = off.copy()
    bad[3] = bad[2] - 1
    _expect(-2, lambda: bp.partition(n, bad, pins, 2, 0.05))
    bad0 = off.copy()
    bad0[0] = 1
    _expect(-2, lambda: bp.partition(n, bad0, pins, 2, 0.05))
    p2 = pins.copy()
    p2[0] = n
    _expect(-2, lambda: bp.partition(n, off, p2, 2, 0.05))
    p3 = pins.copy()
    p3[1] = p3[0]  # node repeated inside hyperedge 0
    _expect(-2, lambda: bp.partition(n, off, p3, 2, 0.05))
    _expect(-1, lambda: bp.partition(n, off, pins, 0, 0.05))
    _expect(-1, lambda: bp.partition(n, off, pins, 2, -0.1))
    _expect(-1, lambda: bp.partition(n, off, pins, 2, float("nan")))
    _expect(-3, lambda: bp.partition(n, off, pins, 2, 0.05, nw=-np.ones(n, np.int32)))
    _expect(-3, lambda: bp.partition(n, off, pins, 2, 0.05,
                                     nw=np.full(n, 2 ** 30, np.int32)))
    _expect(-3, lambda: bp.partition(n, off, pins, 2, 0.05,
                                     hw=np.full(len(off) - 1, 2 ** 29, np.int32)))
    _expect(-1, lambda: bp.partition(n, off, pins, 2, 0.05, prm=bp.params(policy=9)))
    _expect(-1, lambda: bp.partition(n, off, pins, 2, 0.05, prm=bp.params(refine_iters=-1)))
    _expect(-1, lambda: bp.compute_cut(n, off, pins, np.full(n, 5, np.int32), 2))


def test_library_has_no_cpu_fallback():
    # On a machine without a GPU the device work must fail loudly.
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = I.random_small(20, 15, 2, 4, 0)
    _expect(-5, lambda: bp.partition(h.num_nodes, h.offsets, h.pins, 2, 0.05))


def test_batch_host_validation_errors():
    a = I.random_small(30, 20, 2, 4, 1)
    b = I.random_small(30, 20, 2, 4, 2)
    bad = I.Hypergraph(b.num_nodes, b.offsets, b.pins.copy(), b.node_w, b.hedge_w)
    bad.pins[0] = -1
    with pytest.raises(bp.BipartError) as ei:
        bp.partition_batch([a, bad], [2, 2], [0.05, 0.05])
    assert ei.value.status == -2 and "graph 1" in str(ei.value)
    _expect(-1, lambda: bp.partition_batch([a, b], [2, 0], [0.05, 0.05]))
    _expect(-1, lambda: bp.partition_batch([a, b], [2, 2], [0.05, float("inf")]))
    _expect(-3, lambda: bp.partition_batch(
        [a, I.Hypergraph(30, b.offsets, b.pins, np.full(30, 2 ** 27, np.int32), b.hedge_w)],
        [2, 2], [0.05, 0.05]))
    with pytest.raises(ValueError):
        bp.partition_batch([a, b], [2], [0.05, 0.05])


def test_schedule_defaults_and_validation():
    d = bp.schedule_default()
    assert d.as_dict() == {"incremental_min_pins": 1 << 16, "seg_select_max_nodes": 1 << 14,
                           "round_chunk_max": 32, "fused_pick_lists": 8, "fuse_max_pins": 1 << 17,
                           "chunk_select_max_nodes": 1 << 18, "graph_rounds": 0}
    old = bp.schedule_get()
    try:
        s = bp.schedule_default()
        s.round_chunk_max = 8
        bp.schedule_set(s)
        assert bp.schedule_get().round_chunk_max == 8
        for field, bad in [("round_chunk_max", 0), ("round_chunk_max", 65), ("fused_pick_lists", -1),
                           ("incremental_min_pins", -5), ("seg_select_max_nodes", -1), ("fuse_max_pins", -1),
                           ("chunk_select_max_nodes", -1), ("graph_rounds", 2)]:
            s = bp.schedule_default()
            setattr(s, field, bad)
            _expect(-1, lambda: bp.schedule_set(s))
    finally:
        bp.schedule_set(old)


def test_memory_limit_argument_check():
    _expect(-1, lambda: bp.set_memory_limit(-1))
    bp.set_memory_limit(0)
