"""Rounds replayed from captured hipGraphs (schedule knob graph_rounds) give
exactly the results of launching every kernel, for single calls and the
batched form; and the report's per-tree-level depths and imbalance."""
import sys

import numpy as np
import pytest

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


def _with_graphs(bp, on, fn):
    old = bp.schedule_get()
    try:
        s = bp.schedule_get()
        s.graph_rounds = on
        bp.schedule_set(s)
        return fn()
    finally:
        bp.schedule_set(old)


def test_graph_replay_is_bit_identical(bp):
    import torch
    cases = [(I.column_net(n=1_000_000), 8, 0.03), (I.vlsi(seed=13, n=200_000), 2, 0.05)]
    replayed = 0
    for h, k, eps in cases:
        dh = bp.DeviceHypergraph.from_host(h)
        out = {}
        for on in (0, 1):
            part = torch.empty(h.num_nodes, dtype=torch.int32, device="cuda")
            _, cut, st, rep = _with_graphs(bp, on, lambda: bp.partition_device(dh, k, eps, part_out=part))
            out[on] = (part.cpu().numpy(), cut, rep)
            say(h.name, "graphs", on, "cut", cut, "replays", rep.graph_replays, "launches", rep.kernel_launches)
        assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]
        assert out[0][2].graph_replays == 0
        replayed += out[1][2].graph_replays
    assert replayed > 0
    # the batched form, both graphs at once
    dev = [bp.DeviceHypergraph.from_host(h) for h, _, _ in cases]
    ks, es = [k for _, k, _ in cases], [e for _, _, e in cases]
    a = _with_graphs(bp, 0, lambda: bp.partition_batch_device(dev, ks, es))
    b = _with_graphs(bp, 1, lambda: bp.partition_batch_device(dev, ks, es))
    assert a[1] == b[1]
    for x, y in zip(a[0], b[0]):
        assert torch.equal(x, y)
    assert b[3][0].graph_replays > 0


def test_report_levels_and_imbalance(bp):
    import torch
    h = I.column_net(n=200_000)
    dh = bp.DeviceHypergraph.from_host(h)
    part, cut, st, rep = bp.partition_device(dh, 8, 0.03)
    d = rep.as_dict()
    assert len(d["levels"]) == rep.tree_levels == 3
    assert d["levels"][0] == rep.coarsen_levels and all(x >= 0 for x in d["levels"])
    W = int(h.node_w.sum())
    assert abs(rep.imbalance - (rep.max_part_weight * 8 / W - 1.0)) < 1e-12
    assert rep.balanced == (rep.max_part_weight <= rep.part_weight_limit)
