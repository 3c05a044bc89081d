"""Batched form: many graphs partitioned in one device run.

Every graph of a batch must get exactly the partition and cut that the
oracle gives it alone (and that the single-graph entry point gives it), for
any mix of sizes, k, eps, weights and degenerate members.  At the full
256-graph size the oracle is run on a sample of members and the remaining
members are compared with the single-graph GPU path.
"""
import sys

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


def _empty(n):
    return I.Hypergraph(n, np.zeros(1, np.int32), np.zeros(0, np.int32), np.ones(n, np.int32),
                        np.ones(0, np.int32), name=f"empty-{n}")


def _mixed():
    """(graph, k, eps) triples covering the member kinds a batch can hold."""
    g = []
    g.append((I.random_small(300, 400, 2, 6, 1), 2, 0.05))
    g.append((I.random_small(1000, 900, 1, 40, 2, weighted_nodes=True, weighted_hedges=True), 3, 0.1))
    g.append((I.random_small(40, 30, 1, 1, 3), 2, 0.0))          # only 1-pin hyperedges
    g.append((I.random_small(500, 600, 2, 300, 4, isolated=50), 4, 0.03))
    g.append((I.random_small(200, 150, 2, 8, 5), 1, 0.05))        # k = 1: copied only
    g.append((_empty(0), 2, 0.05))                                 # no nodes
    g.append((_empty(25), 2, 0.05))                                # nodes, no hyperedges
    g.append((I.random_small(2500, 3000, 2, 12, 6), 7, 0.05))
    g.append((I.random_small(60, 50, 2, 5, 7), 64, 0.2))           # k > n
    g.append((I.random_small(3000, 2500, 2, 600, 8, weighted_hedges=True), 8, 0.05))
    g.append((I.random_small(800, 1000, 2, 5, 9, weighted_nodes=True, max_w=40), 2, 0.0))
    return g


def _dev(bp, h):
    return bp.DeviceHypergraph.from_host(h)


def test_batch_mixed_matches_oracle(bp):
    items = _mixed()
    say("batch mixed", len(items))
    hs = [h for h, _, _ in items]
    ks = [k for _, k, _ in items]
    es = [e for _, _, e in items]
    parts, cuts, st, reps = bp.partition_batch_device([_dev(bp, h) for h in hs], ks, es)
    for i, (h, k, e) in enumerate(items):
        ref_part, ref_cut = oracle.partition(h.num_nodes, h.offsets, h.pins, k, e, h.node_w, h.hedge_w)
        got = parts[i].cpu().numpy()
        assert np.array_equal(got, ref_part), (i, h.name, k)
        assert cuts[i] == ref_cut, (i, h.name, k)
        assert reps[i].cut == ref_cut
        _, _, st1, rep1 = bp.partition_device(_dev(bp, h), k, e)
        assert reps[i].max_part_weight == rep1.max_part_weight
        assert reps[i].part_weight_limit == rep1.part_weight_limit
        assert reps[i].balanced == rep1.balanced
    # the host entry point gives the same
    parts2, cuts2, st2, _ = bp.partition_batch(hs, ks, es)
    assert st2 == st and cuts2 == cuts
    for i in range(len(items)):
        assert np.array_equal(parts2[i], parts[i].cpu().numpy())


def test_batch_order_and_neighbours_do_not_matter(bp):
    items = _mixed()
    say("batch permuted")
    rng = np.random.default_rng(11)
    perm = rng.permutation(len(items))
    hs = [items[i][0] for i in perm]
    ks = [items[i][1] for i in perm]
    es = [items[i][2] for i in perm]
    parts, cuts, _, _ = bp.partition_batch(hs, ks, es)
    for j, i in enumerate(perm):
        h, k, e = items[i]
        alone, cut_alone, _, _ = bp.partition(h.num_nodes, h.offsets, h.pins, k, e, h.node_w, h.hedge_w)
        assert np.array_equal(parts[j], alone) and cuts[j] == cut_alone, (i, h.name)


def test_batch_single_and_empty(bp):
    say("batch of one / zero")
    h = I.random_small(700, 800, 2, 10, 21)
    parts, cuts, _, _ = bp.partition_batch([h], [3], [0.05])
    ref = oracle.partition(h.num_nodes, h.offsets, h.pins, 3, 0.05)
    assert np.array_equal(parts[0], ref[0]) and cuts[0] == ref[1]
    parts, cuts, st, _ = bp.partition_batch([], [], [])
    assert parts == [] and cuts == [] and st == 0


def test_batch_policies(bp):
    say("batch policies")
    hs = [I.random_small(900, 1100, 2, 30, 40 + i, weighted_hedges=True) for i in range(4)]
    for pol in (bp.HDH, bp.LWD, bp.RAND):
        prm = bp.params(policy=pol)
        oprm = oracle.params(policy=pol)
        parts, cuts, _, _ = bp.partition_batch(hs, [2, 4, 2, 5], [0.05] * 4, prm=prm)
        for i, (h, k) in enumerate(zip(hs, [2, 4, 2, 5])):
            ref = oracle.partition(h.num_nodes, h.offsets, h.pins, k, 0.05, h.node_w, h.hedge_w, oprm)
            assert np.array_equal(parts[i], ref[0]) and cuts[i] == ref[1], (pol, i)


def test_batch_invalid_member_is_named(bp):
    say("batch invalid member")
    a = I.random_small(50, 40, 2, 4, 1)
    b = I.random_small(50, 40, 2, 4, 2)
    bad = b.pins.copy()
    bad[0] = 50
    dev = [_dev(bp, a), bp.DeviceHypergraph(50, b.offsets, bad)]
    with pytest.raises(bp.BipartError) as ei:
        bp.partition_batch_device(dev, [2, 2], [0.05, 0.05])
    assert ei.value.status == -2 and "graph 1" in str(ei.value)


def test_full_batch_256(bp):
    """The 256-graph batch (k = 2 for even members, 4 for odd): the batched run
    equals the single-graph GPU path on every member and the oracle on the
    eight smallest and the eight largest members."""
    import torch
    say("full batch 256: generating")
    hs = [I.batch_member(i) for i in range(256)]
    ks = [h.meta["k"] for h in hs]
    es = [h.meta["eps"] for h in hs]
    dev = [_dev(bp, h) for h in hs]
    say("full batch 256: running", sum(h.num_pins for h in hs), "pins")
    parts, cuts, st, reps = bp.partition_batch_device(dev, ks, es)
    torch.cuda.synchronize()
    say("  launches", reps[0].kernel_launches, "syncs", reps[0].host_syncs)
    by_size = sorted(range(256), key=lambda i: hs[i].num_pins)
    for i in by_size[:8] + by_size[-8:]:
        say("  oracle on member", i, hs[i].num_pins, "pins")
        ref_part, ref_cut = oracle.partition_hg(hs[i])
        assert np.array_equal(parts[i].cpu().numpy(), ref_part), i
        assert cuts[i] == ref_cut, i
    for i in range(256):
        p1, c1, _, r1 = bp.partition_device(dev[i], ks[i], es[i])
        assert torch.equal(parts[i], p1), i
        assert cuts[i] == c1 and reps[i].max_part_weight == r1.max_part_weight, i


def test_schedules_never_change_results(bp):
    """Every launch schedule gives the same partitions and cuts."""
    items = _mixed() + [(I.batch_member(3), 4, 0.05), (I.batch_member(10), 2, 0.05)]
    hs = [h for h, _, _ in items]
    ks = [k for _, k, _ in items]
    es = [e for _, _, e in items]
    dev = [_dev(bp, h) for h in hs]
    ref_parts, ref_cuts, _, _ = bp.partition_batch_device(dev, ks, es)
    ref_parts = [p.cpu().numpy() for p in ref_parts]
    old = bp.schedule_get()
    try:
        # fuse_max_pins 0: no segment balances in one workgroup; 1 << 30: every
        # segment of <= 8192 nodes does; 5000: a mix within one level.
        # chunk_select_max_nodes 0: balance selections of large segments on the
        # multi-workgroup passes; else in chunks up to that size
        for inc, seg, chunk, fused, fuse, csel in [(0, 0, 1, 0, 0, 0),
                                                   (1 << 30, 16384, 64, 4096, 1 << 30, 1 << 18),
                                                   (1 << 16, 4096, 7, 2, 5000, 50000),
                                                   (2 ** 31 - 1, 100, 3, 64, 1 << 17, 20000)]:
            s = bp.schedule_default()
            s.incremental_min_pins, s.seg_select_max_nodes, s.round_chunk_max, s.fused_pick_lists = \
                inc, seg, chunk, fused
            s.fuse_max_pins = fuse
            s.chunk_select_max_nodes = csel
            bp.schedule_set(s)
            say("schedule", s.as_dict())
            parts, cuts, _, _ = bp.partition_batch_device(dev, ks, es)
            assert cuts == ref_cuts
            for a, b in zip(parts, ref_parts):
                assert np.array_equal(a.cpu().numpy(), b)
            h = hs[-1]
            p1, c1, _, _ = bp.partition_device(dev[-1], ks[-1], es[-1])
            assert np.array_equal(p1.cpu().numpy(), ref_parts[-1]) and c1 == ref_cuts[-1]
    finally:
        bp.schedule_set(old)


def test_autotune_returns_a_valid_schedule(bp):
    hs = [I.batch_member(i) for i in range(6)]
    dev = [_dev(bp, h) for h in hs]
    ks = [h.meta["k"] for h in hs]
    es = [h.meta["eps"] for h in hs]
    best, ms = bp.autotune_batch_device(dev, ks, es)
    say("autotune", best.as_dict(), ms)
    assert ms > 0 and 1 <= best.round_chunk_max <= 64
    old = bp.schedule_get()
    try:
        ref = bp.partition_batch_device(dev, ks, es)
        bp.schedule_set(best)
        got = bp.partition_batch_device(dev, ks, es)
        assert got[1] == ref[1]
        for a, b in zip(got[0], ref[0]):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    finally:
        bp.schedule_set(old)
