"""Parity of the HIP path with the sequential oracle, element by element.

Integer work throughout, so every comparison is exact: gains, matchings,
coarse hypergraphs, bisection sides, part vectors and cuts must be identical.
Inputs are seeded and synthetic; they span all hyperedge schedules (one
thread up to degree 8, one wavefront up to 256, one workgroup up to 8192, and
the global-memory path above that), weighted and unweighted graphs, isolated
nodes, 1-pin hyperedges and the degenerate cases.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2012_13618_amd import inputs as I
from tests.conftest import golden

pytestmark = pytest.mark.gpu

F105 = 4509715660


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


def _huge_graph(seed=5):
    """A graph with one 9000-pin hyperedge (global-memory sort path) plus a
    few hundred small and medium ones."""
    n = 12000
    base = I.random_small(n, 400, 2, 300, seed)
    rng = np.random.default_rng(seed)
    big = np.sort(rng.choice(n, 9000, replace=False)).astype(np.int32)
    off = np.concatenate([base.offsets, [base.offsets[-1] + 9000]]).astype(np.int32)
    pins = np.concatenate([base.pins, big]).astype(np.int32)
    return I.Hypergraph(n, off, pins, np.ones(n, np.int32), np.ones(len(off) - 1, np.int32),
                        name="huge-hedge")


def _golden_graph(name):
    g = golden(name)
    n = g["n"]
    nw = np.asarray(g.get("node_w", [1] * n), np.int32)
    e = len(g["offsets"]) - 1
    hw = np.asarray(g.get("hedge_w", [1] * e), np.int32)
    return I.Hypergraph(n, np.asarray(g["offsets"], np.int32), np.asarray(g["pins"], np.int32),
                        nw, hw, name=name)


def graph_cases():
    yield _golden_graph("fig2_coarsen.json")
    yield _golden_graph("singleton_dedup.json")
    yield _golden_graph("initial_refine.json")
    yield I.random_small(300, 400, 2, 8, 1)
    yield I.random_small(500, 300, 2, 40, 2, weighted_nodes=True, weighted_hedges=True, isolated=7)
    yield I.random_small(3000, 120, 2, 700, 3, weighted_hedges=True)
    yield I.random_small(800, 900, 1, 6, 4, isolated=20)
    yield I.vlsi(seed=12, n=20000)
    yield _huge_graph()


CASES = list(graph_cases())
IDS = [c.name for c in CASES]


def _dev(bp, h):
    return bp.DeviceHypergraph.from_host(h)


@pytest.mark.parametrize("h", CASES, ids=IDS)
def test_gains(bp, h):
    import torch
    say("gains", h.name)
    dh = _dev(bp, h)
    rng = np.random.default_rng(0)
    for t in range(3):
        side = (rng.random(h.num_nodes) < (0.1, 0.5, 0.9)[t]).astype(np.uint8)
        got = bp.step_gains(dh, torch.as_tensor(side).cuda()).cpu().numpy()
        ref = oracle.gains(h.num_nodes, h.offsets, h.pins, side, hw=h.hedge_w)
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("h", CASES, ids=IDS)
@pytest.mark.parametrize("policy", [0, 1, 2, 3, 4])
def test_match(bp, h, policy):
    say("match", h.name, policy)
    got = bp.step_match(_dev(bp, h), policy).cpu().numpy()
    ref = oracle.match(h.num_nodes, h.offsets, h.pins, hw=h.hedge_w, policy=policy)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("h", CASES, ids=IDS)
@pytest.mark.parametrize("policy", [0, 1, 4])
def test_coarsen(bp, h, policy):
    say("coarsen", h.name, policy)
    got = [t.cpu().numpy() for t in bp.step_coarsen(_dev(bp, h), policy)]
    ref = oracle.coarsen(h.num_nodes, h.offsets, h.pins, h.node_w, h.hedge_w, policy=policy)
    for name, a, b in zip(["parent", "offsets", "pins", "node_w", "hedge_w"], got, ref):
        assert np.array_equal(a, b), name


def test_coarsen_chain_vlsi(bp):
    say("coarsen chain vlsi-50k")
    h = I.vlsi(seed=21, n=50000)
    n, off, pins, nw, hw = h.num_nodes, h.offsets, h.pins, h.node_w, h.hedge_w
    for lvl in range(6):
        hh = I.Hypergraph(n, np.asarray(off, np.int32), np.asarray(pins, np.int32),
                          np.asarray(nw, np.int32), np.asarray(hw, np.int32))
        got = [t.cpu().numpy() for t in bp.step_coarsen(_dev(bp, hh))]
        ref = oracle.coarsen(n, off, pins, nw, hw)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), lvl
        _, off, pins, nw, hw = ref
        n = len(nw)
        if len(off) == 1:
            break


@pytest.mark.parametrize("h", CASES, ids=IDS)
def test_initial(bp, h):
    say("initial", h.name)
    dh = _dev(bp, h)
    for k0, k1 in [(1, 1), (2, 1), (1, 3)]:
        got = bp.step_initial(dh, k0, k1).cpu().numpy()
        ref = oracle.initial(h.num_nodes, h.offsets, h.pins, k0, k1, nw=h.node_w, hw=h.hedge_w)
        assert np.array_equal(got, ref), (k0, k1)


@pytest.mark.parametrize("h", CASES, ids=IDS)
def test_refine(bp, h):
    import torch
    say("refine", h.name)
    dh = _dev(bp, h)
    rng = np.random.default_rng(3)
    total = int(h.node_w.sum())
    for t, (frac, iters) in enumerate([(0.5, 2), (0.85, 1), (0.2, 0), (0.5, 3)]):
        side = (rng.random(h.num_nodes) < frac).astype(np.uint8)
        m0, m1 = oracle.bounds(total, 1, 1, F105)
        ref, rstuck = oracle.refine(h.num_nodes, h.offsets, h.pins, side, m0, m1, iters=iters,
                                    nw=h.node_w, hw=h.hedge_w)
        ds = torch.as_tensor(side).cuda()
        stuck = bp.step_refine(dh, ds, m0, m1, iters=iters)
        assert np.array_equal(ds.cpu().numpy(), ref), t
        assert stuck == rstuck


@pytest.mark.parametrize("fuse", [0, 1 << 30], ids=["rounds", "one-workgroup"])
def test_balance_paths(bp, fuse):
    """Both forms of the balance step (a launch per round, or every round of
    a segment in one workgroup) against the oracle, whichever the default
    schedule picks."""
    import torch
    old = bp.schedule_get()
    try:
        s = bp.schedule_default()
        s.fuse_max_pins = fuse
        bp.schedule_set(s)
        say("balance paths", s.as_dict())
        rng = np.random.default_rng(17)
        for h in CASES[3:]:
            dh = _dev(bp, h)
            total = int(h.node_w.sum())
            for frac, iters in [(0.9, 0), (0.12, 1)]:
                side = (rng.random(h.num_nodes) < frac).astype(np.uint8)
                m0, m1 = oracle.bounds(total, 1, 1, F105)
                ref, rstuck = oracle.refine(h.num_nodes, h.offsets, h.pins, side, m0, m1, iters=iters,
                                            nw=h.node_w, hw=h.hedge_w)
                ds = torch.as_tensor(side).cuda()
                stuck = bp.step_refine(dh, ds, m0, m1, iters=iters)
                assert np.array_equal(ds.cpu().numpy(), ref), (h.name, frac)
                assert stuck == rstuck
        for name, make, k, eps in [PARTITION_CASES[1], PARTITION_CASES[4]]:
            h = make()
            ref_part, ref_cut = oracle.partition(h.num_nodes, h.offsets, h.pins, k, eps, h.node_w, h.hedge_w)
            part, cut, _, _ = bp.partition_device(_dev(bp, h), k, eps)
            assert np.array_equal(part.cpu().numpy(), ref_part) and cut == ref_cut, name
    finally:
        bp.schedule_set(old)


@pytest.mark.parametrize("h", CASES, ids=IDS)
def test_bisect(bp, h):
    say("bisect", h.name)
    dh = _dev(bp, h)
    for k0, k1, prm in [(1, 1, oracle.params()), (2, 1, oracle.params(min_coarse_nodes=10)),
                        (1, 1, oracle.params(max_levels=3, refine_iters=1)),
                        (3, 2, oracle.params(policy=oracle.HDH, min_coarse_nodes=0))]:
        F = oracle.eps_factor(k0 + k1, 0.05)
        ref, rlv = oracle.bisect(h.num_nodes, h.offsets, h.pins, k0, k1, F, nw=h.node_w,
                                 hw=h.hedge_w, prm=prm)
        p = bp.params(prm.policy, prm.max_levels, prm.refine_iters, prm.min_coarse_nodes)
        got, lv = bp.step_bisect(dh, k0, k1, F, p)
        assert np.array_equal(got.cpu().numpy(), ref), (k0, k1)
        assert lv == rlv


PARTITION_CASES = [
    ("tiny", lambda: I.tiny(), 2, 0.05),
    ("rand-k3", lambda: I.random_small(2000, 2400, 2, 9, 7, weighted_hedges=True), 3, 0.05),
    ("rand-k4-w", lambda: I.random_small(3000, 3000, 1, 12, 8, weighted_nodes=True), 4, 0.03),
    ("rand-k5", lambda: I.random_small(1500, 2500, 2, 30, 9), 5, 0.1),
    ("vlsi20k-k8", lambda: I.vlsi(seed=13, n=20000), 8, 0.03),
    ("colnet50k-k8", lambda: I.column_net(seed=14, n=50000), 8, 0.03),
    ("huge-k2", lambda: _huge_graph(6), 2, 0.05),
    ("vlsi20k-k16", lambda: I.vlsi(seed=15, n=20000), 16, 0.05),
    ("tiny-k7", lambda: I.tiny(), 7, 0.05),
    # hyperedge weights at the edge of the 16-bit contribution encoding: the
    # finest level has w(e) up to 2^15 - 1 (packed), coarser levels sum
    # merged duplicates past it (int2); and weights past it from the start
    ("hw-32767", lambda: I.random_small(60000, 70000, 2, 6, 12, weighted_hedges=True, max_w=32767), 4, 0.05),
    ("hw-60000", lambda: I.random_small(6000, 7000, 2, 10, 11, weighted_hedges=True, max_w=60000), 4, 0.05),
]


@pytest.mark.parametrize("name,make,k,eps", PARTITION_CASES, ids=[c[0] for c in PARTITION_CASES])
def test_partition(bp, name, make, k, eps):
    say("partition", name, k, eps)
    h = make()
    ref_part, ref_cut = oracle.partition(h.num_nodes, h.offsets, h.pins, k, eps, h.node_w,
                                         h.hedge_w)
    part, cut, st, rep = bp.partition_device(_dev(bp, h), k, eps)
    assert np.array_equal(part.cpu().numpy(), ref_part)
    assert cut == ref_cut
    # host entry point gives the same
    part2, cut2, st2, _ = bp.partition(h.num_nodes, h.offsets, h.pins, k, eps, h.node_w, h.hedge_w)
    assert np.array_equal(part2, ref_part) and cut2 == ref_cut and st2 == st


def test_full_size_vlsi(bp):
    say("partition full vlsi 1M")
    h = I.vlsi()
    ref_part, ref_cut = oracle.partition_hg(h)
    part, cut, st, rep = bp.partition_device(_dev(bp, h), 2, 0.05)
    assert np.array_equal(part.cpu().numpy(), ref_part)
    assert cut == ref_cut
    say("  levels", rep.coarsen_levels, "launches", rep.kernel_launches, "syncs", rep.host_syncs)


@pytest.mark.parametrize("k", [2, 7, 64, 100])
def test_compute_cut(bp, k):
    import torch
    say("cut", k)
    h = I.random_small(5000, 4000, 1, 300, 31, weighted_hedges=True, weighted_nodes=True)
    rng = np.random.default_rng(k)
    part = rng.integers(0, k, h.num_nodes).astype(np.int32)
    ref = oracle.cut(h.num_nodes, h.offsets, h.pins, part, k, hw=h.hedge_w, nw=h.node_w)
    assert bp.compute_cut(h.num_nodes, h.offsets, h.pins, part, k, h.node_w, h.hedge_w) == ref
    got = bp.compute_cut_device(_dev(bp, h), torch.as_tensor(part).cuda(), k)
    assert got == ref


def test_determinism_and_pin_order(bp):
    say("determinism")
    h = I.vlsi(seed=16, n=30000)
    a = bp.partition_device(_dev(bp, h), 4, 0.05)
    b = bp.partition_device(_dev(bp, h), 4, 0.05)
    c = bp.partition_device(_dev(bp, I.shuffle_pins(h, 3)), 4, 0.05)
    pa = a[0].cpu().numpy()
    assert np.array_equal(pa, b[0].cpu().numpy()) and a[1] == b[1]
    assert np.array_equal(pa, c[0].cpu().numpy()) and a[1] == c[1]


def test_degenerate_inputs(bp):
    say("degenerate")
    # no nodes
    part, cut, st, _ = bp.partition(0, [0], [], 2, 0.05)
    assert len(part) == 0 and cut == 0
    # no hyperedges
    ref = oracle.partition(10, [0], [], 2, 0.05)
    part, cut, st, _ = bp.partition(10, [0], [], 2, 0.05)
    assert np.array_equal(part, ref[0]) and cut == ref[1] == 0
    # only 1-pin hyperedges, k = 1, k > n, eps = 0
    h = I.random_small(40, 30, 1, 1, 2)
    for k, eps in [(2, 0.0), (1, 0.05), (64, 0.05), (3, 0.0)]:
        ref = oracle.partition(h.num_nodes, h.offsets, h.pins, k, eps)
        got = bp.partition(h.num_nodes, h.offsets, h.pins, k, eps)
        assert np.array_equal(got[0], ref[0]) and got[1] == ref[1], (k, eps)
    h = I.random_small(50, 60, 2, 5, 3)
    for k, eps in [(1, 0.05), (50, 0.0), (64, 0.2), (2, 0.0)]:
        ref = oracle.partition(h.num_nodes, h.offsets, h.pins, k, eps)
        got = bp.partition(h.num_nodes, h.offsets, h.pins, k, eps)
        assert np.array_equal(got[0], ref[0]) and got[1] == ref[1], (k, eps)


def _zero_weights(h, every=3):
    """Same hypergraph with every `every`-th node weighing 0 (the balance
    prefix then has steps of zero weight)."""
    nw = h.node_w.copy()
    nw[::every] = 0
    return I.Hypergraph(h.num_nodes, h.offsets, h.pins, nw, h.hedge_w, name=h.name + "-w0")


CHUNKS = 1 << 18  # the chunked selection's default (and largest) segment size


SEG = 1 << 15  # the one-workgroup selections' largest segment (balance)


@pytest.mark.parametrize("n,fuse,chunk,zw,seg", [
    (8192, 1 << 30, CHUNKS, False, SEG), (8193, 1 << 30, CHUNKS, False, SEG), (20000, 0, CHUNKS, False, SEG),
    (30000, 0, CHUNKS, False, SEG), (6000, 1 << 30, CHUNKS, True, SEG), (40000, 0, CHUNKS, False, SEG),
    (40000, 0, 0, False, SEG), (CHUNKS, 0, CHUNKS, False, SEG), (CHUNKS + 1, 0, CHUNKS, False, SEG),
    (50000, 0, CHUNKS, True, SEG), (32769, 0, CHUNKS, False, SEG), (20000, 0, CHUNKS, False, 1 << 14)],
    ids=["fused-at-limit", "fused-over-limit", "select-768", "select-1024", "fused-zero-w", "chunked",
         "multi-workgroup", "chunked-at-limit", "chunked-over-limit", "chunked-zero-w", "chunked-one-node-tail",
         "chunked-two"])
def test_balance_size_limits(bp, n, fuse, chunk, zw, seg):
    """Balance steps at the size limits of the one-workgroup kernels (the fused
    rounds at 8192 nodes, the 768- and 1024-thread selections, the chunked
    selection at 16 chunks of 16384 nodes and at two), on the multi-workgroup
    passes, and with zero-weight nodes, against the oracle."""
    import torch
    h = I.random_small(n, int(1.1 * n), 2, 12, 40 + n % 97, weighted_nodes=True, weighted_hedges=True)
    if zw:
        h = _zero_weights(h)
    old = bp.schedule_get()
    try:
        s = bp.schedule_default()
        s.fuse_max_pins = fuse
        s.chunk_select_max_nodes = chunk
        s.seg_select_max_nodes = seg
        s.incremental_min_pins = 0  # the later rounds update their gains from the moves
        bp.schedule_set(s)
        say("balance limits", h.name, s.as_dict())
        dh = _dev(bp, h)
        total = int(h.node_w.sum())
        rng = np.random.default_rng(n)
        for frac, iters in [(0.93, 0), (0.08, 2), (0.6, 1)]:
            side = (rng.random(n) < frac).astype(np.uint8)
            m0, m1 = oracle.bounds(total, 1, 1, F105)
            ref, rstuck = oracle.refine(n, h.offsets, h.pins, side, m0, m1, iters=iters, nw=h.node_w,
                                        hw=h.hedge_w)
            ds = torch.as_tensor(side).cuda()
            stuck = bp.step_refine(dh, ds, m0, m1, iters=iters)
            assert np.array_equal(ds.cpu().numpy(), ref), (frac, iters)
            assert stuck == rstuck
    finally:
        bp.schedule_set(old)
