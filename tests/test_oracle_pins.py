"""Pins of the sequential oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
hash test vectors, hand-derived worked examples (tests/golden, each citing the
passage it follows), closed forms, exact identities (gain = change of cut,
cut preservation under contraction, cut decomposition over recursive
bisection) and brute force on tiny inputs.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2012_13618_amd import inputs as I
from tests.conftest import golden

F105 = 4509715660  # floor(1.05 * 2**32)


# ---- hash ---------------------------------------------------------------------

def test_hash_published_vectors():
    # MurmurHash3_x86_32 of the empty key equals fmix32(seed): SMHasher's
    # published vectors for seeds 1 and 0xffffffff.
    assert oracle.hash32(1) == 0x514E28B7
    assert oracle.hash32(0xFFFFFFFF) == 0x81F16F39
    assert oracle.hash32(0) == 0


def _unxorshift(x, s):
    r = x
    for _ in range(32 // s + 1):
        r = x ^ (r >> s)
    return r & 0xFFFFFFFF


def test_hash_is_a_bijection():
    inv1 = pow(0x85EBCA6B, -1, 1 << 32)
    inv2 = pow(0xC2B2AE35, -1, 1 << 32)
    rng = np.random.default_rng(0)
    for x in [0, 1, 2, 3, 0xFFFFFFFF] + [int(v) for v in rng.integers(0, 1 << 32, 500)]:
        h = oracle.hash32(x)
        y = _unxorshift(h, 16)
        y = (y * inv2) & 0xFFFFFFFF
        y = _unxorshift(y, 13)
        y = (y * inv1) & 0xFFFFFFFF
        y = _unxorshift(y, 16)
        assert y == x


# ---- cut (problem statement) -----------------------------------------------------

def test_cut_golden_cases():
    for c in golden("cut_cases.json")["cases"]:
        got, _ = oracle.cut(c["n"], c["offsets"], c["pins"], c["part"], c["k"], hw=c["hedge_w"])
        assert got == c["cut"], c["name"]


@pytest.mark.parametrize("seed", range(5))
def test_cut_invariants(seed):
    h = I.random_small(40, 60, 1, 7, seed, weighted_hedges=True)
    rng = np.random.default_rng(seed)
    k = 4
    part = rng.integers(0, k, h.num_nodes).astype(np.int32)
    c, mw = oracle.cut(h.num_nodes, h.offsets, h.pins, part, k, hw=h.hedge_w, nw=h.node_w)
    # all in one part -> 0
    assert oracle.cut(h.num_nodes, h.offsets, h.pins, np.zeros(h.num_nodes, np.int32), k,
                      hw=h.hedge_w)[0] == 0
    # relabelling parts leaves the cut unchanged
    perm = rng.permutation(k).astype(np.int32)
    assert oracle.cut(h.num_nodes, h.offsets, h.pins, perm[part], k, hw=h.hedge_w)[0] == c
    # upper bound: each hyperedge spans at most min(|e|, k) parts
    d = np.diff(h.offsets)
    assert c <= int(np.sum(h.hedge_w.astype(np.int64) * np.maximum(np.minimum(d, k) - 1, 0)))
    assert mw == max(int(h.node_w[part == p].sum()) for p in range(k))


# ---- gains (Algorithm 4) ---------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_gain_is_exact_change_of_cut(seed):
    h = I.random_small(30, 45, 2, 6, seed, weighted_hedges=(seed % 2 == 1), isolated=2)
    rng = np.random.default_rng(100 + seed)
    side = rng.integers(0, 2, h.num_nodes).astype(np.uint8)
    g = oracle.gains(h.num_nodes, h.offsets, h.pins, side, hw=h.hedge_w)
    base, _ = oracle.cut(h.num_nodes, h.offsets, h.pins, side.astype(np.int32), 2, hw=h.hedge_w)
    for u in range(h.num_nodes):
        s2 = side.astype(np.int32).copy()
        s2[u] ^= 1
        moved, _ = oracle.cut(h.num_nodes, h.offsets, h.pins, s2, 2, hw=h.hedge_w)
        assert g[u] == base - moved


def test_gains_golden():
    gd = golden("initial_refine.json")
    n, off, pins = gd["n"], gd["offsets"], gd["pins"]
    assert list(oracle.gains(n, off, pins, np.ones(n, np.uint8))) == gd["gains_all_side1"]
    assert list(oracle.gains(n, off, pins, gd["initial_side"])) == gd["gains_initial_side"]
    assert list(oracle.gains(n, off, pins, [1, 0, 0, 1, 1, 0])) == gd["gains_after_swap1"]


# ---- matching (Algorithm 1) ------------------------------------------------------

@pytest.mark.parametrize("name", ["fig2_coarsen.json", "singleton_dedup.json", "singleton_candidates.json"])
def test_match_golden(name):
    gd = golden(name)
    m = oracle.match(gd["n"], gd["offsets"], gd["pins"], hw=gd["hedge_w"])
    assert list(m) == gd["match"]


def _priority(policy, e, d, w):
    if policy == oracle.HDH:
        return 0xFFFFFFFF - d
    if policy == oracle.LWD:
        return w
    if policy == oracle.HWD:
        return 0xFFFFFFFF - w
    if policy == oracle.RAND:
        return oracle.hash32(e + 1)
    return d


@pytest.mark.parametrize("policy", [oracle.LDH, oracle.HDH, oracle.LWD, oracle.HWD, oracle.RAND])
@pytest.mark.parametrize("seed", range(3))
def test_match_is_lexicographic_argmin(policy, seed):
    # Algorithm 1's three passes must equal a single argmin of the pair
    # (priority, hash) per node, because the hash of distinct ids differs.
    h = I.random_small(60, 80, 1, 6, seed, weighted_hedges=True, isolated=3)
    m = oracle.match(h.num_nodes, h.offsets, h.pins, hw=h.hedge_w, policy=policy)
    best = {}
    for e in range(h.num_hedges):
        key = (_priority(policy, e, int(h.offsets[e + 1] - h.offsets[e]), int(h.hedge_w[e])),
               oracle.hash32(e + 1))
        for v in h.pins[h.offsets[e]:h.offsets[e + 1]]:
            if int(v) not in best or key < best[int(v)][0]:
                best[int(v)] = (key, e)
    for v in range(h.num_nodes):
        assert m[v] == (best[v][1] if v in best else -1)


# ---- coarsening (Algorithm 2) ----------------------------------------------------

@pytest.mark.parametrize("name", ["fig2_coarsen.json", "singleton_dedup.json", "singleton_candidates.json"])
def test_coarsen_golden(name):
    gd = golden(name)
    parent, coff, cpins, cnw, chw = oracle.coarsen(gd["n"], gd["offsets"], gd["pins"],
                                                   gd["node_w"], gd["hedge_w"])
    assert list(parent) == gd["parent"]
    assert list(coff) == gd["coarse_offsets"]
    assert list(cpins) == gd["coarse_pins"]
    assert list(cnw) == gd["coarse_node_w"]
    assert list(chw) == gd["coarse_hedge_w"]


def _check_coarse(h, parent, coff, cpins, cnw, chw, rng):
    n = h.num_nodes
    nc = len(cnw)
    # every coarse id used, weight conserved
    assert parent.min(initial=0) >= 0 and (n == 0 or parent.max() == nc - 1)
    assert len(np.unique(parent)) == nc
    assert int(cnw.sum()) == int(h.node_w.sum())
    # ids follow the smallest member
    first = np.full(nc, n, np.int64)
    np.minimum.at(first, parent, np.arange(n))
    assert np.all(np.diff(first) > 0)
    # coarse hyperedges: >= 2 distinct sorted pins, no repeated pin sets
    sets = set()
    for e in range(len(coff) - 1):
        q = cpins[coff[e]:coff[e + 1]]
        assert len(q) >= 2 and np.all(np.diff(q) > 0) and q[-1] < nc
        t = tuple(int(x) for x in q)
        assert t not in sets
        sets.add(t)
    # cut preservation for random coarse bisections and 3-way splits
    for k in (2, 3):
        for _ in range(4):
            pc = rng.integers(0, k, nc).astype(np.int32)
            cc, _ = oracle.cut(nc, coff, cpins, pc, k, hw=chw)
            cf, _ = oracle.cut(n, h.offsets, h.pins, pc[parent], k, hw=h.hedge_w)
            assert cc == cf


@pytest.mark.parametrize("seed", range(8))
def test_coarsen_invariants(seed):
    h = I.random_small(80, 90, 2, 7, seed, weighted_nodes=(seed % 2 == 0),
                       weighted_hedges=(seed % 3 == 0), isolated=4)
    rng = np.random.default_rng(seed)
    parent, coff, cpins, cnw, chw = oracle.coarsen(h.num_nodes, h.offsets, h.pins, h.node_w,
                                                   h.hedge_w)
    _check_coarse(h, parent, coff, cpins, cnw, chw, rng)
    # at least one hyperedge -> strictly fewer nodes
    assert len(cnw) < h.num_nodes
    # step-one groups are a multi-node matching: each lies inside its hyperedge
    m = oracle.match(h.num_nodes, h.offsets, h.pins)
    for v in range(h.num_nodes):
        if m[v] >= 0:
            assert v in h.pins[h.offsets[m[v]]:h.offsets[m[v] + 1]]


def test_coarsen_chain_on_vlsi_shape():
    h = I.vlsi(seed=11, n=20000)
    rng = np.random.default_rng(1)
    n, off, pins, nw, hw = h.num_nodes, h.offsets, h.pins, h.node_w, h.hedge_w
    for _ in range(3):
        parent, coff, cpins, cnw, chw = oracle.coarsen(n, off, pins, nw, hw)
        hh = I.Hypergraph(n, np.asarray(off, np.int32), np.asarray(pins, np.int32), nw, hw)
        _check_coarse(hh, parent, coff, cpins, cnw, chw, rng)
        n, off, pins, nw, hw = len(cnw), coff, cpins, cnw, chw


# ---- initial partitioning, refinement, balance (Algorithms 3 and 5) --------------

def test_initial_and_refine_golden():
    gd = golden("initial_refine.json")
    n, off, pins = gd["n"], gd["offsets"], gd["pins"]
    side = oracle.initial(n, off, pins, 1, 1)
    assert list(side) == gd["initial_side"]
    mx = gd["max_side_weight"]
    assert oracle.bounds(6, 1, 1, F105) == (mx, mx)
    s2, stuck = oracle.refine(n, off, pins, side, mx, mx, iters=2)
    assert list(s2) == gd["refined_side"] and stuck == 0
    assert oracle.cut(n, off, pins, side.astype(np.int32), 2)[0] == gd["cut_initial"]
    assert oracle.cut(n, off, pins, s2.astype(np.int32), 2)[0] == gd["cut_refined"]


def test_balance_golden():
    gd = golden("balance.json")
    for c in gd["cases"]:
        s, stuck = oracle.refine(6, gd["offsets"], gd["pins"], c["side"], c["max0"], c["max1"],
                                 iters=0, nw=c["node_w"])
        assert list(s) == c["expect_side"] and stuck == c["expect_stuck"], c["derivation"]


def test_bisect_without_hyperedges_closed_form():
    # No hyperedges: all gains are 0, so every ordering is by id.  Initial
    # moves 4 then 4 more nodes (m = ceil(sqrt 10) = 4) to reach half; swaps
    # exchange {0,1}<->{8,9} then {2,3}<->{0,1}; balance moves 0,1,4 back.
    n = 10
    side, levels = oracle.bisect(n, [0], [], 1, 1, F105)
    assert levels == 0
    assert list(side) == [1, 1, 1, 1, 1, 0, 0, 0, 0, 0]
    assert list(oracle.initial(n, [0], [], 1, 1)) == [0] * 8 + [1, 1]


@pytest.mark.parametrize("seed", range(6))
def test_initial_invariants(seed):
    h = I.random_small(50, 60, 2, 5, seed, weighted_nodes=True)
    for k0, k1 in [(1, 1), (2, 1), (3, 5)]:
        side = oracle.initial(h.num_nodes, h.offsets, h.pins, k0, k1, nw=h.node_w)
        w0 = int(h.node_w[side == 0].sum())
        total = int(h.node_w.sum())
        assert w0 * (k0 + k1) >= total * k0 or np.all(side == 0)
        # the moved set came in batches of ceil(sqrt n) unless P1 emptied
        m = int(np.ceil(np.sqrt(h.num_nodes)))
        moved = int((side == 0).sum())
        assert moved % m == 0 or moved == h.num_nodes


@pytest.mark.parametrize("seed", range(6))
def test_swap_keeps_side_sizes(seed):
    # The swap moves l nodes each way, so side node counts never change.
    h = I.random_small(60, 80, 2, 6, seed)
    rng = np.random.default_rng(seed)
    side = rng.integers(0, 2, h.num_nodes).astype(np.uint8)
    big = 10 ** 9
    s2, stuck = oracle.refine(h.num_nodes, h.offsets, h.pins, side, big, big, iters=3)
    assert stuck == 0
    assert int(s2.sum()) == int(side.sum())


@pytest.mark.parametrize("seed", range(6))
def test_balance_postcondition(seed):
    h = I.random_small(60, 70, 2, 6, seed, weighted_nodes=(seed % 2 == 1))
    rng = np.random.default_rng(seed)
    side = (rng.random(h.num_nodes) < 0.8).astype(np.uint8)
    total = int(h.node_w.sum())
    m0, m1 = oracle.bounds(total, 1, 1, F105)
    s2, stuck = oracle.refine(h.num_nodes, h.offsets, h.pins, side, m0, m1, iters=1, nw=h.node_w)
    w0 = int(h.node_w[s2 == 0].sum())
    w1 = total - w0
    if not stuck:
        assert w0 <= m0 and w1 <= m1
    if seed % 2 == 0:  # unit weights can always be balanced
        assert not stuck


# ---- the multilevel bisection (Section 2.3, Algorithm 5, Section 3.4) ---------------

def _arr(x):
    return np.asarray(x, np.int32)


def test_multilevel_golden_trace():
    gd = golden("multilevel.json")
    lv = gd["levels"]
    mx = gd["max_side_weight"]
    assert oracle.bounds(9, 1, 1, F105) == (mx, mx)
    # coarsening: every level's parents and the next level's graph
    for j in range(len(lv) - 1):
        f, c = lv[j], lv[j + 1]
        parent, coff, cpins, cnw, chw = oracle.coarsen(f["n"], f["offsets"], f["pins"], nw=f["node_w"])
        assert list(parent) == f["parent"], f"level {j} parents"
        assert list(coff) == c["offsets"] and list(cpins) == c["pins"], f"level {j + 1} hyperedges"
        assert list(cnw) == c["node_w"] and len(cnw) == c["n"], f"level {j + 1} weights"
        assert np.all(chw == 1)
    # the coarsest level: initial bisection, then its own refinement
    top = lv[-1]
    side = oracle.initial(top["n"], top["offsets"], top["pins"], 1, 1, nw=top["node_w"])
    assert list(side) == gd["coarsest_initial"]
    side, _ = oracle.refine(top["n"], top["offsets"], top["pins"], side, mx, mx, nw=top["node_w"])
    assert list(side) == gd["coarsest_refined"]
    # uncoarsening: projection through the parents, refinement of every level
    for step in gd["uncoarsen"]:
        L = lv[step["level"]]
        side = side[_arr(L["parent"])]
        assert list(side) == step["projected"], f"level {step['level']} projection"
        side, _ = oracle.refine(L["n"], L["offsets"], L["pins"], side, mx, mx, nw=L["node_w"])
        assert list(side) == step["refined"], f"level {step['level']} refinement"
    # the whole bisection in one call follows the same trace
    got, levels = oracle.bisect(gd["n"], gd["offsets"], gd["pins"], 1, 1, F105,
                                prm=oracle.params(min_coarse_nodes=0))
    assert levels == len(lv) - 1
    assert list(got) == gd["final_side"]
    assert oracle.cut(gd["n"], gd["offsets"], gd["pins"], got.astype(np.int32), 2)[0] == gd["final_cut"]


def test_multilevel_golden_coarsest_at_threshold():
    gd = golden("multilevel.json")
    c = gd["coarsest_level1"]
    L1 = gd["levels"][1]
    mx = gd["max_side_weight"]
    side = oracle.initial(L1["n"], L1["offsets"], L1["pins"], 1, 1, nw=L1["node_w"])
    assert list(side) == c["initial"]
    side, _ = oracle.refine(L1["n"], L1["offsets"], L1["pins"], side, mx, mx, nw=L1["node_w"])
    assert list(side) == c["refined"]
    got, levels = oracle.bisect(gd["n"], gd["offsets"], gd["pins"], 1, 1, F105,
                                prm=oracle.params(min_coarse_nodes=4))
    assert levels == 1 and list(got) == c["final_side"]


def test_stop_rule_closed_forms():
    gd = golden("multilevel.json")
    for c in gd["stop_rule"]["cases"]:
        prm = oracle.params(max_levels=c["max_levels"], min_coarse_nodes=c["min_coarse_nodes"])
        _, levels = oracle.bisect(gd["n"], gd["offsets"], gd["pins"], 1, 1, F105, prm=prm)
        assert levels == c["levels"], c
    # disjoint pairs: one step merges every pair and leaves no hyperedge, so
    # coarsening stops there whatever the node threshold and level limit
    off, pins = [0, 2, 4, 6, 8], list(range(8))
    for t in (0, 1, 3):
        _, levels = oracle.bisect(8, off, pins, 1, 1, F105, prm=oracle.params(min_coarse_nodes=t))
        assert levels == 1
    # one hyperedge over every node: one step to a single node
    _, levels = oracle.bisect(6, [0, 6], list(range(6)), 1, 1, F105, prm=oracle.params(min_coarse_nodes=0))
    assert levels == 1


def _vcycle(h, k0, k1, F, prm):
    """The multilevel scheme re-driven from Python over the single steps:
    coarsen while the stop rule allows, partition the coarsest graph, then
    project and refine every level up to the input."""
    W = int(h.node_w.sum())
    m0, m1 = oracle.bounds(W, k0, k1, F)
    lv = [(h.num_nodes, h.offsets, h.pins, h.node_w, h.hedge_w)]
    parents = []
    while (len(parents) < prm.max_levels and len(lv[-1][1]) > 1
           and lv[-1][0] > prm.min_coarse_nodes):
        n, off, pins, nw, hw = lv[-1]
        parent, coff, cpins, cnw, chw = oracle.coarsen(n, off, pins, nw, hw, policy=prm.policy)
        parents.append(parent)
        lv.append((len(cnw), coff, cpins, cnw, chw))
    n, off, pins, nw, hw = lv[-1]
    side = oracle.initial(n, off, pins, k0, k1, nw=nw, hw=hw)
    side, _ = oracle.refine(n, off, pins, side, m0, m1, prm.refine_iters, nw=nw, hw=hw)
    for j in range(len(parents) - 1, -1, -1):
        side = side[parents[j]]
        n, off, pins, nw, hw = lv[j]
        side, _ = oracle.refine(n, off, pins, side, m0, m1, prm.refine_iters, nw=nw, hw=hw)
    return side, len(parents)


@pytest.mark.parametrize("seed", range(4))
def test_bisect_is_the_multilevel_scheme(seed):
    h = I.random_small(300, 330, 2, 6, seed, weighted_nodes=(seed % 2 == 1),
                       weighted_hedges=(seed >= 2))
    for t, maxl, k0, k1 in [(0, 25, 1, 1), (20, 25, 2, 1), (40, 2, 1, 1), (0, 1, 3, 2), (5, 4, 1, 1)]:
        prm = oracle.params(max_levels=maxl, min_coarse_nodes=t, policy=seed % 5)
        want, wl = _vcycle(h, k0, k1, F105, prm)
        got, gl = oracle.bisect(h.num_nodes, h.offsets, h.pins, k0, k1, F105, nw=h.node_w, hw=h.hedge_w,
                                prm=prm)
        assert gl == wl and np.array_equal(got, want), (t, maxl, k0, k1)
    assert wl >= 1


# ---- bounds and eps ---------------------------------------------------------------

def test_bounds_closed_forms():
    two32 = 1 << 32
    assert oracle.bounds(101, 1, 1, two32) == (51, 51)           # eps = 0: ceil(W/2)
    assert oracle.bounds(100, 2, 1, two32 * 3 // 2) == (100, 50)  # floor(1.5 * share)
    assert oracle.bounds(100, 2, 1, two32) == (67, 34)
    assert oracle.bounds(0, 1, 1, F105) == (0, 0)
    # no overflow at the largest weight sum
    w = 2 ** 31 - 1
    assert oracle.bounds(w, 1, 1, F105) == (w * F105 // (2 * two32), w * F105 // (2 * two32))


def test_eps_factor():
    assert oracle.eps_factor(2, 0.05) == F105
    assert oracle.eps_factor(2, 0.0) == 1 << 32
    f = oracle.eps_factor(8, 0.03) / 2 ** 32
    assert abs(f ** 3 - 1.03) < 1e-8
    f = oracle.eps_factor(5, 0.1) / 2 ** 32   # ceil(log2 5) = 3 tree levels
    assert abs(f ** 3 - 1.1) < 1e-8


def test_huge_eps_is_unconstrained():
    # A per-bisection factor of 2^30 or more lets either side hold the whole
    # weight, so all such factors give the same result; they are capped at 2^62.
    assert oracle.eps_factor(2, 1e12) == 1 << 62
    assert oracle.eps_factor(8, 1e300) == 1 << 62
    assert oracle.eps_factor(2, 2.0 ** 30 - 2) == (2 ** 30 - 1) << 32
    h = I.random_small(200, 240, 2, 6, 3, weighted_nodes=True)
    W = int(h.node_w.sum())
    assert min(oracle.bounds(W, 2, 1, 1 << 62)) >= W
    a = oracle.partition_hg(h, k=3, eps=1e12)
    b = oracle.partition_hg(h, k=3, eps=1e6)     # bound already above W, uncapped
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]


# ---- k-way (Algorithm 6) and the whole method --------------------------------------

@pytest.mark.parametrize("k", [2, 3, 4, 5, 8])
@pytest.mark.parametrize("seed", range(3))
def test_kway_cut_decomposition(k, seed):
    h = I.random_small(300, 360, 1, 8, seed, weighted_hedges=True, weighted_nodes=(seed == 2))
    # Sum over all bisections of the cut-net cut inside each subgraph equals the
    # connectivity-1 cut of the final partition; the tree is re-driven from
    # Python with cut-net splitting written independently of the oracle's.
    prm = oracle.params(min_coarse_nodes=20)
    part, cut = oracle.partition_hg(h, k=k, eps=0.05, prm=prm)
    F = oracle.eps_factor(k, 0.05)
    part2, tree_cut = _bisect_tree_prm(h, k, F, prm)
    assert np.array_equal(part, part2)
    assert cut == tree_cut
    assert part.min() >= 0 and part.max() < k


def _bisect_tree_prm(h, k, F, prm):
    """Recursive bisection driven from Python; returns (part, sum of cut-net cuts)."""
    d = np.diff(h.offsets)
    keep = d >= 2
    pins = h.pins[np.repeat(keep, d)]
    off = np.concatenate([[0], np.cumsum(d[keep])]).astype(np.int32)
    hw = h.hedge_w[keep]
    part = np.zeros(h.num_nodes, np.int32)
    total_cut = 0
    tasks = [(np.arange(h.num_nodes), off, pins, h.node_w, hw, 0, k)]
    while tasks:
        orig, off, pins, nw, hw, lo, ks = tasks.pop(0)
        if ks == 1:
            part[orig] = lo
            continue
        k0 = (ks + 1) // 2
        side, _ = oracle.bisect(len(orig), off, pins, k0, ks - k0, F, nw=nw, hw=hw, prm=prm)
        hedge = np.repeat(np.arange(len(off) - 1), np.diff(off))
        ones = np.bincount(hedge, weights=side[pins], minlength=len(off) - 1).astype(np.int64)
        deg = np.diff(off)
        total_cut += int(np.sum(hw[(ones > 0) & (ones < deg)].astype(np.int64)))
        for s, (clo, cks) in enumerate([(lo, k0), (lo + k0, ks - k0)]):
            sel = side == s
            local = np.cumsum(sel) - 1
            pin_in = sel[pins]
            cnt = np.bincount(hedge[pin_in], minlength=len(off) - 1)
            keep_e = cnt >= 2
            cp = local[pins[pin_in & keep_e[hedge]]].astype(np.int32)
            coff = np.concatenate([[0], np.cumsum(cnt[keep_e])]).astype(np.int32)
            tasks.append((orig[sel], coff, cp, nw[sel], hw[keep_e], clo, cks))
    return part, total_cut


def test_k1_and_empty():
    h = I.random_small(20, 30, 2, 4, 0)
    part, cut = oracle.partition_hg(h, k=1, eps=0.05)
    assert np.all(part == 0) and cut == 0
    part, cut = oracle.partition(0, [0], [], 2, 0.05)
    assert len(part) == 0 and cut == 0
    with pytest.raises(ValueError):
        oracle.partition(3, [0], [], 0, 0.05)


@pytest.mark.parametrize("k,eps", [(2, 0.05), (4, 0.03), (3, 0.1), (8, 0.05)])
def test_unit_weights_are_always_balanced(k, eps):
    # With unit weights the finest level can always move a node that fits,
    # so every bisection ends within its bound; the product of the per-level
    # bounds (with ceilings) bounds every part.
    h = I.random_small(500, 600, 2, 6, 7)
    part, _ = oracle.partition_hg(h, k=k, eps=eps)
    F = oracle.eps_factor(k, eps)
    # walk the tree bounds: a part's weight is at most the chained bounds
    def bound(total, ks):
        if ks == 1:
            return total
        k0 = (ks + 1) // 2
        m0, m1 = oracle.bounds(total, k0, ks - k0, F)
        return max(bound(m0, k0), bound(m1, ks - k0))
    sizes = np.bincount(part, minlength=k)
    assert sizes.max() <= bound(h.num_nodes, k)


def _brute_force_opt(h, max0, max1):
    n = h.num_nodes
    masks = np.arange(1 << n, dtype=np.int64)
    bits = ((masks[:, None] >> np.arange(n)) & 1).astype(np.int8)
    w1 = bits @ h.node_w.astype(np.int64)
    total = int(h.node_w.sum())
    ok = (total - w1 <= max0) & (w1 <= max1)
    cut = np.zeros(len(masks), np.int64)
    for e in range(h.num_hedges):
        p = h.pins[h.offsets[e]:h.offsets[e + 1]]
        if len(p) < 2:
            continue
        ones = bits[:, p].sum(axis=1)
        cut += h.hedge_w[e] * ((ones > 0) & (ones < len(p)))
    return int(cut[ok].min())


@pytest.mark.parametrize("seed", range(4))
def test_cut_not_below_brute_force_optimum(seed):
    h = I.random_small(12, 14, 2, 4, seed, weighted_hedges=True)
    part, cut = oracle.partition_hg(h, k=2, eps=0.05)
    m0, m1 = oracle.bounds(int(h.node_w.sum()), 1, 1, F105)
    opt = _brute_force_opt(h, m0, m1)
    w1 = int(h.node_w[part == 1].sum())
    assert w1 <= m1 and int(h.node_w.sum()) - w1 <= m0
    assert cut >= opt


@pytest.mark.parametrize("seed", range(3))
def test_pin_order_and_run_to_run(seed):
    h = I.random_small(400, 500, 2, 9, seed, weighted_hedges=True)
    a = oracle.partition_hg(h, k=4, eps=0.05)
    b = oracle.partition_hg(I.shuffle_pins(h, seed), k=4, eps=0.05)
    c = oracle.partition_hg(h, k=4, eps=0.05)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]
    assert np.array_equal(a[0], c[0]) and a[1] == c[1]


def test_tiny_workload_runs():
    h = I.tiny()
    part, cut = oracle.partition_hg(h)
    assert part.shape == (1000,)
    assert 0 < cut < 2000
    assert np.bincount(part).max() <= 525
