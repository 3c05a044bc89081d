"""Seeded synthetic hypergraph generators.

This module only builds inputs: it holds none of the partitioner's arithmetic
and is shared by the HIP path's tests/bench and by the CPU oracle's tests.

Random numbers come from a counter-based form of SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): for a
(seed, stream) pair the state starts at ``mix(seed ^ mix(stream))`` and value
``i`` is ``mix(state + (i + 1) * 0x9E3779B97F4A7C15)``, where ``mix`` is the
SplitMix64 output function.  Uniform doubles take the top 53 bits; uniform
integers in [0, n) take ``((v >> 32) * n) >> 32``.

Hypergraphs are returned as int32 CSR over hyperedges: ``offsets[E+1]`` and
``pins[P]`` (node ids of each hyperedge, sorted ascending, no repeats), plus
``node_w[N]`` and ``hedge_w[E]`` (int32).  The shapes follow the workloads the
paper measures on (Table 2: VLSI netlists and sparse-matrix column-net models);
the paper's data files themselves are not used.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def _mix1(x: int) -> int:
    return int(_mix(np.array([x & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0])


def rand_u64(seed: int, stream: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 values number ``counters`` of generator (seed, stream)."""
    state = np.uint64(_mix1((seed & 0xFFFFFFFFFFFFFFFF) ^ _mix1(stream)))
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(state + (c + np.uint64(1)) * _GOLDEN)


def rand_double(seed: int, stream: int, counters: np.ndarray) -> np.ndarray:
    v = rand_u64(seed, stream, counters)
    return (v >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def rand_int(seed: int, stream: int, counters: np.ndarray, n) -> np.ndarray:
    """Uniform integers in [0, n); ``n`` may be a scalar or an array (< 2**32)."""
    v = rand_u64(seed, stream, counters) >> np.uint64(32)
    n = np.asarray(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return ((v * n) >> np.uint64(32)).astype(np.int64)


def powerlaw_degrees(seed: int, stream: int, count: int, alpha: float,
                     dmin: int, dmax: int) -> np.ndarray:
    """Discrete power law P(d) ~ d^-alpha on [dmin, dmax] by inverse CDF."""
    d = np.arange(dmin, dmax + 1, dtype=np.float64)
    cdf = np.cumsum(d ** (-alpha))
    cdf /= cdf[-1]
    u = rand_double(seed, stream, np.arange(count, dtype=np.uint64))
    idx = np.searchsorted(cdf, u, side="right")
    return (dmin + np.minimum(idx, len(cdf) - 1)).astype(np.int64)


@dataclass
class Hypergraph:
    num_nodes: int
    offsets: np.ndarray          # int32 [E+1]
    pins: np.ndarray             # int32 [P]
    node_w: np.ndarray           # int32 [N]
    hedge_w: np.ndarray          # int32 [E]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def num_hedges(self) -> int:
        return len(self.offsets) - 1

    @property
    def num_pins(self) -> int:
        return int(self.offsets[-1])


def _draw_pins(seed: int, deg: np.ndarray, n: int, draw) -> tuple[np.ndarray, np.ndarray]:
    """Fill each hyperedge with ``deg`` distinct node ids.

    ``draw(round, slots)`` returns candidate node ids for the given pin slots.
    Slots whose value repeats an earlier slot of the same hyperedge are drawn
    again in the next round (with fresh streams) until none repeat.  Returns
    (offsets, pins sorted within each hyperedge).
    """
    deg = np.minimum(deg.astype(np.int64), n)
    e = len(deg)
    offsets = np.zeros(e + 1, dtype=np.int64)
    np.cumsum(deg, out=offsets[1:])
    p = int(offsets[-1])
    hedge_of = np.repeat(np.arange(e, dtype=np.int64), deg)
    slots = np.arange(p, dtype=np.int64)
    pins = draw(0, slots)
    rnd = 0
    todo = slots
    while True:
        # repeated (hyperedge, node) pairs: keep the lowest slot, redraw the rest
        key = hedge_of * np.int64(n) + pins
        order = np.lexsort((slots, key))
        ks = key[order]
        dup = np.zeros(p, dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        todo = order[dup]
        if todo.size == 0:
            break
        rnd += 1
        if rnd > 10000:
            raise RuntimeError("pin drawing did not converge")
        pins[todo] = draw(rnd, todo)
    key = hedge_of * np.int64(n) + pins
    pins = pins[np.argsort(key, kind="stable")]
    return offsets.astype(np.int32), pins.astype(np.int32)


def uniform_hypergraph(n: int, e: int, dmin: int, dmax: int, seed: int,
                       name: str = "uniform") -> Hypergraph:
    """Degrees uniform in [dmin, dmax], pins uniform without replacement."""
    deg = dmin + rand_int(seed, 0, np.arange(e, dtype=np.uint64), dmax - dmin + 1)
    draw = lambda r, s: rand_int(seed, 1 + r, s.astype(np.uint64), n)
    off, pins = _draw_pins(seed, deg, n, draw)
    return Hypergraph(n, off, pins, np.ones(n, np.int32), np.ones(e, np.int32), name)


def local_powerlaw_hypergraph(n: int, e: int, alpha: float, dmin: int, dmax: int,
                              seed: int, window: int = 2000, p_local: float = 0.8,
                              name: str = "vlsi") -> Hypergraph:
    """Netlist-shaped: power-law degrees; each pin lies within +-window of a
    per-hyperedge anchor (mod n) with probability p_local, else uniform."""
    deg = powerlaw_degrees(seed, 0, e, alpha, dmin, dmax)
    anchor = rand_int(seed, 1, np.arange(e, dtype=np.uint64), n)
    deg_c = np.minimum(deg, n)
    hedge_of = np.repeat(np.arange(e, dtype=np.int64), deg_c)
    width = min(2 * window + 1, n)

    def draw(r, s):
        s64 = s.astype(np.uint64)
        u = rand_double(seed, 16 + 3 * r, s64)
        off = rand_int(seed, 17 + 3 * r, s64, width) - (width // 2)
        far = rand_int(seed, 18 + 3 * r, s64, n)
        near = (anchor[hedge_of[s]] + off) % n
        return np.where(u < p_local, near, far).astype(np.int64)

    off, pins = _draw_pins(seed, deg_c, n, draw)
    return Hypergraph(n, off, pins, np.ones(n, np.int32), np.ones(e, np.int32), name)


def column_net_hypergraph(n_rows: int, n_cols: int, alpha: float, dmin: int, dmax: int,
                          seed: int, name: str = "colnet") -> Hypergraph:
    """Sparse-matrix column-net model: rows are nodes, columns are hyperedges,
    nonzeros per column power-law; node weight = row nonzero count."""
    deg = powerlaw_degrees(seed, 0, n_cols, alpha, dmin, dmax)
    draw = lambda r, s: rand_int(seed, 1 + r, s.astype(np.uint64), n_rows)
    off, pins = _draw_pins(seed, deg, n_rows, draw)
    nw = np.bincount(pins, minlength=n_rows).astype(np.int32)
    return Hypergraph(n_rows, off, pins, nw, np.ones(n_cols, np.int32), name)


# --- the measured workloads -------------------------------------------------

def tiny(seed: int = 1) -> Hypergraph:
    """1,000 unit nodes, 2,000 hyperedges of degree U{2..8}; k=2, eps=0.05."""
    h = uniform_hypergraph(1000, 2000, 2, 8, seed, name="tiny-1k")
    h.meta.update(k=2, eps=0.05)
    return h


def vlsi(seed: int = 2, n: int = 1_000_000) -> Hypergraph:
    """Netlist shape: N=1M unit nodes, E=1.2N, PL(2.5) on [2,1000], +-2000 window."""
    e = int(round(1.2 * n))
    h = local_powerlaw_hypergraph(n, e, 2.5, 2, 1000, seed, name=f"vlsi-{n}")
    h.meta.update(k=2, eps=0.05)
    return h


def column_net(seed: int = 3, n: int = 4_000_000, dmin: int = 1) -> Hypergraph:
    """Column-net shape: N=E=4M, PL(2.1) on [dmin,5000], node weight = row nnz."""
    h = column_net_hypergraph(n, n, 2.1, dmin, 5000, seed, name=f"colnet-{n}-d{dmin}")
    h.meta.update(k=8, eps=0.03)
    return h


def random_10m(seed: int = 6) -> Hypergraph:
    """The shape of the paper's Random-10M input (Table 2): N = E = 10M,
    about 115M pins; degrees uniform in [2, 21] (mean 11.5), pins uniform
    without replacement, unit weights; k=2, eps=0.1 (the 55:45 balance of the
    paper's runs).  The paper does not give its generator."""
    h = uniform_hypergraph(10_000_000, 10_000_000, 2, 21, seed, name="random-10m")
    h.meta.update(k=2, eps=0.1)
    return h


def random_15m(seed: int = 7) -> Hypergraph:
    """The shape of the paper's Random-15M input (Table 2): N = 15M, E = 17M,
    about 281M pins; degrees uniform in [2, 31] (mean 16.5), pins uniform
    without replacement, unit weights; k=2, eps=0.1."""
    h = uniform_hypergraph(15_000_000, 17_000_000, 2, 31, seed, name="random-15m")
    h.meta.update(k=2, eps=0.1)
    return h


def batch_member(i: int, seed: int = 4) -> Hypergraph:
    """Member i of the 256-graph batch: N log-uniform in [1e3, 2e5], E=1.2N,
    netlist structure; k=2 for even i, 4 for odd i; eps=0.05."""
    u = float(rand_double(seed, 0, np.array([i], dtype=np.uint64))[0])
    n = int(round(math.exp(math.log(1e3) + u * (math.log(2e5) - math.log(1e3)))))
    e = int(round(1.2 * n))
    h = local_powerlaw_hypergraph(n, e, 2.5, 2, 1000, _mix1(seed * 1000003 + i + 1),
                                  name=f"batch-{i}")
    h.meta.update(k=2 if i % 2 == 0 else 4, eps=0.05)
    return h


def serve_request(r: int, seed: int = 5, mean_degree: float = 4.536746661367512) -> Hypergraph:
    """Request r of the served stream: target pins log-uniform in [1e4, 2e6],
    N = pins / (1.2 * mean degree), netlist structure, k in {2,4,16}."""
    u = rand_double(seed, r + 1, np.arange(2, dtype=np.uint64))
    target = math.exp(math.log(1e4) + float(u[0]) * (math.log(2e6) - math.log(1e4)))
    n = max(2, int(round(target / (1.2 * mean_degree))))
    e = int(round(1.2 * n))
    h = local_powerlaw_hypergraph(n, e, 2.5, 2, 1000, _mix1(seed * 1000003 + r + 1),
                                  name=f"req-{r}")
    h.meta.update(k=(2, 4, 16)[min(2, int(float(u[1]) * 3))], eps=0.05)
    return h


def poisson_arrivals(count: int, rate: float, seed: int = 5) -> np.ndarray:
    """Arrival times (s) of an open-loop Poisson stream (stream 0 of the seed)."""
    u = rand_double(seed, 0, np.arange(count, dtype=np.uint64))
    return np.cumsum(-np.log1p(-u) / rate)


def random_small(n: int, e: int, dmin: int, dmax: int, seed: int,
                 weighted_nodes: bool = False, weighted_hedges: bool = False,
                 max_w: int = 5, isolated: int = 0) -> Hypergraph:
    """Small random hypergraphs for tests: degrees U[dmin, dmax] (1-pin and
    0-pin hyperedges allowed when dmin < 2), optional random weights and
    ``isolated`` trailing nodes that no hyperedge touches."""
    core = max(1, n - isolated)
    deg = dmin + rand_int(seed, 0, np.arange(e, dtype=np.uint64), dmax - dmin + 1)
    deg = np.minimum(deg, core)
    draw = lambda r, s: rand_int(seed, 1 + r, s.astype(np.uint64), core)
    off, pins = _draw_pins(seed, deg, core, draw)
    nw = (1 + rand_int(seed, 900, np.arange(n, dtype=np.uint64), max_w)).astype(np.int32) \
        if weighted_nodes else np.ones(n, np.int32)
    hw = (1 + rand_int(seed, 901, np.arange(e, dtype=np.uint64), max_w)).astype(np.int32) \
        if weighted_hedges else np.ones(e, np.int32)
    return Hypergraph(n, off, pins, nw, hw, name=f"small-{n}-{e}-{seed}")


def shuffle_pins(h: Hypergraph, seed: int) -> Hypergraph:
    """Same hypergraph with the pin order inside every hyperedge permuted."""
    p = h.num_pins
    hedge_of = np.repeat(np.arange(h.num_hedges, dtype=np.int64), np.diff(h.offsets))
    r = rand_u64(seed, 77, np.arange(p, dtype=np.uint64))
    order = np.lexsort((r, hedge_of))
    return Hypergraph(h.num_nodes, h.offsets.copy(), h.pins[order].copy(), h.node_w.copy(),
                      h.hedge_w.copy(), h.name + "-shuffled", dict(h.meta))
