"""Python binding of libbipart_mi355x.so (the C ABI in include/bipart.h).

Argument marshalling only: every step of the partitioner runs in the HIP
library.  Device entry points take torch tensors on the GPU (PyTorch supplies
device memory and the current stream); host entry points take numpy arrays.
The library must have been built (``__graft_entry__.build()`` or
``python paper_2012_13618_amd/build_lib.py``); importing a function that needs
it raises if it is missing - there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbipart_mi355x.so")

BP_OK = 0
BP_WARN_IMBALANCED = 1
STATUS = {0: "BP_OK", 1: "BP_WARN_IMBALANCED", -1: "BP_ERR_INVALID_ARG", -2: "BP_ERR_INVALID_CSR",
          -3: "BP_ERR_WEIGHT_OVERFLOW", -4: "BP_ERR_OUT_OF_MEMORY", -5: "BP_ERR_DEVICE",
          -6: "BP_ERR_REJECTED", -7: "BP_ERR_SHUTDOWN", -8: "BP_ERR_NOT_FOUND"}
LDH, HDH, LWD, HWD, RAND = 0, 1, 2, 3, 4

EXPORTS = [
    "bp_default_params", "bp_status_string", "bp_last_error", "bp_partition",
    "bp_partition_device", "bp_compute_cut", "bp_compute_cut_device", "bp_step_match",
    "bp_step_coarsen", "bp_step_gains", "bp_step_initial", "bp_step_refine", "bp_step_bisect",
    "bp_profile_enable", "bp_profile_reset", "bp_profile_read", "bp_partition_batch",
    "bp_partition_batch_device", "bp_server_default_config", "bp_request_footprint",
    "bp_server_create", "bp_server_submit", "bp_server_wait", "bp_server_destroy",
    "bp_profile_floor", "bp_schedule_default", "bp_schedule_set", "bp_schedule_get",
    "bp_autotune_batch_device", "bp_release_memory", "bp_set_memory_limit",
    "bp_partition_device_noalloc",
]


class BipartError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Hypergraph(ctypes.Structure):
    _fields_ = [("num_nodes", ctypes.c_int32), ("num_hedges", ctypes.c_int32),
                ("hedge_offsets", ctypes.c_void_p), ("pins", ctypes.c_void_p),
                ("node_weights", ctypes.c_void_p), ("hedge_weights", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("refine_iters", ctypes.c_int32), ("min_coarse_nodes", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("cut", ctypes.c_int64), ("max_part_weight", ctypes.c_int64),
                ("part_weight_limit", ctypes.c_int64), ("balanced", ctypes.c_int32),
                ("tree_levels", ctypes.c_int32), ("bisections", ctypes.c_int32),
                ("coarsen_levels", ctypes.c_int32), ("pins_coarsened", ctypes.c_int64),
                ("pins_refined", ctypes.c_int64), ("host_syncs", ctypes.c_int32),
                ("kernel_launches", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("levels", ctypes.c_int32 * 64), ("imbalance", ctypes.c_double),
                ("graph_replays", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("levels", "reserved")}
        d["levels"] = list(self.levels)[:max(self.tree_levels, 0)]
        return d


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("max_batch_delay_us", ctypes.c_int32), ("device", ctypes.c_int32),
                ("workers", ctypes.c_int32), ("params", Params), ("max_run_pins", ctypes.c_int64)]


class ReqStats(ctypes.Structure):
    _fields_ = [("cut", ctypes.c_int64), ("max_part_weight", ctypes.c_int64),
                ("part_weight_limit", ctypes.c_int64), ("balanced", ctypes.c_int32),
                ("batch_size", ctypes.c_int32), ("footprint_bytes", ctypes.c_int64),
                ("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Schedule(ctypes.Structure):
    _fields_ = [("incremental_min_pins", ctypes.c_int32), ("seg_select_max_nodes", ctypes.c_int32),
                ("round_chunk_max", ctypes.c_int32), ("fused_pick_lists", ctypes.c_int32),
                ("fuse_max_pins", ctypes.c_int32), ("chunk_select_max_nodes", ctypes.c_int32),
                ("graph_rounds", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                 ctypes.c_double)
        L.bp_default_params.argtypes = [P]
        L.bp_default_params.restype = None
        L.bp_status_string.argtypes = [i32]
        L.bp_status_string.restype = ctypes.c_char_p
        L.bp_last_error.argtypes = []
        L.bp_last_error.restype = ctypes.c_char_p
        L.bp_partition.argtypes = [P, i32, f64, P, P, P, P]
        L.bp_partition_device.argtypes = [P, i32, f64, P, P, P, P, P]
        L.bp_compute_cut.argtypes = [P, i32, P, P, P]
        L.bp_compute_cut_device.argtypes = [P, i32, P, P, P, P]
        L.bp_step_match.argtypes = [P, i32, P, P]
        L.bp_step_coarsen.argtypes = [P, i32, P, P, P, P, P, P, P, P]
        L.bp_step_gains.argtypes = [P, P, P, P]
        L.bp_step_initial.argtypes = [P, i32, i32, P, P]
        L.bp_step_refine.argtypes = [P, i32, i64, i64, P, P, P]
        L.bp_step_bisect.argtypes = [P, i32, i32, u64, P, P, P, P]
        L.bp_partition_batch.argtypes = [i32, P, P, P, P, P, P, P]
        L.bp_partition_batch_device.argtypes = [i32, P, P, P, P, P, P, P, P]
        L.bp_server_default_config.argtypes = [P]
        L.bp_server_default_config.restype = None
        L.bp_request_footprint.argtypes = [i32, i32, i64, i32, P]
        L.bp_server_create.argtypes = [P, P]
        L.bp_server_submit.argtypes = [P, P, i32, f64, P]
        L.bp_server_wait.argtypes = [P, u64, P, P, P]
        L.bp_server_destroy.argtypes = [P]
        L.bp_profile_enable.argtypes = [i32]
        L.bp_profile_enable.restype = None
        L.bp_profile_reset.argtypes = []
        L.bp_profile_reset.restype = None
        L.bp_profile_read.argtypes = [P, i32]
        L.bp_profile_floor.argtypes = [i32, P]
        L.bp_schedule_default.argtypes = [P]
        L.bp_schedule_default.restype = None
        L.bp_schedule_set.argtypes = [P]
        L.bp_schedule_get.argtypes = [P]
        L.bp_autotune_batch_device.argtypes = [i32, P, P, P, P, P, i32, P, P, P]
        L.bp_release_memory.argtypes = []
        L.bp_partition_device_noalloc.argtypes = [P, i32, f64, P, P, P, P, P]
        L.bp_set_memory_limit.argtypes = [i64]
        for name in EXPORTS:
            f = getattr(L, name)
            if f.restype is ctypes.c_int:
                f.restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(status):
    if status < 0:
        raise BipartError(status, lib().bp_last_error().decode())
    return status


def default_params() -> Params:
    p = Params()
    lib().bp_default_params(ctypes.byref(p))
    return p


def params(policy=LDH, max_levels=25, refine_iters=2, min_coarse_nodes=100) -> Params:
    return Params(policy, max_levels, refine_iters, min_coarse_nodes)


# ---- host entry points (numpy) -------------------------------------------------------

def _host_hg(n, off, pins, nw, hw, keep):
    off = np.ascontiguousarray(off, dtype=np.int32)
    pins = np.ascontiguousarray(pins, dtype=np.int32)
    nw = None if nw is None else np.ascontiguousarray(nw, dtype=np.int32)
    hw = None if hw is None else np.ascontiguousarray(hw, dtype=np.int32)
    keep.extend([off, pins, nw, hw])
    ptr = lambda a: None if a is None else a.ctypes.data
    return Hypergraph(n, len(off) - 1, ptr(off), ptr(pins), ptr(nw), ptr(hw))


def partition(n, off, pins, k, eps, nw=None, hw=None, prm: Params | None = None):
    """k-way partition of a host hypergraph: returns (part, cut, status, report)."""
    keep = []
    hg = _host_hg(n, off, pins, nw, hw, keep)
    part = np.empty(max(n, 1), np.int32)
    cut = ctypes.c_int64(0)
    rep = Report()
    st = _check(lib().bp_partition(ctypes.byref(hg), k, eps, None if prm is None else ctypes.byref(prm),
                                   part.ctypes.data, ctypes.byref(cut), ctypes.byref(rep)))
    return part[:n], int(cut.value), st, rep


def partition_hg(h, k=None, eps=None, prm: Params | None = None):
    k = h.meta.get("k", 2) if k is None else k
    eps = h.meta.get("eps", 0.05) if eps is None else eps
    return partition(h.num_nodes, h.offsets, h.pins, k, eps, h.node_w, h.hedge_w, prm)


def _batch_arrays(n, ks, epss):
    ks = np.ascontiguousarray(ks, dtype=np.int32)
    epss = np.ascontiguousarray(epss, dtype=np.float64)
    if len(ks) != n or len(epss) != n:
        raise ValueError("k and eps need one entry per graph")
    return ks, epss


def partition_batch(graphs, ks, epss, prm: Params | None = None):
    """Batched form over host hypergraphs (objects with num_nodes, offsets, pins,
    node_w, hedge_w): returns (list of parts, list of cuts, status, list of reports)."""
    n = len(graphs)
    keep = []
    hgs = (Hypergraph * max(n, 1))()
    for i, h in enumerate(graphs):
        hgs[i] = _host_hg(h.num_nodes, h.offsets, h.pins, h.node_w, h.hedge_w, keep)
    ks, epss = _batch_arrays(n, ks, epss)
    parts = [np.empty(max(h.num_nodes, 1), np.int32) for h in graphs]
    outs = (ctypes.c_void_p * max(n, 1))(*[p.ctypes.data for p in parts])
    cuts = np.zeros(max(n, 1), np.int64)
    reps = (Report * max(n, 1))()
    st = _check(lib().bp_partition_batch(n, hgs, ks.ctypes.data, epss.ctypes.data,
                                         None if prm is None else ctypes.byref(prm), outs,
                                         cuts.ctypes.data, reps))
    return ([p[:h.num_nodes] for p, h in zip(parts, graphs)], [int(c) for c in cuts[:n]], st,
            [reps[i] for i in range(n)])


def request_footprint(num_nodes, num_hedges, num_pins, k):
    """Device bytes the library budgets for one partition of these sizes."""
    b = ctypes.c_int64(0)
    _check(lib().bp_request_footprint(num_nodes, num_hedges, num_pins, k, ctypes.byref(b)))
    return int(b.value)


class Server:
    """The served form: submit host hypergraphs, wait for their partitions."""

    def __init__(self, hbm_budget_bytes=None, max_slots=None, max_batch_delay_us=None, device=0,
                 prm: Params | None = None, workers=None, max_run_pins=None):
        cfg = ServerConfig()
        lib().bp_server_default_config(ctypes.byref(cfg))
        if workers is not None:
            cfg.workers = int(workers)
        if max_run_pins is not None:
            cfg.max_run_pins = int(max_run_pins)
        if hbm_budget_bytes is not None:
            cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        if max_slots is not None:
            cfg.max_slots = int(max_slots)
        if max_batch_delay_us is not None:
            cfg.max_batch_delay_us = int(max_batch_delay_us)
        cfg.device = int(device)
        if prm is not None:
            cfg.params = prm
        h = ctypes.c_void_p()
        _check(lib().bp_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._nodes = {}

    def submit(self, h, k=None, eps=None):
        """Queues a copy of h; returns its ticket."""
        k = h.meta.get("k", 2) if k is None else k
        eps = h.meta.get("eps", 0.05) if eps is None else eps
        keep = []
        hg = _host_hg(h.num_nodes, h.offsets, h.pins, h.node_w, h.hedge_w, keep)
        t = ctypes.c_uint64(0)
        _check(lib().bp_server_submit(self._h, ctypes.byref(hg), k, eps, ctypes.byref(t)))
        self._nodes[t.value] = h.num_nodes
        return t.value

    def wait(self, ticket):
        """Blocks until the request is done: returns (part, cut, status, stats)."""
        n = self._nodes.pop(ticket, 0)
        part = np.empty(max(n, 1), np.int32)
        cut = ctypes.c_int64(0)
        st = ReqStats()
        status = _check(lib().bp_server_wait(self._h, ctypes.c_uint64(ticket), part.ctypes.data,
                                             ctypes.byref(cut), ctypes.byref(st)))
        return part[:n], int(cut.value), status, st

    def close(self):
        if self._h:
            _check(lib().bp_server_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def compute_cut(n, off, pins, part, k, nw=None, hw=None):
    keep = []
    hg = _host_hg(n, off, pins, nw, hw, keep)
    part = np.ascontiguousarray(part, dtype=np.int32)
    cut, mw = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().bp_compute_cut(ctypes.byref(hg), k, part.ctypes.data, ctypes.byref(cut),
                                ctypes.byref(mw)))
    return int(cut.value), int(mw.value)


# ---- device entry points (torch tensors on the GPU) -----------------------------------

def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class DeviceHypergraph:
    """A hypergraph resident in device memory (int32 torch tensors)."""

    def __init__(self, num_nodes, offsets, pins, node_w=None, hedge_w=None):
        import torch
        dev = torch.device("cuda")
        t = lambda a: None if a is None else torch.as_tensor(np.asarray(a, np.int32)).to(dev)
        self.num_nodes = int(num_nodes)
        self.offsets = offsets if isinstance(offsets, torch.Tensor) else t(offsets)
        self.pins = pins if isinstance(pins, torch.Tensor) else t(pins)
        self.node_w = node_w if (node_w is None or isinstance(node_w, torch.Tensor)) else t(node_w)
        self.hedge_w = hedge_w if (hedge_w is None or isinstance(hedge_w, torch.Tensor)) else t(hedge_w)
        if self.pins.numel() == 0:
            self.pins = torch.zeros(1, dtype=torch.int32, device=dev)

    @classmethod
    def from_host(cls, h):
        return cls(h.num_nodes, h.offsets, h.pins, h.node_w, h.hedge_w)

    @property
    def num_hedges(self):
        return int(self.offsets.numel()) - 1

    def struct(self) -> Hypergraph:
        p = lambda x: None if x is None else x.data_ptr()
        return Hypergraph(self.num_nodes, self.num_hedges, p(self.offsets), p(self.pins),
                          p(self.node_w), p(self.hedge_w))


def partition_device(dh: DeviceHypergraph, k, eps, prm: Params | None = None, part_out=None):
    """Partition a device hypergraph; returns (part tensor, cut, status, report)."""
    import torch
    if part_out is None:
        part_out = torch.empty(max(dh.num_nodes, 1), dtype=torch.int32, device="cuda")
    hg = dh.struct()
    cut = ctypes.c_int64(0)
    rep = Report()
    st = _check(lib().bp_partition_device(ctypes.byref(hg), k, eps,
                                          None if prm is None else ctypes.byref(prm),
                                          part_out.data_ptr(), ctypes.byref(cut),
                                          ctypes.byref(rep), _stream()))
    return part_out[:dh.num_nodes], int(cut.value), st, rep


def partition_device_noalloc(dh: DeviceHypergraph, k, eps, prm: Params | None = None, part_out=None):
    """As partition_device, through the entry point that allocates no device
    memory (fixed workspace); part_out is required."""
    hg = dh.struct()
    cut = ctypes.c_int64(0)
    rep = Report()
    st = _check(lib().bp_partition_device_noalloc(ctypes.byref(hg), k, eps,
                                                  None if prm is None else ctypes.byref(prm),
                                                  part_out.data_ptr(), ctypes.byref(cut),
                                                  ctypes.byref(rep), _stream()))
    return part_out[:dh.num_nodes], int(cut.value), st, rep


def release_memory():
    """Frees the cached device memory of every idle call context of the current device."""
    _check(lib().bp_release_memory())


def set_memory_limit(nbytes):
    """Caps the device memory one call may hold (0 = no cap)."""
    _check(lib().bp_set_memory_limit(int(nbytes)))


def partition_batch_device(dhs, ks, epss, prm: Params | None = None, parts_out=None):
    """Batched form over DeviceHypergraphs: returns (list of part tensors, list of
    cuts, status, list of reports)."""
    import torch
    n = len(dhs)
    hgs = (Hypergraph * max(n, 1))()
    for i, d in enumerate(dhs):
        hgs[i] = d.struct()
    ks, epss = _batch_arrays(n, ks, epss)
    if parts_out is None:
        parts_out = [torch.empty(max(d.num_nodes, 1), dtype=torch.int32, device="cuda") for d in dhs]
    outs = (ctypes.c_void_p * max(n, 1))(*[p.data_ptr() for p in parts_out])
    cuts = np.zeros(max(n, 1), np.int64)
    reps = (Report * max(n, 1))()
    st = _check(lib().bp_partition_batch_device(n, hgs, ks.ctypes.data, epss.ctypes.data,
                                                None if prm is None else ctypes.byref(prm), outs,
                                                cuts.ctypes.data, reps, _stream()))
    return ([p[:d.num_nodes] for p, d in zip(parts_out, dhs)], [int(c) for c in cuts[:n]], st,
            [reps[i] for i in range(n)])


def schedule_default() -> Schedule:
    s = Schedule()
    lib().bp_schedule_default(ctypes.byref(s))
    return s


def schedule_get() -> Schedule:
    s = Schedule()
    _check(lib().bp_schedule_get(ctypes.byref(s)))
    return s


def schedule_set(s: Schedule):
    _check(lib().bp_schedule_set(ctypes.byref(s)))


def autotune_batch_device(dhs, ks, epss, prm: Params | None = None, trials=1):
    """Fastest launch schedule for this batch: returns (Schedule, best ms)."""
    import torch
    n = len(dhs)
    hgs = (Hypergraph * max(n, 1))()
    for i, d in enumerate(dhs):
        hgs[i] = d.struct()
    ks, epss = _batch_arrays(n, ks, epss)
    scratch = [torch.empty(max(d.num_nodes, 1), dtype=torch.int32, device="cuda") for d in dhs]
    outs = (ctypes.c_void_p * max(n, 1))(*[p.data_ptr() for p in scratch])
    best = Schedule()
    ms = ctypes.c_double(0)
    _check(lib().bp_autotune_batch_device(n, hgs, ks.ctypes.data, epss.ctypes.data,
                                          None if prm is None else ctypes.byref(prm), outs, trials,
                                          ctypes.byref(best), ctypes.byref(ms), _stream()))
    return best, float(ms.value)


def compute_cut_device(dh: DeviceHypergraph, part, k):
    hg = dh.struct()
    cut, mw = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().bp_compute_cut_device(ctypes.byref(hg), k, part.data_ptr(), ctypes.byref(cut),
                                       ctypes.byref(mw), _stream()))
    return int(cut.value), int(mw.value)


def step_match(dh: DeviceHypergraph, policy=LDH):
    import torch
    out = torch.empty(max(dh.num_nodes, 1), dtype=torch.int32, device="cuda")
    hg = dh.struct()
    _check(lib().bp_step_match(ctypes.byref(hg), policy, out.data_ptr(), _stream()))
    return out[:dh.num_nodes]


def step_coarsen(dh: DeviceHypergraph, policy=LDH):
    """Returns (parent, c_offsets, c_pins, c_node_w, c_hedge_w) as tensors."""
    import torch
    n, e = dh.num_nodes, dh.num_hedges
    p = int(dh.offsets[-1].item())
    mk = lambda m: torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
    parent, coff, cpins, cnw, chw = mk(n), mk(e + 1), mk(p), mk(n), mk(e)
    cn, ce = ctypes.c_int32(0), ctypes.c_int32(0)
    hg = dh.struct()
    _check(lib().bp_step_coarsen(ctypes.byref(hg), policy, parent.data_ptr(), coff.data_ptr(),
                                 cpins.data_ptr(), cnw.data_ptr(), chw.data_ptr(), ctypes.byref(cn),
                                 ctypes.byref(ce), _stream()))
    cn, ce = cn.value, ce.value
    coff = coff[:ce + 1]
    return parent[:n], coff, cpins[:int(coff[-1].item())], cnw[:cn], chw[:ce]


def step_gains(dh: DeviceHypergraph, side):
    import torch
    out = torch.empty(max(dh.num_nodes, 1), dtype=torch.int32, device="cuda")
    hg = dh.struct()
    _check(lib().bp_step_gains(ctypes.byref(hg), side.data_ptr(), out.data_ptr(), _stream()))
    return out[:dh.num_nodes]


def step_initial(dh: DeviceHypergraph, k0, k1):
    import torch
    side = torch.empty(max(dh.num_nodes, 1), dtype=torch.uint8, device="cuda")
    hg = dh.struct()
    _check(lib().bp_step_initial(ctypes.byref(hg), k0, k1, side.data_ptr(), _stream()))
    return side[:dh.num_nodes]


def step_refine(dh: DeviceHypergraph, side, max0, max1, iters=2):
    """Refines side (uint8 tensor) in place; returns the stuck flag."""
    stuck = ctypes.c_int32(0)
    hg = dh.struct()
    _check(lib().bp_step_refine(ctypes.byref(hg), iters, max0, max1, side.data_ptr(),
                                ctypes.byref(stuck), _stream()))
    return stuck.value


def step_bisect(dh: DeviceHypergraph, k0, k1, F, prm: Params | None = None):
    import torch
    side = torch.empty(max(dh.num_nodes, 1), dtype=torch.uint8, device="cuda")
    lv = ctypes.c_int32(0)
    hg = dh.struct()
    _check(lib().bp_step_bisect(ctypes.byref(hg), k0, k1, F, None if prm is None else ctypes.byref(prm),
                                side.data_ptr(), ctypes.byref(lv), _stream()))
    return side[:dh.num_nodes], lv.value


def profile_enable(on=True):
    lib().bp_profile_enable(1 if on else 0)


def profile_reset():
    lib().bp_profile_reset()


def profile_floor(n=200):
    """Times n empty launches under the family "event_floor"."""
    _check(lib().bp_profile_floor(n, _stream()))


def profile_read():
    n = lib().bp_profile_read(None, 0)
    arr = (KernelStat * max(n, 1))()
    n = lib().bp_profile_read(ctypes.cast(arr, ctypes.c_void_p), n)
    return [{"name": arr[i].name.decode(), "launches": arr[i].launches,
             "total_ms": arr[i].total_ms, "bytes": arr[i].bytes} for i in range(n)]
