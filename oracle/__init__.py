"""ctypes wrapper of the sequential C oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It compiles ``bipart_oracle.c`` with gcc into
``liboracle.so`` next to it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bipart_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

LDH, HDH, LWD, HWD, RAND = 0, 1, 2, 3, 4


def build() -> str:
    """Compile the oracle (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared", _SRC,
           "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("refine_iters", ctypes.c_int32), ("min_coarse_nodes", ctypes.c_int32)]


def params(policy=LDH, max_levels=25, refine_iters=2, min_coarse_nodes=100) -> Params:
    return Params(policy, max_levels, refine_iters, min_coarse_nodes)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        _lib.oracle_hash32.argtypes = [ctypes.c_uint32]
        _lib.oracle_hash32.restype = ctypes.c_uint32
        _lib.oracle_cut.argtypes = [i32, i32, P, P, P, P, i32, P, P]
        _lib.oracle_cut.restype = i64
        _lib.oracle_match.argtypes = [i32, i32, P, P, P, i32, P]
        _lib.oracle_coarsen.argtypes = [i32, i32, P, P, P, P, i32, P, P, P, P, P, P, P]
        _lib.oracle_gains.argtypes = [i32, i32, P, P, P, P, P]
        _lib.oracle_bounds.argtypes = [i64, i32, i32, u64, P, P]
        _lib.oracle_initial.argtypes = [i32, i32, P, P, P, P, i32, i32, P]
        _lib.oracle_refine.argtypes = [i32, i32, P, P, P, P, i32, i64, i64, P]
        _lib.oracle_refine.restype = i32
        _lib.oracle_bisect.argtypes = [i32, i32, P, P, P, P, i32, i32, u64, P, P, P]
        _lib.oracle_eps_factor.argtypes = [i32, f64]
        _lib.oracle_eps_factor.restype = u64
        _lib.oracle_partition.argtypes = [i32, i32, P, P, P, P, i32, f64, P, P, P]
        _lib.oracle_partition.restype = i32
    return _lib


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def hash32(x: int) -> int:
    return int(_load().oracle_hash32(x & 0xFFFFFFFF))


def cut(n, off, pins, part, k, hw=None, nw=None):
    """Returns (cut, heaviest part weight)."""
    off, pins, part, hw, nw = _i32(off), _i32(pins), _i32(part), _i32(hw), _i32(nw)
    mw = ctypes.c_int64(0)
    c = _load().oracle_cut(n, len(off) - 1, _ptr(off), _ptr(pins), _ptr(nw), _ptr(hw), k,
                           _ptr(part), ctypes.byref(mw))
    return int(c), int(mw.value)


def match(n, off, pins, hw=None, policy=LDH):
    off, pins, hw = _i32(off), _i32(pins), _i32(hw)
    out = np.empty(n, np.int32)
    _load().oracle_match(n, len(off) - 1, _ptr(off), _ptr(pins), _ptr(hw), policy, _ptr(out))
    return out


def coarsen(n, off, pins, nw=None, hw=None, policy=LDH):
    """One coarsening step: returns (parent, c_off, c_pins, c_nw, c_hw)."""
    off, pins, nw, hw = _i32(off), _i32(pins), _i32(nw), _i32(hw)
    e = len(off) - 1
    p = int(off[-1]) if e else 0
    parent = np.empty(n, np.int32)
    c_off = np.empty(e + 1, np.int32)
    c_pins = np.empty(max(p, 1), np.int32)
    c_nw = np.empty(max(n, 1), np.int32)
    c_hw = np.empty(max(e, 1), np.int32)
    cn, ce = ctypes.c_int32(0), ctypes.c_int32(0)
    _load().oracle_coarsen(n, e, _ptr(off), _ptr(pins), _ptr(nw), _ptr(hw), policy,
                           _ptr(parent), ctypes.byref(cn), ctypes.byref(ce), _ptr(c_off),
                           _ptr(c_pins), _ptr(c_nw), _ptr(c_hw))
    cn, ce = cn.value, ce.value
    c_off = c_off[:ce + 1].copy()
    return parent, c_off, c_pins[:c_off[-1]].copy(), c_nw[:cn].copy(), c_hw[:ce].copy()


def gains(n, off, pins, side, hw=None):
    off, pins, hw = _i32(off), _i32(pins), _i32(hw)
    side = np.ascontiguousarray(side, dtype=np.uint8)
    out = np.empty(n, np.int32)
    _load().oracle_gains(n, len(off) - 1, _ptr(off), _ptr(pins), _ptr(hw), _ptr(side), _ptr(out))
    return out


def bounds(total_w, k0, k1, F):
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    _load().oracle_bounds(total_w, k0, k1, F, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def eps_factor(k, eps) -> int:
    return int(_load().oracle_eps_factor(k, eps))


def initial(n, off, pins, k0, k1, nw=None, hw=None):
    off, pins, nw, hw = _i32(off), _i32(pins), _i32(nw), _i32(hw)
    side = np.empty(n, np.uint8)
    _load().oracle_initial(n, len(off) - 1, _ptr(off), _ptr(pins), _ptr(nw), _ptr(hw), k0, k1,
                           _ptr(side))
    return side


def refine(n, off, pins, side, max0, max1, iters=2, nw=None, hw=None):
    """Returns (new side, stuck flag)."""
    off, pins, nw, hw = _i32(off), _i32(pins), _i32(nw), _i32(hw)
    s = np.array(side, dtype=np.uint8, copy=True)
    stuck = _load().oracle_refine(n, len(off) - 1, _ptr(off), _ptr(pins), _ptr(nw), _ptr(hw),
                                  iters, max0, max1, _ptr(s))
    return s, int(stuck)


def bisect(n, off, pins, k0, k1, F, nw=None, hw=None, prm: Params | None = None):
    """Returns (side, coarsening steps taken)."""
    off, pins, nw, hw = _i32(off), _i32(pins), _i32(nw), _i32(hw)
    side = np.empty(n, np.uint8)
    lv = ctypes.c_int32(0)
    prm = prm or params()
    _load().oracle_bisect(n, len(off) - 1, _ptr(off), _ptr(pins), _ptr(nw), _ptr(hw), k0, k1, F,
                          ctypes.byref(prm), _ptr(side), ctypes.byref(lv))
    return side, lv.value


def partition(n, off, pins, k, eps, nw=None, hw=None, prm: Params | None = None):
    """Full k-way partition: returns (part, cut)."""
    off, pins, nw, hw = _i32(off), _i32(pins), _i32(nw), _i32(hw)
    part = np.empty(max(n, 1), np.int32)
    c = ctypes.c_int64(0)
    prm = prm or params()
    rc = _load().oracle_partition(n, len(off) - 1, _ptr(off), _ptr(pins), _ptr(nw), _ptr(hw), k,
                                  eps, ctypes.byref(prm), _ptr(part), ctypes.byref(c))
    if rc != 0:
        raise ValueError("oracle_partition rejected its arguments")
    return part[:n].copy(), int(c.value)


def partition_hg(h, k=None, eps=None, prm: Params | None = None):
    """Convenience: partition an inputs.Hypergraph with its own k/eps."""
    k = h.meta.get("k", 2) if k is None else k
    eps = h.meta.get("eps", 0.05) if eps is None else eps
    return partition(h.num_nodes, h.offsets, h.pins, k, eps, h.node_w, h.hedge_w, prm)
